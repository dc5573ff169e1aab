// lbcg_mlp.hip -- host side of the surrogate MLP (include/lbcg.h, lbcg_mlp_*): workspace layout,
// forward / backward / Adam sequencing of the kernels in mlp.hpp on the caller's stream.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <stdexcept>
#include <string>
#include <vector>

#include "../../include/lbcg.h"
#include "errors.hpp"
#include "mlp.hpp"

using namespace lbcg::mlp;

namespace {

struct MErr : std::runtime_error {
    lbcg_status code;
    MErr(lbcg_status c, const std::string& m) : std::runtime_error(m), code(c) {}
};

#define MCHK(call)                                                                                    \
    do {                                                                                              \
        hipError_t e_ = (call);                                                                       \
        if (e_ != hipSuccess) throw MErr(LBCG_EDEVICE, std::string(#call) + ": " + hipGetErrorString(e_)); \
    } while (0)

template <typename F> lbcg_status mguard(F&& fn) {
    try {
        fn();
        lbcg::last_error_slot().clear();
        return LBCG_OK;
    } catch (const MErr& e) {
        lbcg::last_error_slot() = e.what();
        return e.code;
    } catch (const std::exception& e) {
        lbcg::last_error_slot() = e.what();
        return LBCG_EDEVICE;
    }
}

size_t a256(size_t b) { return (b + 255) & ~size_t(255); }

constexpr int SPLIT_MAX = 8;  // most K splits of a weight-gradient GEMM

struct Layer {
    int in, out;
    float *W, *b, *mW, *vW, *mb, *vb, *gW, *gb;
    bf16* Wb;
};

struct Plan {
    std::vector<size_t> off;  // offsets of every buffer, in creation order
    size_t total = 0;
    size_t take(size_t bytes) {
        size_t o = total;
        total += a256(bytes);
        off.push_back(o);
        return o;
    }
};

void check_shape(int nl, const int* w, int max_batch) {
    if (nl < 1 || nl > 16) throw MErr(LBCG_EINVAL, "number of layers must be in [1, 16]");
    if (!w) throw MErr(LBCG_EINVAL, "widths is NULL");
    for (int i = 0; i <= nl; i++)
        if (w[i] < 1 || w[i] > 4096) throw MErr(LBCG_EINVAL, "layer widths must be in [1, 4096]");
    if (w[nl] % 2) throw MErr(LBCG_EINVAL, "the output width must be even (mean and log-variance heads)");
    if (max_batch < 1 || max_batch > (1 << 20)) throw MErr(LBCG_EINVAL, "max_batch must be in [1, 2^20]");
}

int maxw(int nl, const int* w) {
    int m = 0;
    for (int i = 0; i <= nl; i++) m = w[i] > m ? w[i] : m;
    return m;
}

}  // namespace

struct lbcg_mlp {
    int nl;
    std::vector<int> w;
    int maxB;
    char* ws;
    hipStream_t stream;
    std::vector<Layer> layers;
    std::vector<float*> z;   // pre-activations of the hidden layers [maxB x w[l+1]]
    std::vector<bf16*> a;    // a[0] = input, a[l] = activation of hidden layer l-1 (bf16)
    float* y;                // output [maxB x w[nl]]
    float* t;                // gathered targets [maxB x w[nl]/2]
    bf16* dz[2];             // back-propagated gradients (bf16) [maxB x max width]
    float* partial;          // loss partial sums
    float* split;            // split-K partial sums of a weight gradient [SPLIT_MAX x max in*out]
    int64_t step;
};

namespace {

Plan plan_of(int nl, const int* w, int maxB) {
    Plan P;
    for (int l = 0; l < nl; l++) {
        const size_t nw = (size_t)w[l] * w[l + 1], nb = w[l + 1];
        P.take(nw * 4);  // W
        P.take(nb * 4);  // b
        P.take(nw * 4);  // mW
        P.take(nw * 4);  // vW
        P.take(nb * 4);  // mb
        P.take(nb * 4);  // vb
        P.take(nw * 4);  // gW
        P.take(nb * 4);  // gb
        P.take(nw * 2);  // Wb
    }
    for (int l = 0; l + 1 < nl; l++) P.take((size_t)maxB * w[l + 1] * 4);  // z
    for (int l = 0; l < nl; l++) P.take((size_t)maxB * w[l] * 2);          // a
    P.take((size_t)maxB * w[nl] * 4);                                      // y
    P.take((size_t)maxB * (w[nl] / 2) * 4);                                // t
    const int mw = maxw(nl, w);
    P.take((size_t)maxB * mw * 2);
    P.take((size_t)maxB * mw * 2);
    P.take((size_t)((maxB * (w[nl] / 2) + 255) / 256 + 1) * 4);  // partials
    size_t nwmax = 0;
    for (int l = 0; l < nl; l++) nwmax = std::max(nwmax, (size_t)w[l] * w[l + 1]);
    P.take((size_t)SPLIT_MAX * nwmax * 4);  // split-K partial sums
    return P;
}

int blocks(long long n) { return (int)((n + 255) / 256); }

void gemm(int epi, GemmArgs g, hipStream_t s) {
    constexpr int TK = 32;
    if (g.kchunk <= 0) g.kchunk = (g.K + TK - 1) / TK * TK;  // one split
    dim3 grid((g.N + 63) / 64, (g.M + 63) / 64, (g.K + g.kchunk - 1) / g.kchunk);
    switch (epi) {
        case EPI_FWD_HIDDEN: hipLaunchKernelGGL(gemm_bf16<EPI_FWD_HIDDEN>, grid, dim3(256), 0, s, g); break;
        case EPI_FWD_OUT: hipLaunchKernelGGL(gemm_bf16<EPI_FWD_OUT>, grid, dim3(256), 0, s, g); break;
        case EPI_BWD_DX: hipLaunchKernelGGL(gemm_bf16<EPI_BWD_DX>, grid, dim3(256), 0, s, g); break;
        default: hipLaunchKernelGGL(gemm_bf16<EPI_DW>, grid, dim3(256), 0, s, g); break;
    }
}

// forward of a batch already in m->a[0]; output in m->y
void forward(lbcg_mlp* m, int B) {
    for (int l = 0; l < m->nl; l++) {
        const Layer& L = m->layers[l];
        GemmArgs g{};
        g.M = B;
        g.N = L.out;
        g.K = L.in;
        g.A = m->a[l];
        g.lda_i = L.in;
        g.lda_k = 1;
        g.B = L.Wb;  // B(k, n) = W[n, k]
        g.ldb_k = 1;
        g.ldb_n = L.in;
        g.bias = L.b;
        if (l + 1 < m->nl) {
            g.z = m->z[l];
            g.out_bf16 = m->a[l + 1];
            gemm(EPI_FWD_HIDDEN, g, m->stream);
        } else {
            g.out_f32 = m->y;
            gemm(EPI_FWD_OUT, g, m->stream);
        }
    }
}

// loss + backward for the batch in m->a[0] / m->t (forward already run); the loss stays on the
// device as per-block partial sums (loss_of reads it back)
void backward(lbcg_mlp* m, int B) {
    const int D = m->w[m->nl] / 2;
    const int nb = blocks((long long)B * D);
    hipLaunchKernelGGL(nll_kernel, dim3(nb), dim3(256), 0, m->stream, B, D, m->y, m->t, m->dz[0], m->partial);
    int cur = 0;
    for (int l = m->nl - 1; l >= 0; l--) {
        const Layer& L = m->layers[l];
        // gW = dz^T a_l
        GemmArgs gw{};
        gw.M = L.out;
        gw.N = L.in;
        gw.K = B;
        gw.A = m->dz[cur];  // A(i = n, k = b) = dz[b, n]
        gw.lda_i = 1;
        gw.lda_k = L.out;
        gw.B = m->a[l];  // B(k = b, j) = a[b, j]
        gw.ldb_k = L.in;
        gw.ldb_n = 1;
        // split K = B over up to SPLIT_MAX workgroup layers (B = 1024: 8 x 128): a weight
        // gradient has only (out/64) x (in/64) output tiles
        const int S = std::max(1, std::min(SPLIT_MAX, B / 128));
        gw.kchunk = ((B + S - 1) / S + 31) / 32 * 32;
        const int nsplit = (B + gw.kchunk - 1) / gw.kchunk;
        const long long nw = (long long)L.out * L.in;
        if (nsplit > 1) {
            gw.out_f32 = m->split;
            gw.split_stride = nw;
            gemm(EPI_DW, gw, m->stream);
            hipLaunchKernelGGL(split_sum_kernel, dim3(blocks(nw)), dim3(256), 0, m->stream, nw, nsplit, m->split, L.gW);
        } else {
            gw.out_f32 = L.gW;
            gemm(EPI_DW, gw, m->stream);
        }
        hipLaunchKernelGGL(bias_grad_kernel, dim3((L.out + 63) / 64), dim3(64 * BG_WAVES), 0, m->stream, B, L.out,
                           m->dz[cur], L.gb);
        if (l > 0) {
            // dz_{l-1} = (dz W) * silu'(z_{l-1})
            GemmArgs gx{};
            gx.M = B;
            gx.N = L.in;
            gx.K = L.out;
            gx.A = m->dz[cur];
            gx.lda_i = L.out;
            gx.lda_k = 1;
            gx.B = L.Wb;  // B(k = n, j) = W[n, j]
            gx.ldb_k = L.in;
            gx.ldb_n = 1;
            gx.z = m->z[l - 1];
            gx.out_bf16 = m->dz[cur ^ 1];
            gemm(EPI_BWD_DX, gx, m->stream);
            cur ^= 1;
        }
    }
}

// the last batch's loss: sum of the partials in block order (synchronises)
float loss_of(lbcg_mlp* m, int B) {
    const int nb = blocks((long long)B * (m->w[m->nl] / 2));
    std::vector<float> part(nb);
    MCHK(hipMemcpyAsync(part.data(), m->partial, sizeof(float) * nb, hipMemcpyDeviceToHost, m->stream));
    MCHK(hipStreamSynchronize(m->stream));
    double loss = 0;
    for (float p : part) loss += p;
    return (float)loss;
}

void gather(lbcg_mlp* m, int B, const float* X, const float* T, const int* idx, int rows) {
    const int in = m->w[0], D = m->w[m->nl] / 2;
    hipLaunchKernelGGL(gather_kernel, dim3(blocks((long long)B * in)), dim3(256), 0, m->stream, B, in, idx, X, m->a[0],
                       (float*)nullptr, rows);
    if (T)
        hipLaunchKernelGGL(gather_kernel, dim3(blocks((long long)B * D)), dim3(256), 0, m->stream, B, D, idx, T,
                           (bf16*)nullptr, m->t, rows);
}

}  // namespace

extern "C" {

size_t lbcg_mlp_workspace_bytes(int nlayers, const int* widths, int max_batch) {
    try {
        check_shape(nlayers, widths, max_batch);
        return plan_of(nlayers, widths, max_batch).total;
    } catch (...) {
        return 0;
    }
}

lbcg_status lbcg_mlp_create(int nlayers, const int* widths, int max_batch, void* dev_workspace, size_t bytes,
                            void* hip_stream, lbcg_mlp** out) {
    if (out) *out = nullptr;
    lbcg_mlp* m = nullptr;
    lbcg_status st = mguard([&] {
        if (!out) throw MErr(LBCG_EINVAL, "out is NULL");
        check_shape(nlayers, widths, max_batch);
        Plan P = plan_of(nlayers, widths, max_batch);
        if (!dev_workspace || ((uintptr_t)dev_workspace & 255)) throw MErr(LBCG_EINVAL, "workspace NULL or unaligned");
        if (bytes < P.total) throw MErr(LBCG_ENOMEM, "workspace too small: need " + std::to_string(P.total));
        m = new lbcg_mlp();
        m->nl = nlayers;
        m->w.assign(widths, widths + nlayers + 1);
        m->maxB = max_batch;
        m->ws = (char*)dev_workspace;
        m->stream = (hipStream_t)hip_stream;
        m->step = 0;
        size_t k = 0;
        auto nxt = [&]() { return m->ws + P.off[k++]; };
        for (int l = 0; l < nlayers; l++) {
            Layer L;
            L.in = widths[l];
            L.out = widths[l + 1];
            L.W = (float*)nxt();
            L.b = (float*)nxt();
            L.mW = (float*)nxt();
            L.vW = (float*)nxt();
            L.mb = (float*)nxt();
            L.vb = (float*)nxt();
            L.gW = (float*)nxt();
            L.gb = (float*)nxt();
            L.Wb = (bf16*)nxt();
            m->layers.push_back(L);
        }
        for (int l = 0; l + 1 < nlayers; l++) m->z.push_back((float*)nxt());
        for (int l = 0; l < nlayers; l++) m->a.push_back((bf16*)nxt());
        m->y = (float*)nxt();
        m->t = (float*)nxt();
        m->dz[0] = (bf16*)nxt();
        m->dz[1] = (bf16*)nxt();
        m->partial = (float*)nxt();
        m->split = (float*)nxt();
        MCHK(hipMemsetAsync(m->ws, 0, P.total, m->stream));
        MCHK(hipStreamSynchronize(m->stream));
    });
    if (st != LBCG_OK) {
        delete m;
        return st;
    }
    *out = m;
    return LBCG_OK;
}

int64_t lbcg_mlp_num_params(const lbcg_mlp* m) {
    if (!m) return -1;
    int64_t n = 0;
    for (const Layer& L : m->layers) n += (int64_t)L.in * L.out + L.out;
    return n;
}

lbcg_status lbcg_mlp_set_params(lbcg_mlp* m, const float* host_params) {
    return mguard([&] {
        if (!m || !host_params) throw MErr(LBCG_EINVAL, "NULL argument");
        const float* p = host_params;
        for (Layer& L : m->layers) {
            const size_t nw = (size_t)L.in * L.out;
            MCHK(hipMemcpyAsync(L.W, p, nw * 4, hipMemcpyHostToDevice, m->stream));
            p += nw;
            MCHK(hipMemcpyAsync(L.b, p, L.out * 4, hipMemcpyHostToDevice, m->stream));
            p += L.out;
            hipLaunchKernelGGL(to_bf16_kernel, dim3(blocks((long long)nw)), dim3(256), 0, m->stream, (long long)nw, L.W,
                               L.Wb);
            MCHK(hipMemsetAsync(L.mW, 0, nw * 4, m->stream));
            MCHK(hipMemsetAsync(L.vW, 0, nw * 4, m->stream));
            MCHK(hipMemsetAsync(L.mb, 0, L.out * 4, m->stream));
            MCHK(hipMemsetAsync(L.vb, 0, L.out * 4, m->stream));
        }
        MCHK(hipGetLastError());
        MCHK(hipStreamSynchronize(m->stream));
        m->step = 0;
    });
}

lbcg_status lbcg_mlp_get_params(lbcg_mlp* m, float* host_params) {
    return mguard([&] {
        if (!m || !host_params) throw MErr(LBCG_EINVAL, "NULL argument");
        float* p = host_params;
        for (Layer& L : m->layers) {
            const size_t nw = (size_t)L.in * L.out;
            MCHK(hipMemcpyAsync(p, L.W, nw * 4, hipMemcpyDeviceToHost, m->stream));
            p += nw;
            MCHK(hipMemcpyAsync(p, L.b, L.out * 4, hipMemcpyDeviceToHost, m->stream));
            p += L.out;
        }
        MCHK(hipStreamSynchronize(m->stream));
    });
}

lbcg_status lbcg_mlp_forward(lbcg_mlp* m, int B, const float* x, float* y) {
    return mguard([&] {
        if (!m || !x || !y) throw MErr(LBCG_EINVAL, "NULL argument");
        if (B < 1 || B > m->maxB) throw MErr(LBCG_EINVAL, "batch size out of range");
        const int in = m->w[0], out = m->w[m->nl];
        hipLaunchKernelGGL(to_bf16_kernel, dim3(blocks((long long)B * in)), dim3(256), 0, m->stream,
                           (long long)B * in, x, m->a[0]);
        forward(m, B);
        MCHK(hipMemcpyAsync(y, m->y, sizeof(float) * B * out, hipMemcpyDeviceToDevice, m->stream));
        MCHK(hipGetLastError());
    });
}

lbcg_status lbcg_mlp_grads(lbcg_mlp* m, int B, const float* X, const float* T, const int* idx, int rows,
                           float* host_grads, float* loss_out) {
    return mguard([&] {
        if (!m || !X || !T || !idx) throw MErr(LBCG_EINVAL, "NULL argument");
        if (B < 1 || B > m->maxB || rows < 1) throw MErr(LBCG_EINVAL, "batch size out of range");
        gather(m, B, X, T, idx, rows);
        forward(m, B);
        backward(m, B);
        if (loss_out) *loss_out = loss_of(m, B);
        if (host_grads) {
            float* p = host_grads;
            for (Layer& L : m->layers) {
                const size_t nw = (size_t)L.in * L.out;
                MCHK(hipMemcpyAsync(p, L.gW, nw * 4, hipMemcpyDeviceToHost, m->stream));
                p += nw;
                MCHK(hipMemcpyAsync(p, L.gb, L.out * 4, hipMemcpyDeviceToHost, m->stream));
                p += L.out;
            }
            MCHK(hipStreamSynchronize(m->stream));
        }
    });
}

lbcg_status lbcg_mlp_train_step(lbcg_mlp* m, int B, const float* X, const float* T, const int* idx, int rows,
                                float lr, float beta1, float beta2, float eps, float* loss_out) {
    return mguard([&] {
        if (!m || !X || !T || !idx) throw MErr(LBCG_EINVAL, "NULL argument");
        if (B < 1 || B > m->maxB || rows < 1) throw MErr(LBCG_EINVAL, "batch size out of range");
        if (!(lr > 0) || !(beta1 >= 0 && beta1 < 1) || !(beta2 >= 0 && beta2 < 1) || !(eps > 0))
            throw MErr(LBCG_EINVAL, "bad Adam hyper-parameters");
        gather(m, B, X, T, idx, rows);
        forward(m, B);
        backward(m, B);
        m->step++;
        const float c1 = 1.f - std::pow(beta1, (float)m->step), c2 = 1.f - std::pow(beta2, (float)m->step);
        for (Layer& L : m->layers) {
            const long long nw = (long long)L.in * L.out;
            hipLaunchKernelGGL(adam_kernel, dim3(blocks(nw)), dim3(256), 0, m->stream, nw, L.W, L.Wb, L.gW, L.mW, L.vW,
                               lr, beta1, beta2, eps, c1, c2);
            hipLaunchKernelGGL(adam_kernel, dim3(blocks(L.out)), dim3(256), 0, m->stream, (long long)L.out, L.b,
                               (bf16*)nullptr, L.gb, L.mb, L.vb, lr, beta1, beta2, eps, c1, c2);
        }
        MCHK(hipGetLastError());
        if (loss_out) *loss_out = loss_of(m, B);  // the partials are not touched by the update
    });
}

lbcg_status lbcg_mlp_destroy(lbcg_mlp* m) {
    delete m;
    return LBCG_OK;
}

}  // extern "C"
