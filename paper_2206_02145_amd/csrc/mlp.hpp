// mlp.hpp -- kernels of the growth-rate surrogate: a multilayer perceptron trained and evaluated
// with bf16 MFMA (v_mfma_f32_16x16x32_bf16, fp32 accumulation) on gfx950.
//
// Precision contract (the CPU reference mirrors it exactly): every GEMM operand is bf16 (weights
// rounded from fp32 master copies; activations and back-propagated gradients rounded after their
// fp32 epilogue), every accumulation and every elementwise op is fp32.
#pragma once

#include <hip/hip_bf16.h>
#include <hip/hip_runtime.h>

namespace lbcg {
namespace mlp {

typedef __bf16 bf16;
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float f32x4 __attribute__((ext_vector_type(4)));

__device__ __forceinline__ float silu(float z) { return z / (1.0f + expf(-z)); }
__device__ __forceinline__ float dsilu(float z) {
    const float s = 1.0f / (1.0f + expf(-z));
    return s * (1.0f + z * (1.0f - s));
}
__device__ __forceinline__ bf16 to_bf16(float v) { return (bf16)v; }  // round to nearest even

enum Epi { EPI_FWD_HIDDEN = 0, EPI_FWD_OUT = 1, EPI_BWD_DX = 2, EPI_DW = 3 };

struct GemmArgs {
    int M, N, K;
    const bf16* A;  // A(i, k) = A[i * lda_i + k * lda_k]
    long long lda_i, lda_k;
    const bf16* B;  // B(k, n) = B[k * ldb_k + n * ldb_n]
    long long ldb_k, ldb_n;
    // epilogue operands (row-major M x N unless noted)
    const float* bias;  // [N]            (forward)
    float* z;           // pre-activation (forward: written; backward: read, previous layer)
    bf16* out_bf16;     // activation / back-propagated gradient
    float* out_f32;     // output layer / weight gradient
    int kchunk;          // K range of one split (blockIdx.z), a multiple of the K tile; >= K: no split
    long long split_stride;  // weight gradient: elements between the partial sums of two splits
};

constexpr int GEMM_TK = 32;

// Stage a 64 x 32 operand tile X(r, k) = X[r * ld_r + k * ld_k], rows r0 .. r0 + 63 (< R) and
// k0 .. k0 + 31 (< kend), into sX[r][k], zero outside. The 256 threads take 8 consecutive elements
// each along the operand's unit-stride index (one 16-byte load when vec: that stride is 1, the
// other a multiple of 8 and the base 16-byte aligned); neither stride 1: one element at a time.
__device__ inline void stage_tile(bf16 (*sX)[GEMM_TK + 8], const bf16* X, long long ld_r, long long ld_k, int r0,
                                  int R, int k0, int kend, bool kfast, bool rfast, bool vec, int tid) {
    if (kfast) {  // 8 consecutive k of one row
        const int r = tid >> 2, k = (tid & 3) * 8;
        const int gr = r0 + r, gk = k0 + k;
        bf16x8 v;
        if (vec && gr < R && gk + 8 <= kend) {
            v = *reinterpret_cast<const bf16x8*>(X + gr * ld_r + gk);
        } else {
#pragma unroll
            for (int j = 0; j < 8; j++) v[j] = (gr < R && gk + j < kend) ? X[gr * ld_r + gk + j] : (bf16)0.0f;
        }
        *reinterpret_cast<bf16x8*>(&sX[r][k]) = v;
    } else if (rfast) {  // 8 consecutive rows of one k
        const int r = (tid & 7) * 8, k = tid >> 3;
        const int gr = r0 + r, gk = k0 + k;
        bf16x8 v;
        if (vec && gk < kend && gr + 8 <= R) {
            v = *reinterpret_cast<const bf16x8*>(X + gk * ld_k + gr);
        } else {
#pragma unroll
            for (int j = 0; j < 8; j++) v[j] = (gk < kend && gr + j < R) ? X[gk * ld_k + gr + j] : (bf16)0.0f;
        }
#pragma unroll
        for (int j = 0; j < 8; j++) sX[r + j][k] = v[j];
    } else {
#pragma unroll
        for (int e = 0; e < 8; e++) {
            const int idx = tid + 256 * e;
            const int r = idx / GEMM_TK, k = idx % GEMM_TK;
            const int gr = r0 + r, gk = k0 + k;
            sX[r][k] = (gr < R && gk < kend) ? X[gr * ld_r + gk * ld_k] : (bf16)0.0f;
        }
    }
}

// C = A B for a 64 x 64 tile per workgroup (4 wavefronts x 16 rows, 4 MFMA blocks of 16 columns).
template <int EPI>
__global__ __launch_bounds__(256) void gemm_bf16(GemmArgs g) {
    constexpr int TM = 64, TN = 64, TK = GEMM_TK;
    __shared__ __align__(16) bf16 sA[TM][TK + 8];  // A tile, k contiguous
    __shared__ __align__(16) bf16 sB[TN][TK + 8];  // B tile transposed (n, k), k contiguous
    const int tid = threadIdx.x;
    const int lane = tid & 63, wv = tid >> 6;
    const int m0 = blockIdx.y * TM, n0 = blockIdx.x * TN;
    f32x4 acc[4];
#pragma unroll
    for (int b = 0; b < 4; b++) acc[b] = f32x4{0.f, 0.f, 0.f, 0.f};

    const int kbeg = blockIdx.z * g.kchunk;
    const int kend = min(g.K, kbeg + g.kchunk);
    // consecutive threads walk each operand's unit-stride index (coalesced, 16-byte loads)
    const bool a_kf = g.lda_k == 1, a_rf = !a_kf && g.lda_i == 1;
    const bool b_kf = g.ldb_k == 1, b_rf = !b_kf && g.ldb_n == 1;
    const auto aligned = [](const bf16* p) { return (reinterpret_cast<uintptr_t>(p) & 15) == 0; };
    const bool a_vec = aligned(g.A) && (a_kf ? g.lda_i % 8 == 0 : g.lda_k % 8 == 0);
    const bool b_vec = aligned(g.B) && (b_kf ? g.ldb_n % 8 == 0 : g.ldb_k % 8 == 0);
    for (int k0 = kbeg; k0 < kend; k0 += TK) {
        // stage: 64x32 of A and 32x64 of B (8 elements each per thread), zero outside the matrix
        stage_tile(sA, g.A, g.lda_i, g.lda_k, m0, g.M, k0, kend, a_kf, a_rf, a_vec, tid);
        stage_tile(sB, g.B, g.ldb_n, g.ldb_k, n0, g.N, k0, kend, b_kf, b_rf, b_vec, tid);
        __syncthreads();
        // fragments: lane holds A(i = lane%16, k = 8*(lane/16) + j), B(k = 8*(lane/16) + j, n = lane%16)
        const int r = lane & 15, kq = 8 * (lane >> 4);
        bf16x8 af;
#pragma unroll
        for (int j = 0; j < 8; j++) af[j] = sA[16 * wv + r][kq + j];
#pragma unroll
        for (int b = 0; b < 4; b++) {
            bf16x8 bfr;
#pragma unroll
            for (int j = 0; j < 8; j++) bfr[j] = sB[16 * b + r][kq + j];
            acc[b] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(af, bfr, acc[b], 0, 0, 0);
        }
        __syncthreads();
    }
    // epilogue: lane holds C(i = 4*(lane/16) + q, n = lane%16) of each 16x16 block
#pragma unroll
    for (int b = 0; b < 4; b++) {
#pragma unroll
        for (int q = 0; q < 4; q++) {
            const int i = m0 + 16 * wv + 4 * (lane >> 4) + q;
            const int n = n0 + 16 * b + (lane & 15);
            if (i >= g.M || n >= g.N) continue;
            const long long o = (long long)i * g.N + n;
            const float c = acc[b][q];
            if constexpr (EPI == EPI_FWD_HIDDEN) {
                const float zz = c + g.bias[n];
                g.z[o] = zz;
                g.out_bf16[o] = to_bf16(silu(zz));
            } else if constexpr (EPI == EPI_FWD_OUT) {
                g.out_f32[o] = c + g.bias[n];
            } else if constexpr (EPI == EPI_BWD_DX) {
                // dA of the previous layer times the derivative of its activation
                g.out_bf16[o] = to_bf16(c * dsilu(g.z[o]));
            } else {
                g.out_f32[blockIdx.z * g.split_stride + o] = c;
            }
        }
    }
}

// Gaussian negative log-likelihood with a mean head y[:, :D] and a log-variance head y[:, D:]
// (log-variance clamped to [-12, 12]): L = (1/(B D)) sum 0.5 (exp(-s) (t - mu)^2 + s).
// Writes dL/dy (bf16, B x 2D) and per-block partial sums of L.
__global__ __launch_bounds__(256) void nll_kernel(int B, int D, const float* y, const float* t, bf16* dy,
                                                  float* partial) {
    const int idx = blockIdx.x * 256 + threadIdx.x;
    float l = 0.f;
    if (idx < B * D) {
        const int b = idx / D, d = idx % D;
        const float mu = y[(long long)b * 2 * D + d];
        const float s_raw = y[(long long)b * 2 * D + D + d];
        const bool in = s_raw > -12.f && s_raw < 12.f;
        const float s = in ? s_raw : (s_raw <= -12.f ? -12.f : 12.f);
        const float e = expf(-s);
        const float r = t[idx] - mu;
        const float inv = 1.0f / (float)(B * D);
        l = 0.5f * (e * r * r + s) * inv;
        dy[(long long)b * 2 * D + d] = to_bf16(-e * r * inv);
        dy[(long long)b * 2 * D + D + d] = to_bf16(in ? 0.5f * (1.0f - e * r * r) * inv : 0.f);
    }
    __shared__ float sh[256];
    sh[threadIdx.x] = l;
    __syncthreads();
    for (int o = 128; o > 0; o >>= 1) {
        if (threadIdx.x < o) sh[threadIdx.x] += sh[threadIdx.x + o];
        __syncthreads();
    }
    if (threadIdx.x == 0) partial[blockIdx.x] = sh[0];
}

// Sum of the split-K partial products of the weight gradient, in split order.
__global__ __launch_bounds__(256) void split_sum_kernel(long long n, int S, const float* part, float* out) {
    const long long i = blockIdx.x * 256LL + threadIdx.x;
    if (i >= n) return;
    float s = part[i];
    for (int k = 1; k < S; k++) s += part[k * n + i];
    out[i] = s;
}

// Bias gradient db[n] = sum_b dz[b, n]: a workgroup of 16 wavefronts takes 64 columns (lane =
// column, coalesced rows); wavefront w sums rows w, w + 16, ..., then the 16 partial sums are added
// in wavefront order (a fixed order for a given B).
constexpr int BG_WAVES = 16;
__global__ __launch_bounds__(64 * BG_WAVES) void bias_grad_kernel(int B, int N, const bf16* dz, float* db) {
    __shared__ float s[BG_WAVES][64];
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    const int n = blockIdx.x * 64 + lane;
    float acc = 0.f;
    if (n < N) {
#pragma unroll 8
        for (int b = wv; b < B; b += BG_WAVES) acc += (float)dz[(long long)b * N + n];
    }
    s[wv][lane] = acc;
    __syncthreads();
    if (wv == 0 && n < N) {
        float t = 0.f;
        for (int w = 0; w < BG_WAVES; w++) t += s[w][lane];
        db[n] = t;
    }
}

// Gather rows idx[b] of the dataset X (rows of width W) into out (fp32 -> bf16 for the input layer).
__global__ __launch_bounds__(256) void gather_kernel(int B, int W, const int* idx, const float* X, bf16* out_bf,
                                                     float* out_f, int rows_total) {
    const long long e = blockIdx.x * 256LL + threadIdx.x;
    if (e >= (long long)B * W) return;
    const int b = (int)(e / W), w = (int)(e % W);
    int r = idx[b];
    r = r < 0 ? 0 : (r >= rows_total ? rows_total - 1 : r);
    const float v = X[(long long)r * W + w];
    if (out_bf) out_bf[e] = to_bf16(v);
    if (out_f) out_f[e] = v;
}

// Adam on the fp32 master copy; refreshes the bf16 copy of weights (wb may be null for biases).
__global__ __launch_bounds__(256) void adam_kernel(long long n, float* w, bf16* wb, const float* g, float* m, float* v,
                                                   float lr, float b1, float b2, float eps, float c1, float c2) {
    const long long i = blockIdx.x * 256LL + threadIdx.x;
    if (i >= n) return;
    const float gi = g[i];
    const float mi = b1 * m[i] + (1.f - b1) * gi;
    const float vi = b2 * v[i] + (1.f - b2) * gi * gi;
    m[i] = mi;
    v[i] = vi;
    const float mh = mi / c1, vh = vi / c2;
    const float wi = w[i] - lr * mh / (sqrtf(vh) + eps);
    w[i] = wi;
    if (wb) wb[i] = to_bf16(wi);
}

__global__ __launch_bounds__(256) void to_bf16_kernel(long long n, const float* src, bf16* dst) {
    const long long i = blockIdx.x * 256LL + threadIdx.x;
    if (i < n) dst[i] = to_bf16(src[i]);
}

}  // namespace mlp
}  // namespace lbcg
