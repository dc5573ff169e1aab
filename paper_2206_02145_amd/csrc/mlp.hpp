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
};

// C = A B for a 64 x 64 tile per workgroup (4 wavefronts x 16 rows, 4 MFMA blocks of 16 columns).
template <int EPI>
__global__ __launch_bounds__(256) void gemm_bf16(GemmArgs g) {
    constexpr int TM = 64, TN = 64, TK = 32;
    __shared__ bf16 sA[TM][TK + 8];  // A tile, k contiguous
    __shared__ bf16 sB[TN][TK + 8];  // B tile transposed (n, k), k contiguous
    const int tid = threadIdx.x;
    const int lane = tid & 63, wv = tid >> 6;
    const int m0 = blockIdx.y * TM, n0 = blockIdx.x * TN;
    f32x4 acc[4];
#pragma unroll
    for (int b = 0; b < 4; b++) acc[b] = f32x4{0.f, 0.f, 0.f, 0.f};

    for (int k0 = 0; k0 < g.K; k0 += TK) {
        // stage: 64x32 of A and 32x64 of B (8 elements each per thread), zero outside the matrix
#pragma unroll
        for (int e = 0; e < 8; e++) {
            const int idx = tid + 256 * e;  // 0 .. 2047
            const int i = idx / TK, k = idx % TK;
            const int gi = m0 + i, gk = k0 + k;
            sA[i][k] = (gi < g.M && gk < g.K) ? g.A[gi * g.lda_i + gk * g.lda_k] : (bf16)0.0f;
            const int n = idx / TK;  // 0 .. 63
            const int gn = n0 + n;
            sB[n][k] = (gn < g.N && gk < g.K) ? g.B[gk * g.ldb_k + gn * g.ldb_n] : (bf16)0.0f;
        }
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
                g.out_f32[o] = c;
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

// Bias gradient: db[n] = sum_b dz[b, n] (fixed order), one thread per column.
__global__ __launch_bounds__(256) void bias_grad_kernel(int B, int N, const bf16* dz, float* db) {
    const int n = blockIdx.x * 256 + threadIdx.x;
    if (n >= N) return;
    float s = 0.f;
    for (int b = 0; b < B; b++) s += (float)dz[(long long)b * N + n];
    db[n] = s;
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
