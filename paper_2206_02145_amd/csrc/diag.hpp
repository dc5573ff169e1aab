// diag.hpp -- initial state, field read-back, raw population I/O and the diagnostics
// (binary64 reductions of mass, volume and velocity; crystal-size ray-march).
#pragma once

#include <hip/hip_fp16.h>
#include <hip/hip_runtime.h>

#include "lattice.hpp"
#include "mem.hpp"
#include "step.hpp"

namespace lbcg {

struct SeedArgs {
    double cx, cy, cz, R, W0, U0, u_in, tilt;
    int shape;  // lbcg_seed_shape
};

// Signed distance to the seed surface (negative inside) for the offset (dx, dy, dz) from its
// centre: the sphere, or the largest distance to the face planes of the tilted polygon (and, in
// 3-D, to the planes z = +-apothem of its prism).
template <int DIM>
__device__ inline double seed_distance(const SeedArgs& s, double dx, double dy, double dz) {
    if (s.shape == 0) return sqrt(dx * dx + dy * dy + dz * dz) - s.R;
    const double pi = 3.141592653589793;
    const int n = s.shape == 1 ? 6 : 4;
    const double a = s.R * cos(pi / (s.shape == 1 ? 6 : 3));  // apothem
    double d = -1e300;
    for (int k = 0; k < n; k++) {
        // hexagon: normals at 30 + 60 k degrees; rhombus: 30, 150, 210, 330 degrees (four of them)
        const double deg = s.shape == 1 ? 30.0 + 60.0 * k : (k < 2 ? 30.0 + 120.0 * k : 210.0 + 120.0 * (k - 2));
        const double t = deg * (pi / 180.0) + s.tilt;
        d = fmax(d, cos(t) * dx + sin(t) * dy - a);
    }
    if (DIM == 3) d = fmax(d, fabs(dz) - a);
    return d;
}

// Initial state: phi0 = tanh((R - |x - c|) / (sqrt(2) W0)), h = w phi0, g = w U0,
// f = f_eq(rho = 1, u* = u_in (1 - phi0)/2 x^), phi_prev = phi0; evaluated in binary64 and
// rounded once into the stored deviations (h + w, g - w U0, f - w, phi_prev + 1).
template <int DIM, bool FLOW, typename real, typename fst>
__global__ __launch_bounds__(256) void init_kernel(InstDev I, int par, SeedArgs s) {
    using S = typename Lattices<DIM>::S;
    using V = typename Lattices<DIM>::V;
    const long long N = I.N;
    const Planes<real> h(pick(I.h, par), I.Np), g(pick(I.g, par), I.Np), pp(I.phi_prev, I.Nm);
    const Planes<fst> f(pick(I.f, par), I.Np);
    for (long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x; i < N;
         i += (long long)gridDim.x * blockDim.x) {
        const int x = (int)(i % I.nx);
        const long long r = i / I.nx;
        const int y = (int)(r % I.ny);
        const int z = (int)(r / I.ny);
        const unsigned row = (unsigned)(r * I.pitch);
        const double dx = x - s.cx, dy = y - s.cy, dz = (DIM == 3) ? z - s.cz : 0.0;
        const double phi0 = tanh(-seed_distance<DIM>(s, dx, dy, dz) / (sqrt(2.0) * s.W0));
        pp.st(0, row + (unsigned)x, (real)(phi0 + 1.0));
#pragma unroll
        for (int a = 0; a < S::Q; a++) {
            const unsigned m = row + xmem(x, S::c(a, 0), I.nx);
            h.st(a, m, (real)(S::w(a) * (phi0 + 1.0)));  // h + w
            g.st(a, m, (real)0);                         // g - w U0
        }
        if constexpr (FLOW) {
            const double ux = s.u_in * 0.5 * (1.0 - phi0);
#pragma unroll
            for (int a = 0; a < V::Q; a++) {
                const double cu = V::c(a, 0) * ux;
                const double dev = V::w(a) * (3.0 * cu + 4.5 * cu * cu - 1.5 * ux * ux);  // f_eq - w
                f.st(a, row + xmem(x, V::c(a, 0), I.nx), (real)dev);
            }
        }
    }
}

// Stored index of the node with dense index i = (z ny + y) nx + x.
__device__ __forceinline__ long long stored_node(const InstDev& I, long long i) {
    return (i / I.nx) * I.pitch + i % I.nx;
}

// Moments of one node in the compute precision: psi = phi + 1, Ut = U - U0, rho and u*.
template <int DIM, bool FLOW, typename real, typename fst>
__device__ inline void node_moments(const InstDev& I, int par, long long i, real& psi, real& Ut,
                                    real& rho, real& usx, real& usy, real& usz) {
    using S = typename Lattices<DIM>::S;
    using V = typename Lattices<DIM>::V;
    const Planes<real> h(pick(I.h, par), I.Np), g(pick(I.g, par), I.Np);
    const int x = (int)(i % I.nx);
    const unsigned row = (unsigned)((i / I.nx) * I.pitch);
    psi = 0;
    Ut = 0;
#pragma unroll
    for (int a = 0; a < S::Q; a++) {
        const unsigned m = row + xmem(x, S::c(a, 0), I.nx);
        psi += h.template ld<real>(a, m);
        Ut += g.template ld<real>(a, m);
    }
    rho = 1;
    usx = usy = usz = 0;
    if constexpr (FLOW) {
        const Planes<fst> f(pick(I.f, par), I.Np);
        real drho = 0, mx = 0, my = 0, mz = 0;
#pragma unroll
        for (int a = 0; a < V::Q; a++) {
            const real fa = f.template ld<real>(a, row + xmem(x, V::c(a, 0), I.nx));
            drho += fa;
            if (V::c(a, 0)) mx += (real)V::c(a, 0) * fa;
            if (V::c(a, 1)) my += (real)V::c(a, 1) * fa;
            if (DIM == 3 && V::c(a, 2)) mz += (real)V::c(a, 2) * fa;
        }
        rho = (real)1 + drho;
        const real two_m_psi = (real)2 - psi;
        const real K = (real)I.kdrag * psi * psi * two_m_psi;
        const real iden = (real)1 / (rho + (real)0.5 * K);
        const real hs = (real)0.5 * two_m_psi;
        usx = hs * mx * iden;
        usy = hs * my * iden;
        usz = hs * mz * iden;
    }
}

// One macroscopic field (0 phi, 1 U, 2 rho, 3-5 u*, 6 phi_prev) into out.
template <int DIM, bool FLOW, typename real, typename fst, typename out_t>
__global__ __launch_bounds__(256) void field_kernel(InstDev I, int par, int field, out_t* out) {
    const long long N = I.N;
    const real* pp = static_cast<const real*>(I.phi_prev);
    for (long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x; i < N;
         i += (long long)gridDim.x * blockDim.x) {
        if (field == 6) {
            out[i] = (out_t)((double)pp[stored_node(I, i)] - 1.0);  // psi_prev = phi_prev + 1 (no column shift)
            continue;
        }
        real psi, Ut, rho, ux, uy, uz;
        node_moments<DIM, FLOW, real, fst>(I, par, i, psi, Ut, rho, ux, uy, uz);
        const double v = field == 0 ? (double)psi - 1.0 : field == 1 ? (double)Ut + I.U0
                       : field == 2 ? (double)rho : field == 3 ? (double)ux : field == 4 ? (double)uy : (double)uz;
        out[i] = (out_t)v;
    }
}

// One stored plane to out, decoded to the plain layout: value(x) = stored(column xmem(x, cx)) + shift
// (h: -w, g: w U0, f: w).
template <typename real, typename st, typename out_t>
__global__ __launch_bounds__(256) void raw_read_kernel(const st* src, long long n, int nx, int pitch, long long nm,
                                                       int cx, double shift, out_t* out) {
    const Planes<st> P(src, nm);
    for (long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x; i < n;
         i += (long long)gridDim.x * blockDim.x) {
        const int x = (int)(i % nx);
        const unsigned row = (unsigned)((i / nx) * pitch);
        out[i] = (out_t)((double)P.template ld<real>(0, row + xmem(x, cx, nx)) + shift);
    }
}

// One plane from the plain layout, encoded: stored(column xmem(x, cx)) = value(x) - shift, rounded once.
template <typename real, typename st, typename in_t>
__global__ __launch_bounds__(256) void raw_write_kernel(st* dst, long long n, int nx, int pitch, long long nm, int cx,
                                                        double shift, const in_t* in) {
    const Planes<st> P(dst, nm);
    for (long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x; i < n;
         i += (long long)gridDim.x * blockDim.x) {
        const int x = (int)(i % nx);
        const unsigned row = (unsigned)((i / nx) * pitch);
        P.st(0, row + xmem(x, cx, nx), (real)((double)in[i] - shift));
    }
}

// ---- reductions (binary64 accumulation) ----
constexpr int RED_THREADS = 256;
constexpr int RED_VALUES = 6;  // sumU, sumPhiPrev, Vs, M', max|u*|, nonfinite

__device__ inline double wave_sum(double v) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
    return v;
}
__device__ inline double wave_max(double v) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v = fmax(v, __shfl_xor(v, o, 64));
    return v;
}

template <int DIM, bool FLOW, typename real, typename fst>
__global__ __launch_bounds__(RED_THREADS) void reduce_kernel(InstDev I, int par, double* partials) {
    const long long N = I.N;
    const real* pp = static_cast<const real*>(I.phi_prev);
    double acc[RED_VALUES] = {0, 0, 0, 0, 0, 0};
    for (long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x; i < N;
         i += (long long)gridDim.x * blockDim.x) {
        const long long m = stored_node(I, i);
        if (I.wall && I.wall[m]) continue;  // the sums cover the fluid and the crystal
        real psi, Ut, rho, ux, uy, uz;
        node_moments<DIM, FLOW, real, fst>(I, par, i, psi, Ut, rho, ux, uy, uz);
        const double U = (double)Ut + I.U0;
        const double psi_prev = (double)pp[m];  // phi_prev + 1
        acc[0] += U;
        acc[1] += psi_prev - 1.0;
        acc[2] += 0.5 * (double)psi;      // (1 + phi) / 2
        acc[3] += U + I.kd[K_SRC] * psi_prev;  // U + B (1 + phi_prev)
        const double um = sqrt((double)ux * ux + (double)uy * uy + (double)uz * uz);
        acc[4] = fmax(acc[4], um);
        if (!isfinite((double)psi) || !isfinite((double)Ut) || !isfinite((double)rho)) acc[5] += 1.0;
    }
    __shared__ double s[RED_THREADS / 64][RED_VALUES];
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
#pragma unroll
    for (int k = 0; k < RED_VALUES; k++) {
        const double v = (k == 4) ? wave_max(acc[k]) : wave_sum(acc[k]);
        if (lane == 0) s[wv][k] = v;
    }
    __syncthreads();
    if (threadIdx.x < RED_VALUES) {
        const int k = threadIdx.x;
        double v = s[0][k];
        for (int w = 1; w < RED_THREADS / 64; w++) v = (k == 4) ? fmax(v, s[w][k]) : v + s[w][k];
        partials[blockIdx.x * RED_VALUES + k] = v;
    }
}

// Fixed-order sum of the block partials (deterministic for a given launch shape): lane l sums the
// partials of blocks l, l + 64, l + 128, ... in that order, then lane k combines value k of the 64
// lane sums in lane order. (One lane walking all partials in order waits on one dependent load per
// block: ~150 us for 1024 blocks.)
static __global__ __launch_bounds__(64) void reduce_final(const double* partials, int nblocks, double* out) {
    __shared__ double s[RED_VALUES][64];
    const int l = threadIdx.x;
    double v[RED_VALUES];
#pragma unroll
    for (int k = 0; k < RED_VALUES; k++) v[k] = 0;
    for (int b = l; b < nblocks; b += 64) {
#pragma unroll
        for (int k = 0; k < RED_VALUES; k++) {
            const double p = partials[b * RED_VALUES + k];
            v[k] = (k == 4) ? fmax(v[k], p) : v[k] + p;
        }
    }
#pragma unroll
    for (int k = 0; k < RED_VALUES; k++) s[k][l] = v[k];
    __syncthreads();
    if (l < RED_VALUES) {
        double a = 0;
        for (int j = 0; j < 64; j++) a = (l == 4) ? fmax(a, s[l][j]) : a + s[l][j];
        out[l] = a;
    }
}

// ---- crystal size: ray-march along directions from the seed centre ----
template <int DIM, typename real>
__device__ inline double phi_node(const InstDev& I, const real* h, int x, int y, int z) {
    using S = typename Lattices<DIM>::S;
    const long long row = ((long long)z * I.ny + y) * I.pitch;
    double psi = 0;
#pragma unroll
    for (int a = 0; a < S::Q; a++) psi += (double)h[a * I.Np + row + xmem(x, S::c(a, 0), I.nx)];
    return psi - 1.0;
}

template <int DIM, typename real>
__device__ inline double phi_interp(const InstDev& I, const real* h, const double* pt) {
    const int n[3] = {I.nx, I.ny, I.nz};
    int i0[3], i1[3];
    double t[3];
    for (int d = 0; d < 3; d++) {
        const double fl = floor(pt[d]);
        i0[d] = (int)fl;
        t[d] = pt[d] - fl;
        if (i0[d] > n[d] - 1) i0[d] = n[d] - 1;
        if (i0[d] < 0) i0[d] = 0;
        i1[d] = (i0[d] + 1 < n[d]) ? i0[d] + 1 : n[d] - 1;
    }
    double v = 0;
    for (int cz = 0; cz < (DIM == 3 ? 2 : 1); cz++)
        for (int cy = 0; cy < 2; cy++)
            for (int cx = 0; cx < 2; cx++) {
                const double wgt = (cx ? t[0] : 1 - t[0]) * (cy ? t[1] : 1 - t[1]) *
                                   (DIM == 3 ? (cz ? t[2] : 1 - t[2]) : 1.0);
                if (wgt == 0.0) continue;
                v += wgt * phi_node<DIM, real>(I, h, cx ? i1[0] : i0[0], cy ? i1[1] : i0[1],
                                               DIM == 3 ? (cz ? i1[2] : i0[2]) : 0);
            }
    return v;
}

// Crystal extent along one direction dv from centre c, computed by one 64-lane wavefront. Lane j
// of a round tests sample j+1: the first sample that leaves the domain or has phi <= 0 ends the
// ray (all earlier samples have phi > 0). Lane 0 writes the result.
template <int DIM, typename real>
__device__ inline void raymarch_one(const InstDev& I, int par, const double* dv_in, const double* c_in,
                                    double* L_out) {
    const int lane = threadIdx.x;
    const real* h = static_cast<const real*>(pick(I.h, par));
    const double ds = 0.25;
    const double c[3] = {c_in[0], c_in[1], DIM == 3 ? c_in[2] : 0.0};
    const double dv[3] = {dv_in[0], dv_in[1], DIM == 3 ? dv_in[2] : 0.0};
    const double n[3] = {(double)I.nx, (double)I.ny, (double)I.nz};
    const double phic = phi_interp<DIM, real>(I, h, c);
    if (!(phic > 0.0)) {
        if (lane == 0) *L_out = 0.0;
        return;
    }
    for (long long base = 0;; base += 64) {
        const long long j = base + lane;
        const double s1 = (double)(j + 1) * ds;
        const double pt[3] = {c[0] + s1 * dv[0], c[1] + s1 * dv[1], c[2] + s1 * dv[2]};
        bool out = false;
        for (int d = 0; d < (DIM == 3 ? 3 : 2); d++)
            if (pt[d] < 0.0 || pt[d] > n[d] - 1) out = true;
        double cur = 1.0;
        if (!out) cur = phi_interp<DIM, real>(I, h, pt);
        const bool ev = out || !(cur > 0.0);
        const unsigned long long mask = __ballot(ev);
        if (mask) {
            const int first = __ffsll((long long)mask) - 1;
            if (lane == first) {
                const double sj = (double)j * ds;
                double L;
                if (out) {
                    L = sj;
                } else {
                    const double p0[3] = {c[0] + sj * dv[0], c[1] + sj * dv[1], c[2] + sj * dv[2]};
                    const double prev = (j == 0) ? phic : phi_interp<DIM, real>(I, h, p0);
                    L = sj + ds * prev / (prev - cur);
                }
                *L_out = L;
            }
            return;
        }
    }
}

// One workgroup per direction.
template <int DIM, typename real>
__global__ __launch_bounds__(64) void raymarch_kernel(InstDev I, int par, const double* dirs,
                                                      double cx, double cy, double cz, double* L_out) {
    const int k = blockIdx.x;
    const double c[3] = {cx, cy, cz};
    raymarch_one<DIM, real>(I, par, dirs + 3 * k, c, L_out + k);
}

// Batched: workgroup (k, i) marches direction k of instance i from that instance's seed centre;
// out[i * ndirs + k].
template <int DIM, typename real>
__global__ __launch_bounds__(64) void raymarch_batch_kernel(const InstDev* __restrict__ insts, int par,
                                                            const double* dirs, int ndirs,
                                                            const double* centers, double* out) {
    const int k = blockIdx.x, i = blockIdx.y;
    const InstDev I = insts[i];
    raymarch_one<DIM, real>(I, par, dirs + 3 * k, centers + 3 * i, out + (size_t)i * ndirs + k);
}

}  // namespace lbcg
