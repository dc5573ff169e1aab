// step.hpp -- the fused coupled time step (phase field h, solute g, flow f) for gfx950.
//
// One workgroup updates one tile of TX x TY (x TZ) nodes. Every collision of a step uses time-n
// data only (Section 2.2 couples the lattices through phi, U and u* of the same step), so the three
// lattices are collided and streamed in one pass:
//
//   phase 1: the workgroup loads h^n on the tile plus a one-node halo into LDS and forms
//            phi = sum h there (the halo serves the isotropic gradient and the old-value term of
//            the a_s^2-weighted stream, Eq. (d));
//   phase 2: each thread owns one node: grad phi from LDS, the anisotropy a_s and its flux N
//            (Eq. e), the three collisions, and a push stream of h, g and f into the other
//            ping-pong buffer; phi_prev <- phi in place.
//
// Stream (push) with the a_s^2 weighting of Eq. (d), both a_s^2 taken at the collision node:
//   h^{n+1}_a(x + c_a) = (h*_a(x) - (1 - a_s^2(x)) h^n_a(x + c_a)) / a_s^2(x).
// Open x faces: the inlet (x = 0) bounces back the populations leaving through it (velocity
// bounce-back for f, anti-bounce-back with U = U_in for g, plain bounce-back of Eq. (d) for h);
// at the outlet (x = nx-1) the unknown incoming populations take the value streamed into
// x = nx-2, which the push writes twice; with the pressure outlet (I.xpress) the flow populations
// leaving through x = nx-1 come back instead by anti-bounce-back at rho = 1.
// Flow collision: BGK with Guo forcing, or (CHM) the central-Hermite MRT of chmrt.hpp. Solid walls
// (WALLS): a node mask staged in LDS with the halo; populations aimed at a wall bounce back.
//
// Storage: every population array holds its deviation from a fixed reference, which keeps the
// low-order bits where the dynamics happens and is what the binary16 mode stores:
//   h~ = h + w   (so sum h~ = psi = phi + 1, ~0 in the liquid),
//   g~ = g - w U0 (sum g~ = U - U0, 0 at the start),
//   f~ = f - w   (sum f~ = rho - 1),
// and phi_prev is kept as psi_prev = phi_prev + 1. The collisions are written in these variables;
// the a_s^2-weighted stream is unchanged by the shift because w_a = w_{opposite(a)}.
//
// Layout: a population with velocity component c_x = +-1 is stored shifted along its row, the
// value of node x at memory column (x - c_x) mod nx (xmem below). The push stream then writes every
// population of node x at memory column x of the destination row -- whole, aligned cache lines
// per wavefront -- and the one-column shift moves to the loads, where a line split between two
// wavefronts costs nothing extra. Rows, planes and lattice order are otherwise the plain SoA
// [a][z][y][x]; the read/write entry points of the library convert to and from the plain layout.
//
// HBM traffic per node: every population read once and written once, plus phi_prev read and
// written; halo re-reads of h are served by LDS and L2.
#pragma once

#include <hip/hip_fp16.h>
#include <hip/hip_runtime.h>

#include "chmrt.hpp"
#include "exact.hpp"
#include "lattice.hpp"
#include "mem.hpp"

namespace lbcg {

// Per-instance descriptor, shared by the single-grid and the batched launches.
struct InstDev {
    int nx, ny, nz, xopen;
    int xpress;                   // the outlet of the flow is a pressure (rho = 1) outlet
    int tiles_x, tiles_y, tiles_z, tile_begin;
    int zc;                       // planes per workgroup of the z-marching kernel
    int zband;                    // block tiles: z tile-layers per band of the tile order (<= 1: none)
    long long N;                  // nodes
    int pitch;                    // stored row length (nodes; >= nx): node (x, y, z) at (z ny + y) pitch + x
    long long Nm;                 // stored nodes of a plane, nz ny pitch
    long long Np;                 // plane stride of the population arrays (>= Nm)
    void* h[2];                   // ping-pong population arrays, planes [a][z][y][x]
    void* g[2];
    void* f[2];
    void* phi_prev;
    const unsigned char* wall;    // solid-wall flags per node (plain layout), or null
    double k;                     // W0^2 / tau0
    double inv_tau0, lambda, eps, grad_eps2, D;
    double tau_f, kdrag;          // kdrag = h_drag tau_f / (4 W0^2)
    double u_in, U_in, U0;
    // Constants of the fused step, derived once on the host in binary64 and rounded to binary32
    // (the kernel reads those of its precision); indices K_*.
    double kd[16];
    float kf[16];
};

enum : int {
    K_EPS = 0,    // anisotropy strength eps
    K_GEPS2,      // |grad phi|^2 threshold of the anisotropy
    K_KC,         // (W0^2 / tau0) / cs^2 of the phase-field / solute lattice
    K_LAMBDA,     // coupling constant lambda
    K_ITAU0,      // 1 / tau0
    K_U0,         // reference supersaturation U0 (g is stored as g - w U0)
    K_KDRAG,      // h_drag tau_f / (4 W0^2)
    K_ITAUF,      // 1 / tau_f
    K_GUO,        // 1 - 1 / (2 tau_f)
    K_UIN,        // inlet velocity
    K_DQ,         // D / cs^2
    K_UIN2,       // 2 (U_in - U0), the anti-bounce-back term
    K_OMB,        // trace relaxation rate of the central-Hermite MRT flow collision
    K_CT,         // cos and sin of the crystal's orientation (the anisotropy's frame)
    K_ST,
    K_SRC,        // B of the solute source -B dphi/dt: 1, or 1/2 (both exact scalings)
};
template <typename real> __device__ __forceinline__ real kconst(const InstDev& I, int k) {
    if constexpr (sizeof(real) == 4) return I.kf[k];
    else return I.kd[k];
}

// Copy `par` of a ping-pong pair. A select, not an index: indexing a local copy of the record
// with a run-time value would move the record into private (scratch) memory.
__host__ __device__ __forceinline__ void* pick(void* const (&a)[2], int par) { return par ? a[1] : a[0]; }

// Memory column of node column x for a population with x-velocity cx (see the layout note).
__host__ __device__ __forceinline__ int xmem(int x, int cx, int nx) {
    return cx == 0 ? x : (cx > 0 ? (x == 0 ? nx - 1 : x - 1) : (x == nx - 1 ? 0 : x + 1));
}

// Wall flag of node idx, the index clamped to the grid: a halo box of a grid smaller than the tile
// reaches rows past the last one, which only nodes outside the grid read (branch-free clamp).
__device__ __forceinline__ unsigned char wall_at(const InstDev& I, unsigned idx) {
    return I.wall[__builtin_elementwise_min(idx, (unsigned)(I.Nm - 1))];
}

__device__ __forceinline__ int wrap_coord(int v, int n) {
    if (v < 0) v += n;
    if (v >= n) v -= n;
    if (v < 0 || v >= n) {
        v %= n;
        if (v < 0) v += n;
    }
    return v;
}

// Workgroup -> tile map that gives each of the 8 XCDs (workgroups are dealt round-robin to
// them) one contiguous range of tiles, so halo re-reads stay in that XCD's L2.
__device__ __forceinline__ int xcd_tile(int b, int nblocks) {
    const int xcd = b & 7, idx = b >> 3;
    const int per = nblocks >> 3, rem = nblocks & 7;
    return xcd * per + (xcd < rem ? xcd : rem) + idx;
}

// PF: issue the own node's g, f and phi_prev loads before the barrier, so that their latency
// overlaps the halo load of h. AUX: cache-policy bits of the population stores (0, or 2 = stream).
// LAUX: cache-policy bits of the loads of g, f and phi_prev, which are read once (h keeps the
// default policy: its halo is read again by the neighbouring tiles).
//
// WALLS: honour the solid-wall mask I.wall (zero-flux / no-slip bounce-back, see lbcg_set_walls).
//
// HAUX: cache-policy bits of the h stores (-1: AUX). h is read again by the next step with its halo
// (each row by three tiles), while g and f are read once per step: with HAUX = 0, AUX = 2 and
// LAUX = 2 only h and phi_prev take room in the L2 and last-level caches, whose 256 MB then hold
// them between the steps (on the 192 x 128 x 128 flow grid: 158.8 instead of 184.6 us).
// GC (with HAUX = 0): the first GC planes of g keep the default policy too, so that the next step
// reads them from the last-level cache as well; that pays while everything kept there stays below
// about 128 MiB (on the same grid, 2 planes: 153.9 us, 3: 151.4 us, 4: 163.1 us).
//
// Tile order: x fastest, so that the x-neighbours, which share the halo's cache lines, run
// together. With I.zband = B > 1 the z tile-layers are grouped in bands of B: within a band the
// order is x, then z, then y, so the tiles above and below run B * tiles_x apart instead of a whole
// layer apart and the z-halo of h is still in L2 when it is read again.
template <int DIM, bool FLOW, typename real, typename fst, int TX, int TY, int TZ, bool PF = false, int AUX = 0,
          int LAUX = 0, bool WALLS = false, bool CHM = false, int HAUX = -1, int GC = 0>
__device__ __forceinline__ void step_tile(const InstDev& I, const int tile, const int par) {
    using S = typename Lattices<DIM>::S;
    using V = typename Lattices<DIM>::V;
    constexpr int NT = TX * TY * TZ;
    constexpr int BX = TX + 2, BY = TY + 2, BZ = (DIM == 3) ? TZ + 2 : 1;
    constexpr int NB = BX * BY * BZ;
    constexpr int SY = BX, SZ = BX * BY;  // LDS strides
    // One wavefront per x-row segment: its y and z are the same in every lane, so row offsets are
    // scalar (computed by the scalar unit, passed in the buffer instructions' scalar offset) and a
    // lane's address arithmetic reduces to its column.
    constexpr bool ROW = (TX == 64);
    __shared__ real s_phi[NB];
    __shared__ real s_h[S::Q][NB];
    __shared__ unsigned char s_wall[WALLS ? NB : 1];

    const int tid = threadIdx.x;
    const int nx = I.nx, ny = I.ny, nz = I.nz, pitch = I.pitch;
    const int tix = tile % I.tiles_x;
    const int trest = tile / I.tiles_x;
    int tiy, tiz;
    if (I.zband <= 1) {
        tiy = trest % I.tiles_y;
        tiz = trest / I.tiles_y;
    } else {
        const int per_band = I.tiles_y * I.zband;
        const int band = trest / per_band;
        const int q = trest - band * per_band;
        const int rem = I.tiles_z - band * I.zband;  // the last band may be partial
        const int bz = rem < I.zband ? rem : I.zband;
        tiz = band * I.zband + q % bz;
        tiy = q / bz;
    }
    const int x0 = tix * TX, y0 = tiy * TY, z0 = tiz * TZ;

    constexpr int HA = HAUX < 0 ? AUX : HAUX;
    const Planes<real, HA> hin(pick(I.h, par), I.Np), hout(pick(I.h, par ^ 1), I.Np);
    const Planes<real, AUX, LAUX, (HAUX == 0 ? GC : 0)> gin(pick(I.g, par), I.Np), gout(pick(I.g, par ^ 1), I.Np);
    // phi_prev (one plane, re-read by its own node the next step) stays cacheable with h
    const Planes<real, 0, (HAUX == 0 ? 0 : LAUX)> pprev(I.phi_prev, I.Nm);
    const Planes<fst, AUX, LAUX> fin(pick(I.f, par), I.Np), fout(pick(I.f, par ^ 1), I.Np);
    // node (row + col) of plane a; with ROW the row is wave-uniform
    auto LD = [&](const auto& P, int a, unsigned row, int col) -> real {
        if constexpr (ROW) return P.template ldr<real>(a, row, (unsigned)col);
        else return P.template ld<real>(a, row + (unsigned)col);
    };
    auto ST = [&](const auto& P, int a, unsigned row, int col, real v) {
        if constexpr (ROW) P.str(a, row, (unsigned)col, v);
        else P.st(a, row + (unsigned)col, v);
    };

    const int lx = tid % TX;
    int lyz = tid / TX;
    if constexpr (ROW) lyz = __builtin_amdgcn_readfirstlane(lyz);
    const int ly = lyz % TY, lz = lyz / TY;
    const int x = x0 + lx, y = y0 + ly, z = z0 + lz;
    const bool row_ok = y < ny && z < nz;
    const bool valid = row_ok && x < nx;
    const int xv = x < nx ? x : 0;
    const unsigned rowO = row_ok ? (unsigned)((z * ny + y) * pitch) : 0u;  // own row
    // memory columns of this node for populations with c_x = 0, +1, -1 (x-shifted layout)
    const int xc0 = xv, xcp = xmem(xv, 1, nx), xcm = xmem(xv, -1, nx);
    auto xcol = [&](int cx) { return cx > 0 ? xcp : (cx < 0 ? xcm : xc0); };
    real gv[S::Q];
    real fv[V::Q];
    real pp = 0;
    auto load_own = [&]() {
#pragma unroll
        for (int a = 0; a < S::Q; a++) gv[a] = LD(gin, a, rowO, xcol(S::c(a, 0)));
        if constexpr (FLOW) {
#pragma unroll
            for (int a = 0; a < V::Q; a++) fv[a] = LD(fin, a, rowO, xcol(V::c(a, 0)));  // f - w
        }
        pp = LD(pprev, 0, rowO, xc0);
    };
    if constexpr (PF) load_own();

    // ---- phase 1: h and phi on the tile + halo ----
    auto box_x = [&](int bx) {  // grid column of box column bx; at an open face the ghost is the face node
        int gx = x0 + bx - 1;
        if (I.xopen) gx = gx < 0 ? 0 : (gx > nx - 1 ? nx - 1 : gx);
        else gx = wrap_coord(gx, nx);
        return gx;
    };
    if constexpr (ROW) {
        // box rows are dealt to the wavefronts; lane l loads box column l, lanes 0 and 1 also 64 + l
        constexpr int NW = NT / 64;
        const int ga = box_x(lx), gb = box_x(64 + (lx & 1));
        const int ca[3] = {ga, xmem(ga, 1, nx), xmem(ga, -1, nx)};
        const int cb[3] = {gb, xmem(gb, 1, nx), xmem(gb, -1, nx)};
        auto csel = [](const int* c, int cx) { return cx > 0 ? c[1] : (cx < 0 ? c[2] : c[0]); };
        for (int r = lyz; r < BY * BZ; r += NW) {
            const int by = r % BY, bz = r / BY;
            const int gy = wrap_coord(y0 + by - 1, ny);
            const int gz = (DIM == 3) ? wrap_coord(z0 + bz - 1, nz) : 0;
            const unsigned rb = (unsigned)((gz * ny + gy) * pitch);
            const int b = r * BX + lx;
            real phi = 0;
#pragma unroll
            for (int a = 0; a < S::Q; a++) {
                const real v = LD(hin, a, rb, csel(ca, S::c(a, 0)));
                s_h[a][b] = v;
                phi += v;
            }
            s_phi[b] = phi;
            if constexpr (WALLS) s_wall[b] = wall_at(I, rb + (unsigned)ga);
        }
        // box columns 64 and 65 of the wavefront's rows in one load per plane: lanes 2j and 2j + 1
        // take its j-th row (the row base is then per lane: a vector offset, not the scalar one)
        constexpr int RW = (BY * BZ + NW - 1) / NW;  // box rows per wavefront
        static_assert(2 * RW <= 64, "x-halo lanes");
        const int rj = lyz + (lx >> 1) * NW;
        if (lx < 2 * RW && rj < BY * BZ) {
            const int by = rj % BY, bz = rj / BY;
            const int gy = wrap_coord(y0 + by - 1, ny);
            const int gz = (DIM == 3) ? wrap_coord(z0 + bz - 1, nz) : 0;
            const unsigned rb = (unsigned)((gz * ny + gy) * pitch);
            const int b = rj * BX + 64 + (lx & 1);
            real phi = 0;
#pragma unroll
            for (int a = 0; a < S::Q; a++) {
                const real v = hin.template ld<real>(a, rb + (unsigned)csel(cb, S::c(a, 0)));
                s_h[a][b] = v;
                phi += v;
            }
            s_phi[b] = phi;
            if constexpr (WALLS) s_wall[b] = wall_at(I, rb + (unsigned)gb);
        }
    } else {
        for (int b = tid; b < NB; b += NT) {
            const int bx = b % BX;
            const int br = b / BX;
            const int by = br % BY;
            const int bz = br / BY;
            const int gx = box_x(bx);
            const int gy = wrap_coord(y0 + by - 1, ny);
            const int gz = (DIM == 3) ? wrap_coord(z0 + bz - 1, nz) : 0;
            const unsigned rb = (unsigned)((gz * ny + gy) * pitch);
            real phi = 0;
#pragma unroll
            for (int a = 0; a < S::Q; a++) {
                const real v = LD(hin, a, rb, xmem(gx, S::c(a, 0), nx));
                s_h[a][b] = v;
                phi += v;
            }
            s_phi[b] = phi;
            if constexpr (WALLS) s_wall[b] = wall_at(I, rb + (unsigned)gx);
        }
    }
    __syncthreads();

    // ---- phase 2: one node per thread ----
    if (!valid) return;
    const int bo = (DIM == 3 ? (lz + 1) * SZ : 0) + (ly + 1) * SY + (lx + 1);
    if constexpr (WALLS) {
        if (s_wall[bo]) return;  // wall nodes are frozen
    }
    if constexpr (!PF) load_own();

    // Push targets. Every population is written at memory column x of its destination row, except
    // at an open x face: the inlet node (x = 0) pushes nothing with c_x < 0 (those slots are
    // bounced back into the opposite populations of the same node) and the outlet node
    // (x = nx - 1) nothing with c_x > 0; the outlet also copies its c_x < 0 values into the
    // populations entering through the outlet (memory column 0). Those boundary stores come after
    // each collision loop, apart from the regular pushes.
    const bool xopen = I.xopen != 0;
    const bool at_inlet = xopen && x == 0;
    const bool at_outlet = xopen && x == nx - 1 && !at_inlet;
    const bool push_p = !(xopen && x == nx - 1);  // c_x > 0 allowed
    const bool push_m = !at_inlet;                 // c_x < 0 allowed
    auto push_ok = [&](int cx) { return cx == 0 || (cx > 0 ? push_p : push_m); };
    const int yp = (y + 1 < ny) ? y + 1 : 0;
    const int ym = (y > 0) ? y - 1 : ny - 1;
    const int zp = (DIM == 3) ? ((z + 1 < nz) ? z + 1 : 0) : 0;
    const int zm = (DIM == 3) ? ((z > 0) ? z - 1 : nz - 1) : 0;
    auto row = [&](int cy, int cz) -> unsigned {
        const int yy = cy > 0 ? yp : (cy < 0 ? ym : y);
        const int zz = cz > 0 ? zp : (cz < 0 ? zm : z);
        return (unsigned)((zz * ny + yy) * pitch);
    };

    const real psi = s_phi[bo];  // phi + 1
    const real phi = psi - (real)1;
    const real two_m_psi = (real)2 - psi;  // 1 - phi
    const real p2 = psi * two_m_psi;       // 1 - phi^2

    // directions whose destination inside the domain is a wall node (bit a of swall / vwall)
    unsigned swall = 0, vwall = 0;
    if constexpr (WALLS) {
#pragma unroll
        for (int a = 1; a < S::Q; a++)
            if (push_ok(S::c(a, 0)) && s_wall[bo + S::c(a, 0) + S::c(a, 1) * SY + (DIM == 3 ? S::c(a, 2) * SZ : 0)])
                swall |= 1u << a;
        if constexpr (FLOW) {
#pragma unroll
            for (int a = 1; a < V::Q; a++)
                if (push_ok(V::c(a, 0)) && s_wall[bo + V::c(a, 0) + V::c(a, 1) * SY + (DIM == 3 ? V::c(a, 2) * SZ : 0)])
                    vwall |= 1u << a;
        }
    }
    auto to_wall = [](unsigned bits, int a) { return WALLS && ((bits >> a) & 1u) != 0; };
    // A value bounced back at x = nx - 2 into a population with c_x < 0 is also what the outlet
    // copy gives node nx - 1 of the same row (memory column 0 there).
    const bool pre_outlet = WALLS && xopen && x == nx - 2;

    // grad phi = (1/cs^2) sum_b w_b c_b phi(x + c_b), D2Q9 / D3Q19 stencil (the shift cancels)
    real px = 0, py = 0, pz = 0;
#pragma unroll
    for (int b = 1; b < V::Q; b++) {
        const int nb = bo + V::c(b, 0) + V::c(b, 1) * SY + (DIM == 3 ? V::c(b, 2) * SZ : 0);
        const real ph = (WALLS && s_wall[nb]) ? psi : s_phi[nb];  // a wall neighbour: zero normal derivative
        const real wc = (real)(V::w(b) * V::inv_cs2);
        if (V::c(b, 0)) px += (real)V::c(b, 0) * wc * ph;
        if (V::c(b, 1)) py += (real)V::c(b, 1) * wc * ph;
        if (DIM == 3 && V::c(b, 2)) pz += (real)V::c(b, 2) * wc * ph;
    }

    // anisotropy a_s = 1 + eps Re((nx + i ny)^6) and its flux N = 2 eps a_s |p| (grad P - 6 P n),
    // in the frame of the crystal turned by its orientation (n and N turned about z)
    const real eps = kconst<real>(I, K_EPS);
    const real ct = kconst<real>(I, K_CT), st = kconst<real>(I, K_ST);
    real as = 1, Nx = 0, Ny = 0, Nz = 0;
    const real s2 = px * px + py * py + pz * pz;
    if (s2 > kconst<real>(I, K_GEPS2)) {
        const real m = sqrt(s2);
        const real im = (real)1 / m;
        const real ux_ = (ct * px + st * py) * im, uy_ = (ct * py - st * px) * im, uz_ = pz * im;
        const real z2r = ux_ * ux_ - uy_ * uy_, z2i = (real)2 * ux_ * uy_;
        const real z4r = z2r * z2r - z2i * z2i, z4i = (real)2 * z2r * z2i;
        const real z5r = z4r * ux_ - z4i * uy_, z5i = z4r * uy_ + z4i * ux_;
        const real P6 = z5r * ux_ - z5i * uy_;
        as = (real)1 + eps * P6;
        const real c2 = (real)2 * eps * as * m;
        const real nx_ = c2 * ((real)6 * z5r - (real)6 * P6 * ux_);
        const real ny_ = c2 * ((real)-6 * z5i - (real)6 * P6 * uy_);
        Nx = ct * nx_ - st * ny_;
        Ny = st * nx_ + ct * ny_;
        Nz = c2 * ((real)-6 * P6 * uz_);
    }
    const real a2 = as * as;
    const real inv_a2 = (real)1 / a2;
    const real one_m_a2 = (real)1 - a2;

    // solute moment: Ut = U - U0
    real Ut = 0;
#pragma unroll
    for (int a = 0; a < S::Q; a++) Ut += gv[a];
    const real U = Ut + kconst<real>(I, K_U0);

    // ---- phase field: Eq. (d) with the equilibrium of Eq. (e) ----
    {
        const real kc = kconst<real>(I, K_KC);  // (W0^2/tau0)/cs^2
        const real inv_tau_phi = (real)1 / (a2 * kc + (real)0.5);
        // Q = phi - phi^3 + lambda U (1 - phi^2)^2 = (1 - phi^2)(phi + lambda U (1 - phi^2))
        const real Qs = p2 * (phi + kconst<real>(I, K_LAMBDA) * U * p2) * kconst<real>(I, K_ITAU0);
        real hk[S::Q], vk[S::Q];  // post-collision values; pushed values (c_x < 0 ones reused at the open faces)
        real hv[S::Q];
#pragma unroll
        for (int a = 0; a < S::Q; a++) {
            const int cx = S::c(a, 0), cy = S::c(a, 1), cz = S::c(a, 2);
            const real wa = (real)S::w(a);
            const real cN = (real)cx * Nx + (real)cy * Ny + (real)cz * Nz;
            const real heq = wa * (psi - cN * kc);  // h_eq + w
            const real ha = s_h[a][bo];
            hv[a] = ha;
            hk[a] = ha - (ha - heq) * inv_tau_phi + wa * Qs;
        }
        // The collision's zeroth moment is psi + Q/tau0 exactly; taking the rest population from it
        // (with the rounding errors of the sums carried, rest_closure) keeps each node's phase
        // balance closed in the working precision (in binary32 this stops a drift of the interface
        // that would otherwise grow linearly with the step count, and a drift of U in the solid).
        hk[0] = rest_closure<real, S::Q>(hv, psi, Qs, hk);
#pragma unroll
        for (int a = 0; a < S::Q; a++) {
            const int cx = S::c(a, 0), cy = S::c(a, 1), cz = S::c(a, 2);
            const real hnb = s_h[a][bo + cx + cy * SY + (DIM == 3 ? cz * SZ : 0)];
            vk[a] = (hk[a] - one_m_a2 * hnb) * inv_a2;
            if (push_ok(cx) && !to_wall(swall, a)) ST(hout, a, row(cy, cz), x, vk[a]);  // memory column of x + cx is x
        }
        if constexpr (WALLS) {
            if (swall) {  // zero-flux bounce-back off walls, old value of the slot written (as at the inlet)
#pragma unroll
                for (int a = 1; a < S::Q; a++)
                    if (to_wall(swall, a)) {
                        const int b = S::opp(a);
                        const real v = (hk[a] - one_m_a2 * s_h[b][bo]) * inv_a2;
                        ST(hout, b, rowO, xcol(S::c(b, 0)), v);
                        if (S::c(b, 0) < 0 && pre_outlet) ST(hout, b, rowO, 0, v);
                    }
            }
        }
        if (xopen) {
#pragma unroll
            for (int a = 0; a < S::Q; a++) {
                if (S::c(a, 0) >= 0) continue;
                if (at_inlet) {  // bounce back into the opposite slot of this node (old value of that slot)
                    const int b = S::opp(a);
                    ST(hout, b, rowO, xcp, (hk[a] - one_m_a2 * s_h[b][bo]) * inv_a2);
                }
                if (at_outlet && !to_wall(swall, a)) ST(hout, a, row(S::c(a, 1), S::c(a, 2)), xcm, vk[a]);
            }
        }
    }

    // ---- flow: BGK + Guo forcing of the drag, u* in the equilibrium (or the central-Hermite MRT) ----
    real usx = 0, usy = 0, usz = 0;
    if constexpr (FLOW) {
        real drho = 0, mx = 0, my = 0, mz = 0;
#pragma unroll
        for (int a = 0; a < V::Q; a++) {
            drho += fv[a];
            if (V::c(a, 0)) mx += (real)V::c(a, 0) * fv[a];
            if (V::c(a, 1)) my += (real)V::c(a, 1) * fv[a];
            if (DIM == 3 && V::c(a, 2)) mz += (real)V::c(a, 2) * fv[a];
        }
        const real rho = (real)1 + drho;
        const real K = kconst<real>(I, K_KDRAG) * psi * psi * two_m_psi;  // (1+phi)^2 (1-phi)
        const real iden = (real)1 / (rho + (real)0.5 * K);
        const real ux = mx * iden, uy = my * iden, uz = mz * iden;
        const real Fx = -K * ux, Fy = -K * uy, Fz = -K * uz;
        const real hs_ = (real)0.5 * two_m_psi;
        usx = hs_ * ux;
        usy = hs_ * uy;
        usz = hs_ * uz;
        const real uu = usx * usx + usy * usy + usz * usz;
        const real uF = usx * Fx + usy * Fy + usz * Fz;
        const real inv_tau_f = kconst<real>(I, K_ITAUF);
        const real guo = kconst<real>(I, K_GUO);
        const real uinx = kconst<real>(I, K_UIN);
        real fk[V::Q];
        real fsum = 0;
        if constexpr (CHM) {
            chm_collide<DIM, V, real>(fv, drho, rho, mx, my, mz, usx, usy, usz, Fx, Fy, Fz, inv_tau_f, guo,
                                      kconst<real>(I, K_OMB), fk);
#pragma unroll
            for (int a = 1; a < V::Q; a++) fsum += fk[a];
        } else {
#pragma unroll
            for (int a = 0; a < V::Q; a++) {
                const int cx = V::c(a, 0), cy = V::c(a, 1), cz = V::c(a, 2);
                const real wa = (real)V::w(a);
                const real cu = (real)cx * usx + (real)cy * usy + (real)cz * usz;
                const real cF = (real)cx * Fx + (real)cy * Fy + (real)cz * Fz;
                // f_eq - w = w [rho - 1 + rho (cu/cs2 + cu^2/(2 cs2^2) - uu/(2 cs2))]
                const real feq = wa * (drho + rho * ((real)3 * cu + (real)4.5 * cu * cu - (real)1.5 * uu));
                const real Sa = wa * guo * ((real)3 * cF + (real)9 * cu * cF - (real)3 * uF);
                fk[a] = fv[a] - (fv[a] - feq) * inv_tau_f + Sa;
                if (a) fsum += fk[a];
            }
        }
        fk[0] = drho - fsum;  // mass: the collision and the Guo term leave sum_a (f_a - w_a) = rho - 1
#pragma unroll
        for (int a = 0; a < V::Q; a++)
            if (push_ok(V::c(a, 0)) && !to_wall(vwall, a)) ST(fout, a, row(V::c(a, 1), V::c(a, 2)), x, fk[a]);
        if constexpr (WALLS) {
            if (vwall) {  // no-slip halfway bounce-back off walls at rest
#pragma unroll
                for (int a = 1; a < V::Q; a++)
                    if (to_wall(vwall, a)) {
                        ST(fout, V::opp(a), rowO, xcol(-V::c(a, 0)), fk[a]);
                        if (V::c(a, 0) > 0 && pre_outlet && !I.xpress) ST(fout, V::opp(a), rowO, 0, fk[a]);
                    }
            }
        }
        if (xopen) {
#pragma unroll
            for (int a = 0; a < V::Q; a++) {
                const int cx = V::c(a, 0);
                if (cx >= 0) continue;
                if (at_inlet)  // velocity bounce-back, wall density 1
                    ST(fout, V::opp(a), rowO, xcp, fk[a] - (real)6 * (real)V::w(a) * (real)cx * uinx);
                if (at_outlet && !I.xpress && !to_wall(vwall, a)) ST(fout, a, row(V::c(a, 1), V::c(a, 2)), xcm, fk[a]);
            }
            if (I.xpress && at_outlet) {  // pressure outlet: anti-bounce-back at rho = 1 and the node's u*
#pragma unroll
                for (int a = 0; a < V::Q; a++) {
                    const int cx = V::c(a, 0);
                    if (cx <= 0) continue;
                    const real cu = (real)cx * usx + (real)V::c(a, 1) * usy + (real)V::c(a, 2) * usz;
                    // f_opp - w = -(f*_a - w) + 2 w (cu^2 / (2 cs^4) - uu / (2 cs^2))
                    ST(fout, V::opp(a), rowO, xcm, -fk[a] + (real)2 * (real)V::w(a) * ((real)4.5 * cu * cu - (real)1.5 * uu));
                }
            }
        }
    }

    // ---- solute: advection-diffusion LB with source -w B dphi/dt ----
    {
        real q = two_m_psi;  // 1 - phi, clamped to [0, 2]
        q = q < (real)0 ? (real)0 : (q > (real)2 ? (real)2 : q);
        const real inv_tau_U = (real)1 / (kconst<real>(I, K_DQ) * q + (real)0.5);
        const real dphi = kconst<real>(I, K_SRC) * (psi - pp);
        const real Uin2 = kconst<real>(I, K_UIN2);
        real gk[S::Q];
        real gsum = 0;
#pragma unroll
        for (int a = 0; a < S::Q; a++) {
            const int cx = S::c(a, 0), cy = S::c(a, 1), cz = S::c(a, 2);
            const real wa = (real)S::w(a);
            const real cu = (real)cx * usx + (real)cy * usy + (real)cz * usz;
            const real geq = wa * (Ut + U * cu * (real)S::inv_cs2);  // g_eq - w U0
            gk[a] = gv[a] - (gv[a] - geq) * inv_tau_U - wa * dphi;
            if (a) gsum += gk[a];
        }
        gk[0] = (Ut - dphi) - gsum;  // solute balance of the node: sum_a g*_a - U0 = U - U0 - B dphi
#pragma unroll
        for (int a = 0; a < S::Q; a++)
            if (push_ok(S::c(a, 0)) && !to_wall(swall, a)) ST(gout, a, row(S::c(a, 1), S::c(a, 2)), x, gk[a]);
        if constexpr (WALLS) {
            if (swall) {  // zero-flux bounce-back off walls
#pragma unroll
                for (int a = 1; a < S::Q; a++)
                    if (to_wall(swall, a)) {
                        ST(gout, S::opp(a), rowO, xcol(-S::c(a, 0)), gk[a]);
                        if (S::c(a, 0) > 0 && pre_outlet) ST(gout, S::opp(a), rowO, 0, gk[a]);
                    }
            }
        }
        if (xopen) {
#pragma unroll
            for (int a = 0; a < S::Q; a++) {
                if (S::c(a, 0) >= 0) continue;
                if (at_inlet)  // anti-bounce-back, U = U_in on the inlet wall
                    ST(gout, S::opp(a), rowO, xcp, -gk[a] + (real)S::w(a) * Uin2);
                if (at_outlet && !to_wall(swall, a)) ST(gout, a, row(S::c(a, 1), S::c(a, 2)), xcm, gk[a]);
            }
        }
    }
    ST(pprev, 0, rowO, xc0, psi);
}

template <int DIM, bool FLOW, typename real, typename fst, int TX, int TY, int TZ, bool PF, int AUX, int LAUX,
          bool WALLS = false, bool CHM = false, int HAUX = -1, int GC = 0>
__global__ __launch_bounds__(TX* TY* TZ) void step_single(InstDev I, int par) {
    step_tile<DIM, FLOW, real, fst, TX, TY, TZ, PF, AUX, LAUX, WALLS, CHM, HAUX, GC>(I, xcd_tile(blockIdx.x, gridDim.x), par);
}

// Batched launch: the tiles of all instances form one list; each workgroup finds its instance
// by binary search over the tile offsets.
template <int DIM, bool FLOW, typename real, typename fst, int TX, int TY, int TZ, bool PF, int AUX, int LAUX = 0,
          bool CHM = false, int HAUX = -1>
__global__ __launch_bounds__(TX* TY* TZ) void step_batch(const InstDev* __restrict__ insts, int ninst,
                                                         int par) {
    const int t = xcd_tile(blockIdx.x, gridDim.x);
    int lo = 0, hi = ninst - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (__builtin_amdgcn_readfirstlane(insts[mid].tile_begin) <= t) lo = mid;
        else hi = mid - 1;
    }
    // The record is the same for the whole workgroup: read it word by word into scalar registers,
    // so that the buffer descriptors and the grid constants stay scalar as in the one-grid kernel.
    static_assert(sizeof(InstDev) % 4 == 0, "InstDev is read as 32-bit words");
    unsigned w[sizeof(InstDev) / 4];
    const unsigned* src = reinterpret_cast<const unsigned*>(insts + lo);
#pragma unroll
    for (int k = 0; k < (int)(sizeof(InstDev) / 4); k++) w[k] = __builtin_amdgcn_readfirstlane(src[k]);
    InstDev I;
    __builtin_memcpy(&I, w, sizeof(InstDev));
    step_tile<DIM, FLOW, real, fst, TX, TY, TZ, PF, AUX, LAUX, false, CHM, HAUX>(I, t - I.tile_begin, par);
}

}  // namespace lbcg
