// march.hpp -- the fused coupled step as a z-marching kernel for 3-D grids with nx <= 64 NW.
//
// A workgroup owns TY full x-rows (y0 .. y0+TY-1) and marches over the planes z0 .. z0+ZC-1. It
// keeps, in LDS, a ring of three planes of psi = phi + 1 on rows y0-1 .. y0+TY (the isotropic
// gradient needs phi on the D3Q19 stencil) and the in-plane components (+-x, +-y) of h^n of the
// current plane (the old-value term of the a_s^2-weighted stream, Eq. (d)); the +-z components
// stay in the registers of the thread that owns the column. Per plane:
//
//   A  load h^n of plane z+1 (own row + the two halo rows), form psi, fill the LDS ring;
//      own f, g and psi_prev of plane z are loaded before the barrier so their latency overlaps;
//   B  barrier;
//   C  collide the own node of plane z (three lattices, identical arithmetic to step.hpp) and
//      push; with the x-shifted layout of step.hpp every store of a wavefront is a whole, aligned
//      row segment (only the inlet bounce-back and the outlet copy write single columns).
//
// HBM traffic per node is the algorithmic one (each population read and written once, psi_prev
// read and written); the halo rows of h and the planes z0-1, z0+ZC are re-read through L2.
#pragma once

#include <hip/hip_fp16.h>
#include <hip/hip_runtime.h>

#include "lattice.hpp"
#include "mem.hpp"
#include "step.hpp"

namespace lbcg {

template <bool FLOW, typename real, typename fst, int NW, int TY>
__device__ __forceinline__ void march3d_tile(const InstDev& I, const int tile, const int par, const int ZC) {
    using S = D3Q7;
    using V = D3Q19;
    constexpr int NXP = 64 * NW;       // padded row length
    constexpr int NT = NXP * TY;       // threads
    constexpr int NR = TY + 2;         // rows with halo
    __shared__ real s_psi[3][NR][NXP];    // psi ring over planes
    __shared__ real s_hh[2][4][NR][NXP];  // h^n components +x, -x, +y, -y; slot = plane parity

    const int tid = threadIdx.x;
    const int x = tid % NXP;
    const int ly = tid / NXP;
    const int nx = I.nx, ny = I.ny, nz = I.nz;
    const int tiy = tile % I.tiles_y;
    const int tiz = tile / I.tiles_y;
    const int y0 = tiy * TY;
    const int z0 = tiz * ZC;
    const int z1 = min(z0 + ZC, nz);
    const int y = y0 + ly;
    const bool xin = x < nx;
    const bool active = xin && y < ny;
    const bool xopen = I.xopen != 0;

    const Planes<real> hin(pick(I.h, par), I.Np), hout(pick(I.h, par ^ 1), I.Np);
    const Planes<real> gin(pick(I.g, par), I.Np), gout(pick(I.g, par ^ 1), I.Np);
    const Planes<fst> fin(pick(I.f, par), I.Np), fout(pick(I.f, par ^ 1), I.Np);
    const Planes<real> pprev(I.phi_prev, I.Nm);

    auto wrapz = [&](int v) { return wrap_coord(v, nz); };
    auto wrapy = [&](int v) { return wrap_coord(v, ny); };
    auto node = [&](int xx, int yy, int zz) { return (unsigned)((zz * ny + yy) * I.pitch + xx); };
    // x neighbour inside the row for phi and the old-value term: wrap, or the face copy at an open face
    const int xm = x > 0 ? x - 1 : (xopen ? 0 : nx - 1);
    const int xp = x < nx - 1 ? x + 1 : (xopen ? nx - 1 : 0);

    // Load h^n of plane zz on the own row and, for the first / last row of the tile, the halo row
    // beyond it; write psi into ring slot `ring` and the in-plane components into s_hh[hs]; return
    // the own node's seven values in hv.
    auto load_plane = [&](int zz, int ring, int hs, real* hv) {
        const int zw = wrapz(zz);
        for (int k = 0; k < 2; k++) {
            int r;  // LDS row 0 .. NR-1 (row r is y0 + r - 1)
            if (k == 0) r = ly + 1;
            else if (ly == 0) r = 0;
            else if (ly == TY - 1) r = NR - 1;
            else break;
            real v[S::Q];
            real psi = 0;
            if (xin) {
                const unsigned rb = node(0, wrapy(y0 + r - 1), zw);
#pragma unroll
                for (int a = 0; a < S::Q; a++) {
                    v[a] = hin.template ld<real>(a, rb + xmem(x, S::c(a, 0), nx));
                    psi += v[a];
                }
            } else {
#pragma unroll
                for (int a = 0; a < S::Q; a++) v[a] = 0;
            }
            s_psi[ring][r][x] = psi;
#pragma unroll
            for (int c = 0; c < 4; c++) s_hh[hs][c][r][x] = v[1 + c];
            if (k == 0) {
#pragma unroll
                for (int a = 0; a < S::Q; a++) hv[a] = v[a];
            }
            if (TY == 1 && k == 1) {  // a one-row tile loads both halo rows
                const int r2 = NR - 1;
                real w2[S::Q];
                real psi2 = 0;
                if (xin) {
                    const unsigned rb = node(0, wrapy(y0 + r2 - 1), zw);
#pragma unroll
                    for (int a = 0; a < S::Q; a++) {
                        w2[a] = hin.template ld<real>(a, rb + xmem(x, S::c(a, 0), nx));
                        psi2 += w2[a];
                    }
                } else {
#pragma unroll
                    for (int a = 0; a < S::Q; a++) w2[a] = 0;
                }
                s_psi[ring][r2][x] = psi2;
#pragma unroll
                for (int c = 0; c < 4; c++) s_hh[hs][c][r2][x] = w2[1 + c];
            }
        }
    };

    // prologue: planes z0-1 and z0
    real hmz;  // h^n_{-z} of plane z-1 at the own column
    real hc[S::Q];
    {
        real tmp[S::Q];
        load_plane(z0 - 1, (z0 + 2) % 3, (z0 + 1) & 1, tmp);
        hmz = tmp[6];
        load_plane(z0, z0 % 3, z0 & 1, hc);
    }

    const real kc = (real)(I.k * S::inv_cs2);
    const real eps = (real)I.eps;
    const real geps2 = (real)I.grad_eps2;
    const real ct = kconst<real>(I, K_CT), st = kconst<real>(I, K_ST);
    const real lam = (real)I.lambda, itau0 = (real)I.inv_tau0;
    const real DU = (real)(I.D * S::inv_cs2);
    const real U0 = (real)I.U0;
    const real Uin2 = (real)2 * (real)(I.U_in - I.U0);
    const real inv_tau_f = (real)(1.0 / I.tau_f);
    const real guo = (real)(1.0 - 0.5 / I.tau_f);
    const real kdrag = (real)I.kdrag;
    const real uinx = (real)I.u_in;

    for (int z = z0; z < z1; z++) {
        const int zw = z;  // z < nz
        const unsigned rowO = active ? node(0, y, zw) : 0u;
        const unsigned gi = rowO + (active ? (unsigned)x : 0u);
        // own g, f, psi_prev of plane z (issued before the barrier)
        real gv[S::Q];
        real fv[V::Q];
        real pp = 0;
        if (active) {
#pragma unroll
            for (int a = 0; a < S::Q; a++) gv[a] = gin.template ld<real>(a, rowO + xmem(x, S::c(a, 0), nx));
            if constexpr (FLOW) {
#pragma unroll
                for (int a = 0; a < V::Q; a++) fv[a] = fin.template ld<real>(a, rowO + xmem(x, V::c(a, 0), nx));
            }
            pp = pprev.template ld<real>(0, gi);
        } else {
#pragma unroll
            for (int a = 0; a < S::Q; a++) gv[a] = 0;
#pragma unroll
            for (int a = 0; a < V::Q; a++) fv[a] = 0;
        }
        // A: plane z+1
        real hn[S::Q];
        load_plane(z + 1, (z + 1) % 3, (z + 1) & 1, hn);
        __syncthreads();  // B (psi ring has planes z-1, z, z+1; s_hin holds plane z)

        const int rm = (z + 2) % 3, r0 = z % 3, rp = (z + 1) % 3, hsl = z & 1;
        const int row = ly + 1;
        // ---- C: collide ----
        if (active) {
            const real psi = s_psi[r0][row][x];
            const real phi = psi - (real)1;
            const real two_m_psi = (real)2 - psi;
            const real p2 = psi * two_m_psi;
            // gradient, D3Q19 stencil (planes rm / r0 / rp, rows row-1 .. row+1, columns xm / x / xp)
            real px = 0, py = 0, pz = 0;
#pragma unroll
            for (int b = 1; b < V::Q; b++) {
                const int cx = V::c(b, 0), cy = V::c(b, 1), cz = V::c(b, 2);
                const int rr = cz > 0 ? rp : (cz < 0 ? rm : r0);
                const int xx = cx > 0 ? xp : (cx < 0 ? xm : x);
                const real ph = s_psi[rr][row + cy][xx];
                const real wc = (real)(V::w(b) * V::inv_cs2);
                if (cx) px += (real)cx * wc * ph;
                if (cy) py += (real)cy * wc * ph;
                if (cz) pz += (real)cz * wc * ph;
            }
            real as = 1, Nx = 0, Ny = 0, Nz = 0;
            const real s2 = px * px + py * py + pz * pz;
            if (s2 > geps2) {  // in the frame of the crystal turned by its orientation
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

            real Ut = 0;
#pragma unroll
            for (int a = 0; a < S::Q; a++) Ut += gv[a];
            const real U = Ut + U0;

            // phase field
            const real inv_tau_phi = (real)1 / (a2 * kc + (real)0.5);
            const real Qs = p2 * (phi + lam * U * p2) * itau0;
            // old values h^n_a(x + c_a): +x, -x, +y, -y from LDS, +z / -z from registers
            const real hnb[7] = {hc[0],
                                 s_hh[hsl][0][row][xp],
                                 s_hh[hsl][1][row][xm],
                                 s_hh[hsl][2][row + 1][x],
                                 s_hh[hsl][3][row - 1][x],
                                 hn[5],
                                 hmz};
            real hk[S::Q];
#pragma unroll
            for (int a = 0; a < S::Q; a++) {
                const int cx = S::c(a, 0), cy = S::c(a, 1), cz = S::c(a, 2);
                const real wa = (real)S::w(a);
                const real cN = (real)cx * Nx + (real)cy * Ny + (real)cz * Nz;
                const real heq = wa * (psi - cN * kc);
                hk[a] = hc[a] - (hc[a] - heq) * inv_tau_phi + wa * Qs;
            }
            // rest population from the exact zeroth moment psi + Q/tau0 (rounding errors carried)
            hk[0] = rest_closure<real, S::Q>(hc, psi, Qs, hk);
#pragma unroll
            for (int a = 0; a < S::Q; a++) {
                const int cx = S::c(a, 0), cy = S::c(a, 1), cz = S::c(a, 2);
                const real hs = hk[a];
                const unsigned drow = node(0, wrapy(y + cy), wrapz(z + cz));
                if (cx < 0 && xopen && x == 0) {  // inlet: bounce-back into the opposite slot, old value of that slot
                    const int b = S::opp(a);
                    hout.st(b, rowO + xmem(0, S::c(b, 0), nx), (hs - one_m_a2 * hc[b]) * inv_a2);
                } else if (!(cx > 0 && xopen && x == nx - 1)) {  // (leaves through the outlet)
                    const real v = (hs - one_m_a2 * hnb[a]) * inv_a2;
                    hout.st(a, drow + x, v);
                    if (cx < 0 && xopen && x == nx - 1) hout.st(a, drow + xmem(x, cx, nx), v);  // outlet copy
                }
            }

            // flow
            real usx = 0, usy = 0, usz = 0;
            if constexpr (FLOW) {
                real drho = 0, mx = 0, my = 0, mz = 0;
#pragma unroll
                for (int a = 0; a < V::Q; a++) {
                    drho += fv[a];
                    if (V::c(a, 0)) mx += (real)V::c(a, 0) * fv[a];
                    if (V::c(a, 1)) my += (real)V::c(a, 1) * fv[a];
                    if (V::c(a, 2)) mz += (real)V::c(a, 2) * fv[a];
                }
                const real rho = (real)1 + drho;
                const real K = kdrag * psi * psi * two_m_psi;
                const real iden = (real)1 / (rho + (real)0.5 * K);
                const real ux = mx * iden, uy = my * iden, uz = mz * iden;
                const real Fx = -K * ux, Fy = -K * uy, Fz = -K * uz;
                const real hs_ = (real)0.5 * two_m_psi;
                usx = hs_ * ux;
                usy = hs_ * uy;
                usz = hs_ * uz;
                const real uu = usx * usx + usy * usy + usz * usz;
                const real uF = usx * Fx + usy * Fy + usz * Fz;
                real fk[V::Q];
                real fsum = 0;
#pragma unroll
                for (int a = 0; a < V::Q; a++) {
                    const int cx = V::c(a, 0), cy = V::c(a, 1), cz = V::c(a, 2);
                    const real wa = (real)V::w(a);
                    const real cu = (real)cx * usx + (real)cy * usy + (real)cz * usz;
                    const real cF = (real)cx * Fx + (real)cy * Fy + (real)cz * Fz;
                    const real feq = wa * (drho + rho * ((real)3 * cu + (real)4.5 * cu * cu - (real)1.5 * uu));
                    const real Sa = wa * guo * ((real)3 * cF + (real)9 * cu * cF - (real)3 * uF);
                    fk[a] = fv[a] - (fv[a] - feq) * inv_tau_f + Sa;
                    if (a) fsum += fk[a];
                }
                fk[0] = drho - fsum;  // mass of the node, rho - 1
#pragma unroll
                for (int a = 0; a < V::Q; a++) {
                    const int cx = V::c(a, 0), cy = V::c(a, 1), cz = V::c(a, 2);
                    const real wa = (real)V::w(a);
                    const real fs = fk[a];
                    const unsigned drow = node(0, wrapy(y + cy), wrapz(z + cz));
                    if (cx < 0 && xopen && x == 0) {  // inlet: velocity bounce-back, wall density 1
                        const int b = V::opp(a);
                        fout.st(b, rowO + xmem(0, V::c(b, 0), nx), fs - (real)6 * wa * (real)cx * uinx);
                    } else if (!(cx > 0 && xopen && x == nx - 1)) {
                        fout.st(a, drow + x, fs);
                        if (cx < 0 && xopen && x == nx - 1) fout.st(a, drow + xmem(x, cx, nx), fs);
                    }
                }
            }

            // solute
            {
                real q = two_m_psi;
                q = q < (real)0 ? (real)0 : (q > (real)2 ? (real)2 : q);
                const real inv_tau_U = (real)1 / (DU * q + (real)0.5);
                const real dphi = kconst<real>(I, K_SRC) * (psi - pp);
                real gk[S::Q];
                real gsum = 0;
#pragma unroll
                for (int a = 0; a < S::Q; a++) {
                    const int cx = S::c(a, 0), cy = S::c(a, 1), cz = S::c(a, 2);
                    const real wa = (real)S::w(a);
                    const real cu = (real)cx * usx + (real)cy * usy + (real)cz * usz;
                    const real geq = wa * (Ut + U * cu * (real)S::inv_cs2);
                    gk[a] = gv[a] - (gv[a] - geq) * inv_tau_U - wa * dphi;
                    if (a) gsum += gk[a];
                }
                gk[0] = (Ut - dphi) - gsum;  // solute balance of the node
#pragma unroll
                for (int a = 0; a < S::Q; a++) {
                    const int cx = S::c(a, 0), cy = S::c(a, 1), cz = S::c(a, 2);
                    const real wa = (real)S::w(a);
                    const real gs = gk[a];
                    const unsigned drow = node(0, wrapy(y + cy), wrapz(z + cz));
                    if (cx < 0 && xopen && x == 0) {  // inlet: anti-bounce-back, U = U_in on the wall
                        const int b = S::opp(a);
                        gout.st(b, rowO + xmem(0, S::c(b, 0), nx), -gs + wa * Uin2);
                    } else if (!(cx > 0 && xopen && x == nx - 1)) {
                        gout.st(a, drow + x, gs);
                        if (cx < 0 && xopen && x == nx - 1) gout.st(a, drow + xmem(x, cx, nx), gs);
                    }
                }
            }
            pprev.st(0, gi, psi);
        }
        // roll the column registers and the in-plane LDS slot
        hmz = hc[6];
#pragma unroll
        for (int a = 0; a < S::Q; a++) hc[a] = hn[a];
        // the next iteration's loads overwrite s_psi[(z+2)%3] and s_hh[z & 1], read in C above
        __syncthreads();
    }
}

template <bool FLOW, typename real, typename fst, int NW, int TY>
__global__ __launch_bounds__(64 * NW * TY) void march3d_single(InstDev I, int par, int ZC) {
    march3d_tile<FLOW, real, fst, NW, TY>(I, xcd_tile(blockIdx.x, gridDim.x), par, ZC);
}

}  // namespace lbcg
