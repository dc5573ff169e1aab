// chmrt.hpp -- central-Hermite multiple-relaxation-time collision of the flow populations
// (the stabilised collision the flow paragraph of Section 2.2 names; moment set and rates as below).
//
// Relaxation rule, in central Hermite moments about u* (He0 = 1, He1 = xi, He2 = xi^2 - cs2 per
// direction, the multi-indices the lattice carries: n_x, n_y <= 2 on D2Q9; each n_d <= 2 with at
// most two non-zero on D3Q19):
//   order 0  rho, kept;
//   order 1  (1 - w) k + (1 - w/2) F       (the momentum update of BGK with Guo forcing);
//   order 2  deviatoric part times (1 - w), trace part times (1 - w_b), w = 1/tau_f;
//   order 3, 4  zero (their equilibrium value; the forcing has no central moment there).
//
// Closed form used here instead of a moment matrix: only the second-order central moments of the
// incoming populations are needed. The post-collision central monomials follow from the rule
// (K_iij = cs2 K_j, K_iijj = cs2 (K_ii + K_jj) - cs2^2 rho where the Hermite moments vanish), the
// raw monomials from the binomial expansion of c = (c - u*) + u*, and the populations from the
// raw monomials by the lattice's explicit inverse:
//   edge (d, e), signs (s_d, s_e):  f = [M_ddee + s_d M_dee + s_e M_dde + s_d s_e M_de] / 4
//   axis d, sign s:                 f = [(M_dd - sum_e M_ddee) + s (M_d - sum_e M_dee)] / 2
//   rest:                           f = M_0 - sum_d M_dd + sum_{d<e} M_ddee
// (M_dee = sum_a f_a c_d c_e^2). Every quantity is carried as a deviation from the rest state
// f = w (whose non-zero raw monomials are M_0 = 1, M_dd = cs2, M_ddee = cs2^2), so binary32 keeps
// the digits of the small deviations.
#pragma once

#include "lattice.hpp"

namespace lbcg {

// M_eed - the raw moment sum_a f_a c_e^2 c_d (d != e) of the post-collision populations
// (K_eed = cs2 K_d).
template <typename real>
__device__ __forceinline__ real chm_m3(real Kd, real Ke, real Kee_full, real Kde, real ud, real ue, real rho) {
    const real cs2 = (real)(1.0 / 3.0);
    return cs2 * Kd + ud * Kee_full + (real)2 * ue * Kde + (real)2 * ue * ud * Ke + ue * ue * Kd + rho * ue * ue * ud;
}

// M_iijj - cs2^2 (i != j): Ki, Kj first-order, Aii, Ajj, Aij post-collision Hermite second-order
// central moments (K_ii = A_ii + rho cs2).
template <typename real>
__device__ __forceinline__ real chm_m4(real Ki, real Kj, real Aii, real Ajj, real Aij, real ui, real uj, real rho,
                                       real drho) {
    const real cs2 = (real)(1.0 / 3.0);
    const real Kii = Aii + rho * cs2, Kjj = Ajj + rho * cs2;
    const real dK4 = cs2 * (Aii + Ajj) + cs2 * cs2 * drho;  // K_iijj - cs2^2
    return dK4 + (real)2 * ui * cs2 * Ki + (real)2 * uj * cs2 * Kj + ui * ui * Kjj + uj * uj * Kii +
           (real)4 * ui * uj * Aij + (real)2 * ui * uj * uj * Ki + (real)2 * ui * ui * uj * Kj + rho * ui * ui * uj * uj;
}

// fv: incoming populations f - w; drho = rho - 1; m: raw first moments; u: u*; F: drag force;
// om = 1/tau_f, guo = 1 - om/2, omb: trace rate. Writes the post-collision f - w to fk.
template <int DIM, class V, typename real>
__device__ __forceinline__ void chm_collide(const real (&fv)[V::Q], real drho, real rho, real mx, real my, real mz,
                                            real ux, real uy, real uz, real Fx, real Fy, real Fz, real om, real guo,
                                            real omb, real (&fk)[V::Q]) {
    const real cs2 = (real)(1.0 / 3.0);
    // raw second moments of the deviations, S_ij = sum_a (f_a - w_a) c_ai c_aj
    real sxx = 0, syy = 0, szz = 0, sxy = 0, sxz = 0, syz = 0;
#pragma unroll
    for (int a = 1; a < V::Q; a++) {
        const int cx = V::c(a, 0), cy = V::c(a, 1), cz = V::c(a, 2);
        if (cx) sxx += fv[a];
        if (cy) syy += fv[a];
        if (DIM == 3 && cz) szz += fv[a];
        if (cx && cy) sxy += (real)(cx * cy) * fv[a];
        if (DIM == 3 && cx && cz) sxz += (real)(cx * cz) * fv[a];
        if (DIM == 3 && cy && cz) syz += (real)(cy * cz) * fv[a];
    }
    if constexpr (DIM == 2) uz = 0, mz = 0, Fz = 0;
    // central Hermite second moments about u*: S_ij - drho cs2 d_ij - u_i m_j - m_i u_j + rho u_i u_j
    const real hxx = sxx - drho * cs2 - (real)2 * ux * mx + rho * ux * ux;
    const real hyy = syy - drho * cs2 - (real)2 * uy * my + rho * uy * uy;
    const real hzz = DIM == 3 ? szz - drho * cs2 - (real)2 * uz * mz + rho * uz * uz : (real)0;
    const real hxy = sxy - ux * my - mx * uy + rho * ux * uy;
    const real hxz = DIM == 3 ? sxz - ux * mz - mx * uz + rho * ux * uz : (real)0;
    const real hyz = DIM == 3 ? syz - uy * mz - my * uz + rho * uy * uz : (real)0;
    const real t = (hxx + hyy + hzz) * (real)(1.0 / DIM);
    const real as = (real)1 - om, ab = (real)1 - omb;
    const real Axx = as * (hxx - t) + ab * t, Ayy = as * (hyy - t) + ab * t;
    const real Azz = DIM == 3 ? as * (hzz - t) + ab * t : (real)0;
    const real Axy = as * hxy, Axz = as * hxz, Ayz = as * hyz;
    // post-collision first-order central moments
    const real Kx = as * (mx - rho * ux) + guo * Fx;
    const real Ky = as * (my - rho * uy) + guo * Fy;
    const real Kz = DIM == 3 ? as * (mz - rho * uz) + guo * Fz : (real)0;
    // raw monomials (minus the rest state's value where that is non-zero)
    const real Mx = Kx + rho * ux, My = Ky + rho * uy, Mz = Kz + rho * uz;
    const real dMxx = Axx + drho * cs2 + (real)2 * ux * Kx + rho * ux * ux;
    const real dMyy = Ayy + drho * cs2 + (real)2 * uy * Ky + rho * uy * uy;
    const real dMzz = DIM == 3 ? Azz + drho * cs2 + (real)2 * uz * Kz + rho * uz * uz : (real)0;
    const real Mxy = Axy + ux * Ky + uy * Kx + rho * ux * uy;
    const real Mxz = DIM == 3 ? Axz + ux * Kz + uz * Kx + rho * ux * uz : (real)0;
    const real Myz = DIM == 3 ? Ayz + uy * Kz + uz * Ky + rho * uy * uz : (real)0;
    const real Kxx = Axx + rho * cs2, Kyy = Ayy + rho * cs2, Kzz = Azz + rho * cs2;
    // M_dee: d linear, e squared
    const real Mxyy = chm_m3(Kx, Ky, Kyy, Axy, ux, uy, rho);
    const real Myxx = chm_m3(Ky, Kx, Kxx, Axy, uy, ux, rho);
    const real Mxzz = DIM == 3 ? chm_m3(Kx, Kz, Kzz, Axz, ux, uz, rho) : (real)0;
    const real Mzxx = DIM == 3 ? chm_m3(Kz, Kx, Kxx, Axz, uz, ux, rho) : (real)0;
    const real Myzz = DIM == 3 ? chm_m3(Ky, Kz, Kzz, Ayz, uy, uz, rho) : (real)0;
    const real Mzyy = DIM == 3 ? chm_m3(Kz, Ky, Kyy, Ayz, uz, uy, rho) : (real)0;
    const real dMxxyy = chm_m4(Kx, Ky, Axx, Ayy, Axy, ux, uy, rho, drho);
    const real dMxxzz = DIM == 3 ? chm_m4(Kx, Kz, Axx, Azz, Axz, ux, uz, rho, drho) : (real)0;
    const real dMyyzz = DIM == 3 ? chm_m4(Ky, Kz, Ayy, Azz, Ayz, uy, uz, rho, drho) : (real)0;
    const real half = (real)0.5, quarter = (real)0.25;
#pragma unroll
    for (int a = 0; a < V::Q; a++) {
        const int cx = V::c(a, 0), cy = V::c(a, 1), cz = V::c(a, 2);
        const int n = (cx != 0) + (cy != 0) + (cz != 0);
        real v;
        if (n == 0) {
            v = drho - (dMxx + dMyy + dMzz) + (dMxxyy + dMxxzz + dMyyzz);
        } else if (n == 1) {
            if (cx) v = half * ((dMxx - dMxxyy - dMxxzz) + (real)cx * (Mx - Mxyy - Mxzz));
            else if (cy) v = half * ((dMyy - dMxxyy - dMyyzz) + (real)cy * (My - Myxx - Myzz));
            else v = half * ((dMzz - dMxxzz - dMyyzz) + (real)cz * (Mz - Mzxx - Mzyy));
        } else {
            if (!cz) v = quarter * (dMxxyy + (real)cx * Mxyy + (real)cy * Myxx + (real)(cx * cy) * Mxy);
            else if (!cy) v = quarter * (dMxxzz + (real)cx * Mxzz + (real)cz * Mzxx + (real)(cx * cz) * Mxz);
            else v = quarter * (dMyyzz + (real)cy * Myzz + (real)cz * Mzyy + (real)(cy * cz) * Myz);
        }
        fk[a] = v;
    }
}

}  // namespace lbcg
