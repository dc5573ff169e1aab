// exact.hpp -- error-free addition for the closure of the phase-field collision.
//
// two_sum (Knuth's TwoSum): s = fl(a + b) and e with s + e = a + b exactly, in any binary floating
// point format with round-to-nearest (six additions, no branch, valid without |a| >= |b|).
#pragma once

#include <hip/hip_runtime.h>

namespace lbcg {

template <typename real> __device__ __forceinline__ real two_sum(real a, real b, real& e) {
    const real s = a + b;
    const real bb = s - a;
    e = (a - (s - bb)) + (b - bb);
    return s;
}

// The rest population of the phase-field collision from the collision's exact zeroth moment:
// hk0 = (psi + Qs) - sum_{a>0} hk[a], where psi = h[0] + ... + h[Q-1] was summed in that order.
// The rounding errors of psi's sum, of psi + Qs and of the sum of the moving populations are
// carried along and added back once, so that the node's stored phase balance is
// psi_exact + Qs up to the one final rounding. In binary32 the uncompensated closure changes the
// crystal's phi by a few units in the last place every step, and that change reaches the solute
// through the source -dphi/dt, where tau_U = 1/2 in the solid leaves it undamped.
template <typename real, int Q>
__device__ __forceinline__ real rest_closure(const real (&h)[Q], real psi, real Qs, const real (&hk)[Q]) {
    real psi_lo = 0;
    real ps = h[0];
#pragma unroll
    for (int a = 1; a < Q; a++) {
        real e;
        ps = two_sum(ps, h[a], e);
        psi_lo += e;
    }
    real hsum = hk[1], hsum_lo = 0;
#pragma unroll
    for (int a = 2; a < Q; a++) {
        real e;
        hsum = two_sum(hsum, hk[a], e);
        hsum_lo += e;
    }
    real e_q;
    const real psq = two_sum(psi, Qs, e_q);
    return (psq - hsum) + ((psi_lo + e_q) - hsum_lo);
}

}  // namespace lbcg
