// kits.hpp -- the step-kernel tiling descriptor and the batched-launch kits, shared by the host
// runtime (lbcg_capi.hip) and the translation unit that instantiates the batched kernels
// (batch_kits.hip).
#pragma once

#include <hip/hip_runtime.h>

#include <vector>

#include "step.hpp"

namespace lbcg {

// Tiling of the step kernel: a TX x TY x TZ block, or (march) TY full rows x TZ planes.
struct Tiling {
    bool march;
    int TX, TY, TZ;
    bool prefetch;  // own populations loaded before the halo barrier
    int aux;        // store cache policy
    int laux = 0;   // cache policy of the single-use loads (g, f, phi_prev)
    int zband = 0;  // z tile-layers per band of the block tile order (0: plain x, y, z order)
    bool walls = false;  // the kernel honours the solid-wall mask
    bool chm = false;    // central-Hermite MRT flow collision
    int haux = -1;       // cache policy of the h stores (-1: aux)
    int gcache = 0;      // with haux = 0: planes of g that keep the default policy as well
};

// One compiled tiling of the batched step (every instance's tiles in one launch) and its
// batched ray-march.
struct BatchKit {
    Tiling tiling;
    void (*step)(const InstDev* d, int n, int tiles, int par, hipStream_t);
    void (*ray)(const InstDev* d, int n, int par, const double* dirs, int ndirs, const double* centers,
                double* out, hipStream_t);
};

// The candidate tilings of the batched step for (dim, kind: 0 no flow, 1 BGK flow, 2 central-Hermite
// MRT flow, precision); the first is the default. The batch autotuner times them.
const std::vector<BatchKit>& batch_kits_for(int dim, int kind, int prec);

}  // namespace lbcg
