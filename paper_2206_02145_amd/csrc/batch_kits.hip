// batch_kits.hip -- instantiations of the batched step kernel (step.hpp, step_batch) and the
// batched ray-march (diag.hpp) for every tiling the batch autotuner may choose. A translation unit
// of its own so that the build compiles it next to the host runtime.
#include <hip/hip_fp16.h>
#include <hip/hip_runtime.h>

#include "../../include/lbcg.h"
#include "diag.hpp"
#include "kits.hpp"
#include "step.hpp"

namespace lbcg {
namespace {

template <int DIM, bool FLOW, typename real, typename fst, int TX, int TY, int TZ, bool PF, int AUX, bool CHM = false,
          int LAUX = 0, int HAUX = -1>
struct BatchImpl {
    static void step(const InstDev* d, int n, int tiles, int par, hipStream_t s) {
        hipLaunchKernelGGL((step_batch<DIM, FLOW, real, fst, TX, TY, TZ, PF, AUX, LAUX, CHM, HAUX>), dim3(tiles),
                           dim3(TX * TY * TZ), 0, s, d, n, par);
    }
    static void ray(const InstDev* d, int n, int par, const double* dirs, int ndirs, const double* centers,
                    double* out, hipStream_t s) {
        hipLaunchKernelGGL((raymarch_batch_kernel<DIM, real>), dim3(ndirs, n), dim3(64), 0, s, d, par, dirs, ndirs,
                           centers, out);
    }
    static BatchKit kit() {
        Tiling t{false, TX, TY, TZ, PF, AUX, LAUX, 0};
        t.chm = CHM;
        t.haux = HAUX;
        return BatchKit{t, step, ray};
    }
};

// Candidates per kind. The BGK flow kind (the parametric sweeps) gets the same tilings the single-grid
// kernel offers (so every batch tiling has a single-grid twin computing bit for bit the same
// update); no flow and the MRT get the default and one alternative.
template <int DIM, typename real, typename fst, bool FLOW, bool CHM>
std::vector<BatchKit> kits_of() {
    constexpr int S = sizeof(real) == 8 ? 0 : 2;  // streaming stores in binary32
    std::vector<BatchKit> v;
    if constexpr (DIM == 2) {
        // binary32 flow: streaming loads and stores of g and f with h and phi_prev kept in the
        // caches first (the 256 sweep instances' 1 GB exceed the last-level cache; 64 x 8 and
        // 64 x 4 tiles measured fastest among these for them, ~199 against 216 us per step for
        // streaming stores alone)
        if constexpr (FLOW && !CHM && S != 0) v.push_back(BatchImpl<2, FLOW, real, fst, 64, 8, 1, false, 2, CHM, 2, 0>::kit());
        v.push_back(BatchImpl<2, FLOW, real, fst, 64, 4, 1, false, S, CHM>::kit());
        if constexpr (FLOW && !CHM) {
            if constexpr (S != 0) v.push_back(BatchImpl<2, FLOW, real, fst, 64, 4, 1, false, 0, CHM>::kit());
            v.push_back(BatchImpl<2, FLOW, real, fst, 64, 4, 1, true, 0, CHM>::kit());
            v.push_back(BatchImpl<2, FLOW, real, fst, 64, 2, 1, true, 2, CHM>::kit());
            v.push_back(BatchImpl<2, FLOW, real, fst, 64, 8, 1, false, 2, CHM>::kit());
            v.push_back(BatchImpl<2, FLOW, real, fst, 128, 2, 1, false, 2, CHM>::kit());
            v.push_back(BatchImpl<2, FLOW, real, fst, 64, 4, 1, false, 2, CHM, 2, 0>::kit());
            if constexpr (S == 0) v.push_back(BatchImpl<2, FLOW, real, fst, 64, 8, 1, false, 2, CHM, 2, 0>::kit());
        } else {
            v.push_back(BatchImpl<2, FLOW, real, fst, 64, 8, 1, false, 2, CHM>::kit());
        }
    } else if constexpr (sizeof(real) == 8) {
        v.push_back(BatchImpl<3, FLOW, real, fst, 16, 4, 4, false, 0, CHM>::kit());
        v.push_back(BatchImpl<3, FLOW, real, fst, 32, 2, 4, true, 0, CHM>::kit());
    } else {
        v.push_back(BatchImpl<3, FLOW, real, fst, 64, 2, 4, false, 2, CHM>::kit());
        if constexpr (FLOW && !CHM) {
            v.push_back(BatchImpl<3, FLOW, real, fst, 64, 2, 4, false, 0, CHM>::kit());
            v.push_back(BatchImpl<3, FLOW, real, fst, 64, 4, 2, true, 0, CHM>::kit());
            v.push_back(BatchImpl<3, FLOW, real, fst, 64, 2, 2, true, 0, CHM>::kit());
            v.push_back(BatchImpl<3, FLOW, real, fst, 64, 2, 4, false, 2, CHM, 2, 0>::kit());
        } else {
            v.push_back(BatchImpl<3, FLOW, real, fst, 64, 2, 2, true, 0, CHM>::kit());
        }
    }
    return v;
}

template <int DIM>
const std::vector<BatchKit>& kits_dim(int kind, int prec) {
    static const std::vector<BatchKit> k[3][3] = {
        {kits_of<DIM, double, double, false, false>(), kits_of<DIM, float, float, false, false>(),
         kits_of<DIM, float, float, false, false>()},
        {kits_of<DIM, double, double, true, false>(), kits_of<DIM, float, float, true, false>(),
         kits_of<DIM, float, __half, true, false>()},
        {kits_of<DIM, double, double, true, true>(), kits_of<DIM, float, float, true, true>(),
         kits_of<DIM, float, __half, true, true>()}};
    return k[kind][prec];
}

}  // namespace

const std::vector<BatchKit>& batch_kits_for(int dim, int kind, int prec) {
    return dim == 2 ? kits_dim<2>(kind, prec) : kits_dim<3>(kind, prec);
}

}  // namespace lbcg
