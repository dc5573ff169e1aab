// lattice.hpp -- velocity sets of the solver, as compile-time tables for device code.
//
// phi and U use D2Q5 / D3Q7 (rest weight 1/3, cs^2 = 1/3 / rest weight 1/4, cs^2 = 1/4); the flow
// uses D2Q9 / D3Q19 (cs^2 = 1/3), whose weights also define the isotropic gradient stencil
// grad phi = (1/cs^2) sum_b w_b c_b phi(x + c_b). The velocity order is part of the C ABI
// (population planes of RAW read/write) and is listed in include/lbcg.h.
#pragma once

#include <hip/hip_runtime.h>

namespace lbcg {

struct D2Q5 {
    static constexpr int Q = 5;
    __host__ __device__ static constexpr int c(int a, int d) {
        constexpr int t[5][3] = {{0, 0, 0}, {1, 0, 0}, {-1, 0, 0}, {0, 1, 0}, {0, -1, 0}};
        return t[a][d];
    }
    __host__ __device__ static constexpr double w(int a) { return a == 0 ? 1.0 / 3.0 : 1.0 / 6.0; }
    __host__ __device__ static constexpr int opp(int a) { return a == 0 ? 0 : ((a & 1) ? a + 1 : a - 1); }
    static constexpr double inv_cs2 = 3.0;
};

struct D3Q7 {
    static constexpr int Q = 7;
    __host__ __device__ static constexpr int c(int a, int d) {
        constexpr int t[7][3] = {{0, 0, 0},  {1, 0, 0}, {-1, 0, 0}, {0, 1, 0},
                                 {0, -1, 0}, {0, 0, 1}, {0, 0, -1}};
        return t[a][d];
    }
    __host__ __device__ static constexpr double w(int a) { return a == 0 ? 0.25 : 0.125; }
    __host__ __device__ static constexpr int opp(int a) { return a == 0 ? 0 : ((a & 1) ? a + 1 : a - 1); }
    static constexpr double inv_cs2 = 4.0;
};

struct D2Q9 {
    static constexpr int Q = 9;
    __host__ __device__ static constexpr int c(int a, int d) {
        constexpr int t[9][3] = {{0, 0, 0},  {1, 0, 0},   {-1, 0, 0}, {0, 1, 0}, {0, -1, 0},
                                 {1, 1, 0},  {-1, -1, 0}, {1, -1, 0}, {-1, 1, 0}};
        return t[a][d];
    }
    __host__ __device__ static constexpr double w(int a) {
        return a == 0 ? 4.0 / 9.0 : (a < 5 ? 1.0 / 9.0 : 1.0 / 36.0);
    }
    __host__ __device__ static constexpr int opp(int a) { return a == 0 ? 0 : ((a & 1) ? a + 1 : a - 1); }
    static constexpr double inv_cs2 = 3.0;
};

struct D3Q19 {
    static constexpr int Q = 19;
    __host__ __device__ static constexpr int c(int a, int d) {
        constexpr int t[19][3] = {{0, 0, 0},   {1, 0, 0},   {-1, 0, 0},  {0, 1, 0},   {0, -1, 0},
                                  {0, 0, 1},   {0, 0, -1},  {1, 1, 0},   {-1, -1, 0}, {1, -1, 0},
                                  {-1, 1, 0},  {1, 0, 1},   {-1, 0, -1}, {1, 0, -1},  {-1, 0, 1},
                                  {0, 1, 1},   {0, -1, -1}, {0, 1, -1},  {0, -1, 1}};
        return t[a][d];
    }
    __host__ __device__ static constexpr double w(int a) {
        return a == 0 ? 1.0 / 3.0 : (a < 7 ? 1.0 / 18.0 : 1.0 / 36.0);
    }
    __host__ __device__ static constexpr int opp(int a) { return a == 0 ? 0 : ((a & 1) ? a + 1 : a - 1); }
    static constexpr double inv_cs2 = 3.0;
};

template <int DIM> struct Lattices;
template <> struct Lattices<2> { using S = D2Q5; using V = D2Q9; };
template <> struct Lattices<3> { using S = D3Q7; using V = D3Q19; };

}  // namespace lbcg
