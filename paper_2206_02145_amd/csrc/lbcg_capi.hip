// lbcg_capi.hip -- host runtime and C ABI of the coupled LB crystal-growth solver (include/lbcg.h).
//
// The host side validates parameters, lays the caller's device workspace out into ping-pong
// population arrays, picks the kernel instantiation for (dimension, flow, precision), enqueues
// kernels on the caller's stream, and keeps the crystal-size history for the growth-rate fit.
#include <hip/hip_fp16.h>
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdio>
#include <algorithm>
#include <cstring>
#include <map>
#include <mutex>
#include <stdexcept>
#include <string>
#include <type_traits>
#include <vector>

#include "../../include/lbcg.h"
#include "diag.hpp"
#include "errors.hpp"
#include "kits.hpp"
#include "lattice.hpp"
#include "march.hpp"
#include "step.hpp"

using namespace lbcg;

namespace {


struct Error : std::runtime_error {
    lbcg_status code;
    Error(lbcg_status c, const std::string& m) : std::runtime_error(m), code(c) {}
};

#define HIPCHK(call)                                                                          \
    do {                                                                                      \
        hipError_t e_ = (call);                                                               \
        if (e_ != hipSuccess)                                                                 \
            throw Error(LBCG_EDEVICE, std::string(#call) + ": " + hipGetErrorString(e_));     \
    } while (0)

template <typename F> lbcg_status guarded(F&& fn) {
    try {
        fn();
        lbcg::last_error_slot().clear();
        return LBCG_OK;
    } catch (const Error& e) {
        lbcg::last_error_slot() = e.what();
        return e.code;
    } catch (const std::exception& e) {
        lbcg::last_error_slot() = e.what();
        return LBCG_EDEVICE;
    }
}

size_t align256(size_t b) { return (b + 255) & ~size_t(255); }

int qs_of(int dim) { return dim == 2 ? 5 : 7; }
int qf_of(int dim) { return dim == 2 ? 9 : 19; }
size_t real_size(int prec) { return prec == LBCG_FP64 ? 8 : 4; }
size_t fstore_size(int prec) { return prec == LBCG_FP64 ? 8 : (prec == LBCG_FP32 ? 4 : 2); }

constexpr int MAX_DIRS = 256;
constexpr int RED_BLOCKS = 1024;
constexpr int HIST_DOUBLES = 4096;  // on-device measurement history of lbcg_run (32 KB)

// Validation shared by single and batched creation; throws Error.
void validate(const lbcg_params* p) {
    if (!p) throw Error(LBCG_EINVAL, "params is NULL");
    if (p->dim != 2 && p->dim != 3) throw Error(LBCG_EINVAL, "dim must be 2 or 3");
    if (p->nx < 1 || p->ny < 1 || p->nz < 1) throw Error(LBCG_EINVAL, "grid sizes must be >= 1");
    if (p->dim == 2 && p->nz != 1) throw Error(LBCG_EINVAL, "nz must be 1 when dim = 2");
    if (p->flow != 0 && p->flow != 1) throw Error(LBCG_EINVAL, "flow must be 0 or 1");
    if (p->precision < LBCG_FP64 || p->precision > LBCG_FP32_F16SHIFT)
        throw Error(LBCG_EINVAL, "unknown precision");
    if (p->precision == LBCG_FP32_F16SHIFT && !p->flow)
        throw Error(LBCG_EINVAL, "the binary16 shifted storage applies to the flow populations (flow = 1)");
    if (p->xbc != LBCG_PERIODIC && p->xbc != LBCG_INFLOW_OUTFLOW && p->xbc != LBCG_INFLOW_PRESSURE)
        throw Error(LBCG_EINVAL, "unknown xbc");
    if (p->xbc != LBCG_PERIODIC && p->nx < 3) throw Error(LBCG_EINVAL, "open x faces need nx >= 3");
    if (p->walls != 0 && p->walls != 1) throw Error(LBCG_EINVAL, "walls must be 0 or 1");
    if (p->seed_shape < LBCG_SEED_CIRCLE || p->seed_shape > LBCG_SEED_RHOMBUS) throw Error(LBCG_EINVAL, "unknown seed shape");
    if (p->collision != LBCG_COLLISION_BGK && p->collision != LBCG_COLLISION_CHMRT)
        throw Error(LBCG_EINVAL, "unknown collision");
    if (p->collision == LBCG_COLLISION_CHMRT && !p->flow)
        throw Error(LBCG_EINVAL, "the central-Hermite MRT collision applies to the flow populations (flow = 1)");
    const double N = (double)p->nx * p->ny * p->nz;
    if (N >= 536870912.0)  // each population plane is addressed with 32-bit byte offsets
        throw Error(LBCG_EINVAL, "grid too large (at most 2^29 - 1 nodes)");
    const double vals[] = {p->W0, p->tau0, p->lambda, p->D, p->eps_aniso, p->nu, p->h_drag,
                           p->u_inlet, p->U0, p->U_inlet, p->seed_center[0], p->seed_center[1],
                           p->seed_center[2], p->seed_radius, p->grad_eps2, p->seed_tilt, p->omega_bulk};
    for (double v : vals)
        if (!std::isfinite(v)) throw Error(LBCG_EINVAL, "non-finite parameter");
    if (!(p->tau0 > 0) || !(p->W0 > 0))
        throw Error(LBCG_EUNSTABLE, "tau0 and W0 must be > 0 (tau_phi = a_s^2 W0^2/(tau0 cs^2) + 1/2 > 1/2)");
    if (!(p->eps_aniso >= 0 && p->eps_aniso < 1))
        throw Error(LBCG_EUNSTABLE, "eps_aniso must lie in [0, 1) so that a_s > 0");
    if (!(p->D >= 0)) throw Error(LBCG_EUNSTABLE, "D must be >= 0 (tau_U >= 1/2)");
    if (p->flow && !(p->nu > 0)) throw Error(LBCG_EUNSTABLE, "nu must be > 0 (tau_f > 1/2)");
    if (!(p->grad_eps2 >= 0)) throw Error(LBCG_EINVAL, "grad_eps2 must be >= 0");
    if (p->collision == LBCG_COLLISION_CHMRT && !(p->omega_bulk > 0 && p->omega_bulk < 2))
        throw Error(LBCG_EUNSTABLE, "omega_bulk must lie in (0, 2)");
    if (p->solute_source != LBCG_SOURCE_FULL && p->solute_source != LBCG_SOURCE_HALF)
        throw Error(LBCG_EINVAL, "solute_source must be 0 (full) or 1 (half)");
}

struct Layout {
    size_t h[2], g[2], f[2], phi_prev, staging, partials, dirs, out, hist, wall, total;  // wall: 0 = none
};

// Plane stride of the population arrays: N rounded up to 64 nodes, plus 64. Planes whose byte size
// is a multiple of a large power of two otherwise all start at the same offset of the memory
// interleave, and the step's concurrent plane streams collide there (256 x 128 x 128: 289 ->
// 255 us per step on MI355X; other grids unchanged). Dropped when a binary64 plane would reach
// 2^32 bytes, the reach of the kernels' 32-bit byte offsets.
size_t plane_stride(size_t N) {
    const size_t s = (N + 63) / 64 * 64 + 64;
    return s * 8 < (size_t(1) << 32) ? s : N;
}

// Stored row length: nx rounded up to 64 nodes, so that every row starts on a 256-byte boundary in
// binary32 (128 bytes for binary16 flow storage) and a wavefront's 64-node segment covers whole
// cache lines (rows of other lengths cost up to 1.5x per node on MI355X). nx itself where the
// padded binary64 plane would reach 2^32 bytes.
int row_pitch(const lbcg_params* p) {
    const size_t r = ((size_t)p->nx + 63) / 64 * 64;
    return (size_t)p->nz * p->ny * r * 8 < (size_t(1) << 32) ? (int)r : p->nx;
}
size_t stored_nodes(const lbcg_params* p) { return (size_t)p->nz * p->ny * row_pitch(p); }

Layout layout_of(const lbcg_params* p) {
    const size_t N0 = (size_t)p->nx * p->ny * p->nz, Nm = stored_nodes(p), N = plane_stride(Nm);
    const size_t rs = real_size(p->precision), fs = fstore_size(p->precision);
    Layout L{};
    size_t off = 0;
    auto take = [&](size_t bytes) {
        size_t o = off;
        off += align256(bytes);
        return o;
    };
    for (int k = 0; k < 2; k++) L.h[k] = take(qs_of(p->dim) * N * rs);
    for (int k = 0; k < 2; k++) L.g[k] = take(qs_of(p->dim) * N * rs);
    for (int k = 0; k < 2; k++) L.f[k] = p->flow ? take(qf_of(p->dim) * N * fs) : 0;
    L.phi_prev = take(Nm * rs);
    L.staging = take(N0 * 8);
    L.partials = take((RED_BLOCKS + 1) * RED_VALUES * 8);  // block partials, then the final values
    L.dirs = take(MAX_DIRS * 3 * 8);
    L.out = take((RED_VALUES + MAX_DIRS) * 8);
    L.hist = take(HIST_DOUBLES * 8);
    L.wall = p->walls ? take(Nm) : 0;
    L.total = off;
    return L;
}


InstDev make_inst(const lbcg_params* p, char* ws, const Layout& L, const Tiling& T) {
    InstDev I{};
    I.nx = p->nx;
    I.ny = p->ny;
    I.nz = p->nz;
    I.xopen = p->xbc != LBCG_PERIODIC;
    I.xpress = p->xbc == LBCG_INFLOW_PRESSURE;
    I.tiles_x = T.march ? 1 : (p->nx + T.TX - 1) / T.TX;
    I.tiles_y = (p->ny + T.TY - 1) / T.TY;
    I.tiles_z = p->dim == 3 ? (p->nz + T.TZ - 1) / T.TZ : 1;
    I.tile_begin = 0;
    I.zc = T.TZ;
    I.zband = T.march ? 0 : T.zband;
    I.N = (long long)p->nx * p->ny * p->nz;
    I.pitch = row_pitch(p);
    I.Nm = (long long)stored_nodes(p);
    I.Np = (long long)plane_stride((size_t)I.Nm);
    for (int k = 0; k < 2; k++) {
        I.h[k] = ws + L.h[k];
        I.g[k] = ws + L.g[k];
        I.f[k] = p->flow ? ws + L.f[k] : nullptr;
    }
    I.phi_prev = ws + L.phi_prev;
    I.wall = p->walls ? reinterpret_cast<const unsigned char*>(ws + L.wall) : nullptr;
    I.k = p->W0 * p->W0 / p->tau0;
    I.inv_tau0 = 1.0 / p->tau0;
    I.lambda = p->lambda;
    I.eps = p->eps_aniso;
    I.grad_eps2 = p->grad_eps2;
    I.D = p->D;
    I.tau_f = p->flow ? p->nu * 3.0 + 0.5 : 1.0;
    I.kdrag = p->h_drag * I.tau_f / (4.0 * p->W0 * p->W0);
    I.u_in = p->u_inlet;
    I.U_in = p->U_inlet;
    I.U0 = p->U0;
    const double inv_cs2 = p->dim == 3 ? 4.0 : 3.0;  // D3Q7 / D2Q5
    I.kd[K_EPS] = I.eps;
    I.kd[K_GEPS2] = I.grad_eps2;
    I.kd[K_KC] = I.k * inv_cs2;
    I.kd[K_LAMBDA] = I.lambda;
    I.kd[K_ITAU0] = I.inv_tau0;
    I.kd[K_U0] = I.U0;
    I.kd[K_KDRAG] = I.kdrag;
    I.kd[K_ITAUF] = 1.0 / I.tau_f;
    I.kd[K_GUO] = 1.0 - 0.5 / I.tau_f;
    I.kd[K_UIN] = I.u_in;
    I.kd[K_DQ] = I.D * inv_cs2;
    I.kd[K_UIN2] = 2.0 * (I.U_in - I.U0);
    I.kd[K_OMB] = p->collision == LBCG_COLLISION_CHMRT ? p->omega_bulk : 1.0;
    I.kd[K_CT] = p->seed_tilt == 0.0 ? 1.0 : std::cos(p->seed_tilt);
    I.kd[K_ST] = p->seed_tilt == 0.0 ? 0.0 : std::sin(p->seed_tilt);
    I.kd[K_SRC] = p->solute_source == LBCG_SOURCE_HALF ? 0.5 : 1.0;
    for (int k = 0; k < 16; k++) I.kf[k] = (float)I.kd[k];
    return I;
}

// ---- kernel dispatch per (dim, flow, precision, row length) ----
struct Ops {
    Tiling tiling;
    void (*step)(const InstDev&, int par, hipStream_t);
    void (*init)(const InstDev&, int par, const SeedArgs&, hipStream_t);
    void (*field)(const InstDev&, int par, int field, void* out, int dtype, hipStream_t);
    void (*reduce)(const InstDev&, int par, double* partials, int nblocks, double* out, hipStream_t);
    void (*ray)(const InstDev&, int par, const double* dirs, int ndirs, const double* c, double* out,
                hipStream_t);
};

// Stored plane = value - shift: h is kept as h + w, g as g - w U0, f as f - w, phi_prev as phi_prev + 1.
double plane_shift(const lbcg_params& p, int field, int a) {
    const double ws = p.dim == 2 ? D2Q5::w(a) : D3Q7::w(a);
    switch (field) {
        case LBCG_FIELD_RAW_H: return -ws;
        case LBCG_FIELD_RAW_G: return ws * p.U0;
        case LBCG_FIELD_RAW_F: return p.dim == 2 ? D2Q9::w(a) : D3Q19::w(a);
        default: return -1.0;  // PHI_PREV
    }
}

// x-velocity of plane a of a population array (its column shift in the stored layout).
int plane_cx(const lbcg_params& p, int field, int a) {
    switch (field) {
        case LBCG_FIELD_RAW_H:
        case LBCG_FIELD_RAW_G: return p.dim == 2 ? D2Q5::c(a, 0) : D3Q7::c(a, 0);
        case LBCG_FIELD_RAW_F: return p.dim == 2 ? D2Q9::c(a, 0) : D3Q19::c(a, 0);
        default: return 0;  // PHI_PREV
    }
}

int grid_for(long long n, int threads, int cap) {
    long long b = (n + threads - 1) / threads;
    if (b > cap) b = cap;
    if (b < 1) b = 1;
    return (int)b;
}

// Everything except the step kernel: shared by every tiling of one (dim, flow, precision).
template <int DIM, bool FLOW, typename real, typename fst>
struct CommonOps {
    static void init(const InstDev& I, int par, const SeedArgs& a, hipStream_t s) {
        hipLaunchKernelGGL((init_kernel<DIM, FLOW, real, fst>), dim3(grid_for(I.N, 256, 65536)), dim3(256),
                           0, s, I, par, a);
    }
    static void field(const InstDev& I, int par, int field, void* out, int dtype, hipStream_t s) {
        const int nb = grid_for(I.N, 256, 65536);
        if (dtype == LBCG_DTYPE_F64)
            hipLaunchKernelGGL((field_kernel<DIM, FLOW, real, fst, double>), dim3(nb), dim3(256), 0, s, I, par,
                               field, (double*)out);
        else
            hipLaunchKernelGGL((field_kernel<DIM, FLOW, real, fst, float>), dim3(nb), dim3(256), 0, s, I, par,
                               field, (float*)out);
    }
    static void reduce(const InstDev& I, int par, double* partials, int nblocks, double* out, hipStream_t s) {
        hipLaunchKernelGGL((reduce_kernel<DIM, FLOW, real, fst>), dim3(nblocks), dim3(RED_THREADS), 0, s, I,
                           par, partials);
        hipLaunchKernelGGL(reduce_final, dim3(1), dim3(64), 0, s, partials, nblocks, out);
    }
    static void ray(const InstDev& I, int par, const double* dirs, int ndirs, const double* c, double* out,
                    hipStream_t s) {
        hipLaunchKernelGGL((raymarch_kernel<DIM, real>), dim3(ndirs), dim3(64), 0, s, I, par, dirs, c[0], c[1],
                           c[2], out);
    }
};

template <int DIM, bool FLOW, typename real, typename fst, int TX, int TY, int TZ, bool PF = false, int AUX = 0,
          int LAUX = 0, bool WALLS = false, bool CHM = false, int HAUX = -1, int GC = 0>
struct BlockOps : CommonOps<DIM, FLOW, real, fst> {
    using C = CommonOps<DIM, FLOW, real, fst>;
    static void step(const InstDev& I, int par, hipStream_t s) {
        const int nblocks = I.tiles_x * I.tiles_y * I.tiles_z;
        hipLaunchKernelGGL((step_single<DIM, FLOW, real, fst, TX, TY, TZ, PF, AUX, LAUX, WALLS, CHM, HAUX, GC>),
                           dim3(nblocks), dim3(TX * TY * TZ), 0, s, I, par);
    }
    static Ops ops() {
        Tiling t{false, TX, TY, TZ, PF, AUX, LAUX, 0};
        t.walls = WALLS;
        t.chm = CHM;
        t.haux = HAUX;
        t.gcache = HAUX == 0 ? GC : 0;
        return Ops{t, step, C::init, C::field, C::reduce, C::ray};
    }
};

template <bool FLOW, typename real, typename fst, int NW, int TY>
struct MarchOps : CommonOps<3, FLOW, real, fst> {
    using C = CommonOps<3, FLOW, real, fst>;
    static void step(const InstDev& I, int par, hipStream_t s) {
        const int nblocks = I.tiles_y * I.tiles_z;
        hipLaunchKernelGGL((march3d_single<FLOW, real, fst, NW, TY>), dim3(nblocks), dim3(64 * NW * TY), 0, s,
                           I, par, I.zc);
    }
    static Ops ops() { return Ops{Tiling{true, 64 * NW, TY, 16, true, 0, 0, 0}, step, C::init, C::field, C::reduce, C::ray}; }
};

// A variant = kernel instantiation + tiling (the z-marching kernel takes its plane count at run time).
struct Variant {
    const Ops* ops;
    Tiling tiling;
};

template <bool FLOW, typename real, typename fst, int TY>
const Ops* march_ops(int nx) {
    static const Ops m1 = MarchOps<FLOW, real, fst, 1, TY>::ops();
    static const Ops m2 = MarchOps<FLOW, real, fst, 2, TY>::ops();
    static const Ops m3 = MarchOps<FLOW, real, fst, 3, TY>::ops();
    static const Ops m4 = MarchOps<FLOW, real, fst, 4, TY>::ops();
    return nx <= 64 ? &m1 : nx <= 128 ? &m2 : nx <= 192 ? &m3 : &m4;
}

constexpr int MARCH_MAX_NX = 256;

// Non-temporal population stores pay off once the two population copies exceed what the 256 MB
// last-level (Infinity) cache holds; below that the next step re-reads them from that cache.
constexpr double LLC_BYTES = 256.0 * 1024 * 1024;

template <int DIM, bool FLOW, typename real, typename fst>
void block_variants(std::vector<Variant>& v, bool large, int gdef, int zdef) {
    auto add = [&](const Ops& o) { v.push_back({&o, o.tiling}); };
    if constexpr (DIM == 2) {
        static const Ops a = BlockOps<2, FLOW, real, fst, 64, 4, 1, false, sizeof(real) == 8 ? 0 : 2>::ops();
        static const Ops a0 = BlockOps<2, FLOW, real, fst, 64, 4, 1, false, 0>::ops();
        static const Ops b = BlockOps<2, FLOW, real, fst, 64, 4, 1, true>::ops();
        static const Ops c = BlockOps<2, FLOW, real, fst, 64, 2, 1, true, 2>::ops();
        static const Ops d = BlockOps<2, FLOW, real, fst, 64, 8, 1, false, 2>::ops();
        static const Ops e = BlockOps<2, FLOW, real, fst, 128, 2, 1, false, 2>::ops();
        // streaming loads and stores of g and f, h and phi_prev kept in the caches (see step_tile)
        static const Ops k = BlockOps<2, FLOW, real, fst, 64, 4, 1, false, 2, 2, false, false, 0>::ops();
        static const Ops k8 = BlockOps<2, FLOW, real, fst, 64, 8, 1, false, 2, 2, false, false, 0>::ops();
        if (large) for (const Ops* o : {&k, &a, &a0, &b, &c, &d, &e, &k8}) add(*o);
        else if (sizeof(real) == 8) for (const Ops* o : {&a, &a0, &b, &c, &d, &e, &k, &k8}) add(*o);
        else for (const Ops* o : {&a0, &a, &b, &c, &d, &e, &k, &k8}) add(*o);
    } else if constexpr (sizeof(real) == 8) {
        static const Ops a = BlockOps<3, FLOW, real, fst, 16, 4, 4>::ops();
        static const Ops b = BlockOps<3, FLOW, real, fst, 32, 2, 4, true>::ops();
        static const Ops k = BlockOps<3, FLOW, real, fst, 16, 4, 4, false, 2, 2, false, false, 0>::ops();
        if (large) for (const Ops* o : {&k, &a, &b}) add(*o);
        else for (const Ops* o : {&a, &b, &k}) add(*o);
    } else {
        static const Ops a0 = BlockOps<3, FLOW, real, fst, 64, 2, 4, false, 0>::ops();
        static const Ops a1 = BlockOps<3, FLOW, real, fst, 64, 2, 4, true, 0>::ops();
        static const Ops a2 = BlockOps<3, FLOW, real, fst, 64, 2, 4, false, 2>::ops();
        static const Ops a3 = BlockOps<3, FLOW, real, fst, 64, 2, 4, true, 2>::ops();
        static const Ops b0 = BlockOps<3, FLOW, real, fst, 64, 4, 2, true>::ops();
        static const Ops b1 = BlockOps<3, FLOW, real, fst, 64, 1, 8, true>::ops();
        static const Ops b2 = BlockOps<3, FLOW, real, fst, 64, 4, 4, true>::ops();
        static const Ops b3 = BlockOps<3, FLOW, real, fst, 64, 2, 2, true>::ops();
        static const Ops c0 = BlockOps<3, FLOW, real, fst, 32, 8, 2>::ops();
        static const Ops c1 = BlockOps<3, FLOW, real, fst, 32, 8, 2, true>::ops();
        static const Ops c2 = BlockOps<3, FLOW, real, fst, 32, 4, 4, true>::ops();
        static const Ops d0 = BlockOps<3, FLOW, real, fst, 64, 2, 4, false, 2, 2>::ops();
        // streaming loads and stores of g and f, h and phi_prev kept in the caches (see step_tile)
        static const Ops k0 = BlockOps<3, FLOW, real, fst, 64, 2, 4, false, 2, 2, false, false, 0>::ops();
        // the same with 2 or 3 planes of g kept in the caches as well
        static const Ops k2 = BlockOps<3, FLOW, real, fst, 64, 2, 4, false, 2, 2, false, false, 0, 2>::ops();
        static const Ops k3 = BlockOps<3, FLOW, real, fst, 64, 2, 4, false, 2, 2, false, false, 0, 3>::ops();
        const Ops* kd = gdef >= 3 ? &k3 : (gdef == 2 ? &k2 : &k0);
        auto band = [&](const Ops& o, int zband) {  // the same kernel with a banded tile order
            Tiling t = o.tiling;
            t.zband = zband;
            v.push_back({&o, t});
        };
        // first = default: 64 x 2 x 4 (one wavefront per x-row); when the two population copies
        // exceed the last-level cache, streaming loads and stores of g and f with h and phi_prev
        // kept in the caches, and gdef planes of g with them (the fastest measured on the
        // 192 x 128 x 128 flow grid, also with binary16 flow storage); when not even h and phi_prev
        // fit (gdef < 0), streaming stores in bands of zdef z tile-layers, whose halo re-reads of h
        // then still find it in L2 (384 x 256 x 256, bands of 16: 1464 against 1583 us for h kept
        // in the caches; 512 x 512 x 256, bands of 8: 3794 against 3957); below the cache size,
        // the default policy
        if (large && gdef < 0) {
            band(a2, zdef);
            for (const Ops* o : {&k0, &k2, &k3, &a2, &a3, &a0, &a1, &d0}) add(*o);
        } else if (large) {
            add(*kd);
            for (const Ops* o : {&k0, &k2, &k3})
                if (o != kd) add(*o);
            for (const Ops* o : {&a2, &a3, &a0, &a1, &d0}) add(*o);
        } else for (const Ops* o : {&a0, &a1, &a2, &a3, &d0, &k0, &k2, &k3}) add(*o);
        for (int zb : {2, 4, 8, 16})
            if (!(large && gdef < 0 && zb == zdef)) band(large ? a2 : a0, zb);
        band(large ? a3 : a1, 4);
        for (const Ops* o : {&b0, &b1, &b2, &b3, &c0, &c1, &c2}) add(*o);
    }
}

// Tilings of the kernel that honours a wall mask (the first is the default).
template <int DIM, bool FLOW, typename real, typename fst>
std::vector<Variant> wall_variants(bool large, int gdef, int zdef) {
    std::vector<Variant> v;
    auto add = [&](const Ops& o) { v.push_back({&o, o.tiling}); };
    if constexpr (DIM == 2) {
        static const Ops a = BlockOps<2, FLOW, real, fst, 64, 4, 1, false, 0, 0, true>::ops();
        add(a);
    } else if constexpr (sizeof(real) == 8) {
        static const Ops a = BlockOps<3, FLOW, real, fst, 16, 4, 4, false, 0, 0, true>::ops();
        add(a);
    } else {
        static const Ops a = BlockOps<3, FLOW, real, fst, 64, 2, 4, false, 0, 0, true>::ops();
        static const Ops b = BlockOps<3, FLOW, real, fst, 64, 2, 4, false, 2, 0, true>::ops();
        static const Ops k = BlockOps<3, FLOW, real, fst, 64, 2, 4, false, 2, 2, true, false, 0>::ops();
        static const Ops k2 = BlockOps<3, FLOW, real, fst, 64, 2, 4, false, 2, 2, true, false, 0, 2>::ops();
        Tiling banded = b.tiling;  // streaming stores in bands of z tile-layers (see block_variants)
        banded.zband = zdef;
        if (large && gdef < 0) {
            v.push_back({&b, banded});
            for (const Ops* o : {&k, &k2, &b, &a}) add(*o);
            return v;
        }
        if (large && gdef >= 2) for (const Ops* o : {&k2, &k, &b, &a}) add(*o);
        else if (large) for (const Ops* o : {&k, &k2, &b, &a}) add(*o);
        else for (const Ops* o : {&a, &b, &k, &k2}) add(*o);
        v.push_back({&b, banded});
    }
    return v;
}

// Tilings of the central-Hermite MRT flow kernel, with or without walls (the first is the default).
template <int DIM, typename real, typename fst>
std::vector<Variant> chm_variants(bool large, bool walls, int gdef, int zdef) {
    std::vector<Variant> v;
    auto add = [&](const Ops& o) { v.push_back({&o, o.tiling}); };
    if constexpr (DIM == 2) {
        static const Ops a = BlockOps<2, true, real, fst, 64, 4, 1, false, 0, 0, false, true>::ops();
        static const Ops b = BlockOps<2, true, real, fst, 64, 4, 1, false, 2, 0, false, true>::ops();
        static const Ops w = BlockOps<2, true, real, fst, 64, 4, 1, false, 0, 0, true, true>::ops();
        static const Ops k = BlockOps<2, true, real, fst, 64, 4, 1, false, 2, 2, false, true, 0>::ops();
        if (walls) add(w);
        else if (large) for (const Ops* o : {&k, &b, &a}) add(*o);
        else if (sizeof(real) == 8) for (const Ops* o : {&b, &a, &k}) add(*o);
        else for (const Ops* o : {&a, &b, &k}) add(*o);
    } else if constexpr (sizeof(real) == 8) {
        static const Ops a = BlockOps<3, true, real, fst, 16, 4, 4, false, 0, 0, false, true>::ops();
        static const Ops w = BlockOps<3, true, real, fst, 16, 4, 4, false, 0, 0, true, true>::ops();
        add(walls ? w : a);
    } else {
        static const Ops a0 = BlockOps<3, true, real, fst, 64, 2, 4, false, 0, 0, false, true>::ops();
        static const Ops a2 = BlockOps<3, true, real, fst, 64, 2, 4, false, 2, 0, false, true>::ops();
        static const Ops a3 = BlockOps<3, true, real, fst, 64, 2, 4, true, 2, 0, false, true>::ops();
        static const Ops w = BlockOps<3, true, real, fst, 64, 2, 4, false, 0, 0, true, true>::ops();
        static const Ops k = BlockOps<3, true, real, fst, 64, 2, 4, false, 2, 2, false, true, 0>::ops();
        static const Ops k2 = BlockOps<3, true, real, fst, 64, 2, 4, false, 2, 2, false, true, 0, 2>::ops();
        static const Ops wk = BlockOps<3, true, real, fst, 64, 2, 4, false, 2, 2, true, true, 0>::ops();
        Tiling banded = a2.tiling;  // streaming stores in bands of z tile-layers (see block_variants)
        banded.zband = zdef;
        if (walls && large) {
            add(wk);
            add(w);
        } else if (walls) {
            add(w);
            add(wk);
        } else if (large && gdef < 0) {
            v.push_back({&a2, banded});
            for (const Ops* o : {&k, &k2, &a2, &a3, &a0}) add(*o);
        } else if (large && gdef >= 2) for (const Ops* o : {&k2, &k, &a2, &a3, &a0}) add(*o);
        else if (large) for (const Ops* o : {&k, &k2, &a2, &a3, &a0}) add(*o);
        else for (const Ops* o : {&a0, &a2, &a3, &k, &k2}) add(*o);
        if (!walls && !(large && gdef < 0)) v.push_back({&a2, banded});
    }
    return v;
}

template <int DIM, bool FLOW, typename real, typename fst>
std::vector<Variant> variants_of(int nx, double pop_bytes, bool walls, bool chm, int gdef, int zdef) {
    if constexpr (FLOW) {
        if (chm) return chm_variants<DIM, real, fst>(pop_bytes > LLC_BYTES, walls, gdef, zdef);
    }
    if (walls) return wall_variants<DIM, FLOW, real, fst>(pop_bytes > LLC_BYTES, gdef, zdef);
    std::vector<Variant> v;
    block_variants<DIM, FLOW, real, fst>(v, pop_bytes > LLC_BYTES, gdef, zdef);
    if constexpr (DIM == 3) {
        if (nx > 0 && nx <= MARCH_MAX_NX) {  // (nx = 0: not offered)
            // z-marching kernels (rows of up to 256 nodes) as further candidates
            const int zcs[] = {8, 16, 4, 32};
            for (int zc : zcs) {
                const Ops* o = march_ops<FLOW, real, fst, 2>(nx);
                v.push_back({o, Tiling{true, o->tiling.TX, 2, zc, true, 0, 0, 0}});
            }
            for (int zc : zcs) {
                const Ops* o = march_ops<FLOW, real, fst, 1>(nx);
                v.push_back({o, Tiling{true, o->tiling.TX, 1, zc, true, 0, 0, 0}});
            }
            if constexpr (sizeof(real) == 4) {
                for (int zc : zcs) {
                    const Ops* o = march_ops<FLOW, real, fst, 4>(nx);
                    v.push_back({o, Tiling{true, o->tiling.TX, 4, zc, true, 0, 0, 0}});
                }
            }
        }
    }
    return v;
}

// Candidate tilings for one grid kind; the first is the default. pop_bytes: both population copies;
// gdef: planes of g the default keeps in the caches beside h and phi_prev (default_gcache); zdef:
// the z-band of the default where not even h and phi_prev fit (default_zband).
std::vector<Variant> variants_for(int dim, int flow, int prec, int nx, double pop_bytes, bool walls, bool chm,
                                  int gdef, int zdef) {
    const double b = pop_bytes;
    const int g = gdef, zb = zdef;
    if (dim == 2) {
        if (!flow) return prec == LBCG_FP64 ? variants_of<2, false, double, double>(nx, b, walls, false, g, zb) : variants_of<2, false, float, float>(nx, b, walls, false, g, zb);
        return prec == LBCG_FP64   ? variants_of<2, true, double, double>(nx, b, walls, chm, g, zb)
               : prec == LBCG_FP32 ? variants_of<2, true, float, float>(nx, b, walls, chm, g, zb)
                                   : variants_of<2, true, float, __half>(nx, b, walls, chm, g, zb);
    }
    if (!flow) return prec == LBCG_FP64 ? variants_of<3, false, double, double>(nx, b, walls, false, g, zb) : variants_of<3, false, float, float>(nx, b, walls, false, g, zb);
    return prec == LBCG_FP64   ? variants_of<3, true, double, double>(nx, b, walls, chm, g, zb)
           : prec == LBCG_FP32 ? variants_of<3, true, float, float>(nx, b, walls, chm, g, zb)
                               : variants_of<3, true, float, __half>(nx, b, walls, chm, g, zb);
}

// What the step keeps in the caches between steps (h, phi_prev and the first planes of g) pays only
// while it fits well inside the 256 MB last-level cache: on the 192 x 128 x 128 flow grid 10 planes
// (126 MB) gained 3.8 %, 11 (138 MB) 5.3 %, 12 (151 MB) lost 2 %, and on 256 x 128 x 128 a ninth
// plane (151 MB) lost 4 %. The default keeps 3 or 2 planes of g when everything kept stays within
// 128 MiB, else none, and -1 says that not even h and phi_prev fit; the autotuner can choose
// otherwise.
constexpr double CACHE_KEEP_BYTES = 128.0 * 1024 * 1024;
int default_gcache(const lbcg_params& p) {
    const double plane = (double)stored_nodes(&p) * real_size(p.precision);
    for (int k : {3, 2})
        if ((qs_of(p.dim) + 1 + k) * plane <= CACHE_KEEP_BYTES) return k;
    return (qs_of(p.dim) + 1) * plane <= CACHE_KEEP_BYTES ? 0 : -1;
}

// The z-band of the tile order where h no longer stays in the caches between steps: a tile's y
// neighbours then run (x tiles) x (band) tiles apart, and both they and its z neighbours should
// still be among the tiles that an XCD holds at once (some 96 of 64 x 2 x 4, whose halo rows then
// come from its L2): the largest power of two up to 96 / (x tiles), between 4 and 16 (measured:
// 6 x tiles, 16 best; 8 x tiles, 8 best).
int default_zband(const lbcg_params& p) {
    const int ntx = (p.nx + 63) / 64;
    int b = 16;
    while (b > 4 && b * ntx > 96) b /= 2;
    return b;
}

double population_bytes(const lbcg_params& p) {
    const double N = (double)p.nx * p.ny * p.nz;
    return 2.0 * N * (2.0 * qs_of(p.dim) * real_size(p.precision) + (p.flow ? qf_of(p.dim) * fstore_size(p.precision) : 0.0));
}

std::string variant_name(const Variant& v) {
    const Tiling& t = v.tiling;
    char buf[96];
    if (t.march)
        std::snprintf(buf, sizeof buf, "march rows=%d x %d planes (row %d)", t.TY, t.TZ, t.TX);
    else
        std::snprintf(buf, sizeof buf, "block %dx%dx%d%s%s%s", t.TX, t.TY, t.TZ, t.prefetch ? " prefetch" : "",
                      t.aux ? " nt-stores" : "", t.laux ? " nt-loads" : "");
        if (t.zband > 1) std::snprintf(buf + std::strlen(buf), sizeof buf - std::strlen(buf), " zband %d", t.zband);
        if (t.walls) std::snprintf(buf + std::strlen(buf), sizeof buf - std::strlen(buf), " walls");
        if (t.chm) std::snprintf(buf + std::strlen(buf), sizeof buf - std::strlen(buf), " chmrt");
        if (t.haux >= 0 && t.haux != t.aux)
            std::snprintf(buf + std::strlen(buf), sizeof buf - std::strlen(buf), " h-cached");
        if (t.gcache > 0) std::snprintf(buf + std::strlen(buf), sizeof buf - std::strlen(buf), " g%d-cached", t.gcache);
    return buf;
}

// Plane a of a raw array (base = the array) into out, decoded to the plain layout.
template <typename real, typename st>
void raw_read_t(const lbcg_params& p, const void* base, int field, int a, long long N, void* out, int dtype,
                hipStream_t s) {
    const int pitch = row_pitch(&p);
    const long long nm = (long long)stored_nodes(&p);
    const st* src = (const st*)base + (size_t)a * plane_stride((size_t)nm);
    const int nb = grid_for(N, 256, 65536);
    const int cx = plane_cx(p, field, a);
    const double sh = plane_shift(p, field, a);
    if (dtype == LBCG_DTYPE_F64)
        hipLaunchKernelGGL((raw_read_kernel<real, st, double>), dim3(nb), dim3(256), 0, s, src, N, p.nx, pitch, nm, cx, sh,
                           (double*)out);
    else
        hipLaunchKernelGGL((raw_read_kernel<real, st, float>), dim3(nb), dim3(256), 0, s, src, N, p.nx, pitch, nm, cx, sh,
                           (float*)out);
}

template <typename real, typename st>
void raw_write_t(const lbcg_params& p, void* base, int field, int a, long long N, const void* in, int dtype,
                 hipStream_t s) {
    const int pitch = row_pitch(&p);
    const long long nm = (long long)stored_nodes(&p);
    st* dst = (st*)base + (size_t)a * plane_stride((size_t)nm);
    const int nb = grid_for(N, 256, 65536);
    const int cx = plane_cx(p, field, a);
    const double sh = plane_shift(p, field, a);
    if (dtype == LBCG_DTYPE_F64)
        hipLaunchKernelGGL((raw_write_kernel<real, st, double>), dim3(nb), dim3(256), 0, s, dst, N, p.nx, pitch, nm, cx, sh,
                           (const double*)in);
    else
        hipLaunchKernelGGL((raw_write_kernel<real, st, float>), dim3(nb), dim3(256), 0, s, dst, N, p.nx, pitch, nm, cx, sh,
                           (const float*)in);
}

int storage_kind(const lbcg_params& p, int field) {  // 0 double, 1 float, 2 half
    if (p.precision == LBCG_FP64) return 0;
    return (field == LBCG_FIELD_RAW_F && p.precision == LBCG_FP32_F16SHIFT) ? 2 : 1;
}


// ---- batched launches (many independent grids of one kind; kernels in batch_kits.hip) ----

// Per-instance population buffers inside a batch workspace (the single-grid layout without its
// staging and diagnostics areas).
Layout instance_layout(const lbcg_params* p, size_t& off) {
    const size_t Nm = stored_nodes(p), N = plane_stride(Nm);
    const size_t rs = real_size(p->precision), fs = fstore_size(p->precision);
    Layout L{};
    auto take = [&](size_t bytes) {
        size_t o = off;
        off += align256(bytes);
        return o;
    };
    for (int k = 0; k < 2; k++) L.h[k] = take(qs_of(p->dim) * N * rs);
    for (int k = 0; k < 2; k++) L.g[k] = take(qs_of(p->dim) * N * rs);
    for (int k = 0; k < 2; k++) L.f[k] = p->flow ? take(qf_of(p->dim) * N * fs) : 0;
    L.phi_prev = take(Nm * rs);
    return L;
}

struct BatchLayout {
    std::vector<Layout> inst;
    size_t table, centers, dirs, Lout, staging, total;
};

BatchLayout batch_layout(int n, const lbcg_params* p) {
    BatchLayout B;
    size_t off = 0, maxN = 0;
    for (int i = 0; i < n; i++) {
        B.inst.push_back(instance_layout(&p[i], off));
        maxN = std::max(maxN, (size_t)p[i].nx * p[i].ny * p[i].nz);
    }
    auto take = [&](size_t bytes) {
        size_t o = off;
        off += align256(bytes);
        return o;
    };
    B.table = take(sizeof(InstDev) * n);
    B.centers = take(sizeof(double) * 3 * n);
    B.dirs = take(sizeof(double) * 3 * MAX_DIRS);
    B.Lout = take(sizeof(double) * MAX_DIRS * n);
    B.staging = take(maxN * 8);
    B.total = off;
    return B;
}

void validate_batch(int n, const lbcg_params* p) {
    if (n < 1 || n > 65535) throw Error(LBCG_EINVAL, "batch size must be in [1, 65535]");
    if (!p) throw Error(LBCG_EINVAL, "params is NULL");
    long long tiles = 0;
    for (int i = 0; i < n; i++) {
        validate(&p[i]);
        if (p[i].dim != p[0].dim || p[i].flow != p[0].flow || p[i].precision != p[0].precision ||
            p[i].collision != p[0].collision)
            throw Error(LBCG_EINVAL, "all instances of a batch need the same dim, flow, precision and collision");
        if (p[i].walls) throw Error(LBCG_EINVAL, "batches do not take walls");
        tiles += (long long)p[i].nx * p[i].ny * p[i].nz;
    }
    if (tiles > (1LL << 31)) throw Error(LBCG_EINVAL, "batch too large");
}

// ---- autotuning cache ----
// The tiling the autotuner found fastest, keyed by the kernel kind, the grid shape (or a batch's
// mix of shapes), the precision and the GPU architecture, stored by name. Kept for the life of the
// process; with the environment variable LBCG_TUNE_CACHE naming a file, also read from that file at
// first use and appended to after each tuning (one "key<TAB>tiling" line per choice).
struct TuneCache {
    std::mutex mu;
    bool loaded = false;
    std::map<std::string, std::string> m;
};
TuneCache& tune_cache() {
    static TuneCache c;
    return c;
}

std::string arch_name() {
    int dev = 0;
    hipDeviceProp_t prop;
    if (hipGetDevice(&dev) != hipSuccess || hipGetDeviceProperties(&prop, dev) != hipSuccess) return "unknown";
    const std::string a = prop.gcnArchName;
    return a.substr(0, a.find(':'));
}

void tune_load_locked(TuneCache& c) {
    if (c.loaded) return;
    c.loaded = true;
    const char* path = std::getenv("LBCG_TUNE_CACHE");
    if (!path || !*path) return;
    std::FILE* f = std::fopen(path, "r");
    if (!f) return;
    char line[4096];
    while (std::fgets(line, sizeof line, f)) {
        std::string l(line);
        while (!l.empty() && (l.back() == '\n' || l.back() == '\r')) l.pop_back();
        const size_t t = l.find('\t');
        if (t != std::string::npos) c.m[l.substr(0, t)] = l.substr(t + 1);
    }
    std::fclose(f);
}

bool tune_lookup(const std::string& key, std::string& name) {
    TuneCache& c = tune_cache();
    std::lock_guard<std::mutex> lock(c.mu);
    tune_load_locked(c);
    auto it = c.m.find(key);
    if (it == c.m.end()) return false;
    name = it->second;
    return true;
}

void tune_store(const std::string& key, const std::string& name) {
    TuneCache& c = tune_cache();
    std::lock_guard<std::mutex> lock(c.mu);
    tune_load_locked(c);
    c.m[key] = name;
    const char* path = std::getenv("LBCG_TUNE_CACHE");
    if (path && *path) {
        if (std::FILE* f = std::fopen(path, "a")) {
            std::fprintf(f, "%s\t%s\n", key.c_str(), name.c_str());
            std::fclose(f);
        }
    }
}

// Key of a single grid: kernel kind, shape, precision, architecture.
std::string grid_key(const lbcg_params& p) {
    char buf[256];
    std::snprintf(buf, sizeof buf, "grid %s dim=%d flow=%d prec=%d xbc=%d walls=%d coll=%d %dx%dx%d",
                  arch_name().c_str(), p.dim, p.flow, p.precision, p.xbc, p.walls, p.collision, p.nx, p.ny, p.nz);
    return buf;
}

// Key of a batch: kernel kind, precision, architecture and the mix of instance shapes (each distinct
// nx x ny x nz with its x-face kind and count; a 64-bit FNV-1a digest of that list if it is long).
std::string batch_key(int n, const lbcg_params* p) {
    std::map<std::string, int> mix;
    for (int i = 0; i < n; i++) {
        char b[96];
        std::snprintf(b, sizeof b, "%dx%dx%d/%d", p[i].nx, p[i].ny, p[i].nz, p[i].xbc);
        mix[b]++;
    }
    std::string m;
    for (const auto& kv : mix) m += kv.first + "*" + std::to_string(kv.second) + ",";
    if (m.size() > 400) {
        unsigned long long hsh = 1469598103934665603ull;
        for (unsigned char ch : m) hsh = (hsh ^ ch) * 1099511628211ull;
        char b[40];
        std::snprintf(b, sizeof b, "fnv:%016llx", hsh);
        m = b;
    }
    char buf[160];
    std::snprintf(buf, sizeof buf, "batch %s dim=%d flow=%d prec=%d coll=%d n=%d ", arch_name().c_str(), p[0].dim,
                  p[0].flow, p[0].precision, p[0].collision, n);
    return buf + m;
}

int variant_index_by_name(const std::vector<Variant>& v, const std::string& name) {
    for (int i = 0; i < (int)v.size(); i++)
        if (variant_name(v[i]) == name) return i;
    return -1;
}

}  // namespace

struct lbcg_batch {
    int n;
    std::vector<lbcg_params> p;
    std::vector<InstDev> inst;
    BatchLayout L;
    char* ws;
    hipStream_t stream;
    const std::vector<BatchKit>* kits;  // candidate tilings of the batched step
    int kit_idx;
    const BatchKit* kit;                // the selected one
    const Ops* common;  // init / field kernels of the instance kind
    int total_tiles;
    int par;
    int64_t nstep;
    struct Graph {
        hipGraphExec_t exec;
        int par, steps, ndirs;
    };
    std::vector<Graph> graphs;
};

struct lbcg_handle {
    lbcg_params p;
    Layout L;
    char* ws;
    hipStream_t stream;
    std::vector<Variant> variants;
    int variant;
    const Ops* ops;
    InstDev inst;
    int par;
    int64_t nstep;
    int red_blocks;
    bool nonfinite;
    int hist_ndirs;
    std::vector<double> hist_t;
    std::vector<double> hist_L;  // samples x ndirs
    int device;                  // current device at creation
};

extern "C" {

size_t lbcg_workspace_bytes(const lbcg_params* p) {
    try {
        validate(p);
        return layout_of(p).total;
    } catch (...) {
        return 0;
    }
}

lbcg_status lbcg_create(const lbcg_params* p, void* dev_workspace, size_t bytes, void* hip_stream,
                        lbcg_handle** out) {
    if (out) *out = nullptr;
    lbcg_handle* hdl = nullptr;
    lbcg_status st = guarded([&] {
        if (!out) throw Error(LBCG_EINVAL, "out is NULL");
        validate(p);
        Layout L = layout_of(p);
        if (!dev_workspace) throw Error(LBCG_EINVAL, "workspace is NULL");
        if (((uintptr_t)dev_workspace & 255) != 0) throw Error(LBCG_EINVAL, "workspace must be 256-byte aligned");
        if (bytes < L.total)
            throw Error(LBCG_ENOMEM, "workspace too small: need " + std::to_string(L.total) + " bytes");
        hdl = new lbcg_handle();
        hdl->p = *p;
        hdl->L = L;
        hdl->ws = (char*)dev_workspace;
        hdl->stream = (hipStream_t)hip_stream;
        const bool chm = p->collision == LBCG_COLLISION_CHMRT;
        hdl->variants = variants_for(p->dim, p->flow, p->precision,
                                     (p->xbc == LBCG_INFLOW_PRESSURE || chm) ? 0 : p->nx,  // (0: no z-marching tiling)
                                     population_bytes(*p), p->walls != 0, chm, default_gcache(*p),
                                     default_zband(*p));
        hdl->variant = 0;
        std::string tuned;  // a tiling the autotuner chose for this grid earlier in the process
        if (tune_lookup(grid_key(*p), tuned)) hdl->variant = std::max(0, variant_index_by_name(hdl->variants, tuned));
        hdl->ops = hdl->variants[hdl->variant].ops;
        hdl->inst = make_inst(p, hdl->ws, L, hdl->variants[hdl->variant].tiling);
        hdl->par = 0;
        hdl->nstep = 0;
        hdl->red_blocks = grid_for(hdl->inst.N, RED_THREADS, RED_BLOCKS);
        hdl->nonfinite = false;
        hdl->hist_ndirs = -1;
        HIPCHK(hipGetDevice(&hdl->device));
        SeedArgs a{p->seed_center[0], p->seed_center[1], p->seed_center[2], p->seed_radius, p->W0, p->U0,
                   p->flow ? p->u_inlet : 0.0, p->seed_tilt, p->seed_shape};
        // unused halves of the ping-pong buffers start defined (zero) so raw reads are reproducible
        HIPCHK(hipMemsetAsync(hdl->ws, 0, L.staging, hdl->stream));
        // the whole mask region, pad columns of the stored rows included (the mask starts empty)
        if (p->walls) HIPCHK(hipMemsetAsync(hdl->ws + L.wall, 0, stored_nodes(p), hdl->stream));
        hdl->ops->init(hdl->inst, 0, a, hdl->stream);
        HIPCHK(hipGetLastError());
    });
    if (st != LBCG_OK) {
        delete hdl;
        return st;
    }
    *out = hdl;
    return LBCG_OK;
}

}  // extern "C"

namespace {
void enqueue_steps(lbcg_handle* h, int64_t nsteps) {
    for (int64_t n = 0; n < nsteps; n++) {
        h->ops->step(h->inst, h->par, h->stream);
        h->par ^= 1;
    }
    h->nstep += nsteps;
}

void check_dirs(const lbcg_handle* h, int ndirs, const double* dirs) {
    if (ndirs < 0 || ndirs > MAX_DIRS) throw Error(LBCG_EINVAL, "ndirs must be in [0, 256]");
    if (ndirs > 0 && !dirs) throw Error(LBCG_EINVAL, "dirs is required when ndirs > 0");
    for (int k = 0; k < ndirs; k++) {
        const double* d = dirs + 3 * k;
        const double n2 = d[0] * d[0] + d[1] * d[1] + d[2] * d[2];
        if (!(std::fabs(n2 - 1.0) < 1e-6)) throw Error(LBCG_EINVAL, "directions must be unit vectors");
        if (h->p.dim == 2 && d[2] != 0.0) throw Error(LBCG_EINVAL, "2-D directions need z = 0");
    }
}

// Keep a measurement's extents in the growth-rate history (restarted when ndirs changes).
void record_history(lbcg_handle* h, double t, int ndirs, const double* L) {
    if (ndirs <= 0) return;
    if (h->hist_ndirs != ndirs) {
        h->hist_ndirs = ndirs;
        h->hist_t.clear();
        h->hist_L.clear();
    }
    h->hist_t.push_back(t);
    h->hist_L.insert(h->hist_L.end(), L, L + ndirs);
}
}  // namespace

extern "C" {

lbcg_status lbcg_step(lbcg_handle* h, int64_t nsteps) {
    return guarded([&] {
        if (!h) throw Error(LBCG_EINVAL, "handle is NULL");
        if (nsteps < 0) throw Error(LBCG_EINVAL, "nsteps must be >= 0");
        if (h->nonfinite) throw Error(LBCG_ENONFINITE, "the last measurement found a non-finite value");
        enqueue_steps(h, nsteps);
        HIPCHK(hipGetLastError());
    });
}

int64_t lbcg_step_count(const lbcg_handle* h) { return h ? h->nstep : -1; }

}  // extern "C"

namespace {

int planes_of(const lbcg_params& p, int field) {
    return field == LBCG_FIELD_RAW_H || field == LBCG_FIELD_RAW_G ? qs_of(p.dim)
           : field == LBCG_FIELD_RAW_F                           ? qf_of(p.dim)
                                                                 : 1;
}

void read_field_impl(const lbcg_params& p, const InstDev& I, int par, void* stage, const Ops* ops,
                     hipStream_t stream, int field, void* dst, size_t dst_bytes, int dst_on_device, int dst_dtype) {
    if (!dst) throw Error(LBCG_EINVAL, "NULL destination");
    if (dst_dtype != LBCG_DTYPE_F64 && dst_dtype != LBCG_DTYPE_F32) throw Error(LBCG_EINVAL, "bad dtype");
    if (field < LBCG_FIELD_PHI || field > LBCG_FIELD_RAW_F) throw Error(LBCG_EINVAL, "bad field id");
    if (field == LBCG_FIELD_RAW_F && !p.flow) throw Error(LBCG_EINVAL, "no flow lattice");
    const long long N = I.N;
    const size_t es = dst_dtype == LBCG_DTYPE_F64 ? 8 : 4;
    const int planes = planes_of(p, field);
    if (dst_bytes < (size_t)planes * N * es) throw Error(LBCG_ENOMEM, "destination too small");
    for (int a = 0; a < planes; a++) {
        void* tgt = dst_on_device ? (char*)dst + (size_t)a * N * es : stage;
        if (field < LBCG_FIELD_RAW_H) {
            ops->field(I, par, field, tgt, dst_dtype, stream);
        } else {
            const void* base = field == LBCG_FIELD_RAW_H ? I.h[par] : field == LBCG_FIELD_RAW_G ? I.g[par] : I.f[par];
            switch (storage_kind(p, field)) {
                case 0: raw_read_t<double, double>(p, base, field, a, N, tgt, dst_dtype, stream); break;
                case 1: raw_read_t<float, float>(p, base, field, a, N, tgt, dst_dtype, stream); break;
                default: raw_read_t<float, __half>(p, base, field, a, N, tgt, dst_dtype, stream); break;
            }
        }
        HIPCHK(hipGetLastError());
        if (!dst_on_device)
            HIPCHK(hipMemcpyAsync((char*)dst + (size_t)a * N * es, stage, N * es, hipMemcpyDeviceToHost, stream));
    }
    HIPCHK(hipStreamSynchronize(stream));
}

void write_field_impl(const lbcg_params& p, const InstDev& I, int par, void* stage, hipStream_t stream, int field,
                      const void* src, size_t src_bytes, int src_on_device, int src_dtype) {
    if (!src) throw Error(LBCG_EINVAL, "NULL source");
    if (src_dtype != LBCG_DTYPE_F64 && src_dtype != LBCG_DTYPE_F32) throw Error(LBCG_EINVAL, "bad dtype");
    if (field != LBCG_FIELD_PHI_PREV && field != LBCG_FIELD_RAW_H && field != LBCG_FIELD_RAW_G &&
        field != LBCG_FIELD_RAW_F)
        throw Error(LBCG_EINVAL, "only RAW_* and PHI_PREV can be written");
    if (field == LBCG_FIELD_RAW_F && !p.flow) throw Error(LBCG_EINVAL, "no flow lattice");
    const long long N = I.N;
    const size_t es = src_dtype == LBCG_DTYPE_F64 ? 8 : 4;
    const int planes = planes_of(p, field);
    if (src_bytes < (size_t)planes * N * es) throw Error(LBCG_ENOMEM, "source too small");
    for (int a = 0; a < planes; a++) {
        const void* in = (const char*)src + (size_t)a * N * es;
        if (!src_on_device) {
            HIPCHK(hipMemcpyAsync(stage, in, N * es, hipMemcpyHostToDevice, stream));
            in = stage;
        }
        void* base = field == LBCG_FIELD_RAW_H   ? I.h[par]
                     : field == LBCG_FIELD_RAW_G ? I.g[par]
                     : field == LBCG_FIELD_RAW_F ? I.f[par]
                                                 : I.phi_prev;
        switch (storage_kind(p, field)) {
            case 0: raw_write_t<double, double>(p, base, field, a, N, in, src_dtype, stream); break;
            case 1: raw_write_t<float, float>(p, base, field, a, N, in, src_dtype, stream); break;
            default: raw_write_t<float, __half>(p, base, field, a, N, in, src_dtype, stream); break;
        }
        HIPCHK(hipGetLastError());
        if (!src_on_device) HIPCHK(hipStreamSynchronize(stream));  // the staging area is reused per plane
    }
    HIPCHK(hipStreamSynchronize(stream));
}

// The diagnostics of lbcg_measure with their device scratch at `part` (block partials, then the
// final values), `ddirs` (the directions) and `dout` (the extents, after RED_VALUES slots).
// Returns true if a non-finite value was found (and marks the handle).
bool measure_into(lbcg_handle* h, int ndirs, const double* dirs, double* L_out, double* mass_out, double* part,
                  double* ddirs, double* dout) {
    check_dirs(h, ndirs, dirs);
    if (ndirs > 0 && !L_out) throw Error(LBCG_EINVAL, "L_out is required when ndirs > 0");
    h->ops->reduce(h->inst, h->par, part, h->red_blocks, part + h->red_blocks * RED_VALUES, h->stream);
    HIPCHK(hipGetLastError());
    if (ndirs > 0) {
        HIPCHK(hipMemcpyAsync(ddirs, dirs, sizeof(double) * 3 * ndirs, hipMemcpyHostToDevice, h->stream));
        h->ops->ray(h->inst, h->par, ddirs, ndirs, h->p.seed_center, dout + RED_VALUES, h->stream);
        HIPCHK(hipGetLastError());
    }
    double host[RED_VALUES + MAX_DIRS];
    HIPCHK(hipMemcpyAsync(host, part + h->red_blocks * RED_VALUES, sizeof(double) * RED_VALUES,
                          hipMemcpyDeviceToHost, h->stream));
    if (ndirs > 0)
        HIPCHK(hipMemcpyAsync(host + RED_VALUES, dout + RED_VALUES, sizeof(double) * ndirs, hipMemcpyDeviceToHost,
                              h->stream));
    HIPCHK(hipStreamSynchronize(h->stream));
    if (mass_out) std::memcpy(mass_out, host, sizeof(double) * RED_VALUES);
    if (ndirs > 0) std::memcpy(L_out, host + RED_VALUES, sizeof(double) * ndirs);
    record_history(h, (double)h->nstep, ndirs, host + RED_VALUES);
    if (host[5] > 0) {
        h->nonfinite = true;
        return true;
    }
    return false;
}

// ---- the diagnostics' scratch as a file-scope device array (lbcg_measure_noalloc) ----
// Offsets (in doubles, 256-byte aligned) of the block partials + final values, the directions and
// the extents inside the array.
constexpr size_t NA_PARTIALS = 0;
constexpr size_t NA_DIRS = ((RED_BLOCKS + 1) * RED_VALUES * 8 + 255) / 256 * 256 / 8;
constexpr size_t NA_OUT = NA_DIRS + ((size_t)MAX_DIRS * 3 * 8 + 255) / 256 * 256 / 8;
constexpr size_t NA_DOUBLES = NA_OUT + RED_VALUES + MAX_DIRS;  // 57.6 KB

}  // namespace

// One copy per device, kept until the process ends. Host code never passes this name to a kernel
// or a copy (on the host it is a stand-in, not a device address): it uses the device address
// hipGetSymbolAddress returns for the current device.
static __device__ __align__(256) double scratch[NA_DOUBLES];

namespace {

std::mutex g_scratch_mu;
std::map<int, double*> g_scratch;  // device -> address of that device's copy of `scratch`

double* static_scratch(int dev) {
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    auto it = g_scratch.find(dev);
    if (it != g_scratch.end()) return it->second;
    void* ptr = nullptr;
    HIPCHK(hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)));
    if (!ptr) throw Error(LBCG_EDEVICE, "hipGetSymbolAddress(scratch) returned NULL");
    g_scratch[dev] = (double*)ptr;
    return (double*)ptr;
}

}  // namespace

extern "C" {

lbcg_status lbcg_read_field(lbcg_handle* h, int field, void* dst, size_t dst_bytes, int dst_on_device,
                            int dst_dtype) {
    return guarded([&] {
        if (!h) throw Error(LBCG_EINVAL, "handle is NULL");
        read_field_impl(h->p, h->inst, h->par, h->ws + h->L.staging, h->ops, h->stream, field, dst, dst_bytes,
                        dst_on_device, dst_dtype);
    });
}

lbcg_status lbcg_write_field(lbcg_handle* h, int field, const void* src, size_t src_bytes, int src_on_device,
                             int src_dtype) {
    return guarded([&] {
        if (!h) throw Error(LBCG_EINVAL, "handle is NULL");
        write_field_impl(h->p, h->inst, h->par, h->ws + h->L.staging, h->stream, field, src, src_bytes,
                         src_on_device, src_dtype);
    });
}

lbcg_status lbcg_measure(lbcg_handle* h, int ndirs, const double* dirs, double* L_out, double* mass_out) {
    bool nonfinite = false;
    lbcg_status st = guarded([&] {
        if (!h) throw Error(LBCG_EINVAL, "handle is NULL");
        nonfinite = measure_into(h, ndirs, dirs, L_out, mass_out, (double*)(h->ws + h->L.partials),
                                 (double*)(h->ws + h->L.dirs), (double*)(h->ws + h->L.out));
    });
    if (st == LBCG_OK && nonfinite) {
        lbcg::last_error_slot() = "non-finite phi, U or rho found";
        return LBCG_ENONFINITE;
    }
    return st;
}

lbcg_status lbcg_measure_noalloc(lbcg_handle* h, int ndirs, const double* dirs, double* L_out, double* mass_out) {
    bool nonfinite = false;
    lbcg_status st = guarded([&] {
        if (!h) throw Error(LBCG_EINVAL, "handle is NULL");
        if (ndirs < 0 || ndirs > MAX_DIRS)
            throw Error(LBCG_EINVAL, "ndirs must be in [0, " + std::to_string(MAX_DIRS) +
                                         "] (the static scratch holds at most that many directions)");
        if (h->red_blocks > RED_BLOCKS) throw Error(LBCG_EINVAL, "reduction larger than the static scratch");
        int dev = -1;
        HIPCHK(hipGetDevice(&dev));
        if (dev != h->device)
            throw Error(LBCG_EINVAL, "the device the handle was created on (" + std::to_string(h->device) +
                                         ") must be current (it is " + std::to_string(dev) + ")");
        double* base = static_scratch(dev);
        nonfinite = measure_into(h, ndirs, dirs, L_out, mass_out, base + NA_PARTIALS, base + NA_DIRS, base + NA_OUT);
    });
    if (st == LBCG_OK && nonfinite) {
        lbcg::last_error_slot() = "non-finite phi, U or rho found";
        return LBCG_ENONFINITE;
    }
    return st;
}

lbcg_status lbcg_run(lbcg_handle* h, int64_t nsteps, int64_t measure_every, int ndirs, const double* dirs,
                     double* L_hist, double* mass_hist) {
    bool nonfinite = false;
    lbcg_status st = guarded([&] {
        if (!h) throw Error(LBCG_EINVAL, "handle is NULL");
        if (nsteps < 0) throw Error(LBCG_EINVAL, "nsteps must be >= 0");
        if (measure_every < 1) throw Error(LBCG_EINVAL, "measure_every must be >= 1");
        check_dirs(h, ndirs, dirs);
        if (h->nonfinite) throw Error(LBCG_ENONFINITE, "the last measurement found a non-finite value");
        const int per = RED_VALUES + ndirs;               // values per sample in the device history
        const int64_t cap = HIST_DOUBLES / per;            // samples per round trip (>= 15)
        const int64_t samples = nsteps / measure_every;
        double* part = (double*)(h->ws + h->L.partials);
        double* ddirs = (double*)(h->ws + h->L.dirs);
        double* dhist = (double*)(h->ws + h->L.hist);
        if (ndirs > 0)
            HIPCHK(hipMemcpyAsync(ddirs, dirs, sizeof(double) * 3 * ndirs, hipMemcpyHostToDevice, h->stream));
        std::vector<double> host((size_t)std::min<int64_t>(cap, std::max<int64_t>(samples, 1)) * per);
        std::vector<double> tsample;
        for (int64_t s0 = 0; s0 < samples && !nonfinite; s0 += cap) {
            const int64_t k = std::min(cap, samples - s0);
            tsample.clear();
            for (int64_t j = 0; j < k; j++) {  // steps and measurements, all on the stream
                enqueue_steps(h, measure_every);
                tsample.push_back((double)h->nstep);
                double* slot = dhist + j * per;
                h->ops->reduce(h->inst, h->par, part, h->red_blocks, slot, h->stream);
                if (ndirs > 0) h->ops->ray(h->inst, h->par, ddirs, ndirs, h->p.seed_center, slot + RED_VALUES, h->stream);
            }
            HIPCHK(hipGetLastError());
            HIPCHK(hipMemcpyAsync(host.data(), dhist, sizeof(double) * k * per, hipMemcpyDeviceToHost, h->stream));
            HIPCHK(hipStreamSynchronize(h->stream));
            for (int64_t j = 0; j < k; j++) {
                const double* v = host.data() + j * per;
                if (mass_hist) std::memcpy(mass_hist + (s0 + j) * RED_VALUES, v, sizeof(double) * RED_VALUES);
                if (ndirs > 0 && L_hist) std::memcpy(L_hist + (s0 + j) * ndirs, v + RED_VALUES, sizeof(double) * ndirs);
                record_history(h, tsample[j], ndirs, v + RED_VALUES);
                if (v[5] > 0) nonfinite = true;
            }
        }
        if (nonfinite) {
            h->nonfinite = true;
            return;
        }
        enqueue_steps(h, nsteps - samples * measure_every);
        HIPCHK(hipGetLastError());
    });
    if (st == LBCG_OK && nonfinite) {
        lbcg::last_error_slot() = "non-finite phi, U or rho found";
        return LBCG_ENONFINITE;
    }
    return st;
}

lbcg_status lbcg_growth_rates(lbcg_handle* h, double* G_out, double* R2_out, double* G_avg_out) {
    return guarded([&] {
        if (!h) throw Error(LBCG_EINVAL, "handle is NULL");
        const int K = h->hist_ndirs;
        const size_t S = h->hist_t.size();
        if (K <= 0 || S < 2) throw Error(LBCG_ESTATE, "need at least two measurements with directions");
        // least squares L = b + G t per direction (Section 4.1.2), centred sums
        double tm = 0;
        for (double t : h->hist_t) tm += t;
        tm /= (double)S;
        double stt = 0;
        for (double t : h->hist_t) stt += (t - tm) * (t - tm);
        if (!(stt > 0)) throw Error(LBCG_ESTATE, "measurements at a single time");
        std::vector<double> avg(S, 0.0);
        for (size_t j = 0; j < S; j++)
            for (int k = 0; k < K; k++) avg[j] += h->hist_L[j * K + k] / K;
        auto fit = [&](auto getL, double& G, double& R2) {
            double Lm = 0;
            for (size_t j = 0; j < S; j++) Lm += getL(j);
            Lm /= (double)S;
            double stl = 0;
            for (size_t j = 0; j < S; j++) stl += (h->hist_t[j] - tm) * (getL(j) - Lm);
            G = stl / stt;
            const double b = Lm - G * tm;
            double ares = 0, atot = 0;
            for (size_t j = 0; j < S; j++) {
                const double r = getL(j) - (b + G * h->hist_t[j]);
                ares += r * r;
                atot += (getL(j) - Lm) * (getL(j) - Lm);
            }
            R2 = atot > 0 ? 1.0 - ares / atot : (ares == 0 ? 1.0 : 0.0);
        };
        for (int k = 0; k < K; k++) {
            double G, R2;
            fit([&](size_t j) { return h->hist_L[j * K + k]; }, G, R2);
            if (G_out) G_out[k] = G;
            if (R2_out) R2_out[k] = R2;
        }
        double Ga, R2a;
        fit([&](size_t j) { return avg[j]; }, Ga, R2a);
        if (G_avg_out) *G_avg_out = Ga;
    });
}

int lbcg_variant_count(const lbcg_handle* h) { return h ? (int)h->variants.size() : -1; }

int lbcg_variant_current(const lbcg_handle* h) { return h ? h->variant : -1; }

lbcg_status lbcg_variant_name(const lbcg_handle* h, int idx, char* buf, size_t buflen) {
    return guarded([&] {
        if (!h || !buf || buflen == 0) throw Error(LBCG_EINVAL, "NULL handle or buffer");
        if (idx < 0 || idx >= (int)h->variants.size()) throw Error(LBCG_EINVAL, "variant index out of range");
        std::snprintf(buf, buflen, "%s", variant_name(h->variants[idx]).c_str());
    });
}

namespace {
void select_variant(lbcg_handle* h, int idx) {
    if (idx < 0 || idx >= (int)h->variants.size()) throw Error(LBCG_EINVAL, "variant index out of range");
    const Variant& v = h->variants[idx];
    InstDev I = make_inst(&h->p, h->ws, h->L, v.tiling);
    h->inst = I;
    h->ops = v.ops;
    h->variant = idx;
}

// Times real coupled steps with variant idx: one untimed step, then `launches` timed ones, with the
// ping-pong parity alternating as in lbcg_step (re-reading one input copy would let the
// last-level cache hold part of it and flatter the variant). The state advances by launches + 1
// steps of variant idx.
// Rounds of the autotuners over all candidates; each candidate keeps its fastest time.
constexpr int TUNE_ROUNDS = 2;

double time_variant(lbcg_handle* h, int idx, int launches) {
    if (h->nonfinite) throw Error(LBCG_ENONFINITE, "the last measurement found a non-finite value");
    const int keep = h->variant;
    select_variant(h, idx);
    hipEvent_t e0, e1;
    HIPCHK(hipEventCreate(&e0));
    HIPCHK(hipEventCreate(&e1));
    h->ops->step(h->inst, h->par, h->stream);  // warm-up
    h->par ^= 1;
    HIPCHK(hipEventRecord(e0, h->stream));
    for (int k = 0; k < launches; k++) {
        h->ops->step(h->inst, h->par, h->stream);
        h->par ^= 1;
    }
    HIPCHK(hipEventRecord(e1, h->stream));
    h->nstep += launches + 1;
    HIPCHK(hipGetLastError());
    HIPCHK(hipEventSynchronize(e1));
    float ms = 0;
    HIPCHK(hipEventElapsedTime(&ms, e0, e1));
    HIPCHK(hipEventDestroy(e0));
    HIPCHK(hipEventDestroy(e1));
    select_variant(h, keep);
    return 1e3 * (double)ms / launches;
}
}  // namespace

lbcg_status lbcg_variant_select(lbcg_handle* h, int idx) {
    return guarded([&] {
        if (!h) throw Error(LBCG_EINVAL, "handle is NULL");
        select_variant(h, idx);
    });
}

lbcg_status lbcg_variant_time(lbcg_handle* h, int idx, int launches, double* us) {
    return guarded([&] {
        if (!h || !us) throw Error(LBCG_EINVAL, "NULL handle or output");
        if (launches < 1) throw Error(LBCG_EINVAL, "launches must be >= 1");
        *us = time_variant(h, idx, launches);
    });
}

lbcg_status lbcg_autotune(lbcg_handle* h, int launches, int* best, double* best_us) {
    return guarded([&] {
        if (!h) throw Error(LBCG_EINVAL, "handle is NULL");
        if (launches < 1) throw Error(LBCG_EINVAL, "launches must be >= 1");
        const int nv = (int)h->variants.size();
        std::vector<double> t(nv, 1e300);
        for (int r = 0; r < TUNE_ROUNDS; r++)
            for (int i = 0; i < nv; i++) t[i] = std::min(t[i], time_variant(h, i, launches));
        int bi = 0;
        for (int i = 1; i < nv; i++)
            if (t[i] < t[bi]) bi = i;
        const double bt = t[bi];
        select_variant(h, bi);
        tune_store(grid_key(h->p), variant_name(h->variants[bi]));
        if (best) *best = bi;
        if (best_us) *best_us = bt;
    });
}

// ---- solid walls ----

lbcg_status lbcg_set_walls(lbcg_handle* h, const uint8_t* mask, size_t bytes, int mask_on_device) {
    return guarded([&] {
        if (!h || !mask) throw Error(LBCG_EINVAL, "NULL handle or mask");
        if (!h->p.walls) throw Error(LBCG_EINVAL, "the solver was created with walls = 0");
        const size_t N = (size_t)h->inst.N, nx = (size_t)h->p.nx;
        if (bytes < N) throw Error(LBCG_EINVAL, "mask smaller than the grid");
        std::vector<uint8_t> host;
        const uint8_t* hm = mask;
        if (mask_on_device) {
            host.resize(N);
            HIPCHK(hipMemcpy(host.data(), mask, N, hipMemcpyDeviceToHost));
            hm = host.data();
        }
        if (h->p.xbc != LBCG_PERIODIC)  // the outlet copy pairs the last two columns of a row
            for (size_t r = 0; r < N / nx; r++)
                if ((hm[r * nx + nx - 2] != 0) != (hm[r * nx + nx - 1] != 0))
                    throw Error(LBCG_EINVAL, "a row's last two columns must be both wall or both fluid");
        // hm is host memory, dense rows of nx; the device mask has rows of the stored pitch
        HIPCHK(hipMemcpy2DAsync(h->ws + h->L.wall, (size_t)h->inst.pitch, hm, nx, nx, N / nx, hipMemcpyHostToDevice,
                                h->stream));
        // Wall nodes are never written: give both ping-pong copies the current state so that they
        // stay frozen whichever copy is current.
        const lbcg_params& p = h->p;
        const size_t rs = real_size(p.precision), fs = fstore_size(p.precision);
        const int cur = h->par, oth = h->par ^ 1;
        const size_t Np = plane_stride(stored_nodes(&p));
        HIPCHK(hipMemcpyAsync(h->ws + h->L.h[oth], h->ws + h->L.h[cur], qs_of(p.dim) * Np * rs,
                              hipMemcpyDeviceToDevice, h->stream));
        HIPCHK(hipMemcpyAsync(h->ws + h->L.g[oth], h->ws + h->L.g[cur], qs_of(p.dim) * Np * rs,
                              hipMemcpyDeviceToDevice, h->stream));
        if (p.flow)
            HIPCHK(hipMemcpyAsync(h->ws + h->L.f[oth], h->ws + h->L.f[cur], qf_of(p.dim) * Np * fs,
                                  hipMemcpyDeviceToDevice, h->stream));
        HIPCHK(hipStreamSynchronize(h->stream));
    });
}

}  // extern "C"

// ---- checkpoints ----

namespace {
struct StateHeader {
    char magic[8];
    int32_t version, dim, nx, ny, nz, flow, precision, xbc;
    int64_t nstep;
    char pad[16];
};
static_assert(sizeof(StateHeader) == 64, "checkpoint header is 64 bytes");
constexpr char STATE_MAGIC[8] = {'L', 'B', 'C', 'G', 'S', 'T', 'A', 'T'};

// (offset in the workspace, bytes) of each stored array of the current copy, in blob order
std::vector<std::pair<size_t, size_t>> state_parts(const lbcg_handle* h) {
    const lbcg_params& p = h->p;
    const size_t Nm = stored_nodes(&p), Np = plane_stride(Nm);
    const size_t rs = real_size(p.precision), fs = fstore_size(p.precision);
    std::vector<std::pair<size_t, size_t>> v;
    v.push_back({h->L.h[h->par], qs_of(p.dim) * Np * rs});
    v.push_back({h->L.g[h->par], qs_of(p.dim) * Np * rs});
    if (p.flow) v.push_back({h->L.f[h->par], qf_of(p.dim) * Np * fs});
    v.push_back({h->L.phi_prev, Nm * rs});
    return v;
}

size_t state_bytes_of(const lbcg_handle* h) {
    size_t b = sizeof(StateHeader);
    for (const auto& q : state_parts(h)) b += q.second;
    return b;
}
}  // namespace

extern "C" {

size_t lbcg_state_bytes(const lbcg_handle* h) { return h ? state_bytes_of(h) : 0; }

lbcg_status lbcg_state_save(lbcg_handle* h, void* dst, size_t dst_bytes, int dst_on_device) {
    return guarded([&] {
        if (!h || !dst) throw Error(LBCG_EINVAL, "NULL handle or destination");
        if (dst_bytes < state_bytes_of(h)) throw Error(LBCG_ENOMEM, "destination smaller than lbcg_state_bytes");
        StateHeader H{};
        std::memcpy(H.magic, STATE_MAGIC, 8);
        H.version = 3;
        H.dim = h->p.dim;
        H.nx = h->p.nx;
        H.ny = h->p.ny;
        H.nz = h->p.nz;
        H.flow = h->p.flow;
        H.precision = h->p.precision;
        H.xbc = h->p.xbc;
        H.nstep = h->nstep;
        char* out = static_cast<char*>(dst);
        if (dst_on_device) HIPCHK(hipMemcpyAsync(out, &H, sizeof H, hipMemcpyHostToDevice, h->stream));
        else std::memcpy(out, &H, sizeof H);
        size_t off = sizeof H;
        for (const auto& q : state_parts(h)) {
            HIPCHK(hipMemcpyAsync(out + off, h->ws + q.first, q.second,
                                  dst_on_device ? hipMemcpyDeviceToDevice : hipMemcpyDeviceToHost, h->stream));
            off += q.second;
        }
        HIPCHK(hipStreamSynchronize(h->stream));
    });
}

lbcg_status lbcg_state_load(lbcg_handle* h, const void* src, size_t src_bytes, int src_on_device) {
    return guarded([&] {
        if (!h || !src) throw Error(LBCG_EINVAL, "NULL handle or source");
        if (src_bytes < state_bytes_of(h)) throw Error(LBCG_ENOMEM, "source smaller than lbcg_state_bytes");
        const char* in = static_cast<const char*>(src);
        StateHeader H{};
        if (src_on_device) {
            HIPCHK(hipMemcpyAsync(&H, in, sizeof H, hipMemcpyDeviceToHost, h->stream));
            HIPCHK(hipStreamSynchronize(h->stream));
        } else {
            std::memcpy(&H, in, sizeof H);
        }
        if (std::memcmp(H.magic, STATE_MAGIC, 8) != 0 || H.version != 3)
            throw Error(LBCG_EINVAL, "not a checkpoint of this library (magic or version)");
        if (H.dim != h->p.dim || H.nx != h->p.nx || H.ny != h->p.ny || H.nz != h->p.nz || H.flow != h->p.flow ||
            H.precision != h->p.precision || H.xbc != h->p.xbc)
            throw Error(LBCG_EINVAL, "checkpoint of a different grid, lattice set, precision or boundary kind");
        if (H.nstep < 0) throw Error(LBCG_EINVAL, "negative step count in the checkpoint");
        size_t off = sizeof H;
        for (const auto& q : state_parts(h)) {
            HIPCHK(hipMemcpyAsync(h->ws + q.first, in + off, q.second,
                                  src_on_device ? hipMemcpyDeviceToDevice : hipMemcpyHostToDevice, h->stream));
            off += q.second;
        }
        HIPCHK(hipStreamSynchronize(h->stream));
        h->nstep = H.nstep;
        h->nonfinite = false;
    });
}

lbcg_status lbcg_destroy(lbcg_handle* h) {
    delete h;
    return LBCG_OK;
}

// ---- batches ----

size_t lbcg_batch_workspace_bytes(int n, const lbcg_params* p) {
    try {
        validate_batch(n, p);
        return batch_layout(n, p).total;
    } catch (...) {
        return 0;
    }
}

lbcg_status lbcg_batch_create(int n, const lbcg_params* p, void* dev_workspace, size_t bytes, void* hip_stream,
                              lbcg_batch** out) {
    if (out) *out = nullptr;
    lbcg_batch* b = nullptr;
    lbcg_status st = guarded([&] {
        if (!out) throw Error(LBCG_EINVAL, "out is NULL");
        validate_batch(n, p);
        BatchLayout L = batch_layout(n, p);
        if (!dev_workspace) throw Error(LBCG_EINVAL, "workspace is NULL");
        if (((uintptr_t)dev_workspace & 255) != 0) throw Error(LBCG_EINVAL, "workspace must be 256-byte aligned");
        if (bytes < L.total) throw Error(LBCG_ENOMEM, "workspace too small: need " + std::to_string(L.total) + " bytes");
        b = new lbcg_batch();
        b->n = n;
        b->p.assign(p, p + n);
        b->L = L;
        b->ws = (char*)dev_workspace;
        b->stream = (hipStream_t)hip_stream;
        const int kind = p[0].flow ? (p[0].collision == LBCG_COLLISION_CHMRT ? 2 : 1) : 0;
        b->kits = &batch_kits_for(p[0].dim, kind, p[0].precision);
        b->kit_idx = 0;
        std::string tuned;  // a tiling the autotuner chose for this mix of instances earlier in the process
        if (tune_lookup(batch_key(n, p), tuned))
            for (int k = 0; k < (int)b->kits->size(); k++)
                if (variant_name(Variant{nullptr, (*b->kits)[k].tiling}) == tuned) b->kit_idx = k;
        b->kit = &(*b->kits)[b->kit_idx];
        b->common = variants_for(p[0].dim, p[0].flow, p[0].precision, p[0].nx, 0.0, false, false, 0, 16)[0].ops;
        b->par = 0;
        b->nstep = 0;
        int tiles = 0;
        std::vector<double> centers(3 * n);
        for (int i = 0; i < n; i++) {
            InstDev I = make_inst(&p[i], b->ws, L.inst[i], b->kit->tiling);
            I.tile_begin = tiles;
            tiles += I.tiles_x * I.tiles_y * I.tiles_z;
            b->inst.push_back(I);
            for (int d = 0; d < 3; d++) centers[3 * i + d] = p[i].seed_center[d];
        }
        b->total_tiles = tiles;
        HIPCHK(hipMemsetAsync(b->ws, 0, L.table, b->stream));
        HIPCHK(hipMemcpyAsync(b->ws + L.table, b->inst.data(), sizeof(InstDev) * n, hipMemcpyHostToDevice, b->stream));
        HIPCHK(hipMemcpyAsync(b->ws + L.centers, centers.data(), sizeof(double) * 3 * n, hipMemcpyHostToDevice,
                              b->stream));
        for (int i = 0; i < n; i++) {
            SeedArgs a{p[i].seed_center[0], p[i].seed_center[1], p[i].seed_center[2], p[i].seed_radius, p[i].W0,
                       p[i].U0, p[i].flow ? p[i].u_inlet : 0.0, p[i].seed_tilt, p[i].seed_shape};
            b->common->init(b->inst[i], 0, a, b->stream);
        }
        HIPCHK(hipGetLastError());
        HIPCHK(hipStreamSynchronize(b->stream));
    });
    if (st != LBCG_OK) {
        delete b;
        return st;
    }
    *out = b;
    return LBCG_OK;
}

namespace {
void check_dirs(int dim, int ndirs, const double* dirs) {
    if (ndirs < 0 || ndirs > MAX_DIRS) throw Error(LBCG_EINVAL, "ndirs must be in [0, 256]");
    if (ndirs > 0 && !dirs) throw Error(LBCG_EINVAL, "dirs is NULL");
    for (int k = 0; k < ndirs; k++) {
        const double* d = dirs + 3 * k;
        const double n2 = d[0] * d[0] + d[1] * d[1] + d[2] * d[2];
        if (!(std::fabs(n2 - 1.0) < 1e-6)) throw Error(LBCG_EINVAL, "directions must be unit vectors");
        if (dim == 2 && d[2] != 0.0) throw Error(LBCG_EINVAL, "2-D directions need z = 0");
    }
}

// Enqueue `steps` batched steps from parity par (and the ray-march into the L slot if ndirs > 0).
void batch_chunk(lbcg_batch* b, int par, int steps, int ndirs) {
    const InstDev* d = (const InstDev*)(b->ws + b->L.table);
    for (int k = 0; k < steps; k++) {
        b->kit->step(d, b->n, b->total_tiles, par, b->stream);
        par ^= 1;
    }
    if (ndirs > 0)
        b->kit->ray(d, b->n, par, (const double*)(b->ws + b->L.dirs), ndirs, (const double*)(b->ws + b->L.centers),
                    (double*)(b->ws + b->L.Lout), b->stream);
}

hipGraphExec_t batch_graph(lbcg_batch* b, int par, int steps, int ndirs) {
    for (auto& g : b->graphs)
        if (g.par == par && g.steps == steps && g.ndirs == ndirs) return g.exec;
    hipGraph_t graph;
    HIPCHK(hipStreamBeginCapture(b->stream, hipStreamCaptureModeRelaxed));
    batch_chunk(b, par, steps, ndirs);
    HIPCHK(hipStreamEndCapture(b->stream, &graph));
    hipGraphExec_t exec;
    const hipError_t e = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0);
    HIPCHK(hipGraphDestroy(graph));
    HIPCHK(e);
    b->graphs.push_back({exec, par, steps, ndirs});
    return exec;
}
}  // namespace

lbcg_status lbcg_batch_run(lbcg_batch* b, int64_t nsteps, int64_t measure_every, int ndirs, const double* dirs,
                           double* L_hist, int use_graph) {
    return guarded([&] {
        if (!b) throw Error(LBCG_EINVAL, "batch is NULL");
        if (nsteps < 0 || measure_every < 0) throw Error(LBCG_EINVAL, "nsteps and measure_every must be >= 0");
        if (measure_every > 1000000) throw Error(LBCG_EINVAL, "measure_every too large");
        check_dirs(b->p[0].dim, ndirs, dirs);
        const bool meas = measure_every > 0 && ndirs > 0;
        if (meas && !L_hist) throw Error(LBCG_EINVAL, "L_hist is NULL");
        if (use_graph && !b->stream) throw Error(LBCG_EINVAL, "graph replay needs a non-null stream");
        if (meas)
            HIPCHK(hipMemcpyAsync(b->ws + b->L.dirs, dirs, sizeof(double) * 3 * ndirs, hipMemcpyHostToDevice, b->stream));
        const int chunk = (int)(measure_every > 0 ? measure_every : 100);
        int64_t done = 0, sample = 0;
        while (done < nsteps) {
            const int steps = (int)std::min<int64_t>(chunk, nsteps - done);
            const bool ray = meas && steps == chunk;
            if (use_graph) HIPCHK(hipGraphLaunch(batch_graph(b, b->par, steps, ray ? ndirs : 0), b->stream));
            else batch_chunk(b, b->par, steps, ray ? ndirs : 0);
            HIPCHK(hipGetLastError());
            if (steps & 1) b->par ^= 1;
            done += steps;
            if (ray) {
                HIPCHK(hipMemcpyAsync(L_hist + sample * (int64_t)b->n * ndirs, b->ws + b->L.Lout,
                                      sizeof(double) * b->n * ndirs, hipMemcpyDeviceToHost, b->stream));
                sample++;
            }
        }
        b->nstep += nsteps;
        HIPCHK(hipStreamSynchronize(b->stream));
    });
}

lbcg_status lbcg_batch_measure(lbcg_batch* b, int ndirs, const double* dirs, double* L_out) {
    return guarded([&] {
        if (!b) throw Error(LBCG_EINVAL, "batch is NULL");
        check_dirs(b->p[0].dim, ndirs, dirs);
        if (ndirs == 0) return;
        if (!L_out) throw Error(LBCG_EINVAL, "L_out is NULL");
        HIPCHK(hipMemcpyAsync(b->ws + b->L.dirs, dirs, sizeof(double) * 3 * ndirs, hipMemcpyHostToDevice, b->stream));
        batch_chunk(b, b->par, 0, ndirs);
        HIPCHK(hipGetLastError());
        HIPCHK(hipMemcpyAsync(L_out, b->ws + b->L.Lout, sizeof(double) * b->n * ndirs, hipMemcpyDeviceToHost, b->stream));
        HIPCHK(hipStreamSynchronize(b->stream));
    });
}

lbcg_status lbcg_batch_read_field(lbcg_batch* b, int inst, int field, void* dst, size_t dst_bytes, int dst_on_device,
                                  int dst_dtype) {
    return guarded([&] {
        if (!b) throw Error(LBCG_EINVAL, "batch is NULL");
        if (inst < 0 || inst >= b->n) throw Error(LBCG_EINVAL, "instance index out of range");
        read_field_impl(b->p[inst], b->inst[inst], b->par, b->ws + b->L.staging, b->common, b->stream, field, dst,
                        dst_bytes, dst_on_device, dst_dtype);
    });
}

int64_t lbcg_batch_step_count(const lbcg_batch* b) { return b ? b->nstep : -1; }

}  // extern "C"

namespace {
std::string batch_variant_name(const lbcg_batch* b, int idx) {
    return variant_name(Variant{nullptr, (*b->kits)[idx].tiling});
}

// Switch the batched step to tiling idx: the instances' tile lists change with the tiling, so the
// table is rebuilt and uploaded (after the kernels already enqueued, which read it, have run) and
// the captured graphs are dropped.
void batch_select(lbcg_batch* b, int idx) {
    if (idx < 0 || idx >= (int)b->kits->size()) throw Error(LBCG_EINVAL, "variant index out of range");
    if (idx == b->kit_idx) return;
    const BatchKit* k = &(*b->kits)[idx];
    int tiles = 0;
    for (int i = 0; i < b->n; i++) {
        InstDev I = make_inst(&b->p[i], b->ws, b->L.inst[i], k->tiling);
        I.tile_begin = tiles;
        tiles += I.tiles_x * I.tiles_y * I.tiles_z;
        b->inst[i] = I;
    }
    HIPCHK(hipStreamSynchronize(b->stream));
    HIPCHK(hipMemcpyAsync(b->ws + b->L.table, b->inst.data(), sizeof(InstDev) * b->n, hipMemcpyHostToDevice,
                          b->stream));
    HIPCHK(hipStreamSynchronize(b->stream));
    for (auto& g : b->graphs) HIPCHK(hipGraphExecDestroy(g.exec));
    b->graphs.clear();
    b->kit = k;
    b->kit_idx = idx;
    b->total_tiles = tiles;
}

// Mean time per batched step (microseconds) of `launches` steps with tiling idx after one untimed
// step; real steps, alternating the ping-pong copies as lbcg_batch_run does. The state advances by
// launches + 1 steps; the selected tiling is left as it was.
double batch_time_variant(lbcg_batch* b, int idx, int launches) {
    const int keep = b->kit_idx;
    batch_select(b, idx);
    hipEvent_t e0, e1;
    HIPCHK(hipEventCreate(&e0));
    HIPCHK(hipEventCreate(&e1));
    batch_chunk(b, b->par, 1, 0);
    b->par ^= 1;
    HIPCHK(hipEventRecord(e0, b->stream));
    batch_chunk(b, b->par, launches, 0);
    if (launches & 1) b->par ^= 1;
    HIPCHK(hipEventRecord(e1, b->stream));
    b->nstep += launches + 1;
    HIPCHK(hipGetLastError());
    HIPCHK(hipEventSynchronize(e1));
    float ms = 0;
    HIPCHK(hipEventElapsedTime(&ms, e0, e1));
    HIPCHK(hipEventDestroy(e0));
    HIPCHK(hipEventDestroy(e1));
    batch_select(b, keep);
    return 1e3 * (double)ms / launches;
}
}  // namespace

extern "C" {

int lbcg_batch_variant_count(const lbcg_batch* b) { return b ? (int)b->kits->size() : -1; }

int lbcg_batch_variant_current(const lbcg_batch* b) { return b ? b->kit_idx : -1; }

lbcg_status lbcg_batch_variant_name(const lbcg_batch* b, int idx, char* buf, size_t buflen) {
    return guarded([&] {
        if (!b || !buf || buflen == 0) throw Error(LBCG_EINVAL, "NULL batch or buffer");
        if (idx < 0 || idx >= (int)b->kits->size()) throw Error(LBCG_EINVAL, "variant index out of range");
        std::snprintf(buf, buflen, "%s", batch_variant_name(b, idx).c_str());
    });
}

lbcg_status lbcg_batch_variant_select(lbcg_batch* b, int idx) {
    return guarded([&] {
        if (!b) throw Error(LBCG_EINVAL, "batch is NULL");
        batch_select(b, idx);
    });
}

lbcg_status lbcg_batch_variant_time(lbcg_batch* b, int idx, int launches, double* us) {
    return guarded([&] {
        if (!b || !us) throw Error(LBCG_EINVAL, "NULL batch or output");
        if (launches < 1) throw Error(LBCG_EINVAL, "launches must be >= 1");
        if (idx < 0 || idx >= (int)b->kits->size()) throw Error(LBCG_EINVAL, "variant index out of range");
        *us = batch_time_variant(b, idx, launches);
    });
}

lbcg_status lbcg_batch_autotune(lbcg_batch* b, int launches, int* best, double* best_us, double* all_us) {
    return guarded([&] {
        if (!b) throw Error(LBCG_EINVAL, "batch is NULL");
        if (launches < 1) throw Error(LBCG_EINVAL, "launches must be >= 1");
        const int nv = (int)b->kits->size();
        std::vector<double> t(nv, 1e300);
        for (int r = 0; r < TUNE_ROUNDS; r++)
            for (int i = 0; i < nv; i++) t[i] = std::min(t[i], batch_time_variant(b, i, launches));
        int bi = 0;
        for (int i = 0; i < nv; i++) {
            if (all_us) all_us[i] = t[i];
            if (t[i] < t[bi]) bi = i;
        }
        const double bt = t[bi];
        batch_select(b, bi);
        tune_store(batch_key(b->n, b->p.data()), batch_variant_name(b, bi));
        if (best) *best = bi;
        if (best_us) *best_us = bt;
    });
}

lbcg_status lbcg_tune_cache_clear(void) {
    return guarded([&] {
        TuneCache& c = tune_cache();
        std::lock_guard<std::mutex> lock(c.mu);
        c.m.clear();
        c.loaded = true;  // the file, if any, is not read again
    });
}

lbcg_status lbcg_batch_destroy(lbcg_batch* b) {
    if (!b) return LBCG_OK;
    for (auto& g : b->graphs) (void)hipGraphExecDestroy(g.exec);
    delete b;
    return LBCG_OK;
}

const char* lbcg_last_error(void) { return lbcg::last_error_slot().c_str(); }

#ifndef LBCG_SOURCE_HASH
#define LBCG_SOURCE_HASH "unknown"
#endif
const char* lbcg_source_hash(void) { return LBCG_SOURCE_HASH; }

}  // extern "C"
