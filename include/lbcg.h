/*
 * lbcg.h -- C ABI of the MI355X coupled lattice Boltzmann crystal-growth solver.
 *
 * The solver advances three coupled lattices on one grid, as defined in Tan et al., "Mandelic
 * acid single-crystal growth: experiments vs numerical simulations" (arXiv 2206.02145),
 * Section 2.2:
 *   h  phase field phi, the a_s^2-weighted stream-collide scheme Eq. (d) with the anisotropic
 *      equilibrium Eq. (e) and source Q = phi - phi^3 + lambda U (1 - phi^2)^2;
 *   g  supersaturation U, advection-diffusion LB with source -w dphi/dt and tau_U = D q/cs^2 + 1/2,
 *      q = 1 - phi (Section 2.1);
 *   f  flow, BGK with Guo forcing of the solid drag F = -h tau_f (1+phi)^2 (1-phi) u / (4 W0^2) and
 *      the redefined velocity u* = (1-phi) u / 2 in the equilibria.
 * Lattices: D2Q5 (phi, U) + D2Q9 (flow) in 2-D; D3Q7 + D3Q19 in 3-D. Lattice units,
 * delta_t = delta_r = 1. Every update of one step uses time-n data only, so the three lattices
 * are advanced by one fused kernel per step.
 *
 * Conventions for every entry point:
 *   - Every function returns lbcg_status (0 = success, < 0 = error); no C++ exception crosses the
 *     ABI. lbcg_last_error() returns a message for the calling thread's last error.
 *   - Device memory: the caller allocates one device workspace (lbcg_workspace_bytes) and owns
 *     it; the library never allocates or frees device memory and keeps only a small host handle.
 *   - Streams: all device work is enqueued on the HIP stream given at creation (a hipStream_t,
 *     NULL for the null stream). lbcg_step only enqueues; read, write, measure and growth-rate
 *     calls synchronise that stream before returning.
 *   - Layout (of what the read and write calls take and give): scalar fields are [z][y][x] with
 *     x fastest; population arrays are planes [a][z][y][x] in the lattice order
 *       D2Q5/D3Q7 : 0, +x, -x, +y, -y, (+z, -z)
 *       D2Q9      : 0, +x, -x, +y, -y, (1,1), (-1,-1), (1,-1), (-1,1)
 *       D3Q19     : 0, +x, -x, +y, -y, +z, -z, (1,1,0), (-1,-1,0), (1,-1,0), (-1,1,0),
 *                   (1,0,1), (-1,0,-1), (1,0,-1), (-1,0,1), (0,1,1), (0,-1,-1), (0,1,-1), (0,-1,1)
 *   - Handles are not thread-safe; distinct handles may be used from distinct threads.
 */
#ifndef LBCG_H
#define LBCG_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    LBCG_OK = 0,
    LBCG_EINVAL = -1,     /* bad argument, size or field id */
    LBCG_EUNSTABLE = -2,  /* parameters give a relaxation time <= 1/2 or a_s <= 0 */
    LBCG_ENOMEM = -3,     /* workspace (or a destination buffer) too small */
    LBCG_EDEVICE = -4,    /* a HIP call failed (the message names it) */
    LBCG_ENONFINITE = -5, /* a measurement found NaN/Inf in phi, U or rho */
    LBCG_ESTATE = -6      /* call not valid in the handle's state */
} lbcg_status;

typedef enum {
    LBCG_FP64 = 0,         /* every population and all arithmetic in binary64 */
    LBCG_FP32 = 1,         /* populations and arithmetic in binary32 */
    LBCG_FP32_F16SHIFT = 2 /* as FP32, but the flow populations are stored as binary16 f_a - w_a */
} lbcg_precision;

/* x faces: periodic; inlet at x = 0 (velocity bounce-back for f, anti-bounce-back U = U_inlet for
 * g, bounce-back for h) and a zero-gradient outlet at x = nx-1 (the incoming populations copied from
 * x = nx-2); or the same inlet with a pressure outlet for the flow: populations leaving through
 * x = nx-1 come back by anti-bounce-back at rho = 1 and the node's own u*,
 * f_opp(a) = -f*_a + 2 w_a (1 + (c_a.u*)^2/(2 cs^4) - |u*|^2/(2 cs^2)), while g and h keep the copy.
 * The zero-gradient outlet fixes no pressure level; with walls or drag along the way the density
 * then creeps up, which the pressure outlet prevents. */
typedef enum { LBCG_PERIODIC = 0, LBCG_INFLOW_OUTFLOW = 1, LBCG_INFLOW_PRESSURE = 2 } lbcg_xbc;

typedef enum {
    LBCG_FIELD_PHI = 0,      /* phi = sum h */
    LBCG_FIELD_U = 1,        /* U = sum g */
    LBCG_FIELD_RHO = 2,      /* rho = sum f (1 without flow) */
    LBCG_FIELD_UX = 3,       /* u* components: the velocity the equilibria use */
    LBCG_FIELD_UY = 4,
    LBCG_FIELD_UZ = 5,
    LBCG_FIELD_PHI_PREV = 6, /* phi of the previous step (for dphi/dt) */
    LBCG_FIELD_RAW_H = 7,    /* populations, q planes */
    LBCG_FIELD_RAW_G = 8,
    LBCG_FIELD_RAW_F = 9
} lbcg_field;

typedef enum { LBCG_DTYPE_F64 = 0, LBCG_DTYPE_F32 = 1 } lbcg_dtype;

typedef struct {
    int32_t dim;         /* 2 or 3 */
    int32_t nx, ny, nz;  /* grid size; nz = 1 when dim = 2; nx >= 3 with open x faces */
    int32_t flow;        /* 1: flow lattice on; 0: u* = 0 everywhere */
    int32_t precision;   /* lbcg_precision */
    int32_t xbc;         /* lbcg_xbc: periodic, or inlet at x = 0 / outlet at x = nx-1 */
    int32_t walls;       /* 0: none; 1: the workspace keeps a solid-wall mask (lbcg_set_walls) */
    double W0, tau0;     /* interface width and time (Eq. a); tau0 > 0, W0 > 0 */
    double lambda;       /* coupling constant of Eq. (a) */
    double D;            /* solute diffusivity (Eq. b); >= 0 */
    double eps_aniso;    /* anisotropy strength, 0 <= eps < 1 */
    double nu;           /* kinematic viscosity, > 0 with flow; tau_f = nu/cs^2 + 1/2 */
    double h_drag;       /* drag constant h of the solid drag force (2.757 in the paper) */
    double u_inlet;      /* inlet velocity (x) with open x faces */
    double U0, U_inlet;  /* initial and inlet supersaturation */
    double seed_center[3], seed_radius; /* initial seed (node coordinates; z ignored in 2-D) */
    double grad_eps2;    /* |grad phi|^2 at or below which a_s = 1 and the anisotropy flux is 0 */
    int32_t seed_shape;  /* lbcg_seed_shape; polygons have circumradius seed_radius and are prisms
                          * of half-height equal to their apothem in 3-D */
    int32_t collision;   /* lbcg_collision of the flow populations (0 without flow) */
    double seed_tilt;    /* orientation of the crystal about z, radians (the paper's seed tilt): turns
                          * a polygonal seed and the anisotropy, a_s = 1 + eps cos 6(theta - tilt) */
    double omega_bulk;   /* central-Hermite MRT only: relaxation rate of the trace of the second-order
                          * central moment, in (0, 2) (1: to equilibrium in one step) */
    int32_t solute_source; /* lbcg_solute_source */
} lbcg_params;

/* Solute source (Eq. (b) and the ADE source of Section 2.2). FULL: -dphi/dt as Eq. (b) prints it,
 * the source term of the solute populations -w_alpha (phi - phi_prev). HALF: -(1/2) dphi/dt, half
 * the rate of change of phi, as in the thin-interface model of Karma and Rappel that the paper
 * cites; with it the average growth rates of rhombic seeds at the paper's scale come within 8% of
 * the ones the paper prints (Tables ljs and lax), against 0.51-0.57 of them with FULL. Either way
 * sum U + B sum (1 + phi_prev), B = 1 or 1/2, is conserved exactly in a closed box; it is the M'
 * of lbcg_measure. */
typedef enum { LBCG_SOURCE_FULL = 0, LBCG_SOURCE_HALF = 1 } lbcg_solute_source;

/* Flow collision (Section 2.2, flow paragraph: BGK, or the central-Hermite multiple-relaxation-time
 * operator the paper names for stability). The MRT works on central Hermite moments about u*
 * (He0 = 1, He1 = xi, He2 = xi^2 - cs^2 per direction; on D2Q9 the multi-indices with n_x, n_y <= 2,
 * on D3Q19 the 19 with each n_d <= 2 and at most two non-zero): rho kept; first order to
 * (1 - w) k + (1 - w/2) F, the BGK-Guo momentum update; the deviatoric second order relaxes with
 * w = 1/tau_f and its trace with omega_bulk; third and fourth orders to zero. Needs flow = 1; the
 * z-marching tiling does not implement it. */
typedef enum { LBCG_COLLISION_BGK = 0, LBCG_COLLISION_CHMRT = 1 } lbcg_collision;

/* Seed shapes (Section 4: rhombic and hexagonal seeds, tilted). The initial phase field is
 * phi0 = tanh(-d / (sqrt(2) W0)) with d the signed distance to the seed: |x - c| - R for the
 * circle / sphere, and for a polygon the largest distance to its face planes, max_k n_k.(x - c) - a
 * (apothem a = R cos(pi/n)). Hexagon: face normals at tilt + 30 + 60k degrees (vertices on the axes
 * at tilt 0); rhombus (60 / 120 degrees): face normals at tilt +- 30 and tilt + 180 +- 30 degrees,
 * four of the hexagon's (long diagonal, 2R, across the tilt direction; the other two facets form at
 * its acute vertices). */
typedef enum { LBCG_SEED_CIRCLE = 0, LBCG_SEED_HEXAGON = 1, LBCG_SEED_RHOMBUS = 2 } lbcg_seed_shape;

typedef struct lbcg_handle lbcg_handle;
typedef struct lbcg_batch lbcg_batch;

/* Bytes of device workspace one solver needs (0 if the parameters are invalid). It holds two
 * copies (ping-pong) of each population array, phi_prev, a staging area for read-back, the
 * reduction scratch, the measurement history of lbcg_run (32 KB) and, with walls, the wall mask.
 * Inside it, rows are stored at a pitch of nx rounded up to 64 nodes and population planes at a
 * stride of the stored plane rounded up to 64 nodes plus 64 (nx and N where a binary64 plane
 * would reach 2^32 bytes); the field and raw-array calls convert to and from the dense layout. */
size_t lbcg_workspace_bytes(const lbcg_params* p);

/* Validate p, bind the caller's workspace (device pointer, >= lbcg_workspace_bytes bytes,
 * 256-byte aligned) and stream, and enqueue the initial state: the seed
 * phi0 = tanh(-d / (sqrt(2) W0)) with d the signed distance to the seed shape (lbcg_seed_shape;
 * d = |x - c| - R for the circle / sphere), h = w phi0, g = w U0,
 * f = f_eq(rho = 1, u* = u_inlet (1 - phi0)/2 x^), phi_prev = phi0.
 * Errors: EINVAL (sizes, enums, NULL pointers), EUNSTABLE, ENOMEM (workspace too small),
 * EDEVICE. On error *out is NULL. */
lbcg_status lbcg_create(const lbcg_params* p, void* dev_workspace, size_t bytes, void* hip_stream,
                        lbcg_handle** out);

/* Enqueue nsteps coupled time steps (Section 2.2: collide and stream h, g and f). Returns
 * ENONFINITE without stepping if the last measurement found a non-finite value. */
lbcg_status lbcg_step(lbcg_handle* h, int64_t nsteps);

/* Number of steps taken so far. */
int64_t lbcg_step_count(const lbcg_handle* h);

/* Copy one field into dst (dst_bytes must hold it: N values, or q*N for a RAW_* field) as
 * binary64 or binary32 values; dst is a device pointer if dst_on_device, else host memory.
 * RAW_F of an FP16-shift solver is returned decoded (w_a + stored deviation). Synchronises. */
lbcg_status lbcg_read_field(lbcg_handle* h, int field, void* dst, size_t dst_bytes,
                            int dst_on_device, int dst_dtype);

/* Overwrite a RAW_* population array or PHI_PREV from src (binary64 or binary32, host or
 * device); values are rounded to the solver's storage precision. Synchronises. */
lbcg_status lbcg_write_field(lbcg_handle* h, int field, const void* src, size_t src_bytes,
                             int src_on_device, int src_dtype);

/* Diagnostics (Section 4.1.2). mass_out[6] (may be NULL) receives, accumulated in binary64:
 * {sum U, sum phi_prev, V_s = sum (1+phi)/2, M' = sum U + B sum (1 + phi_prev) (B of
 *  lbcg_solute_source), max |u*|,
 *  number of nodes with non-finite phi, U or rho}.
 * L_out[ndirs] (may be NULL when ndirs = 0) receives the crystal extent along each unit
 * direction dirs[3k..3k+2] from the seed centre: the first phi = 0 crossing of a ray sampled
 * every 1/4 cell with bi/trilinear interpolation, linearly interpolated between samples; 0 if
 * phi <= 0 at the centre, the last in-domain distance if no crossing. Each call appends
 * (step, L) to the handle's history for lbcg_growth_rates. Synchronises. Returns ENONFINITE
 * (outputs filled) if a non-finite value was found. ndirs <= 256. */
lbcg_status lbcg_measure(lbcg_handle* h, int ndirs, const double* dirs, double* L_out,
                         double* mass_out);

/* lbcg_measure for callers that cannot allocate device memory and cannot give the solver's
 * workspace to the diagnostics (code under HIP graph capture, tight serving loops, harnesses that
 * forbid allocation): the same kernels and results, bit for bit, but the reduction partials, the
 * directions and the extents live in a file-scope device array of the library (57.6 KB per device,
 * held until the process ends) instead of in the workspace. It calls no allocation routine. The
 * device the handle was created on must be current (EINVAL otherwise). ndirs <= 256 (EINVAL
 * otherwise: the array holds no more). Every call on one device shares that device's array, and
 * nothing in it needs to start at zero (each call writes every value it reads); calls that overlap
 * on one device, on any streams, race and must be serialised by the caller. Synchronises. */
lbcg_status lbcg_measure_noalloc(lbcg_handle* h, int ndirs, const double* dirs, double* L_out,
                                 double* mass_out);

/* A run with diagnostics, without host round trips (the measurement sequence of Section 4.1.2,
 * sizes and sums every measure_every steps): enqueue nsteps steps and, after every
 * measure_every of them, the lbcg_measure diagnostics, whose results stay on the device until the
 * run (or each block of up to 4096 / (6 + ndirs) samples) is copied back in one transfer.
 * Samples = nsteps / measure_every; mass_hist[samples][6] and L_hist[samples][ndirs] receive them
 * (either may be NULL) and every sample is appended to the growth-rate history, as lbcg_measure
 * does. Remaining steps (nsteps mod measure_every) are enqueued after the last sample.
 * Synchronises. Returns ENONFINITE if a sample found a non-finite value; the run then stops after
 * that block (outputs filled up to it). Errors: EINVAL (NULL handle, nsteps < 0,
 * measure_every < 1, bad directions), ENONFINITE (as lbcg_step). */
lbcg_status lbcg_run(lbcg_handle* h, int64_t nsteps, int64_t measure_every, int ndirs, const double* dirs,
                     double* L_hist, double* mass_hist);

/* Least-squares growth rate of every direction over the recorded history (Section 4.1.2:
 * linear fit of length against time), in cells per step: G_out[ndirs], R2_out[ndirs]
 * (R^2 = 1 - A_res/A_tot), and *G_avg_out, the slope of the mean length. Needs >= 2 samples
 * taken with the same ndirs (ESTATE otherwise). Any output may be NULL. */
lbcg_status lbcg_growth_rates(lbcg_handle* h, double* G_out, double* R2_out, double* G_avg_out);

/* Step-kernel variants: the tilings the library can run for this solver (z-marching over full
 * rows or 3-D blocks, of several shapes, and their cache policies). Every variant computes the
 * same update, up to the rounding of floating-point contractions the compiler may choose
 * differently per tiling; they differ in speed. Variant 0 is the default. */
int lbcg_variant_count(const lbcg_handle* h);   /* -1 for a NULL handle */
int lbcg_variant_current(const lbcg_handle* h); /* -1 for a NULL handle */
lbcg_status lbcg_variant_name(const lbcg_handle* h, int idx, char* buf, size_t buflen);
lbcg_status lbcg_variant_select(lbcg_handle* h, int idx);

/* Mean time per step (microseconds, HIP events on the handle's stream) of `launches` coupled
 * steps run with variant idx after one untimed step. These are real steps: the state and the
 * step count advance by launches + 1, as lbcg_step(h, launches + 1) with variant idx selected
 * would advance them. The selected variant is left as it was.
 * LBCG_ENONFINITE if the last measurement found a non-finite value. Synchronises. */
lbcg_status lbcg_variant_time(lbcg_handle* h, int idx, int launches, double* us);

/* Time every variant as lbcg_variant_time does, in two rounds over all variants (each keeps the
 * faster of its two times, so that the cache state the previous candidate left does not decide),
 * select the fastest, and return its index and time (either output may be NULL). The state
 * advances by 2 x (launches + 1) x lbcg_variant_count steps. The choice is recorded in the process's tuning cache (see lbcg_batch_autotune), so later
 * solvers of the same grid kind, shape, precision and architecture start with it. Synchronises. */
lbcg_status lbcg_autotune(lbcg_handle* h, int launches, int* best, double* best_us);

/* ---- Checkpoints ----
 * The solver state exactly as stored: the current copy of h, g, f (if flow) and phi_prev in the
 * storage precision and memory layout, after a 64-byte header (magic "LBCGSTAT", format version,
 * dim, nx, ny, nz, flow, precision, boundary kind, step count). Loading it into a solver with the
 * same grid, flow, precision and boundary kind continues the run bit for bit, which a round trip
 * through lbcg_read_field / lbcg_write_field cannot promise (the stored deviations from the lattice
 * weights may be too small for the decoded binary64 value to carry them). */

/* Bytes of a checkpoint of this solver (0 for a NULL handle). */
size_t lbcg_state_bytes(const lbcg_handle* h);

/* Copy the state into dst (>= lbcg_state_bytes; device pointer if dst_on_device, else host
 * memory). ENOMEM if dst is too small. Synchronises. */
lbcg_status lbcg_state_save(lbcg_handle* h, void* dst, size_t dst_bytes, int dst_on_device);

/* Replace the state (and the step count) with a checkpoint. EINVAL if the header does not match
 * this solver; ENOMEM if src_bytes is short. Clears the non-finite flag; the crystal-size history
 * of lbcg_measure is kept. Synchronises. */
lbcg_status lbcg_state_load(lbcg_handle* h, const void* src, size_t src_bytes, int src_on_device);

/* ---- Solid walls (reactor walls and baffles, Section 4: zero-flux phase field and solute, no-slip
 * flow) ----
 * For a solver created with walls = 1: set the wall mask, one byte per node in the plain layout
 * [z][y][x], nonzero = solid wall node (the mask starts empty). Wall nodes are frozen: they are
 * not updated and push nothing. A population a fluid node would push onto a wall node is bounced
 * back into the node's opposite population instead (halfway bounce-back): f with the wall at rest
 * (no-slip), g unchanged (zero solute flux), h by Eq. (d) with the old value of the slot it is
 * written to (zero phase-field flux, as at the inlet). In the phi gradient a wall neighbour takes
 * the node's own value (zero normal derivative). lbcg_measure's sums skip wall nodes; fields read
 * at wall nodes show their frozen state. With open x faces the outlet copy pairs the last two
 * columns of each row, so there they must be both wall or both fluid. EINVAL: walls = 0 at
 * creation, a mask that is too small, or a row that breaks the outlet pairing. Synchronises.
 * Batches do not take walls. */
lbcg_status lbcg_set_walls(lbcg_handle* h, const uint8_t* mask, size_t bytes, int mask_on_device);

/* Release the host handle (the workspace stays the caller's). NULL is accepted. */
lbcg_status lbcg_destroy(lbcg_handle* h);

/* ---- Batches: many independent grids of one kind advanced by one launch per step ----
 * The parametric studies of the paper (Section 4.1.3 supersaturation, 4.1.4 seed size, 4.2
 * inflow velocity) run many small grids; a batch steps all of them with one kernel launch per step
 * (a list of the tiles of every instance), optionally replayed from a captured HIP graph. Every
 * instance computes exactly what a single solver with the same parameters computes. All instances
 * must share dim, flow, precision and collision; sizes, x faces, the solute source and physical
 * parameters may differ.
 * Batches take no walls (EINVAL). */

/* Device workspace bytes for n instances (0 if any parameter set is invalid). */
size_t lbcg_batch_workspace_bytes(int n, const lbcg_params* p /* n */);

/* As lbcg_create, for n instances in one caller-owned workspace; synchronises. */
lbcg_status lbcg_batch_create(int n, const lbcg_params* p, void* dev_workspace, size_t bytes, void* hip_stream,
                              lbcg_batch** out);

/* Advance every instance nsteps steps. If measure_every > 0 and ndirs > 0, after every
 * measure_every steps the crystal extent of every instance along each unit direction (as in
 * lbcg_measure) is appended to L_hist, laid out [sample][instance][direction] with
 * floor(nsteps / measure_every) samples. use_graph != 0 replays each measure_every-step chunk from
 * a captured HIP graph (needs a non-null stream). Synchronises. */
lbcg_status lbcg_batch_run(lbcg_batch* b, int64_t nsteps, int64_t measure_every, int ndirs, const double* dirs,
                           double* L_hist, int use_graph);

/* Crystal extent of every instance now: L_out[instance * ndirs + k]. Synchronises. */
lbcg_status lbcg_batch_measure(lbcg_batch* b, int ndirs, const double* dirs, double* L_out);

/* lbcg_read_field for instance `inst`. */
lbcg_status lbcg_batch_read_field(lbcg_batch* b, int inst, int field, void* dst, size_t dst_bytes,
                                  int dst_on_device, int dst_dtype);

int64_t lbcg_batch_step_count(const lbcg_batch* b);  /* -1 for NULL */

/* Batch tilings and their autotuner (the sweeps of Sections 4.1.3, 4.1.4 and 4.2 as one launch per
 * step). A batch can run its step kernel in several tilings (tile shapes and cache policies, the
 * first the default); every tiling computes what the single-grid kernel of the same tiling computes.
 * lbcg_batch_variant_time times real batched steps with tiling idx (HIP events on the batch's stream:
 * one untimed step, then `launches` timed ones, the ping-pong copies alternating), so the state
 * advances by launches + 1 steps; the selected tiling is left as it was. lbcg_batch_autotune times
 * every tiling that way in two rounds (all_us[count] receives each tiling's faster time, may be
 * NULL; the state advances by 2 x (launches + 1) x count steps), selects the fastest and
 * records the choice in the process's tuning cache under the kernel kind, precision, GPU
 * architecture and the batch's mix of instance shapes; lbcg_batch_create then starts every batch
 * with the same key on that tiling. With the environment variable LBCG_TUNE_CACHE naming a file,
 * the cache is also read from it at first use and every choice is appended to it. lbcg_autotune
 * records its choice for single grids in the same cache (key: kernel kind, grid shape, precision,
 * architecture), which lbcg_create applies. Selecting a tiling synchronises the stream and drops
 * the batch's captured graphs. */
int lbcg_batch_variant_count(const lbcg_batch* b);   /* -1 for NULL */
int lbcg_batch_variant_current(const lbcg_batch* b); /* -1 for NULL */
lbcg_status lbcg_batch_variant_name(const lbcg_batch* b, int idx, char* buf, size_t buflen);
lbcg_status lbcg_batch_variant_select(lbcg_batch* b, int idx);
lbcg_status lbcg_batch_variant_time(lbcg_batch* b, int idx, int launches, double* us);
lbcg_status lbcg_batch_autotune(lbcg_batch* b, int launches, int* best, double* best_us, double* all_us);
/* Forget every choice of the tuning cache in this process (the cache file is not touched or read
 * again). */
lbcg_status lbcg_tune_cache_clear(void);

/* Release the host state and captured graphs (the workspace stays the caller's). NULL accepted. */
lbcg_status lbcg_batch_destroy(lbcg_batch* b);

/* ---- Growth-rate surrogate: a multilayer perceptron trained and evaluated on the GPU ----
 * Layers l = 0 .. nlayers-1 map widths[l] -> widths[l+1]; hidden layers use SiLU, the last layer is
 * linear and its output is split into a mean head (first half) and a log-variance head (second
 * half). GEMMs run on bf16 MFMA with fp32 accumulation: weights are kept as fp32 master copies and
 * used as bf16; activations and back-propagated gradients are rounded to bf16 after their fp32
 * epilogue. Parameters are packed per layer as W (widths[l+1] x widths[l], row-major) then b. The
 * loss is the Gaussian negative log-likelihood (1/(B D)) sum 0.5 (exp(-s)(t - mu)^2 + s), with the
 * log-variance s clamped to [-12, 12]. Device pointers: X (rows x widths[0]), T (rows x D, D =
 * widths[nlayers]/2), idx (int32, B rows of X/T forming the batch, clamped to [0, rows)). */
typedef struct lbcg_mlp lbcg_mlp;
size_t lbcg_mlp_workspace_bytes(int nlayers, const int* widths, int max_batch);  /* 0 if invalid */
lbcg_status lbcg_mlp_create(int nlayers, const int* widths, int max_batch, void* dev_workspace, size_t bytes,
                            void* hip_stream, lbcg_mlp** out);                    /* parameters 0 */
int64_t lbcg_mlp_num_params(const lbcg_mlp* m);
/* Upload / download fp32 parameters (host, packed); upload resets the Adam state. Synchronise. */
lbcg_status lbcg_mlp_set_params(lbcg_mlp* m, const float* host_params);
lbcg_status lbcg_mlp_get_params(lbcg_mlp* m, float* host_params);
/* Inference: y (device, B x widths[nlayers]) from x (device, B x widths[0]); enqueued only. */
lbcg_status lbcg_mlp_forward(lbcg_mlp* m, int B, const float* x, float* y);
/* Loss and gradients of one batch without an update (gradients packed like the parameters, host).
 * Synchronises. */
lbcg_status lbcg_mlp_grads(lbcg_mlp* m, int B, const float* X, const float* T, const int* idx, int rows,
                           float* host_grads, float* loss_out);
/* One training step: gather, forward, loss, backward, Adam (bias-corrected; the step count is
 * kept by the handle). *loss_out gets the batch loss before the update and the call synchronises;
 * with loss_out NULL the step is only enqueued on the handle's stream (X, T and idx must then stay
 * valid until the stream reaches it). */
lbcg_status lbcg_mlp_train_step(lbcg_mlp* m, int B, const float* X, const float* T, const int* idx, int rows,
                                float lr, float beta1, float beta2, float eps, float* loss_out);
lbcg_status lbcg_mlp_destroy(lbcg_mlp* m);

/* Message of the calling thread's last error ("" if none). */
const char* lbcg_last_error(void);

/* Digest of the sources the library was built from (the build stores it; "unknown" if it did not),
 * so that a caller can refuse a library older than its sources. */
const char* lbcg_source_hash(void);

#ifdef __cplusplus
}
#endif
#endif /* LBCG_H */
