/*
 * lbcg_oracle.h -- FP64 CPU oracle of the coupled lattice Boltzmann crystal-growth step.
 *
 * TEST INFRASTRUCTURE ONLY. This is the plain, slow reference that the GPU library is checked
 * against. Only the test suite, the smoke check and the benchmark's CPU-baseline leg load it;
 * the product library neither includes this header nor links this code, and this code uses
 * nothing of the product library.
 *
 * Model: Tan, Hosseini, Seidel-Morgenstern, Thevenin, Lorenz, "Mandelic acid single-crystal
 * growth: experiments vs numerical simulations", arXiv 2206.02145, Section 2 (Eqs. a, b and the
 * three lattice Boltzmann schemes of Section 2.2). Lattice units: delta_t = delta_r = 1.
 *
 * Layout of every array: populations are planes pop[a][z][y][x] with x fastest; scalar fields
 * are field[z][y][x]. Node index i = (z*ny + y)*nx + x. In 2-D, nz = 1.
 */
#ifndef LBCG_ORACLE_H
#define LBCG_ORACLE_H
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct {
    int32_t dim;          /* 2 or 3 */
    int32_t nx, ny, nz;   /* grid; nz = 1 in 2-D */
    int32_t flow;         /* 1: flow lattice (D2Q9 / D3Q19) active; 0: u* = 0 */
    int32_t xbc;          /* 0: periodic in x; 1: inlet at x = 0, zero-gradient outlet at x = nx-1;
                           * 2: as 1 with a pressure outlet (rho = 1) for the flow (R30) */
    double W0, tau0, lambda, D, eps;   /* phase-field width, time, coupling, diffusivity, anisotropy */
    double nu, h_drag, u_in, U0, U_in; /* viscosity, drag constant, inlet velocity, initial / inlet U */
    double seed_c[3], seed_R;          /* seed centre (node coordinates) and radius */
    double grad_eps2;                  /* |grad phi|^2 threshold below which a_s = 1, N = 0 */
    const uint8_t* wall;               /* NULL, or one flag per node (1 = solid wall node, R28):
                                        * walls are frozen, populations aimed at them bounce back */
    int32_t seed_shape;                /* 0 circle / sphere, 1 hexagon, 2 rhombus (60/120 degrees);
                                        * polygons are prisms in 3-D (R29) */
    double seed_tilt;                  /* orientation of the crystal about z (radians): turns a
                                        * polygonal seed and the anisotropy axes (R32) */
    int32_t collision;                 /* flow collision: 0 BGK, 1 central-Hermite MRT (R31) */
    double omega_bulk;                 /* MRT relaxation rate of the trace of the second-order
                                        * central moment, in (0, 2) */
    int32_t solute_source;             /* 0: the source -dphi/dt of Eq. (b) as printed; 1: half
                                        * of it, -(1/2) dphi/dt (R33) */
} orc_params;

/* Lattice tables. kind: 0 = D2Q5, 1 = D3Q7, 2 = D2Q9, 3 = D3Q19.
 * Writes q, the velocities c (q x 3 ints), weights w (q) and cs^2. Returns 0, or -1 for a bad kind. */
int orc_lattice(int kind, int* q, int* c, double* w, double* cs2);

/* Anisotropy a_s and the flux vector N = |p|^2 d(a_s^2)/dp for a gradient p (3 values; p[2] = 0
 * in 2-D). */
void orc_aniso(double eps, double grad_eps2, const double* p, double* a, double* N);

/* Signed distance of the point (dx, dy, dz) (relative to the seed centre) to the seed's surface,
 * negative inside: |x| - R for the circle / sphere; for a polygon of circumradius R the largest
 * distance to its face planes, max_k n_k . x - a (apothem a = R cos(pi/n)), and in 3-D also to the
 * planes z = +-a (R29). */
double orc_seed_distance(const orc_params* P, double dx, double dy, double dz);

/* Initial state: tanh seed, h = w phi0, g = w U0, f = f_eq(1, u_in (1-phi0)/2 x^), phi_prev = phi0,
 * phi0 = tanh(-d / (sqrt(2) W0)) with d = orc_seed_distance.
 * f may be NULL when flow = 0. Returns 0 or -1 on bad parameters. */
int orc_init(const orc_params* P, double* h, double* g, double* f, double* phi_prev);

/* f = f_eq(rho, u) at every node, for given fields rho and u (test set-up). */
int orc_flow_equilibrium(const orc_params* P, const double* rho, const double* ux, const double* uy,
                         const double* uz, double* f);

/* Advance the state nsteps coupled time steps in place. Returns 0 or -1 on bad parameters. */
int orc_step(const orc_params* P, double* h, double* g, double* f, double* phi_prev, int64_t nsteps);

/* Macroscopic fields: phi, U, rho and the velocity u* used by the equilibria (rho = 1 and u* = 0
 * without flow). Any output pointer may be NULL. */
int orc_fields(const orc_params* P, const double* h, const double* g, const double* f, double* phi,
               double* U, double* rho, double* ux, double* uy, double* uz);

/* Diagnostics (sums over the non-wall nodes). mass_out[6] = {sum U, sum phi_prev, V_s = sum (1+phi)/2,
 * M' = sum U + B sum (1 + phi_prev) with B the solute source's coefficient (1, or 1/2 with
 * solute_source = 1), max |u*|, number of non-finite phi/U/rho values}.
 * L_out[ndirs] = crystal extent along each unit direction dirs[3k..3k+2] from the seed centre.
 * Either output may be NULL. */
int orc_measure(const orc_params* P, const double* h, const double* g, const double* f,
                const double* phi_prev, int ndirs, const double* dirs, double* L_out, double* mass_out);

/* Ray-march on a given nodal phi field (exposed for its own tests). */
int orc_raymarch(const orc_params* P, const double* phi, int ndirs, const double* dirs, double* L_out);

int orc_num_threads(void);
/* Threads used by the following oracle calls (OpenMP); n <= 0 leaves the setting alone. */
void orc_set_num_threads(int n);

#ifdef __cplusplus
}
#endif
#endif
