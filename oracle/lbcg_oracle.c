/*
 * lbcg_oracle.c -- FP64 CPU oracle of the coupled lattice Boltzmann crystal-growth step.
 *
 * TEST INFRASTRUCTURE ONLY: the slow, obviously correct reference the GPU library is checked
 * against. Used by the test suite, the smoke check and the benchmark's CPU-baseline leg, never
 * by the product path. It shares no code with the GPU library.
 *
 * Source of every formula: Tan et al., arXiv 2206.02145, Section 2.
 *   Section 2.1, Eq. (a): phase field; Eq. (b): supersaturation U; a_s = 1 + eps cos(6 theta);
 *     q(phi) = 1 - phi.
 *   Section 2.2, flow paragraph: stream-collide with Guo forcing, the solid drag force
 *     F = -h tau_f (1+phi)^2 (1-phi) u / (4 W0^2), the redefined velocity u* = (1-phi) u / 2 used in
 *     the equilibrium, BGK collision, Hermite equilibrium, tau_f = nu/cs^2 + 1/2, rho and rho u
 *     as moments.
 *   Section 2.2, solute paragraph: stream-collide with source -w dphi/dt, BGK with
 *     g_eq = w U (1 + c.u/cs^2), U = sum g, tau_U = D q(phi)/cs^2 + 1/2.
 *   Section 2.2, phase-field paragraph: the a_s^2-weighted stream-collide Eq. (d), source
 *     Q = phi - phi^3 + lambda U (1-phi^2)^2, equilibrium with the anisotropy flux Eq. (e),
 *     phi = sum h, tau_phi = a_s^2 W0^2 / (tau0 cs^2) + 1/2.
 *   Section 4.1.2: zero-flux walls and a constant-U inlet (used for the x faces).
 *
 * Where the paper is silent the oracle takes these readings (numbered as in the design notes):
 *   R1 phi and U on D2Q5 / D3Q7 (rest weights 1/3 and 1/4); R2 second-order Hermite equilibrium,
 *   BGK; R3 a_s = 1 + eps Re((nx + i ny)^6) in 3-D; R4 N = |p|^2 d(a_s^2)/dp in closed form with
 *   a threshold on |p|^2; R5 isotropic D2Q9 / D3Q19 gradient; R6 both a_s^2 of Eq. (d) taken at the
 *   collision (source) node; R8 dphi/dt = phi^n - phi^(n-1); R10 q = clamp(1 - phi, 0, 2);
 *   R13 u = m / (rho + K/2), F = -K u, u* in f_eq, the forcing and g_eq; R15 inlet: velocity
 *   bounce-back for f, anti-bounce-back Dirichlet for g, bounce-back for h; outlet: unknown
 *   populations copied from x = nx-2; R17 equilibrium initial populations; R23 gradient ghost at
 *   an open face = copy of the face node; R27 the h bounce-back at the inlet uses the old value of
 *   the slot it writes; R30 optional pressure outlet; R31 the central-Hermite MRT flow collision;
 *   R32 the anisotropy turns with the crystal's orientation; R33 optional half solute source.
 *
 * Units: lattice units, delta_t = delta_r = 1. Layout: pop[a][z][y][x], x fastest.
 */
#include "lbcg_oracle.h"

#include <complex.h>
#include <math.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

/* ------------------------------------------------------------------------------------------ */
/* Lattices                                                                                    */
/* ------------------------------------------------------------------------------------------ */

/* D2Q5 and D3Q7: the scalar lattices of phi and U (R1). */
static const int C5[5][3] = {{0, 0, 0}, {1, 0, 0}, {-1, 0, 0}, {0, 1, 0}, {0, -1, 0}};
static const double W5[5] = {1.0 / 3, 1.0 / 6, 1.0 / 6, 1.0 / 6, 1.0 / 6};
static const int C7[7][3] = {{0, 0, 0}, {1, 0, 0}, {-1, 0, 0}, {0, 1, 0},
                             {0, -1, 0}, {0, 0, 1}, {0, 0, -1}};
static const double W7[7] = {1.0 / 4, 1.0 / 8, 1.0 / 8, 1.0 / 8, 1.0 / 8, 1.0 / 8, 1.0 / 8};

/* D2Q9 and D3Q19: the flow lattices, and the stencils of the isotropic gradient (R5). */
static const int C9[9][3] = {{0, 0, 0},  {1, 0, 0},   {-1, 0, 0}, {0, 1, 0}, {0, -1, 0},
                             {1, 1, 0},  {-1, -1, 0}, {1, -1, 0}, {-1, 1, 0}};
static const double W9[9] = {4.0 / 9,  1.0 / 9,  1.0 / 9,  1.0 / 9, 1.0 / 9,
                             1.0 / 36, 1.0 / 36, 1.0 / 36, 1.0 / 36};
static const int C19[19][3] = {{0, 0, 0},  {1, 0, 0},  {-1, 0, 0},  {0, 1, 0},  {0, -1, 0},
                               {0, 0, 1},  {0, 0, -1}, {1, 1, 0},   {-1, -1, 0}, {1, -1, 0},
                               {-1, 1, 0}, {1, 0, 1},  {-1, 0, -1}, {1, 0, -1}, {-1, 0, 1},
                               {0, 1, 1},  {0, -1, -1}, {0, 1, -1}, {0, -1, 1}};
static const double W19[19] = {1.0 / 3,  1.0 / 18, 1.0 / 18, 1.0 / 18, 1.0 / 18, 1.0 / 18, 1.0 / 18,
                               1.0 / 36, 1.0 / 36, 1.0 / 36, 1.0 / 36, 1.0 / 36, 1.0 / 36, 1.0 / 36,
                               1.0 / 36, 1.0 / 36, 1.0 / 36, 1.0 / 36, 1.0 / 36};

typedef struct {
    int q;
    const int (*c)[3];
    const double* w;
    double cs2;
} lattice;

static lattice lattice_of_kind(int kind) {
    lattice L;
    switch (kind) {
        case 0: L.q = 5; L.c = C5; L.w = W5; L.cs2 = 1.0 / 3; break;
        case 1: L.q = 7; L.c = C7; L.w = W7; L.cs2 = 1.0 / 4; break;
        case 2: L.q = 9; L.c = C9; L.w = W9; L.cs2 = 1.0 / 3; break;
        default: L.q = 19; L.c = C19; L.w = W19; L.cs2 = 1.0 / 3; break;
    }
    return L;
}
static lattice scalar_lattice(int dim) { return lattice_of_kind(dim == 2 ? 0 : 1); }
static lattice flow_lattice(int dim) { return lattice_of_kind(dim == 2 ? 2 : 3); }

/* Index of the velocity opposite to c_a, found by search. */
static int opposite(const lattice* L, int a) {
    for (int b = 0; b < L->q; b++)
        if (L->c[b][0] == -L->c[a][0] && L->c[b][1] == -L->c[a][1] && L->c[b][2] == -L->c[a][2])
            return b;
    return -1;
}

int orc_lattice(int kind, int* q, int* c, double* w, double* cs2) {
    if (kind < 0 || kind > 3) return -1;
    lattice L = lattice_of_kind(kind);
    *q = L.q;
    for (int a = 0; a < L.q; a++) {
        for (int d = 0; d < 3; d++) c[3 * a + d] = L.c[a][d];
        w[a] = L.w[a];
    }
    *cs2 = L.cs2;
    return 0;
}

int orc_num_threads(void) {
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

void orc_set_num_threads(int n) {
#ifdef _OPENMP
    if (n > 0) omp_set_num_threads(n);
#else
    (void)n;
#endif
}

/* ------------------------------------------------------------------------------------------ */
/* Grid helpers                                                                                */
/* ------------------------------------------------------------------------------------------ */

static long nnodes(const orc_params* P) { return (long)P->nx * P->ny * P->nz; }
static long node(const orc_params* P, int x, int y, int z) {
    return ((long)z * P->ny + y) * P->nx + x;
}
static int wrap(int i, int n) {
    int r = i % n;
    return r < 0 ? r + n : r;
}

static int check_params(const orc_params* P) {
    if (P->dim != 2 && P->dim != 3) return -1;
    if (P->nx < 1 || P->ny < 1 || P->nz < 1) return -1;
    if (P->dim == 2 && P->nz != 1) return -1;
    if (P->xbc < 0 || P->xbc > 2) return -1;
    if (P->xbc != 0 && P->nx < 3) return -1;
    if (P->tau0 <= 0 || P->W0 <= 0) return -1;
    if (P->seed_shape < 0 || P->seed_shape > 2) return -1;
    if (P->collision < 0 || P->collision > 1) return -1;
    if (P->collision == 1 && !(P->omega_bulk > 0.0 && P->omega_bulk < 2.0)) return -1;
    if (P->solute_source < 0 || P->solute_source > 1) return -1;
    return 0;
}

/* ------------------------------------------------------------------------------------------ */
/* Anisotropy (Section 2.1; readings R3, R4)                                                   */
/* ------------------------------------------------------------------------------------------ */

/* a_s(n) = 1 + eps Re((nx + i ny)^6) with n the unit gradient direction; equals
 * 1 + eps cos(6 theta), theta = atan(ny/nx), whenever nz = 0. The sign of n does not matter
 * (even power). N = |p|^2 d(a_s^2)/dp = 2 eps a_s |p| (grad P(n) - 6 P(n) n), where
 * P(n) = Re((nx + i ny)^6) and grad P = (6 Re z^5, -6 Im z^5, 0). */
void orc_aniso(double eps, double grad_eps2, const double* p, double* a, double* N) {
    double s = p[0] * p[0] + p[1] * p[1] + p[2] * p[2];
    if (s <= grad_eps2) {
        *a = 1.0;
        N[0] = N[1] = N[2] = 0.0;
        return;
    }
    double m = sqrt(s);
    double n[3] = {p[0] / m, p[1] / m, p[2] / m};
    double complex z = n[0] + I * n[1];
    double complex z2 = z * z;
    double complex z4 = z2 * z2;
    double complex z5 = z4 * z;
    double complex z6 = z5 * z;
    double P6 = creal(z6);
    double gradP[3] = {6.0 * creal(z5), -6.0 * cimag(z5), 0.0};
    double as = 1.0 + eps * P6;
    *a = as;
    for (int d = 0; d < 3; d++) N[d] = 2.0 * eps * as * m * (gradP[d] - 6.0 * P6 * n[d]);
}

/* The anisotropy of the crystal turned by its orientation seed_tilt about z (R32): a_s and N
 * evaluated in the crystal's frame, a_s = 1 + eps cos(6 (theta - tilt)) in 2-D, N turned back. */
static void crystal_aniso(const orc_params* P, const double* p, double* a, double* N) {
    double c = cos(P->seed_tilt), s = sin(P->seed_tilt);
    double q[3] = {c * p[0] + s * p[1], -s * p[0] + c * p[1], p[2]};
    double Nq[3];
    orc_aniso(P->eps, P->grad_eps2, q, a, Nq);
    N[0] = c * Nq[0] - s * Nq[1];
    N[1] = s * Nq[0] + c * Nq[1];
    N[2] = Nq[2];
}

/* ------------------------------------------------------------------------------------------ */
/* Flow equilibrium and forcing (Section 2.2, flow paragraph; R2, R13, R21)                    */
/* ------------------------------------------------------------------------------------------ */

/* Second-order Hermite equilibrium, f_eq = w rho [1 + c.u/cs2 + (c.u)^2/(2 cs2^2) - u.u/(2 cs2)]. */
static double flow_feq(const lattice* L, int a, double rho, const double* u) {
    double cu = L->c[a][0] * u[0] + L->c[a][1] * u[1] + L->c[a][2] * u[2];
    double uu = u[0] * u[0] + u[1] * u[1] + u[2] * u[2];
    double cs2 = L->cs2;
    return L->w[a] * rho * (1.0 + cu / cs2 + cu * cu / (2.0 * cs2 * cs2) - uu / (2.0 * cs2));
}

/* Guo forcing term, w (1 - 1/(2 tau)) [c.F/cs2 + (u F + F u):(c c - cs2 I)/(2 cs2^2)], whose
 * second part equals ((c.u)(c.F) - cs2 u.F)/cs2^2. */
static double guo_source(const lattice* L, int a, double tau, const double* u, const double* F) {
    double cu = L->c[a][0] * u[0] + L->c[a][1] * u[1] + L->c[a][2] * u[2];
    double cF = L->c[a][0] * F[0] + L->c[a][1] * F[1] + L->c[a][2] * F[2];
    double uF = u[0] * F[0] + u[1] * F[1] + u[2] * F[2];
    double cs2 = L->cs2;
    return L->w[a] * (1.0 - 1.0 / (2.0 * tau)) * (cF / cs2 + (cu * cF - cs2 * uF) / (cs2 * cs2));
}

/* Drag coefficient K with F = -K u (flow paragraph of Section 2.2), the velocity of the
 * Guo scheme u = (m + F/2)/rho solved for the implicit F: u = m / (rho + K/2), and u*. */
static void flow_velocity(const orc_params* P, double tau_f, double phi, double rho, const double* m,
                          double* u, double* F, double* us) {
    double K = P->h_drag * tau_f * (1.0 + phi) * (1.0 + phi) * (1.0 - phi) / (4.0 * P->W0 * P->W0);
    for (int d = 0; d < 3; d++) {
        u[d] = m[d] / (rho + 0.5 * K);
        F[d] = -K * u[d];
        us[d] = 0.5 * (1.0 - phi) * u[d];
    }
}

/* ------------------------------------------------------------------------------------------ */
/* Central-Hermite multiple-relaxation-time flow collision (the stabilised collision Section 2.2 */
/* names for the flow; its moment set and relaxation rates are reading R31)                      */
/* ------------------------------------------------------------------------------------------ */

/* The lattice's Hermite multi-indices (n_x, n_y, n_z), each n_d in {0, 1, 2}: the nine with
 * n_z = 0 on D2Q9, and on D3Q19 the nineteen with at most two non-zero entries. Returns their
 * number (= q). */
static int chm_basis(int dim, int n[19][3]) {
    int m = 0;
    for (int a = 0; a <= 2; a++)
        for (int b = 0; b <= 2; b++)
            for (int c = 0; c <= (dim == 3 ? 2 : 0); c++)
                if ((a > 0) + (b > 0) + (c > 0) <= 2) {
                    n[m][0] = a;
                    n[m][1] = b;
                    n[m][2] = c;
                    m++;
                }
    return m;
}

/* One-dimensional Hermite polynomials of variance cs2: He0 = 1, He1 = xi, He2 = xi^2 - cs2. */
static double he(int n, double xi, double cs2) { return n == 0 ? 1.0 : (n == 1 ? xi : xi * xi - cs2); }

/* Solve A x = b for an n x n row-major A by Gaussian elimination with partial pivoting
 * (A and b are overwritten). */
static void solve_dense(int n, double* A, double* b, double* x) {
    for (int k = 0; k < n; k++) {
        int p = k;
        for (int r = k + 1; r < n; r++)
            if (fabs(A[r * n + k]) > fabs(A[p * n + k])) p = r;
        if (p != k) {
            for (int c = 0; c < n; c++) {
                double t = A[k * n + c];
                A[k * n + c] = A[p * n + c];
                A[p * n + c] = t;
            }
            double t = b[k];
            b[k] = b[p];
            b[p] = t;
        }
        for (int r = k + 1; r < n; r++) {
            double l = A[r * n + k] / A[k * n + k];
            for (int c = k; c < n; c++) A[r * n + c] -= l * A[k * n + c];
            b[r] -= l * b[k];
        }
    }
    for (int k = n - 1; k >= 0; k--) {
        double s = b[k];
        for (int c = k + 1; c < n; c++) s -= A[k * n + c] * x[c];
        x[k] = s / A[k * n + k];
    }
}

/* Post-collision populations of one node (f: the node's q populations). Central Hermite moments
 * about u*: k_n = sum_a f_a prod_d He_{n_d}(c_{a,d} - u*_d). Order 0 is kept (rho); order 1 becomes
 * (1 - omega) k + (1 - omega/2) F, the momentum update of the BGK scheme with Guo forcing; of the
 * order-2 tensor the deviatoric part relaxes with omega = 1/tau_f and the trace with omega_bulk;
 * orders 3 and 4 are set to their equilibrium value 0. The forcing enters the first order only
 * (its central moments vanish from the second order on). The populations solve T f* = k*. */
static void chm_collide(const orc_params* P, const lattice* V, const double* f, const double* us,
                        const double* F, double omega, double* fstar) {
    int n[19][3];
    int q = chm_basis(P->dim, n);
    double T[19 * 19], k[19];
    for (int m = 0; m < q; m++) {
        k[m] = 0.0;
        for (int a = 0; a < q; a++) {
            double t = 1.0;
            for (int d = 0; d < 3; d++) t *= he(n[m][d], V->c[a][d] - us[d], V->cs2);
            T[m * q + a] = t;
            k[m] += t * f[a];
        }
    }
    /* the order-2 tensor, its trace over the dim active directions */
    double K2[3][3] = {{0}};
    for (int m = 0; m < q; m++) {
        int order = n[m][0] + n[m][1] + n[m][2];
        if (order != 2) continue;
        int d = -1, e = -1;
        for (int j = 0; j < 3; j++)
            for (int r = 0; r < n[m][j]; r++) {
                if (d < 0) d = j;
                else e = j;
            }
        K2[d][e] = K2[e][d] = k[m];
    }
    double tr = 0.0;
    for (int d = 0; d < P->dim; d++) tr += K2[d][d];
    tr /= P->dim;
    double ks[19];
    for (int m = 0; m < q; m++) {
        int order = n[m][0] + n[m][1] + n[m][2];
        if (order == 0) {
            ks[m] = k[m];
        } else if (order == 1) {
            int d = n[m][0] ? 0 : (n[m][1] ? 1 : 2);
            ks[m] = (1.0 - omega) * k[m] + (1.0 - 0.5 * omega) * F[d];
        } else if (order == 2) {
            int diag = n[m][0] == 2 || n[m][1] == 2 || n[m][2] == 2;
            ks[m] = diag ? (1.0 - omega) * (k[m] - tr) + (1.0 - P->omega_bulk) * tr : (1.0 - omega) * k[m];
        } else {
            ks[m] = 0.0;
        }
    }
    solve_dense(q, T, ks, fstar);
}

/* ------------------------------------------------------------------------------------------ */
/* Initial state (R11, R17, R26)                                                               */
/* ------------------------------------------------------------------------------------------ */

double orc_seed_distance(const orc_params* P, double dx, double dy, double dz) {
    const double pi = 3.14159265358979323846;
    const double R = P->seed_R;
    if (P->seed_shape == 0) return sqrt(dx * dx + dy * dy + dz * dz) - R;
    /* hexagon: face normals at 30 + 60 k degrees (vertices on the axes); rhombus: face normals at
     * +-30 and 180 +-30 degrees, four of the hexagon's (its long diagonal along y, the acute
     * vertices where the other two facets form); both turned by the tilt (R29) */
    int nf = P->seed_shape == 1 ? 6 : 4;
    static const double hex_deg[6] = {30, 90, 150, 210, 270, 330};
    static const double rho_deg[4] = {30, 150, 210, 330};
    double apothem = R * cos(pi / (P->seed_shape == 1 ? 6.0 : 3.0));
    double d = -1e300;
    for (int k = 0; k < nf; k++) {
        double ang = (P->seed_shape == 1 ? hex_deg[k] : rho_deg[k]) * pi / 180.0 + P->seed_tilt;
        double dk = cos(ang) * dx + sin(ang) * dy - apothem;
        if (dk > d) d = dk;
    }
    if (P->dim == 3) {
        double dzk = fabs(dz) - apothem;
        if (dzk > d) d = dzk;
    }
    return d;
}

int orc_init(const orc_params* P, double* h, double* g, double* f, double* phi_prev) {
    if (check_params(P)) return -1;
    lattice S = scalar_lattice(P->dim);
    lattice V = flow_lattice(P->dim);
    long N = nnodes(P);
#pragma omp parallel for
    for (long r = 0; r < (long)P->nz * P->ny; r++) {
        int z = (int)(r / P->ny), y = (int)(r % P->ny);
        for (int x = 0; x < P->nx; x++) {
            long i = node(P, x, y, z);
            double dx = x - P->seed_c[0], dy = y - P->seed_c[1];
            double dz = (P->dim == 3) ? z - P->seed_c[2] : 0.0;
            double phi0 = tanh(-orc_seed_distance(P, dx, dy, dz) / (sqrt(2.0) * P->W0));
            phi_prev[i] = phi0;
            for (int a = 0; a < S.q; a++) {
                h[a * N + i] = S.w[a] * phi0;
                g[a * N + i] = S.w[a] * P->U0;
            }
            if (P->flow && f) {
                double u0[3] = {P->u_in * 0.5 * (1.0 - phi0), 0.0, 0.0};
                for (int a = 0; a < V.q; a++) f[a * N + i] = flow_feq(&V, a, 1.0, u0);
            }
        }
    }
    return 0;
}

int orc_flow_equilibrium(const orc_params* P, const double* rho, const double* ux, const double* uy,
                         const double* uz, double* f) {
    if (check_params(P)) return -1;
    lattice V = flow_lattice(P->dim);
    long N = nnodes(P);
    for (long i = 0; i < N; i++) {
        double u[3] = {ux[i], uy[i], uz ? uz[i] : 0.0};
        for (int a = 0; a < V.q; a++) f[a * N + i] = flow_feq(&V, a, rho[i], u);
    }
    return 0;
}

/* ------------------------------------------------------------------------------------------ */
/* One coupled time step                                                                       */
/* ------------------------------------------------------------------------------------------ */

typedef struct {
    double *phi, *U, *rho, *mx, *my, *mz, *px, *py, *pz;
    double *hn, *gn, *fn;
} scratch;

/* Phase 1: the zeroth and first moments at every node (phi = sum h, U = sum g, rho = sum f,
 * m = sum c f). */
static void moments(const orc_params* P, const double* h, const double* g, const double* f,
                    scratch* s) {
    lattice S = scalar_lattice(P->dim);
    lattice V = flow_lattice(P->dim);
    long N = nnodes(P);
#pragma omp parallel for
    for (long i = 0; i < N; i++) {
        double phi = 0.0, U = 0.0;
        for (int a = 0; a < S.q; a++) {
            phi += h[a * N + i];
            U += g[a * N + i];
        }
        s->phi[i] = phi;
        s->U[i] = U;
        double rho = 0.0, m[3] = {0.0, 0.0, 0.0};
        if (P->flow) {
            for (int a = 0; a < V.q; a++) {
                double fa = f[a * N + i];
                rho += fa;
                for (int d = 0; d < 3; d++) m[d] += V.c[a][d] * fa;
            }
        }
        s->rho[i] = rho;
        s->mx[i] = m[0];
        s->my[i] = m[1];
        s->mz[i] = m[2];
    }
}

static int is_wall(const orc_params* P, long i) { return P->wall && P->wall[i]; }

/* phi at the node x + c (periodic wrap in y, z, and in x when periodic; at an open x face the
 * ghost takes the value of the face node, R23; a wall neighbour takes the value of the node
 * itself, own, so that the normal derivative vanishes at the wall, R28). */
static double phi_at(const orc_params* P, const double* phi, int x, int y, int z, long own) {
    if (P->xbc == 0) {
        x = wrap(x, P->nx);
    } else {
        if (x < 0) x = 0;
        if (x > P->nx - 1) x = P->nx - 1;
    }
    y = wrap(y, P->ny);
    z = wrap(z, P->nz);
    long j = node(P, x, y, z);
    return is_wall(P, j) ? phi[own] : phi[j];
}

/* Phase 2: grad phi = (1/cs2) sum_b w_b c_b phi(x + c_b) over the D2Q9 / D3Q19 stencil (R5). */
static void gradient(const orc_params* P, scratch* s) {
    lattice G = flow_lattice(P->dim);
#pragma omp parallel for
    for (long r = 0; r < (long)P->nz * P->ny; r++) {
        int z = (int)(r / P->ny), y = (int)(r % P->ny);
        for (int x = 0; x < P->nx; x++) {
            long i = node(P, x, y, z);
            double p[3] = {0.0, 0.0, 0.0};
            for (int b = 0; b < G.q; b++) {
                double phib = phi_at(P, s->phi, x + G.c[b][0], y + G.c[b][1], z + G.c[b][2], i);
                for (int d = 0; d < 3; d++) p[d] += G.w[b] * G.c[b][d] * phib;
            }
            s->px[i] = p[0] / G.cs2;
            s->py[i] = p[1] / G.cs2;
            s->pz[i] = p[2] / G.cs2;
        }
    }
}

/* Where population a leaving node (x,y,z) lands: 0 inside (index in *dst), 1 through the inlet
 * face (x < 0), 2 through the outlet face (x >= nx), 3 onto a wall node. */
static int destination(const orc_params* P, const lattice* L, int a, int x, int y, int z, long* dst) {
    int xd = x + L->c[a][0];
    int yd = wrap(y + L->c[a][1], P->ny);
    int zd = wrap(z + L->c[a][2], P->nz);
    if (P->xbc == 0) {
        xd = wrap(xd, P->nx);
    } else {
        if (xd < 0) return 1;
        if (xd >= P->nx) return 2;
    }
    *dst = node(P, xd, yd, zd);
    return is_wall(P, *dst) ? 3 : 0;
}

/* Phase 3: collide at every node with time-n data only, then stream (push) into the new arrays. */
static void collide_stream(const orc_params* P, const double* h, const double* g, const double* f,
                           const double* phi_prev, scratch* s) {
    lattice S = scalar_lattice(P->dim);
    lattice V = flow_lattice(P->dim);
    long N = nnodes(P);
    double k = P->W0 * P->W0 / P->tau0;                /* W0^2 / tau0 */
    double tau_f = P->nu / V.cs2 + 0.5;                /* flow paragraph, tau_f = nu/cs2 + 1/2 */
    double uw[3] = {P->u_in, 0.0, 0.0};                /* inlet velocity */
#pragma omp parallel for
    for (long r = 0; r < (long)P->nz * P->ny; r++) {
        int z = (int)(r / P->ny), y = (int)(r % P->ny);
        for (int x = 0; x < P->nx; x++) {
            long i = node(P, x, y, z);
            if (is_wall(P, i)) continue; /* walls are frozen (R28) */
            double phi = s->phi[i], U = s->U[i];
            double p[3] = {s->px[i], s->py[i], s->pz[i]};
            double as, Nv[3];
            crystal_aniso(P, p, &as, Nv);
            double a2 = as * as;

            /* Phase field, Eq. (d) with Eq. (e). */
            double tau_phi = a2 * k / S.cs2 + 0.5;
            double Q = phi - phi * phi * phi + P->lambda * U * (1.0 - phi * phi) * (1.0 - phi * phi);
            for (int a = 0; a < S.q; a++) {
                double cN = S.c[a][0] * Nv[0] + S.c[a][1] * Nv[1] + S.c[a][2] * Nv[2];
                double heq = S.w[a] * (phi - cN * k / S.cs2);
                double ha = h[a * N + i];
                double hstar = ha - (ha - heq) / tau_phi + S.w[a] * Q / P->tau0;
                long d;
                int where = destination(P, &S, a, x, y, z, &d);
                if (where == 0) {
                    s->hn[a * N + d] = (hstar - (1.0 - a2) * h[a * N + d]) / a2;
                } else if (where == 1 || where == 3) { /* zero-flux bounce-back: inlet face (R15, R27)
                                                          * or wall (R28) */
                    int b = opposite(&S, a);
                    s->hn[b * N + i] = (hstar - (1.0 - a2) * h[b * N + i]) / a2;
                }
            }

            /* Flow: BGK with Guo forcing of the drag force. */
            double us[3] = {0.0, 0.0, 0.0};
            if (P->flow) {
                double rho = s->rho[i];
                double m[3] = {s->mx[i], s->my[i], s->mz[i]};
                double u[3], F[3];
                flow_velocity(P, tau_f, phi, rho, m, u, F, us);
                double fc[19];
                if (P->collision == 1) { /* central-Hermite MRT (R31) */
                    double fl[19];
                    for (int a = 0; a < V.q; a++) fl[a] = f[a * N + i];
                    chm_collide(P, &V, fl, us, F, 1.0 / tau_f, fc);
                }
                for (int a = 0; a < V.q; a++) {
                    double fa = f[a * N + i];
                    double fstar = P->collision == 1 ? fc[a]
                                                     : fa - (fa - flow_feq(&V, a, rho, us)) / tau_f +
                                                           guo_source(&V, a, tau_f, us, F);
                    long d;
                    int where = destination(P, &V, a, x, y, z, &d);
                    if (where == 0) {
                        s->fn[a * N + d] = fstar;
                    } else if (where == 1) { /* velocity bounce-back, wall density 1 (R15) */
                        int b = opposite(&V, a);
                        double cuw = V.c[a][0] * uw[0] + V.c[a][1] * uw[1] + V.c[a][2] * uw[2];
                        s->fn[b * N + i] = fstar - 2.0 * V.w[a] * 1.0 * cuw / V.cs2;
                    } else if (where == 3) { /* no-slip halfway bounce-back at a wall at rest (R28) */
                        s->fn[opposite(&V, a) * N + i] = fstar;
                    } else if (where == 2 && P->xbc == 2) { /* pressure outlet, rho = 1 (R30):
                                                              * anti-bounce-back at the node's u* */
                        double cu = V.c[a][0] * us[0] + V.c[a][1] * us[1] + V.c[a][2] * us[2];
                        double uu = us[0] * us[0] + us[1] * us[1] + us[2] * us[2];
                        s->fn[opposite(&V, a) * N + i] =
                            -fstar + 2.0 * V.w[a] * 1.0 * (1.0 + cu * cu / (2.0 * V.cs2 * V.cs2) - uu / (2.0 * V.cs2));
                    }
                }
            }

            /* Solute, with q(phi) = 1 - phi clamped to [0, 2] (R10) and dphi/dt = phi^n - phi^(n-1). */
            double q = 1.0 - phi;
            if (q < 0.0) q = 0.0;
            if (q > 2.0) q = 2.0;
            double tau_U = P->D * q / S.cs2 + 0.5;
            /* the source -B dphi/dt: B = 1 as Eq. (b) prints it, or 1/2 (R33) */
            double dphi = (P->solute_source == 1 ? 0.5 : 1.0) * (phi - phi_prev[i]);
            for (int a = 0; a < S.q; a++) {
                double cu = S.c[a][0] * us[0] + S.c[a][1] * us[1] + S.c[a][2] * us[2];
                double geq = S.w[a] * U * (1.0 + cu / S.cs2);
                double ga = g[a * N + i];
                double gstar = ga - (ga - geq) / tau_U - S.w[a] * dphi;
                long d;
                int where = destination(P, &S, a, x, y, z, &d);
                if (where == 0) {
                    s->gn[a * N + d] = gstar;
                } else if (where == 1) { /* anti-bounce-back, Dirichlet U = U_in (R15) */
                    int b = opposite(&S, a);
                    s->gn[b * N + i] = -gstar + 2.0 * S.w[a] * P->U_in;
                } else if (where == 3) { /* zero-flux bounce-back at a wall (R28) */
                    s->gn[opposite(&S, a) * N + i] = gstar;
                }
            }
        }
    }
}

/* Phase 4: at the outlet layer x = nx-1 the populations that would enter from x = nx are unknown;
 * they take the values just streamed into x = nx-2 (zero-gradient outflow, R15). */
static void outlet_fill(const orc_params* P, const lattice* L, double* pn) {
    long N = nnodes(P);
    for (int z = 0; z < P->nz; z++)
        for (int y = 0; y < P->ny; y++) {
            if (is_wall(P, node(P, P->nx - 1, y, z))) continue; /* walls stay frozen (R28) */
            for (int a = 0; a < L->q; a++)
                if (L->c[a][0] < 0)
                    pn[a * N + node(P, P->nx - 1, y, z)] = pn[a * N + node(P, P->nx - 2, y, z)];
        }
}

int orc_step(const orc_params* P, double* h, double* g, double* f, double* phi_prev, int64_t nsteps) {
    if (check_params(P)) return -1;
    if (P->flow && !f) return -1;
    lattice S = scalar_lattice(P->dim);
    lattice V = flow_lattice(P->dim);
    long N = nnodes(P);
    scratch s;
    double* block = (double*)calloc((size_t)N * (9 + 2 * S.q + (P->flow ? V.q : 0)), sizeof(double));
    if (!block) return -1;
    s.phi = block;
    s.U = s.phi + N;
    s.rho = s.U + N;
    s.mx = s.rho + N;
    s.my = s.mx + N;
    s.mz = s.my + N;
    s.px = s.mz + N;
    s.py = s.px + N;
    s.pz = s.py + N;
    s.hn = s.pz + N;
    s.gn = s.hn + (long)S.q * N;
    s.fn = P->flow ? s.gn + (long)S.q * N : NULL;

    for (int64_t n = 0; n < nsteps; n++) {
        if (P->wall) { /* wall nodes are never written: they keep their values */
            memcpy(s.hn, h, sizeof(double) * S.q * N);
            memcpy(s.gn, g, sizeof(double) * S.q * N);
            if (P->flow) memcpy(s.fn, f, sizeof(double) * V.q * N);
        }
        moments(P, h, g, f, &s);
        gradient(P, &s);
        collide_stream(P, h, g, f, phi_prev, &s);
        if (P->xbc != 0) {
            outlet_fill(P, &S, s.hn);
            outlet_fill(P, &S, s.gn);
            if (P->flow && P->xbc == 1) outlet_fill(P, &V, s.fn);
        }
        memcpy(h, s.hn, sizeof(double) * S.q * N);
        memcpy(g, s.gn, sizeof(double) * S.q * N);
        if (P->flow) memcpy(f, s.fn, sizeof(double) * V.q * N);
        memcpy(phi_prev, s.phi, sizeof(double) * N);
    }
    free(block);
    return 0;
}

int orc_fields(const orc_params* P, const double* h, const double* g, const double* f, double* phi,
               double* U, double* rho, double* ux, double* uy, double* uz) {
    if (check_params(P)) return -1;
    lattice S = scalar_lattice(P->dim);
    lattice V = flow_lattice(P->dim);
    long N = nnodes(P);
    double tau_f = P->nu / V.cs2 + 0.5;
    for (long i = 0; i < N; i++) {
        double ph = 0.0, Uv = 0.0;
        for (int a = 0; a < S.q; a++) {
            ph += h[a * N + i];
            Uv += g[a * N + i];
        }
        double r = 1.0, us[3] = {0.0, 0.0, 0.0};
        if (P->flow) {
            double m[3] = {0.0, 0.0, 0.0};
            r = 0.0;
            for (int a = 0; a < V.q; a++) {
                r += f[a * N + i];
                for (int d = 0; d < 3; d++) m[d] += V.c[a][d] * f[a * N + i];
            }
            double u[3], F[3];
            flow_velocity(P, tau_f, ph, r, m, u, F, us);
        }
        if (phi) phi[i] = ph;
        if (U) U[i] = Uv;
        if (rho) rho[i] = r;
        if (ux) ux[i] = us[0];
        if (uy) uy[i] = us[1];
        if (uz) uz[i] = us[2];
    }
    return 0;
}

/* ------------------------------------------------------------------------------------------ */
/* Diagnostics (Section 4.1.2 crystal size; R7, R8, R25)                                       */
/* ------------------------------------------------------------------------------------------ */

/* Tri/bilinear interpolation of the nodal phi at a point inside [0, n-1] on every axis. */
static double interp(const orc_params* P, const double* phi, const double* pt) {
    int i0[3], i1[3];
    double t[3];
    int n[3] = {P->nx, P->ny, P->nz};
    for (int d = 0; d < 3; d++) {
        double fl = floor(pt[d]);
        i0[d] = (int)fl;
        t[d] = pt[d] - fl;
        if (i0[d] > n[d] - 1) i0[d] = n[d] - 1;
        i1[d] = i0[d] + 1 < n[d] ? i0[d] + 1 : n[d] - 1;
    }
    double v = 0.0;
    for (int cz = 0; cz < 2; cz++)
        for (int cy = 0; cy < 2; cy++)
            for (int cx = 0; cx < 2; cx++) {
                double wgt = (cx ? t[0] : 1 - t[0]) * (cy ? t[1] : 1 - t[1]) * (cz ? t[2] : 1 - t[2]);
                if (wgt == 0.0) continue;
                v += wgt * phi[node(P, cx ? i1[0] : i0[0], cy ? i1[1] : i0[1], cz ? i1[2] : i0[2])];
            }
    return v;
}

static int inside(const orc_params* P, const double* pt) {
    int n[3] = {P->nx, P->ny, P->nz};
    for (int d = 0; d < 3; d++)
        if (pt[d] < 0.0 || pt[d] > n[d] - 1) return 0;
    return 1;
}

/* March from the seed centre along each direction with step 1/4 and return the distance of the
 * first phi = 0 crossing (phi_j > 0 >= phi_{j+1}), linearly interpolated between the two samples;
 * 0 if phi <= 0 at the centre, and the last inside sample distance if no crossing is found. */
int orc_raymarch(const orc_params* P, const double* phi, int ndirs, const double* dirs, double* L_out) {
    const double ds = 0.25;
    for (int k = 0; k < ndirs; k++) {
        const double* dv = dirs + 3 * k;
        double c[3] = {P->seed_c[0], P->seed_c[1], P->dim == 3 ? P->seed_c[2] : 0.0};
        double prev = interp(P, phi, c);
        double L = 0.0;
        if (prev > 0.0) {
            double sj = 0.0;
            for (int j = 0;; j++) {
                double s1 = (j + 1) * ds;
                double pt[3] = {c[0] + s1 * dv[0], c[1] + s1 * dv[1], c[2] + s1 * dv[2]};
                if (!inside(P, pt)) {
                    L = sj;
                    break;
                }
                double cur = interp(P, phi, pt);
                if (prev > 0.0 && cur <= 0.0) {
                    L = sj + ds * prev / (prev - cur);
                    break;
                }
                prev = cur;
                sj = s1;
            }
        }
        L_out[k] = L;
    }
    return 0;
}

int orc_measure(const orc_params* P, const double* h, const double* g, const double* f,
                const double* phi_prev, int ndirs, const double* dirs, double* L_out, double* mass_out) {
    if (check_params(P)) return -1;
    long N = nnodes(P);
    double* fld = (double*)malloc(sizeof(double) * 6 * N);
    if (!fld) return -1;
    double *phi = fld, *U = fld + N, *rho = fld + 2 * N, *ux = fld + 3 * N, *uy = fld + 4 * N,
           *uz = fld + 5 * N;
    orc_fields(P, h, g, f, phi, U, rho, ux, uy, uz);
    if (mass_out) {
        double sU = 0.0, sP = 0.0, Vs = 0.0, Mp = 0.0, umax = 0.0, bad = 0.0;
        for (long i = 0; i < N; i++) {
            if (is_wall(P, i)) continue; /* diagnostics cover the fluid and the crystal (R28) */
            sU += U[i];
            sP += phi_prev[i];
            Vs += 0.5 * (1.0 + phi[i]);
            Mp += U[i] + (P->solute_source == 1 ? 0.5 : 1.0) * (1.0 + phi_prev[i]);
            double um = sqrt(ux[i] * ux[i] + uy[i] * uy[i] + uz[i] * uz[i]);
            if (um > umax) umax = um;
            if (!isfinite(phi[i]) || !isfinite(U[i]) || !isfinite(rho[i])) bad += 1.0;
        }
        mass_out[0] = sU;
        mass_out[1] = sP;
        mass_out[2] = Vs;
        mass_out[3] = Mp;
        mass_out[4] = umax;
        mass_out[5] = bad;
    }
    if (L_out && ndirs > 0) orc_raymarch(P, phi, ndirs, dirs, L_out);
    free(fld);
    return 0;
}
