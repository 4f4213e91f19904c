/*
 * mclbm_oracle.c -- plain FP64 CPU oracle for the two-component lattice
 * Boltzmann step of Datadien, Di Staso, Wijshoff and Toschi (arXiv:2110.05197).
 *
 * THIS IS TEST INFRASTRUCTURE, NOT PART OF THE PRODUCT.  Only the tests, the
 * smoke check of the package entry point and the CPU-baseline leg of the
 * benchmark may build, load or call it.  It shares no code, header, table or
 * helper with the HIP library: every lattice constant below is written out
 * here again, from the paper's equations.
 *
 * It is written to be read against the paper, not to be fast: every step of a
 * time step is its own pass over the whole lattice, in the order the paper
 * applies them, on plain double arrays.  OpenMP only splits the node loops
 * over threads; every node's arithmetic is independent of the thread count.
 *
 * Layout shared with the caller (an interface, not code):
 *   node index  n = x + nx*(y + ny*z)            (x fastest)
 *   populations f[(k*Q + i)*N + n]               (k = 0 red / 1 blue)
 *   vectors     v[d*N + n]                        (d = 0,1,2 = x,y,z)
 * Velocity ordering (both lattices): 0 = rest, then opposite pairs
 * (1,2), (3,4), ...: the axis directions first, then the diagonals.
 *
 * Readings of passages where the paper is silent or garbled carry the tag
 * "reading:" and are listed, with their reasons, in the design notes.
 *
 * Every function here is pinned by a CPU test against something other than
 * this file: printed constants, moment identities, closed-form decay rates
 * (including the blended viscosity of Eq. interpVisc), the Laplace law,
 * coexistence densities, the two-component Shan-Chen step's exact relaxation
 * of uniform component momenta and its one-step response to a sinusoidal
 * density, the repulsion force's closed form on planar films, exact
 * multirange forces on quadratic pseudopotentials, invariants.  What no pin
 * can fix is physical calibration the paper leaves open: the repulsion
 * magnitude and range (Pi and chi are free parameters), and the surface
 * tension of the printed multirange couplings, which do not phase-separate
 * under the printed equations.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#ifdef _OPENMP
#include <omp.h>
#endif

/* ------------------------------------------------------------------------ */
/* Parameters (the caller fills this struct through ctypes).                */
/* ------------------------------------------------------------------------ */
typedef struct {
    int32_t lattice;   /* 0 = D2Q9, 1 = D3Q19                               */
    int32_t model;     /* 0 = colour gradient, 1 = SC multiphase, 2 = SC two-component */
    int32_t nx, ny, nz;
    int32_t bc[3];     /* per axis: 0 periodic, 1 wall, 2 outflow           */
    int32_t enhanced_eq; /* 1: Leclaire's enhanced equilibrium (default)    */
    int32_t pad_;
    double rho0_R, rho0_B; /* initial bulk densities of red and blue        */
    double tau_R, tau_B;   /* relaxation times                              */
    double A;              /* perturbation (surface tension) parameter      */
    double beta;           /* recolouring parameter                          */
    double alpha_B;        /* rest fraction of the blue fluid               */
    double g_min;          /* |grad rho^N| below which the interface terms are dropped */
    double G;              /* SC multiphase coupling                        */
    double psi_rho0;       /* SC multiphase reference density rho_0        */
    double G_RB;           /* SC cross-component coupling                   */
    double rho0_X;         /* reference density in the SC cross force       */
    double Pi;             /* CG repulsion magnitude (0 = off)              */
    double chi;            /* CG repulsion exponent                          */
    double Ga_R, Ga_B;     /* SC two-component attraction couplings (belt 1)  */
    double Gr_R, Gr_B;     /* SC two-component repulsion couplings (belts 1+2) */
} orc_params;

/* ------------------------------------------------------------------------ */
/* Lattices.                                                                 */
/* ------------------------------------------------------------------------ */
typedef struct {
    int D, Q;
    int c[19][3];
    double w[19];   /* lattice weights                                      */
    double B[19];   /* perturbation constants B_i                           */
    double ps[19];  /* enhanced-equilibrium constants psi_i                 */
    double xi[19];  /* enhanced-equilibrium constants xi_i                  */
    double phi_a[19]; /* phi_i(alpha) = phi_a[i]*alpha + phi_b[i]           */
    double phi_b[19];
} orc_lattice;

/* D3Q19: velocities (Eq. speeds) and weights (Eq. weights); B_i from the
 * perturbation section, psi_i and xi_i from the enhanced-equilibrium
 * section, phi_i^k from Eq. phi: alpha for the rest population,
 * (1-alpha)/12 on the axes and (1-alpha)/24 on the diagonals. */
static void lattice_d3q19(orc_lattice *L)
{
    static const int c[19][3] = {
        {0, 0, 0},
        {1, 0, 0}, {-1, 0, 0}, {0, 1, 0}, {0, -1, 0}, {0, 0, 1}, {0, 0, -1},
        {1, 1, 0}, {-1, -1, 0}, {1, -1, 0}, {-1, 1, 0},
        {1, 0, 1}, {-1, 0, -1}, {1, 0, -1}, {-1, 0, 1},
        {0, 1, 1}, {0, -1, -1}, {0, 1, -1}, {0, -1, 1}};
    L->D = 3;
    L->Q = 19;
    for (int i = 0; i < 19; ++i) {
        for (int d = 0; d < 3; ++d) L->c[i][d] = c[i][d];
        int c2 = c[i][0] * c[i][0] + c[i][1] * c[i][1] + c[i][2] * c[i][2];
        if (c2 == 0) {
            L->w[i] = 1.0 / 3.0;  L->B[i] = -2.0 / 9.0;
            L->ps[i] = -5.0 / 2.0; L->xi[i] = 0.0;
            L->phi_a[i] = 1.0;    L->phi_b[i] = 0.0;
        } else if (c2 == 1) {
            L->w[i] = 1.0 / 18.0; L->B[i] = 1.0 / 54.0;
            L->ps[i] = -1.0 / 6.0; L->xi[i] = 1.0 / 4.0;
            L->phi_a[i] = -1.0 / 12.0; L->phi_b[i] = 1.0 / 12.0;
        } else {
            L->w[i] = 1.0 / 36.0; L->B[i] = 1.0 / 27.0;
            L->ps[i] = 1.0 / 24.0; L->xi[i] = 1.0 / 8.0;
            L->phi_a[i] = -1.0 / 24.0; L->phi_b[i] = 1.0 / 24.0;
        }
    }
}

/* D2Q9: the paper is D3Q19 only.  reading: the D2Q9 constants obey the same
 * moment conditions the D3Q19 ones do (sum phi = 1, sum B = 1/3,
 * sum B c c = delta/3, sum psi = -3, sum psi c c = 0, sum xi c c = 3/2 delta,
 * sum xi c^4 isotropic with weight 1/2), which fixes
 *   phi: rest alpha, axes (1-alpha)/5, diagonals (1-alpha)/20;
 *   B:   -4/27, 2/27, 5/108;   psi: -8/3, -1/6, 1/12;   xi: 0, 1/2, 1/8. */
static void lattice_d2q9(orc_lattice *L)
{
    static const int c[9][3] = {
        {0, 0, 0}, {1, 0, 0}, {-1, 0, 0}, {0, 1, 0}, {0, -1, 0},
        {1, 1, 0}, {-1, -1, 0}, {1, -1, 0}, {-1, 1, 0}};
    L->D = 2;
    L->Q = 9;
    for (int i = 0; i < 9; ++i) {
        for (int d = 0; d < 3; ++d) L->c[i][d] = c[i][d];
        int c2 = c[i][0] * c[i][0] + c[i][1] * c[i][1];
        if (c2 == 0) {
            L->w[i] = 4.0 / 9.0;  L->B[i] = -4.0 / 27.0;
            L->ps[i] = -8.0 / 3.0; L->xi[i] = 0.0;
            L->phi_a[i] = 1.0;    L->phi_b[i] = 0.0;
        } else if (c2 == 1) {
            L->w[i] = 1.0 / 9.0;  L->B[i] = 2.0 / 27.0;
            L->ps[i] = -1.0 / 6.0; L->xi[i] = 1.0 / 2.0;
            L->phi_a[i] = -1.0 / 5.0; L->phi_b[i] = 1.0 / 5.0;
        } else {
            L->w[i] = 1.0 / 36.0; L->B[i] = 5.0 / 108.0;
            L->ps[i] = 1.0 / 12.0; L->xi[i] = 1.0 / 8.0;
            L->phi_a[i] = -1.0 / 20.0; L->phi_b[i] = 1.0 / 20.0;
        }
    }
}

static void get_lattice(int lattice, orc_lattice *L)
{
    if (lattice == 0) lattice_d2q9(L); else lattice_d3q19(L);
}

static double phi_of(const orc_lattice *L, int i, double alpha)
{
    return L->phi_a[i] * alpha + L->phi_b[i];
}

/* Density ratio through the rest fractions (Eq. gamma):
 * rho_R^0 / rho_B^0 = (1 - alpha_B) / (1 - alpha_R). */
static double alpha_red(const orc_params *p)
{
    return 1.0 - (1.0 - p->alpha_B) * p->rho0_B / p->rho0_R;
}

/* ------------------------------------------------------------------------ */
/* Grid helpers.                                                             */
/* ------------------------------------------------------------------------ */
static int64_t nnodes(const orc_params *p) { return (int64_t)p->nx * p->ny * p->nz; }

static int64_t idx(const orc_params *p, int x, int y, int z)
{
    return (int64_t)x + (int64_t)p->nx * ((int64_t)y + (int64_t)p->ny * z);
}

static void coords(const orc_params *p, int64_t n, int *x, int *y, int *z)
{
    *x = (int)(n % p->nx);
    *y = (int)((n / p->nx) % p->ny);
    *z = (int)(n / ((int64_t)p->nx * p->ny));
}

/* Node that a stencil reads at x + c.  Periodic axes wrap; reading: on wall
 * and outflow axes the node outside the box takes the value of the nearest
 * fluid node (zero normal gradient, neutral wetting). */
static int64_t stencil_node(const orc_params *p, int x, int y, int z,
                            int cx, int cy, int cz)
{
    int q[3] = {x + cx, y + cy, z + cz};
    const int n[3] = {p->nx, p->ny, p->nz};
    for (int d = 0; d < 3; ++d) {
        if (q[d] < 0 || q[d] >= n[d]) {
            if (p->bc[d] == 0) q[d] = (q[d] % n[d] + n[d]) % n[d];
            else q[d] = q[d] < 0 ? 0 : n[d] - 1;
        }
    }
    return idx(p, q[0], q[1], q[2]);
}

/* Isotropic gradient.  reading: the paper names no stencil for grad rho^N and
 * grad rho_k; this uses the same w_i-weighted nearest-neighbour sum as the
 * Shan-Chen force (Eq. interactionforceMP):
 *   grad X(x) = (1/c_s^2) sum_{i != 0} w_i X(x + c_i) c_i,  c_s^2 = 1/3,
 * summed in ascending i. */
static void gradient_at(const orc_params *p, const orc_lattice *L,
                        const double *X, int x, int y, int z, double g[3])
{
    g[0] = g[1] = g[2] = 0.0;
    for (int i = 1; i < L->Q; ++i) {
        double v = X[stencil_node(p, x, y, z, L->c[i][0], L->c[i][1], L->c[i][2])];
        for (int d = 0; d < 3; ++d) g[d] += L->w[i] * v * L->c[i][d];
    }
    for (int d = 0; d < 3; ++d) g[d] *= 3.0;
}

static void gradient_pass(const orc_params *p, const orc_lattice *L,
                          const double *X, double *grad)
{
    const int64_t N = nnodes(p);
#pragma omp parallel for schedule(static)
    for (int64_t n = 0; n < N; ++n) {
        int x, y, z;
        double g[3];
        coords(p, n, &x, &y, &z);
        gradient_at(p, L, X, x, y, z, g);
        for (int d = 0; d < 3; ++d) grad[d * N + n] = g[d];
    }
}

static int ncomp(const orc_params *p) { return p->model == 1 ? 1 : 2; }

/* ------------------------------------------------------------------------ */
/* Moments (Eqs. density, totalDensity, totalMomentum2; Eqs. densitySC,      */
/* totalMomentum for the single-component model).                            */
/* ------------------------------------------------------------------------ */
static void moments_pass(const orc_params *p, const orc_lattice *L, const double *f,
                         double *rhoR, double *rhoB, double *j)
{
    const int64_t N = nnodes(p);
    const int K = ncomp(p);
#pragma omp parallel for schedule(static)
    for (int64_t n = 0; n < N; ++n) {
        double rk[2] = {0.0, 0.0};
        double m[3] = {0.0, 0.0, 0.0};
        for (int k = 0; k < K; ++k)
            for (int i = 0; i < L->Q; ++i) {
                double v = f[((int64_t)k * L->Q + i) * N + n];
                rk[k] += v;
                for (int d = 0; d < 3; ++d) m[d] += v * L->c[i][d];
            }
        rhoR[n] = rk[0];
        rhoB[n] = rk[1];
        for (int d = 0; d < 3; ++d) j[d * N + n] = m[d];
    }
}

/* ------------------------------------------------------------------------ */
/* CG equilibrium of one colour (Eq. equiliCG with Eq. phi and Eq. tensorG). */
/* G_k : c_i c_i = 2 (c_i . u)(c_i . grad rho_k).                             */
/* reading: phi_i^k is kept in the BGK equilibrium as well; with phi = 0 the  */
/* equilibrium would carry no mass.                                           */
/* ------------------------------------------------------------------------ */
static double cg_equilibrium(const orc_lattice *L, int i, double rho_k, double alpha_k,
                             const double u[3], const double grad_k[3], double nubar,
                             int enhanced)
{
    double cu = 0.0, uu = 0.0, ug = 0.0, cg = 0.0;
    for (int d = 0; d < 3; ++d) {
        cu += L->c[i][d] * u[d];
        uu += u[d] * u[d];
        ug += u[d] * grad_k[d];
        cg += L->c[i][d] * grad_k[d];
    }
    double feq = rho_k * (phi_of(L, i, alpha_k)
                          + L->w[i] * (3.0 * cu + 4.5 * cu * cu - 1.5 * uu));
    if (enhanced) feq += nubar * (L->ps[i] * ug + L->xi[i] * 2.0 * cu * cg);
    return feq;
}

/* Interface viscosity (Eq. interpVisc) with nu_k = (tau_k - 1/2)/3. */
static double interface_nu(const orc_params *p, double rR, double rB)
{
    double nuR = (p->tau_R - 0.5) / 3.0, nuB = (p->tau_B - 0.5) / 3.0;
    double r = rR + rB;
    return 1.0 / ((rR / r) / nuR + (rB / r) / nuB);
}

/* Standard equilibrium (Eq. equiliSC). */
static double std_equilibrium(const orc_lattice *L, int i, double rho, const double u[3])
{
    double cu = 0.0, uu = 0.0;
    for (int d = 0; d < 3; ++d) {
        cu += L->c[i][d] * u[d];
        uu += u[d] * u[d];
    }
    return rho * L->w[i] * (1.0 + 3.0 * cu + 4.5 * cu * cu - 1.5 * uu);
}

/* Guo source term (Eq. source) with c_s^2 = 1/3 and relaxation rate om. */
static double guo_source(const orc_lattice *L, int i, double om, const double u[3],
                         const double F[3])
{
    double cu = 0.0, cF = 0.0, cmuF = 0.0;
    for (int d = 0; d < 3; ++d) {
        cu += L->c[i][d] * u[d];
        cF += L->c[i][d] * F[d];
        cmuF += (L->c[i][d] - u[d]) * F[d];
    }
    return L->w[i] * (1.0 - 0.5 * om) * (3.0 * cmuF + 9.0 * cu * cF);
}

/* ------------------------------------------------------------------------ */
/* CG repulsion force (Eq. repForce, Eqs. normal1/normal2).                   */
/* reading: psi_rep = (1 - |rho^N|)^chi so that the force vanishes in the     */
/* bulk and grows as two interfaces approach; a normal is zero where          */
/* |grad rho^N| <= g_min; H(0) = 0.  Direction: the text of section 2.3 sets  */
/* an outward (repulsive) force on the nodes around an extremum of rho^N,     */
/* while the printed sum, with n'_i taken at x + c_i, points from each such   */
/* node toward the extremum; the force is applied outward, as minus that sum. */
/* ------------------------------------------------------------------------ */
static void repulsion_pass(const orc_params *p, const orc_lattice *L, const double *rhoN,
                           const double *gradN, double *F)
{
    const int64_t N = nnodes(p);
#pragma omp parallel for schedule(static)
    for (int64_t n = 0; n < N; ++n) {
        int x, y, z;
        coords(p, n, &x, &y, &z);
        double nv[3] = {gradN[n], gradN[N + n], gradN[2 * N + n]};
        double g = sqrt(nv[0] * nv[0] + nv[1] * nv[1] + nv[2] * nv[2]);
        for (int d = 0; d < 3; ++d) nv[d] = g > p->g_min ? nv[d] / g : 0.0;
        double acc[3] = {0.0, 0.0, 0.0};
        for (int i = 1; i < L->Q; ++i) {
            int64_t m = stencil_node(p, x, y, z, L->c[i][0], L->c[i][1], L->c[i][2]);
            double np[3] = {gradN[m], gradN[N + m], gradN[2 * N + m]};
            double gp = sqrt(np[0] * np[0] + np[1] * np[1] + np[2] * np[2]);
            for (int d = 0; d < 3; ++d) np[d] = gp > p->g_min ? np[d] / gp : 0.0;
            double nc = 0.0, npc = 0.0, cc = 0.0;
            for (int d = 0; d < 3; ++d) {
                nc += nv[d] * L->c[i][d];
                npc += np[d] * L->c[i][d];
                cc += (double)(L->c[i][d] * L->c[i][d]);
            }
            if (-(nc * npc) > 0.0) {
                double inv = 1.0 / sqrt(cc);
                for (int d = 0; d < 3; ++d) acc[d] += (nc * nv[d] + npc * np[d]) * inv;
            }
        }
        double psi_rep = pow(1.0 - fabs(rhoN[n]), p->chi);
        for (int d = 0; d < 3; ++d) F[d * N + n] = -p->Pi * psi_rep * acc[d];
    }
}

/* ------------------------------------------------------------------------ */
/* Scratch for one step.                                                      */
/* ------------------------------------------------------------------------ */
typedef struct {
    double *rhoR, *rhoB, *rhoN, *j, *gN, *gR, *gB, *F, *fpost;
} orc_work;

static int work_alloc(const orc_params *p, const orc_lattice *L, orc_work *w)
{
    const int64_t N = nnodes(p);
    memset(w, 0, sizeof(*w));
    w->rhoR = calloc((size_t)N, sizeof(double));
    w->rhoB = calloc((size_t)N, sizeof(double));
    w->rhoN = calloc((size_t)N, sizeof(double));
    w->j = calloc((size_t)(3 * N), sizeof(double));
    w->gN = calloc((size_t)(3 * N), sizeof(double));
    w->gR = calloc((size_t)(3 * N), sizeof(double));
    w->gB = calloc((size_t)(3 * N), sizeof(double));
    w->F = calloc((size_t)(3 * N), sizeof(double));
    w->fpost = calloc((size_t)(ncomp(p) * L->Q * N), sizeof(double));
    return (w->rhoR && w->rhoB && w->rhoN && w->j && w->gN && w->gR && w->gB && w->F
            && w->fpost) ? 0 : -1;
}

static void work_free(orc_work *w)
{
    free(w->rhoR); free(w->rhoB); free(w->rhoN); free(w->j);
    free(w->gN); free(w->gR); free(w->gB); free(w->F); free(w->fpost);
}

/* ------------------------------------------------------------------------ */
/* Collision passes: each writes the post-collision populations f^{***}.    */
/* ------------------------------------------------------------------------ */

/* Colour gradient: BGK with the enhanced equilibrium (Eq. BGK), the
 * perturbation (Eq. perturbationOp) and the recolouring (Eqs. recoloringOpR,
 * recoloringOpB, cosphi), applied in that order (Eq. threeops).
 *
 * reading of Eq. perturbationOp (printed garbled): each colour receives
 *   (A/2) |grad rho^N| [ w_i (c_i . n)^2 - B_i ],  n = grad rho^N / |grad rho^N|,
 * so the total distribution receives A |grad rho^N| [...]; this is the scale
 * for which Eq. sigmaA, sigma = 4A/(9 omega_eff), holds.
 * reading: both colours relax with omega_eff (Eq. effRelax) of the local
 * interface viscosity; f^eq|_{u=0} in the recolouring is sum_k rho_k phi_i^k;
 * cos(phi_0) = 0; the perturbation and recolouring terms are dropped where
 * |grad rho^N| <= g_min (no defined normal there). */
static void cg_collide_pass(const orc_params *p, const orc_lattice *L, const double *f,
                            orc_work *w, int with_force)
{
    const int64_t N = nnodes(p);
    const int Q = L->Q;
    const double aR = alpha_red(p), aB = p->alpha_B;
#pragma omp parallel for schedule(static)
    for (int64_t n = 0; n < N; ++n) {
        double rR = w->rhoR[n], rB = w->rhoB[n], r = rR + rB;
        double F[3] = {0.0, 0.0, 0.0};
        if (with_force)
            for (int d = 0; d < 3; ++d) F[d] = w->F[d * N + n];
        double u[3];
        for (int d = 0; d < 3; ++d) u[d] = (w->j[d * N + n] + 0.5 * F[d]) / r;
        double gR[3], gB[3], gN[3];
        for (int d = 0; d < 3; ++d) {
            gR[d] = w->gR[d * N + n];
            gB[d] = w->gB[d * N + n];
            gN[d] = w->gN[d * N + n];
        }
        double nubar = interface_nu(p, rR, rB);
        double om = 2.0 / (6.0 * nubar + 1.0);
        double g = sqrt(gN[0] * gN[0] + gN[1] * gN[1] + gN[2] * gN[2]);
        int has_n = g > p->g_min;
        double nv[3] = {0.0, 0.0, 0.0};
        if (has_n)
            for (int d = 0; d < 3; ++d) nv[d] = gN[d] / g;

        for (int i = 0; i < Q; ++i) {
            double fs[2];
            for (int k = 0; k < 2; ++k) {
                double rk = k == 0 ? rR : rB;
                double ak = k == 0 ? aR : aB;
                const double *gk = k == 0 ? gR : gB;
                double fk = f[((int64_t)k * Q + i) * N + n];
                double feq = cg_equilibrium(L, i, rk, ak, u, gk, nubar, p->enhanced_eq);
                double v = fk - om * (fk - feq);                       /* Omega^(1) */
                if (with_force) v += (rk / r) * guo_source(L, i, om, u, F);
                if (has_n) {                                            /* Omega^(2) */
                    double cn = 0.0;
                    for (int d = 0; d < 3; ++d) cn += L->c[i][d] * nv[d];
                    v += 0.5 * p->A * g * (L->w[i] * cn * cn - L->B[i]);
                }
                fs[k] = v;
            }
            /* Omega^(3): recolouring of the total f* = f*_R + f*_B. */
            double ft = fs[0] + fs[1];
            double e0 = rR * phi_of(L, i, aR) + rB * phi_of(L, i, aB);
            double cosphi = 0.0;
            if (i > 0 && has_n) {
                double cn = 0.0, cc = 0.0;
                for (int d = 0; d < 3; ++d) {
                    cn += L->c[i][d] * nv[d];
                    cc += (double)(L->c[i][d] * L->c[i][d]);
                }
                cosphi = cn / sqrt(cc);
            }
            double t = p->beta * (rR * rB / (r * r)) * cosphi * e0;
            w->fpost[(int64_t)i * N + n] = (rR / r) * ft + t;
            w->fpost[((int64_t)Q + i) * N + n] = (rB / r) * ft - t;
        }
    }
}

/* Pseudopotential psi(rho) = rho_0 (1 - exp(-rho/rho_0)) (Eq. pseudopotential). */
static void psi_pass(const orc_params *p, const double *rho, double *psi, int64_t N)
{
#pragma omp parallel for schedule(static)
    for (int64_t n = 0; n < N; ++n) psi[n] = p->psi_rho0 * (1.0 - exp(-rho[n] / p->psi_rho0));
}

/* Shan-Chen force F = -G psi(x) sum_i w_i psi(x + c_i) c_i (Eq. interactionforceMP). */
static void scmp_force_at(const orc_params *p, const orc_lattice *L, const double *psi,
                          int64_t n, double F[3])
{
    int x, y, z;
    coords(p, n, &x, &y, &z);
    double s[3] = {0.0, 0.0, 0.0};
    for (int i = 1; i < L->Q; ++i) {
        double ps = psi[stencil_node(p, x, y, z, L->c[i][0], L->c[i][1], L->c[i][2])];
        for (int d = 0; d < 3; ++d) s[d] += L->w[i] * ps * L->c[i][d];
    }
    for (int d = 0; d < 3; ++d) F[d] = -p->G * psi[n] * s[d];
}

/* The multirange neighbourhood of the two-component Shan-Chen forces
 * (Eq. pweights): the 92 vectors c in {-2..2}^3 with |c|^2 in {1, 2, 3, 4,
 * 5, 6, 8}; belt 1 is |c|^2 <= 2 (the D3Q19 set), belt 2 the rest.  Weights
 * by shell: p = 4/135, 1/63, 2/315, 5/1512, 1/945, 1/1890, 1/15120 for
 * |c|^2 = 1, 2, 3, 4, 5, 6, 8 (p = 0 for the rest vector); w is the D3Q19
 * lattice weight on belt 1 (1/18, 1/36) and 0 on belt 2.  Enumerated with x
 * fastest, then y, then z. */
typedef struct {
    int n;
    int c[92][3];
    double p[92], w[92];
} orc_belts;

static void belts(orc_belts *B)
{
    B->n = 0;
    for (int cz = -2; cz <= 2; ++cz)
        for (int cy = -2; cy <= 2; ++cy)
            for (int cx = -2; cx <= 2; ++cx) {
                const int r2 = cx * cx + cy * cy + cz * cz;
                double p = 0.0, w = 0.0;
                switch (r2) {
                case 1: p = 4.0 / 135.0; w = 1.0 / 18.0; break;
                case 2: p = 1.0 / 63.0; w = 1.0 / 36.0; break;
                case 3: p = 2.0 / 315.0; break;
                case 4: p = 5.0 / 1512.0; break;
                case 5: p = 1.0 / 945.0; break;
                case 6: p = 1.0 / 1890.0; break;
                case 8: p = 1.0 / 15120.0; break;
                default: continue;   /* rest vector, |c|^2 = 9, 12 */
                }
                B->c[B->n][0] = cx; B->c[B->n][1] = cy; B->c[B->n][2] = cz;
                B->p[B->n] = p;
                B->w[B->n] = w;
                ++B->n;
            }
}

static int multirange_on(const orc_params *p)
{
    return p->Ga_R != 0.0 || p->Ga_B != 0.0 || p->Gr_R != 0.0 || p->Gr_B != 0.0;
}

/* Forces on each colour of the two-component Shan-Chen model
 * (Eq. benziforces): the cross-component repulsion (Eq.
 * doublebeltrepulsionforce2, belt 1)
 *   F^X_s = -(G_RB / rho_0^2) rho_s(x) sum_i w_i rho_s'(x + c_i) c_i,
 * plus, when a multirange coupling is set, the attraction on belt 1 (Eq.
 * doublebeltattractiveforce) and the repulsion on belts 1 and 2 (Eq.
 * doublebeltrepulsionforce)
 *   F^a_s = -G^a_s psi_s(x) sum_{belt 1} w_i psi_s(x + c_i) c_i,
 *   F^r_s = -G^r_s psi_s(x) sum_{belts 1,2} p_i psi_s(x + c_i) c_i,
 * with psi_s = rho_0 (1 - exp(-rho_s / rho_0)) (Eq. pseudopotential; reading:
 * the same psi for both species, rho_0 = psi_rho0).  psiR/psiB may be NULL
 * when no multirange coupling is set. */
static void scmc_forces_at(const orc_params *p, const orc_lattice *L, const double *rhoR,
                           const double *rhoB, const double *psiR, const double *psiB,
                           int64_t n, double FR[3], double FB[3])
{
    int x, y, z;
    coords(p, n, &x, &y, &z);
    const double pref = p->G_RB / (p->rho0_X * p->rho0_X);
    double sR[3] = {0.0, 0.0, 0.0}, sB[3] = {0.0, 0.0, 0.0};
    for (int i = 1; i < L->Q; ++i) {
        int64_t m = stencil_node(p, x, y, z, L->c[i][0], L->c[i][1], L->c[i][2]);
        for (int d = 0; d < 3; ++d) {
            sR[d] += L->w[i] * rhoR[m] * L->c[i][d];
            sB[d] += L->w[i] * rhoB[m] * L->c[i][d];
        }
    }
    for (int d = 0; d < 3; ++d) {
        FR[d] = -pref * rhoR[n] * sB[d];
        FB[d] = -pref * rhoB[n] * sR[d];
    }
    if (!multirange_on(p)) return;
    orc_belts B;
    belts(&B);
    double aR[3] = {0, 0, 0}, aB[3] = {0, 0, 0}, rR[3] = {0, 0, 0}, rB[3] = {0, 0, 0};
    for (int b = 0; b < B.n; ++b) {
        int64_t m = stencil_node(p, x, y, z, B.c[b][0], B.c[b][1], B.c[b][2]);
        for (int d = 0; d < 3; ++d) {
            aR[d] += B.w[b] * psiR[m] * B.c[b][d];
            aB[d] += B.w[b] * psiB[m] * B.c[b][d];
            rR[d] += B.p[b] * psiR[m] * B.c[b][d];
            rB[d] += B.p[b] * psiB[m] * B.c[b][d];
        }
    }
    for (int d = 0; d < 3; ++d) {
        FR[d] += -p->Ga_R * psiR[n] * aR[d] - p->Gr_R * psiR[n] * rR[d];
        FB[d] += -p->Ga_B * psiB[n] * aB[d] - p->Gr_B * psiB[n] * rB[d];
    }
}

/* Shan-Chen multiphase: psi force (Eq. interactionforceMP, Eq. pseudopotential),
 * Guo forcing (Eqs. guoforce, source, guoforce2), BGK (Eq. collisSC). */
static void scmp_collide_pass(const orc_params *p, const orc_lattice *L, const double *f,
                              orc_work *w)
{
    const int64_t N = nnodes(p);
    const int Q = L->Q;
    psi_pass(p, w->rhoR, w->rhoN, N); /* psi field in the rhoN scratch */
    const double om = 1.0 / p->tau_R;
#pragma omp parallel for schedule(static)
    for (int64_t n = 0; n < N; ++n) {
        double F[3], u[3];
        scmp_force_at(p, L, w->rhoN, n, F);
        double rho = w->rhoR[n];
        for (int d = 0; d < 3; ++d) u[d] = (w->j[d * N + n] + 0.5 * F[d]) / rho;
        for (int i = 0; i < Q; ++i) {
            double fi = f[(int64_t)i * N + n];
            double feq = std_equilibrium(L, i, rho, u);
            w->fpost[(int64_t)i * N + n] = fi - om * (fi - feq) + guo_source(L, i, om, u, F);
        }
    }
}

/* Shan-Chen two-component with the cross-repulsion only
 * (Eq. doublebeltrepulsionforce2, belt 1 = nearest neighbours).
 * reading: one barycentric velocity u = (sum_s sum_i f^s c_i + sum_s F_s/2)/rho
 * enters both equilibria and both Guo sources, each with its own tau_s. */
static void scmc_collide_pass(const orc_params *p, const orc_lattice *L, const double *f,
                              orc_work *w)
{
    const int64_t N = nnodes(p);
    const int Q = L->Q;
    const double om[2] = {1.0 / p->tau_R, 1.0 / p->tau_B};
    /* psi of both species for the multirange forces (gR / gB scratch) */
    double *psiR = NULL, *psiB = NULL;
    if (multirange_on(p)) {
        psiR = w->gR;
        psiB = w->gB;
        psi_pass(p, w->rhoR, psiR, N);
        psi_pass(p, w->rhoB, psiB, N);
    }
#pragma omp parallel for schedule(static)
    for (int64_t n = 0; n < N; ++n) {
        double rk[2] = {w->rhoR[n], w->rhoB[n]};
        double Fk[2][3], u[3];
        scmc_forces_at(p, L, w->rhoR, w->rhoB, psiR, psiB, n, Fk[0], Fk[1]);
        for (int d = 0; d < 3; ++d)
            u[d] = (w->j[d * N + n] + 0.5 * (Fk[0][d] + Fk[1][d])) / (rk[0] + rk[1]);
        for (int k = 0; k < 2; ++k)
            for (int i = 0; i < Q; ++i) {
                double fi = f[((int64_t)k * Q + i) * N + n];
                double feq = std_equilibrium(L, i, rk[k], u);
                w->fpost[((int64_t)k * Q + i) * N + n] =
                    fi - om[k] * (fi - feq) + guo_source(L, i, om[k], u, Fk[k]);
            }
    }
}

/* ------------------------------------------------------------------------ */
/* Streaming (Eq. streaming), written as a pull: f_i(x, t+1) = f*_i(x - c_i).  */
/* reading (boundaries other than periodic are not in the paper):            */
/*   wall axis:    halfway bounce-back, f_i(x, t+1) = f*_{opp(i)}(x);         */
/*   outflow axis: the population entering from outside is copied from the   */
/*                 node one step inward along that axis (zero gradient).      */
/* A source outside through any wall axis bounces back; otherwise, outside   */
/* through outflow axes only, it is copied.                                   */
/* ------------------------------------------------------------------------ */
static int opposite(const orc_lattice *L, int i)
{
    for (int j = 0; j < L->Q; ++j)
        if (L->c[j][0] == -L->c[i][0] && L->c[j][1] == -L->c[i][1]
            && L->c[j][2] == -L->c[i][2])
            return j;
    return -1;
}

static double pull_one(const orc_params *p, const orc_lattice *L, const double *fpost,
                       int k, int i, int x, int y, int z, int depth)
{
    const int64_t N = nnodes(p);
    const int n[3] = {p->nx, p->ny, p->nz};
    int s[3] = {x - L->c[i][0], y - L->c[i][1], z - L->c[i][2]};
    int wall = 0, outflow = 0;
    int inward[3] = {0, 0, 0};
    int here[3] = {x, y, z};
    for (int d = 0; d < 3; ++d) {
        if (s[d] >= 0 && s[d] < n[d]) continue;
        if (p->bc[d] == 0) s[d] = (s[d] % n[d] + n[d]) % n[d];
        else if (p->bc[d] == 1) wall = 1;
        else { outflow = 1; inward[d] = here[d] == 0 ? 1 : -1; }
    }
    if (wall) {
        int o = opposite(L, i);
        return fpost[((int64_t)k * L->Q + o) * N + idx(p, x, y, z)];
    }
    if (outflow && depth == 0)
        return pull_one(p, L, fpost, k, i, x + inward[0], y + inward[1], z + inward[2], 1);
    return fpost[((int64_t)k * L->Q + i) * N + idx(p, s[0], s[1], s[2])];
}

static void stream_pass(const orc_params *p, const orc_lattice *L, const double *fpost,
                        double *fout)
{
    const int64_t N = nnodes(p);
    const int K = ncomp(p);
#pragma omp parallel for schedule(static)
    for (int64_t n = 0; n < N; ++n) {
        int x, y, z;
        coords(p, n, &x, &y, &z);
        for (int k = 0; k < K; ++k)
            for (int i = 0; i < L->Q; ++i)
                fout[((int64_t)k * L->Q + i) * N + n] = pull_one(p, L, fpost, k, i, x, y, z, 0);
    }
}

/* ------------------------------------------------------------------------ */
/* One full time step: moments -> gradients -> collision -> streaming.        */
/* ------------------------------------------------------------------------ */
static void fill_colour_field(const orc_params *p, orc_work *w)
{
    const int64_t N = nnodes(p);
#pragma omp parallel for schedule(static)
    for (int64_t n = 0; n < N; ++n)
        w->rhoN[n] = (w->rhoR[n] - w->rhoB[n]) / (w->rhoR[n] + w->rhoB[n]);
}

static void step_once(const orc_params *p, const orc_lattice *L, double *f, orc_work *w)
{
    moments_pass(p, L, f, w->rhoR, w->rhoB, w->j);
    if (p->model == 0) {
        fill_colour_field(p, w);
        gradient_pass(p, L, w->rhoN, w->gN);
        gradient_pass(p, L, w->rhoR, w->gR);
        gradient_pass(p, L, w->rhoB, w->gB);
        int with_force = p->Pi != 0.0;
        if (with_force) repulsion_pass(p, L, w->rhoN, w->gN, w->F);
        cg_collide_pass(p, L, f, w, with_force);
    } else if (p->model == 1) {
        scmp_collide_pass(p, L, f, w);
    } else {
        scmc_collide_pass(p, L, f, w);
    }
    stream_pass(p, L, w->fpost, f);
}

/* ======================================================================== */
/* Exported entry points (ctypes).                                           */
/* ======================================================================== */

/* Number of threads the node loops use. */
int orc_num_threads(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

void orc_set_num_threads(int n)
{
#ifdef _OPENMP
    if (n > 0) omp_set_num_threads(n);
#else
    (void)n;
#endif
}

/* Lattice tables: c (Q*3 ints), w, B, psi, xi, phi at the given alpha. */
int orc_lattice_tables(int lattice, double alpha, int32_t *c, double *w, double *B,
                       double *ps, double *xi, double *phi)
{
    orc_lattice L;
    get_lattice(lattice, &L);
    for (int i = 0; i < L.Q; ++i) {
        for (int d = 0; d < 3; ++d) c[i * 3 + d] = L.c[i][d];
        w[i] = L.w[i];
        B[i] = L.B[i];
        ps[i] = L.ps[i];
        xi[i] = L.xi[i];
        phi[i] = phi_of(&L, i, alpha);
    }
    return L.Q;
}

/* CG equilibrium of one colour at one node, for all i (for moment checks). */
void orc_cg_equilibrium(int lattice, double rho_k, double alpha_k, const double *u,
                        const double *grad_k, double nubar, int enhanced, double *feq)
{
    orc_lattice L;
    get_lattice(lattice, &L);
    for (int i = 0; i < L.Q; ++i)
        feq[i] = cg_equilibrium(&L, i, rho_k, alpha_k, u, grad_k, nubar, enhanced);
}

/* Gradient of a scalar field with the model's stencil and boundaries. */
void orc_gradient(const orc_params *p, const double *X, double *grad)
{
    orc_lattice L;
    get_lattice(p->lattice, &L);
    gradient_pass(p, &L, X, grad);
}

/* Moments of f: rho_R, rho_B (zero for the single-component model) and the
 * bare momentum j = sum_k sum_i f c_i. */
void orc_moments(const orc_params *p, const double *f, double *rhoR, double *rhoB, double *j)
{
    orc_lattice L;
    get_lattice(p->lattice, &L);
    moments_pass(p, &L, f, rhoR, rhoB, j);
}

/* Equilibrium initialisation from fields rho_R, rho_B, u (u may be NULL = 0).
 * reading: CG starts from its full equilibrium of the given fields (gradients
 * of the given densities, interface viscosity of the given densities); the SC
 * models start from the standard equilibrium.  For the multiphase model rho_R
 * is the density and rho_B is ignored. */
int orc_init_equilibrium(const orc_params *p, const double *rhoR, const double *rhoB,
                         const double *u, double *f)
{
    orc_lattice L;
    get_lattice(p->lattice, &L);
    const int64_t N = nnodes(p);
    const int Q = L.Q;
    double *gR = NULL, *gB = NULL;
    if (p->model == 0) {
        gR = calloc((size_t)(3 * N), sizeof(double));
        gB = calloc((size_t)(3 * N), sizeof(double));
        if (!gR || !gB) { free(gR); free(gB); return -1; }
        gradient_pass(p, &L, rhoR, gR);
        gradient_pass(p, &L, rhoB, gB);
    }
    const double aR = alpha_red(p);
#pragma omp parallel for schedule(static)
    for (int64_t n = 0; n < N; ++n) {
        double uu[3] = {0.0, 0.0, 0.0};
        if (u)
            for (int d = 0; d < 3; ++d) uu[d] = u[d * N + n];
        for (int i = 0; i < Q; ++i) {
            if (p->model == 0) {
                double g1[3] = {gR[n], gR[N + n], gR[2 * N + n]};
                double g2[3] = {gB[n], gB[N + n], gB[2 * N + n]};
                double nubar = interface_nu(p, rhoR[n], rhoB[n]);
                f[(int64_t)i * N + n] =
                    cg_equilibrium(&L, i, rhoR[n], aR, uu, g1, nubar, p->enhanced_eq);
                f[((int64_t)Q + i) * N + n] =
                    cg_equilibrium(&L, i, rhoB[n], p->alpha_B, uu, g2, nubar, p->enhanced_eq);
            } else if (p->model == 1) {
                f[(int64_t)i * N + n] = std_equilibrium(&L, i, rhoR[n], uu);
            } else {
                f[(int64_t)i * N + n] = std_equilibrium(&L, i, rhoR[n], uu);
                f[((int64_t)Q + i) * N + n] = std_equilibrium(&L, i, rhoB[n], uu);
            }
        }
    }
    free(gR);
    free(gB);
    return 0;
}

/* Post-collision populations f*** (no streaming) of state f, for checks of the
 * collision operator on its own. */
int orc_collide(const orc_params *p, const double *f, double *fpost)
{
    orc_lattice L;
    get_lattice(p->lattice, &L);
    orc_work w;
    if (work_alloc(p, &L, &w)) { work_free(&w); return -1; }
    moments_pass(p, &L, f, w.rhoR, w.rhoB, w.j);
    if (p->model == 0) {
        fill_colour_field(p, &w);
        gradient_pass(p, &L, w.rhoN, w.gN);
        gradient_pass(p, &L, w.rhoR, w.gR);
        gradient_pass(p, &L, w.rhoB, w.gB);
        int with_force = p->Pi != 0.0;
        if (with_force) repulsion_pass(p, &L, w.rhoN, w.gN, w.F);
        cg_collide_pass(p, &L, f, &w, with_force);
    } else if (p->model == 1) {
        scmp_collide_pass(p, &L, f, &w);
    } else {
        scmc_collide_pass(p, &L, f, &w);
    }
    memcpy(fpost, w.fpost, sizeof(double) * (size_t)(ncomp(p) * L.Q * nnodes(p)));
    work_free(&w);
    return 0;
}

/* Streaming alone. */
void orc_stream(const orc_params *p, const double *fpost, double *fout)
{
    orc_lattice L;
    get_lattice(p->lattice, &L);
    stream_pass(p, &L, fpost, fout);
}

/* CG repulsion force field of state f (Eq. repForce under the reading above). */
int orc_repulsion_force(const orc_params *p, const double *f, double *F)
{
    orc_lattice L;
    get_lattice(p->lattice, &L);
    orc_work w;
    if (work_alloc(p, &L, &w)) { work_free(&w); return -1; }
    moments_pass(p, &L, f, w.rhoR, w.rhoB, w.j);
    fill_colour_field(p, &w);
    gradient_pass(p, &L, w.rhoN, w.gN);
    repulsion_pass(p, &L, w.rhoN, w.gN, F);
    work_free(&w);
    return 0;
}

/* Advance f in place by nsteps time steps. */
int orc_run(const orc_params *p, double *f, int64_t nsteps)
{
    orc_lattice L;
    get_lattice(p->lattice, &L);
    orc_work w;
    if (work_alloc(p, &L, &w)) { work_free(&w); return -1; }
    for (int64_t s = 0; s < nsteps; ++s) step_once(p, &L, f, &w);
    work_free(&w);
    return 0;
}

/* ------------------------------------------------------------------------ */
/* Observables.  out[] receives, in order:                                   */
/*   0 mass_R   1 mass_B   2..4 momentum (sum of j)   5 E_kin = sum rho|u|^2/2 */
/*   6 max|u|   7 rho_in   8 rho_out   9 epsilon used   10 red volume          */
/*   11 nodes inside   12 nodes outside   13 diverged (0/1)                    */
/* The momentum sum is of the bare j; E_kin and max|u| use the fluid velocity */
/* u = (j + F/2) / rho, with F the Shan-Chen force for the SC models (Eq.      */
/* guoforce2) and F = 0 for the colour-gradient model.                         */
/* Laplace densities (Eqs. rhoin, rhoout): reading: epsilon is the largest     */
/* 1 - 0.1^n, n = 1..10, for which both {rho^N >= eps} and {rho^N <= -eps} are */
/* non-empty.  Red volume = sum (1 + rho^N)/2.  For the multiphase model       */
/* "inside" is rho >= (rho0_R + rho0_B)/2, rho_in/out are mean densities there */
/* and the red volume counts the inside nodes.                                 */
/* Divergence: any non-finite density or momentum, or rho <= 0 at any node.  */
/* ------------------------------------------------------------------------ */
void orc_observables(const orc_params *p, const double *f, double *out)
{
    orc_lattice L;
    get_lattice(p->lattice, &L);
    const int64_t N = nnodes(p);
    double *rR = calloc((size_t)N, sizeof(double));
    double *rB = calloc((size_t)N, sizeof(double));
    double *j = calloc((size_t)(3 * N), sizeof(double));
    double *psi = calloc((size_t)N, sizeof(double));
    double *psiB = calloc((size_t)N, sizeof(double));
    moments_pass(p, &L, f, rR, rB, j);
    if (p->model == 1 || (p->model == 2 && multirange_on(p))) psi_pass(p, rR, psi, N);
    if (p->model == 2 && multirange_on(p)) psi_pass(p, rB, psiB, N);
    double mR = 0, mB = 0, mom[3] = {0, 0, 0}, ek = 0, umax = 0, vol = 0;
    double sin_[10] = {0}, sout[10] = {0};
    double cin[10] = {0}, cout_[10] = {0};
    int diverged = 0;
    const double mid = 0.5 * (p->rho0_R + p->rho0_B);
    for (int64_t n = 0; n < N; ++n) {
        double r = rR[n] + rB[n];
        double jj[3] = {j[n], j[N + n], j[2 * N + n]};
        double F[3] = {0.0, 0.0, 0.0};
        if (p->model == 1) {
            scmp_force_at(p, &L, psi, n, F);
        } else if (p->model == 2) {
            double FR[3], FB[3];
            scmc_forces_at(p, &L, rR, rB, psi, psiB, n, FR, FB);
            for (int d = 0; d < 3; ++d) F[d] = FR[d] + FB[d];
        }
        double uu[3];
        for (int d = 0; d < 3; ++d) uu[d] = (jj[d] + 0.5 * F[d]) / r;
        if (!isfinite(r) || !isfinite(jj[0]) || !isfinite(jj[1]) || !isfinite(jj[2])
            || !(r > 0.0)) {
            diverged = 1;
            continue;
        }
        mR += rR[n];
        mB += rB[n];
        double u2 = 0.0;
        for (int d = 0; d < 3; ++d) {
            mom[d] += jj[d];
            u2 += uu[d] * uu[d];
        }
        ek += 0.5 * r * u2;
        if (sqrt(u2) > umax) umax = sqrt(u2);
        if (p->model == 1) {
            if (r >= mid) { vol += 1.0; sin_[0] += r; cin[0] += 1.0; }
            else { sout[0] += r; cout_[0] += 1.0; }
        } else {
            double rN = (rR[n] - rB[n]) / r;
            vol += 0.5 * (1.0 + rN);
            for (int m = 0; m < 10; ++m) {
                double eps = 1.0 - pow(0.1, m + 1);
                if (rN >= eps) { sin_[m] += rR[n]; cin[m] += 1.0; }
                if (rN <= -eps) { sout[m] += rB[n]; cout_[m] += 1.0; }
            }
        }
    }
    double rho_in = 0, rho_out = 0, eps_used = 0, nin = 0, nout = 0;
    if (p->model == 1) {
        nin = cin[0]; nout = cout_[0];
        rho_in = nin > 0 ? sin_[0] / nin : 0.0;
        rho_out = nout > 0 ? sout[0] / nout : 0.0;
    } else {
        for (int m = 9; m >= 0; --m) {
            if (cin[m] > 0 && cout_[m] > 0) {
                nin = cin[m]; nout = cout_[m];
                rho_in = sin_[m] / nin;
                rho_out = sout[m] / nout;
                eps_used = 1.0 - pow(0.1, m + 1);
                break;
            }
        }
    }
    out[0] = mR; out[1] = mB; out[2] = mom[0]; out[3] = mom[1]; out[4] = mom[2];
    out[5] = ek; out[6] = umax; out[7] = rho_in; out[8] = rho_out; out[9] = eps_used;
    out[10] = vol; out[11] = nin; out[12] = nout; out[13] = diverged;
    free(rR); free(rB); free(j); free(psi); free(psiB);
}

/* ------------------------------------------------------------------------ */
/* Interface observables (the measurement procedures of the oscillation,     */
/* ligament, coalescence and emulsion studies).                              */
/*                                                                           */
/* Phase indicator per node: phi = rho^N = (rho_R - rho_B)/rho for the two-  */
/* component models, phi = rho - (rho0_R + rho0_B)/2 for SC multiphase (the  */
/* interface definitions of the droplet-oscillation section); a node is      */
/* inside the red (liquid) phase when phi > 0.                               */
/* ------------------------------------------------------------------------ */
void orc_phase_indicator(const orc_params *p, const double *f, double *phi)
{
    orc_lattice L;
    get_lattice(p->lattice, &L);
    const int64_t N = nnodes(p);
    double *rR = calloc((size_t)N, sizeof(double));
    double *rB = calloc((size_t)N, sizeof(double));
    double *j = calloc((size_t)(3 * N), sizeof(double));
    moments_pass(p, &L, f, rR, rB, j);
    const double mid = 0.5 * (p->rho0_R + p->rho0_B);
    for (int64_t n = 0; n < N; ++n) {
        if (p->model == 1) phi[n] = rR[n] - mid;
        else phi[n] = (rR[n] - rB[n]) / (rR[n] + rB[n]);
    }
    free(rR); free(rB); free(j);
}

/* Line along `axis` through the node whose other two coordinates are (c1,
 * c2) in increasing axis order: the positions where the phase indicator
 * changes side, each by linear interpolation between the two nodes of the
 * crossing segment (the radius measurement of the droplet-oscillation
 * section), in ascending order; on a periodic axis the segment from the last
 * node to the first is included (position between n-1 and n).  Returns the
 * number of crossings, of which the first `max` are written. */
int orc_interface_crossings(const orc_params *p, const double *f, int axis, int c1, int c2,
                            double *out, int max)
{
    const int64_t N = nnodes(p);
    double *phi = calloc((size_t)N, sizeof(double));
    orc_phase_indicator(p, f, phi);
    const int len = axis == 0 ? p->nx : (axis == 1 ? p->ny : p->nz);
    double *line = calloc((size_t)len, sizeof(double));
    for (int s = 0; s < len; ++s) {
        int x, y, z;
        if (axis == 0) { x = s; y = c1; z = c2; }
        else if (axis == 1) { x = c1; y = s; z = c2; }
        else { x = c1; y = c2; z = s; }
        line[s] = phi[idx(p, x, y, z)];
    }
    int count = 0;
    const int segs = p->bc[axis] == 0 && len > 1 ? len : len - 1;
    for (int s = 0; s < segs; ++s) {
        const double a = line[s], b = line[(s + 1) % len];
        if ((a > 0.0) != (b > 0.0)) {
            if (count < max) out[count] = s + a / (a - b);
            ++count;
        }
    }
    free(line); free(phi);
    return count;
}

/* Phase area of the lattice plane `pos` normal to `axis`: the sum of the red
 * fraction (1 + rho^N)/2 over the plane for the two-component models, the
 * count of nodes with rho >= (rho0_R + rho0_B)/2 for SC multiphase (the red
 * volume of the observables, restricted to one plane; the bridge radius of
 * the coalescence study is sqrt(area / pi)). */
double orc_plane_area(const orc_params *p, const double *f, int axis, int pos)
{
    orc_lattice L;
    get_lattice(p->lattice, &L);
    const int64_t N = nnodes(p);
    double *rR = calloc((size_t)N, sizeof(double));
    double *rB = calloc((size_t)N, sizeof(double));
    double *j = calloc((size_t)(3 * N), sizeof(double));
    moments_pass(p, &L, f, rR, rB, j);
    const double mid = 0.5 * (p->rho0_R + p->rho0_B);
    double area = 0.0;
    for (int64_t n = 0; n < N; ++n) {
        int x, y, z;
        coords(p, n, &x, &y, &z);
        const int c = axis == 0 ? x : (axis == 1 ? y : z);
        if (c != pos) continue;
        const double r = rR[n] + rB[n];
        if (p->model == 1) area += r >= mid ? 1.0 : 0.0;
        else area += 0.5 * (1.0 + (rR[n] - rB[n]) / r);
    }
    free(rR); free(rB); free(j);
    return area;
}

/* Connected components of the inside nodes (phi > 0) under face adjacency,
 * wrapping across periodic faces (droplet counting of the emulsion study).
 * labels[n] = smallest node index of n's component, -1 outside.  Breadth-
 * first search started from the nodes in ascending index order.  Returns the
 * number of components. */
int64_t orc_label_components(const orc_params *p, const double *f, int64_t *labels)
{
    const int64_t N = nnodes(p);
    double *phi = calloc((size_t)N, sizeof(double));
    orc_phase_indicator(p, f, phi);
    int64_t *queue = malloc((size_t)N * sizeof(int64_t));
    for (int64_t n = 0; n < N; ++n) labels[n] = -1;
    const int dims[3] = {p->nx, p->ny, p->nz};
    int64_t count = 0;
    for (int64_t s = 0; s < N; ++s) {
        if (!(phi[s] > 0.0) || labels[s] >= 0) continue;
        ++count;
        int64_t head = 0, tail = 0;
        queue[tail++] = s;
        labels[s] = s;
        while (head < tail) {
            const int64_t n = queue[head++];
            int c[3];
            coords(p, n, &c[0], &c[1], &c[2]);
            for (int a = 0; a < 3; ++a) {
                if (dims[a] == 1) continue;
                for (int dir = -1; dir <= 1; dir += 2) {
                    int q[3] = {c[0], c[1], c[2]};
                    q[a] += dir;
                    if (q[a] < 0 || q[a] >= dims[a]) {
                        if (p->bc[a] != 0) continue;
                        q[a] = (q[a] + dims[a]) % dims[a];
                    }
                    const int64_t m = idx(p, q[0], q[1], q[2]);
                    if (phi[m] > 0.0 && labels[m] < 0) {
                        labels[m] = s;
                        queue[tail++] = m;
                    }
                }
            }
        }
    }
    free(queue); free(phi);
    return count;
}

/* The multirange neighbourhood as tables: c[3*b + d], p[b], w[b]; returns the
 * number of vectors (92). */
int orc_belts_table(int32_t *c, double *p, double *w)
{
    orc_belts B;
    belts(&B);
    for (int b = 0; b < B.n; ++b) {
        for (int d = 0; d < 3; ++d) c[3 * b + d] = B.c[b][d];
        p[b] = B.p[b];
        w[b] = B.w[b];
    }
    return B.n;
}

/* Per-node forces of the two-component Shan-Chen model on the state f:
 * FR[d*N + n], FB[d*N + n] (cross repulsion plus, when set, the multirange
 * attraction and repulsion). */
void orc_sc_forces(const orc_params *p, const double *f, double *FR, double *FB)
{
    orc_lattice L;
    get_lattice(p->lattice, &L);
    const int64_t N = nnodes(p);
    double *rR = calloc((size_t)N, sizeof(double));
    double *rB = calloc((size_t)N, sizeof(double));
    double *j = calloc((size_t)(3 * N), sizeof(double));
    double *psR = calloc((size_t)N, sizeof(double));
    double *psB = calloc((size_t)N, sizeof(double));
    moments_pass(p, &L, f, rR, rB, j);
    psi_pass(p, rR, psR, N);
    psi_pass(p, rB, psB, N);
    for (int64_t n = 0; n < N; ++n) {
        double a[3], b[3];
        scmc_forces_at(p, &L, rR, rB, psR, psB, n, a, b);
        for (int d = 0; d < 3; ++d) {
            FR[d * N + n] = a[d];
            FB[d * N + n] = b[d];
        }
    }
    free(rR); free(rB); free(j); free(psR); free(psB);
}
