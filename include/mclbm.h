/*
 * mclbm.h -- C ABI of the MI355X two-component lattice Boltzmann library.
 *
 * The library advances the two-component lattice Boltzmann models compared
 * by Datadien, Di Staso, Wijshoff and Toschi (arXiv:2110.05197) on one GPU:
 *
 *   colour gradient (CG)     section 2.2, Eqs. streamingCG ... CGpressure:
 *                            moments -> isotropic gradients -> BGK with the
 *                            enhanced equilibrium -> perturbation ->
 *                            recolouring -> streaming;
 *   CG repulsion variant     section 2.3, Eqs. repForce ... normal2;
 *   Shan-Chen multiphase     section 2.1, Eqs. streamingSC ... guoforce2;
 *   Shan-Chen two-component  section 2.1, Eq. doublebeltrepulsionforce2
 *                            (cross force over the nearest-neighbour belt).
 *
 * on D2Q9 and D3Q19 lattices (the paper uses D3Q19, Eqs. speeds/weights).
 *
 * Conventions
 *   - Every function returns an mclbm_status: MCLBM_OK (0), the outcome
 *     MCLBM_DIVERGED (1), or a negative error.  No function aborts and no
 *     C++ exception crosses the ABI.  mclbm_last_error() holds a message for
 *     the calling thread's last error.
 *   - Pointers named d_* are device pointers (HIP global memory on the
 *     device that is current when the simulation is created); every other
 *     pointer is a host pointer.  The caller owns every buffer it passes;
 *     the library never frees caller memory.  The library owns only the
 *     small scratch it allocates in mclbm_create / mclbm_batch_create
 *     (reduction partials, a status word, descriptors, graphs), freed by the
 *     matching destroy call.
 *   - `stream` arguments are hipStream_t values passed as void*; NULL means
 *     the null stream.  All device work is enqueued on the simulation's
 *     stream and is asynchronous, except where a function says it
 *     synchronises.  One simulation must not be used from two host threads
 *     at once.
 *   - Node index n = x + nx*(y + ny*z), x fastest.  Population arrays are
 *     f[(k*Q + i)*N + n] with k = 0 red (the denser fluid) and k = 1 blue;
 *     the single-component model has k = 0 only.  Vector fields are
 *     v[d*N + n], d = 0, 1, 2 = x, y, z (d = 2 is zero on D2Q9).
 *   - Velocity ordering, both lattices: 0 = rest, then opposite pairs
 *     (1,2), (3,4), ...; axis directions first, then diagonals.
 *       D2Q9 : (1,0) (-1,0) (0,1) (0,-1) (1,1) (-1,-1) (1,-1) (-1,1)
 *       D3Q19: (1,0,0) (-1,0,0) (0,1,0) (0,-1,0) (0,0,1) (0,0,-1)
 *              (1,1,0) (-1,-1,0) (1,-1,0) (-1,1,0) (1,0,1) (-1,0,-1)
 *              (1,0,-1) (-1,0,1) (0,1,1) (0,-1,-1) (0,1,-1) (0,-1,1)
 */
#ifndef MCLBM_H
#define MCLBM_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define MCLBM_VERSION_MAJOR 2
#define MCLBM_VERSION_MINOR 0
#define MCLBM_ABI_VERSION 3

typedef int32_t mclbm_status;
#define MCLBM_OK 0
#define MCLBM_DIVERGED 1          /* outcome: NaN/Inf or rho <= 0 was seen       */
#define MCLBM_EINVAL (-1)         /* invalid argument or parameter               */
#define MCLBM_EUNSUPPORTED (-2)   /* combination not provided                    */
#define MCLBM_EDEVICE (-3)        /* a HIP call failed; text in mclbm_last_error */
#define MCLBM_ENOMEM (-4)         /* buffer too small or scratch allocation failed */

/* Lattices (Eqs. speeds, weights for D3Q19; D2Q9 uses constants obeying the
 * same moment conditions). */
#define MCLBM_D2Q9 0
#define MCLBM_D3Q19 1

/* Models. */
#define MCLBM_CG 0        /* colour gradient, section 2.2                     */
#define MCLBM_SC_MP 1     /* Shan-Chen multiphase, one component, section 2.1 */
#define MCLBM_SC_MC 2     /* Shan-Chen two-component, cross force only        */

/* Precision paths.  FP32/MIXED/FP16 store each population as its deviation
 * g = f - rho_k^0 phi_i^k from the rest equilibrium of the component's
 * initial bulk density (phi_i^k of Eq. phi for CG, w_i for SC). */
#define MCLBM_FP64 0      /* FP64 storage and arithmetic                           */
#define MCLBM_FP32 1      /* FP32 shifted storage, FP32 arithmetic                 */
#define MCLBM_MIXED 2     /* FP32 shifted storage; FP64 moment sums, recolouring   */
                          /* and light-phase (blue) equilibrium                   */
#define MCLBM_FP16 3      /* FP16 shifted storage, FP32 arithmetic                 */

/* Boundary type per axis.  Periodic is the paper's (sections 3.1-3.6); wall
 * (halfway bounce-back, neutral wetting) and outflow (zero-gradient copy of
 * the entering populations) are additions the paper does not define. */
#define MCLBM_PERIODIC 0
#define MCLBM_WALL 1
#define MCLBM_OUTFLOW 2

/* Kernel choice for mclbm_step. */
#define MCLBM_KERNEL_AUTO 0     /* fused where provided (D2Q9: from 2^19 nodes)    */
#define MCLBM_KERNEL_TWO_PASS 1 /* density-field pass + collide/stream pass       */
#define MCLBM_KERNEL_FUSED 2    /* one pass per step: CG/SC without repulsion     */

typedef struct mclbm_params {
    int32_t abi_version;  /* must be MCLBM_ABI_VERSION                              */
    int32_t lattice;      /* MCLBM_D2Q9 or MCLBM_D3Q19                              */
    int32_t model;        /* MCLBM_CG, MCLBM_SC_MP, MCLBM_SC_MC                     */
    int32_t precision;    /* MCLBM_FP64 ... MCLBM_FP16                              */
    int32_t nx, ny, nz;   /* lattice size; nz = 1 on D2Q9; each >= 2 otherwise;     */
                          /* nx * ny * nz < 2^31 (EUNSUPPORTED beyond)              */
    int32_t bc[3];        /* boundary type per axis x, y, z                         */
    int32_t enhanced_eq;  /* CG: 1 = enhanced equilibrium terms of Eq. equiliCG    */
    int32_t kernel;       /* MCLBM_KERNEL_*                                         */
    double rho0_R;        /* initial bulk density of red (>= rho0_B for CG)         */
    double rho0_B;        /* initial bulk density of blue                           */
    double tau_R, tau_B;  /* relaxation times (> 1/2); SC_MP uses tau_R             */
    double A;             /* CG perturbation parameter (Eqs. perturbationOp, sigmaA) */
    double beta;          /* CG recolouring parameter in [0, 1] (Eq. recoloringOpR) */
    double alpha_B;       /* CG rest fraction of blue in [0, 1) (Eq. gamma)         */
    double g_min;         /* |grad rho^N| at or below which the perturbation and    */
                          /* recolouring terms are dropped (no normal defined)      */
    double G;             /* SC_MP coupling, < 0 attractive (Eq. interactionforceMP) */
    double psi_rho0;      /* SC_MP reference density rho_0 (Eq. pseudopotential)    */
    double G_RB;          /* SC_MC cross coupling (Eq. doublebeltrepulsionforce2)   */
    double rho0_X;        /* SC_MC reference density rho_0^(s) in the cross force   */
    double Pi;            /* CG repulsion magnitude (Eq. repForce); 0 = off         */
    double chi;           /* CG repulsion exponent, psi_rep = (1 - |rho^N|)^chi     */
    /* SC_MC multirange couplings (Eq. benziforces): attraction on belt 1     */
    /* (Eq. doublebeltattractiveforce) and repulsion on belts 1 and 2 (Eq.    */
    /* doublebeltrepulsionforce, weights of Eq. pweights), per species, with  */
    /* psi_s = psi_rho0 (1 - exp(-rho_s / psi_rho0)).  All zero = off; any    */
    /* non-zero needs model SC_MC (EINVAL otherwise) and D3Q19 (EUNSUPPORTED  */
    /* on D2Q9), and runs the two-pass kernels (the stencil reaches two       */
    /* nodes).                                                               */
    double Ga_R, Ga_B;    /* attraction couplings G^a of red and blue               */
    double Gr_R, Gr_B;    /* repulsion couplings G^r of red and blue                */
    /* CG with FP32 or mixed storage: 1 = keep each colour's mass at every     */
    /* node to one rounding per step (the rest population is set last from   */
    /* FP64 sums of the node's populations); it removes the steady FP32 drift */
    /* of the colour masses (about 1e-7 of the red mass per step at          */
    /* interfaces, from the rounding of the recolouring exchange, Eqs.       */
    /* recoloringOpR/B) and costs about 4 % of the step.  0 (default) = off; */
    /* ignored by the other models and precisions.  EINVAL unless 0 or 1.     */
    int32_t conserve_mass;
} mclbm_params;

/* Observables (reductions over the whole lattice, FP64 accumulation in a
 * fixed order, so repeated calls on one state give identical results). */
typedef struct mclbm_obs {
    double mass_R, mass_B;  /* sum of rho_R, rho_B                                   */
    double mom[3];          /* sum of j = sum_k sum_i f c_i                          */
    double ekin;            /* sum of rho |u|^2 / 2                                  */
    double umax;            /* max |u|                                               */
    double rho_in, rho_out; /* Eqs. rhoin/rhoout with eps_used (CG, SC_MC); SC_MP:   */
                            /* mean rho where rho >= (rho0_R+rho0_B)/2 and below    */
    double eps_used;        /* largest 1 - 0.1^n (n = 1..10) with both sets non-empty */
    double red_volume;      /* sum (1 + rho^N)/2; SC_MP: number of inside nodes      */
    double n_in, n_out;     /* node counts of the two sets                           */
    double diverged;        /* 1 if any node had non-finite moments or rho <= 0      */
    int64_t step;           /* steps taken since mclbm_init_equilibrium/import       */
} mclbm_obs;
/* u is the fluid velocity (j + F/2)/rho with F the Shan-Chen force (Eq.
 * guoforce2) for SC models; the bare j/rho for CG. */

typedef struct mclbm_sim mclbm_sim;
typedef struct mclbm_batch mclbm_batch;

/* Library version. */
mclbm_status mclbm_version(int32_t *major, int32_t *minor);

/* Static text for a status code (never NULL). */
const char *mclbm_status_str(mclbm_status s);

/* Message of the calling thread's last error ("" if none). */
const char *mclbm_last_error(void);

/* Fill *p with defaults for (lattice, model): 64^3 (64^2 on D2Q9) periodic,
 * FP32, rho0 = 1/1, tau = 1/1, A = 0.005, beta = 0.7 (section 2.2),
 * alpha_B = 0.2 (after Eq. gamma), g_min = 1e-8, enhanced_eq = 1,
 * G = -5, psi_rho0 = 1, G_RB = 0.9, rho0_X = 1, Pi = 0, chi = 1. */
mclbm_status mclbm_params_default(mclbm_params *p, int32_t lattice, int32_t model);

/* CG: set p->A for surface tension sigma by Eq. sigmaA, sigma = 4A/(9 omega),
 * with omega_eff (Eq. effRelax) of the interface viscosity (Eq. interpVisc)
 * at rho^N = 0, i.e. 1/nu = (1/nu_R + 1/nu_B)/2.  EINVAL for SC models. */
mclbm_status mclbm_params_from_sigma(mclbm_params *p, double sigma);

/* Inverse of mclbm_params_from_sigma. */
mclbm_status mclbm_sigma_from_params(const mclbm_params *p, double *sigma);

/* Validate *p and return the device bytes the caller must provide to
 * mclbm_create: two population buffers (ping-pong) plus the per-node fields
 * the stencils read, each 256-byte aligned. */
mclbm_status mclbm_state_bytes(const mclbm_params *p, size_t *bytes);

/* Algorithmic HBM bytes per lattice update of one step (populations read
 * once and written once): 2 * ncomp * Q * sizeof(storage). */
mclbm_status mclbm_bytes_per_update(const mclbm_params *p, double *bytes);

/* Layout of the population buffers inside the state (host only; for tests
 * and diagnostics: callers never index the state themselves).  A buffer
 * holds *arrays population arrays of *word_bytes-byte words (a word is one
 * population of one node; two-colour FP16 storage keeps both colours of a
 * population in one 4-byte word), each array *words words from the previous
 * one.  *words >= N: arrays of large lattices are padded so that the arrays
 * of one buffer do not start a multiple of a large power of two apart (the
 * streams of a step would then fall on the same HBM banks).  EINVAL on NULL
 * or invalid parameters. */
mclbm_status mclbm_population_stride(const mclbm_params *p, int64_t *words, int32_t *word_bytes, int32_t *arrays);

/* Create a simulation on caller memory d_state (>= mclbm_state_bytes, not
 * freed by the library), enqueuing on `stream`.  Allocates the library's
 * small scratch on the current device.  The state is undefined until
 * mclbm_init_equilibrium or mclbm_import_f. */
mclbm_status mclbm_create(const mclbm_params *p, void *d_state, size_t bytes, void *stream,
                          mclbm_sim **out);

/* Release the library's scratch (synchronises the stream). */
mclbm_status mclbm_destroy(mclbm_sim *sim);

/* Initialise the populations to the model's equilibrium of the given fields
 * (device FP64 arrays of N values; d_u is 3*N values or NULL for rest):
 * CG: Eq. equiliCG of each colour with gradients of the given densities;
 * SC: Eq. equiliSC of each component.  SC_MP reads only d_rhoR (its density).
 * Resets the step counter and the divergence flag. */
mclbm_status mclbm_init_equilibrium(mclbm_sim *sim, const double *d_rhoR, const double *d_rhoB,
                                    const double *d_u);

/* Advance nsteps time steps.  check_every > 0: every check_every steps (and
 * at the end) check the current state as mclbm_diverged does (synchronises)
 * and stop early with MCLBM_DIVERGED if it is bad or a step saw a bad state;
 * check_every == 0: fully asynchronous, no early exit.  *steps_done (may be NULL) receives the steps taken.
 * With check_every == 0 the call only enqueues kernel launches on the sim's
 * stream (no copy, fill or synchronisation), so a caller may capture it into
 * a HIP graph.  The ping-pong buffer index and the step counter advance on
 * the host when the launches are enqueued: a graph replayed more than once
 * must hold an even number of steps (so each replay starts from the buffer
 * the previous one wrote), and the counter counts the captured steps, not
 * the replays.  Step once eagerly before capturing: the first launch of a
 * kernel configuration in a process raises its dynamic-LDS limit. */
mclbm_status mclbm_step(mclbm_sim *sim, int64_t nsteps, int64_t check_every, int64_t *steps_done);

/* Per-node moments into device FP64 arrays (any may be NULL): rho_R, rho_B
 * (rho_R = rho for SC_MP, rho_B = 0) and the velocity u (3*N) as in
 * mclbm_obs. */
mclbm_status mclbm_moments(mclbm_sim *sim, double *d_rhoR, double *d_rhoB, double *d_u);

/* Reductions of the current state into *out (synchronises the stream). */
mclbm_status mclbm_observables(mclbm_sim *sim, mclbm_obs *out);

/* Copy the populations f (not deviations) out to / in from a device FP64
 * array of ncomp*Q*N values.  Import converts to the storage precision,
 * resets the divergence flag and keeps the step counter. */
mclbm_status mclbm_export_f(mclbm_sim *sim, double *d_f);
mclbm_status mclbm_import_f(mclbm_sim *sim, const double *d_f);

/* Raw checkpoint: copy the current population buffer in its storage format
 * (bitwise) to/from device memory of mclbm_checkpoint_bytes bytes, with the
 * step counter.  Restoring then stepping reproduces an uninterrupted run
 * bit for bit. */
mclbm_status mclbm_checkpoint_bytes(const mclbm_sim *sim, size_t *bytes);
mclbm_status mclbm_checkpoint(mclbm_sim *sim, void *d_dst, int64_t *step);
mclbm_status mclbm_restore(mclbm_sim *sim, const void *d_src, int64_t step);

/* 1 if the current state has a node with a non-finite moment or rho <= 0,
 * or any earlier state since the last init / import / restore had one (a
 * step flags the state it reads; this call also scans the current one,
 * one read of the populations).  Synchronises. */
mclbm_status mclbm_diverged(mclbm_sim *sim, int32_t *diverged);

/* Interface observables.  The phase indicator of a node is rho^N =
 * (rho_R - rho_B)/rho for the two-component models and rho - (rho0_R +
 * rho0_B)/2 for SC multiphase (the interface definitions of the droplet-
 * oscillation study), computed in FP64 from the stored populations; a node
 * is inside the red (liquid) phase when it is > 0.  All three synchronise the
 * stream; EINVAL on bad arguments, EDEVICE on a HIP error.
 *
 * mclbm_interface_crossings: along the lattice line parallel to `axis` (0 x,
 * 1 y, 2 z) through the node whose other two coordinates are (c1, c2) in
 * increasing axis order, the positions where the indicator changes side,
 * each by linear interpolation between the two nodes of its segment (the
 * radius and endpoint measurements of the oscillation and ligament
 * studies), ascending; a periodic axis includes the segment from its last
 * node to its first (position in [n-1, n)).  *count = number of crossings;
 * the first min(count, max) positions go to host array h_pos.
 *
 * mclbm_plane_area: over the lattice plane `pos` normal to `axis`, the sum of
 * the red fraction (1 + rho^N)/2, or for SC multiphase the number of nodes
 * with rho >= (rho0_R + rho0_B)/2 (the bridge radius of the coalescence
 * study is sqrt(area / pi)); deterministic.
 *
 * mclbm_droplets: connected components of the inside nodes under face
 * adjacency, wrapping across periodic faces (droplet counting of the
 * emulsion study).  *count = number of components; h_sizes receives the
 * node counts of the largest min(count, max), in decreasing order.  The
 * first call allocates 16 bytes per node of device scratch, kept until
 * mclbm_destroy; EUNSUPPORTED for 2^31 - 2 nodes or more. */
mclbm_status mclbm_interface_crossings(mclbm_sim *sim, int32_t axis, int32_t c1, int32_t c2, double *h_pos,
                                       int32_t max, int32_t *count);
mclbm_status mclbm_plane_area(mclbm_sim *sim, int32_t axis, int32_t pos, double *area);

/* mclbm_interface_crossings for callers that cannot allocate device memory
 * (code under HIP graph capture, tight serving or measurement loops,
 * harnesses that forbid hipMalloc): the same arguments, kernels and results,
 * but it calls no hipMalloc, hipFree or other allocating routine.  Its
 * scratch (the sampled line, the positions, the count) is a static device
 * array of 2 * 32768 + 16 doubles (512 KB) that every device holds for the
 * life of the process; the first call on a device looks up its address.
 * EUNSUPPORTED for a line longer than 32768 nodes.  All calls on one device
 * share that array: calls that overlap on one device (other host threads,
 * other streams) race and must be serialised by the caller.  Synchronises
 * the simulation's stream, like mclbm_interface_crossings. */
mclbm_status mclbm_interface_crossings_noalloc(mclbm_sim *sim, int32_t axis, int32_t c1, int32_t c2, double *h_pos,
                                               int32_t max, int32_t *count);
mclbm_status mclbm_droplets(mclbm_sim *sim, int32_t max, int32_t *count, int64_t *h_sizes);

/* The step kernel this simulation runs: MCLBM_KERNEL_FUSED (one pass:
 * without the repulsion or multirange forces; D3Q19 with ny % 4 == 0 and any
 * nx, D2Q9 of any size) or MCLBM_KERNEL_TWO_PASS.  Host only; EINVAL on
 * NULL. */
mclbm_status mclbm_kernel_used(const mclbm_sim *sim, int32_t *kernel);

/* Work of one block of the one-pass kernel: a *tx x *ty column of nodes
 * marching through *tz planes (D3Q19), or a row segment of *tx nodes marching
 * through *tz rows (D2Q9, *ty = 1); blocks at the end of the lattice march
 * fewer.  Host only; EUNSUPPORTED when the simulation runs the two-pass
 * kernels, EINVAL on NULL. */
mclbm_status mclbm_fused_tile(const mclbm_sim *sim, int32_t *tx, int32_t *ty, int32_t *tz);

/* ------------------------------------------------------------------------ */
/* Batched stepping of many independent simulations (sweep serving).         */
/* ------------------------------------------------------------------------ */
/* Batch status words. */
#define MCLBM_RUNNING 0
#define MCLBM_DONE 1
#define MCLBM_STOPPED_DIVERGED 2

/* Group sims (created as above, initialised, on any streams) into a batch
 * that advances them together on `stream`: one launch per kernel per group of
 * equal (lattice, model, precision), with per-lattice parameters, sizes and
 * boundaries in device descriptors.  Groups after the first run on streams
 * the batch creates (default priority), forked from and joined back to
 * `stream` within every step, so that all work of a step is ordered on
 * `stream`.  target_steps[s] (host, n values) is the
 * number of further steps sim s should take; a sim stops when it reaches
 * its target or diverges.  Sims must not be stepped on their own while in a
 * batch.  D3Q19 sims that have a one-pass kernel (no repulsion force, no
 * multirange forces), with ny % 8 == 0 (ny % 4 == 0 in FP64 and mixed
 * precision), and whose kernel is not MCLBM_KERNEL_TWO_PASS, step in batched
 * one-pass launches (64 x 8 columns, 64 x 4 in FP64 and mixed precision, the
 * last column in x masked when 64 does not divide nx, which the batch does
 * when nx >= 3/4 of 64 * ceil(nx / 64); 96 x 4 columns, with ny % 4 == 0,
 * where 96 divides nx and 64 does not, except in FP64 and for the mixed
 * colour gradient; z-chunks sized for the group; one launch per kind present
 * in the group: all faces periodic or not, nx a multiple of 64 or not, 96-wide
 * columns or not); the others in batched two-pass launches.  The
 * per-node arithmetic is the same as mclbm_step's, so a sim's result is
 * bitwise the same alone (either kernel) and in any batch. */
mclbm_status mclbm_batch_create(mclbm_sim *const *sims, int32_t n, const int64_t *target_steps,
                                void *stream, mclbm_batch **out);

/* The kernel each sim runs in the batch: MCLBM_KERNEL_FUSED or
 * MCLBM_KERNEL_TWO_PASS (host array of n, in the order given to
 * mclbm_batch_create).  Host only; EINVAL on NULL. */
mclbm_status mclbm_batch_kernels(const mclbm_batch *b, int32_t *kernels);

/* Enqueue ksteps batch steps.  use_graph != 0 captures the ksteps launches
 * in a HIP graph once (per ksteps value) and replays it. */
mclbm_status mclbm_batch_step(mclbm_batch *b, int32_t ksteps, int32_t use_graph);

/* Status words and steps taken per sim (host arrays of n; synchronises).
 * Also updates each sim's own step counter and current buffer.  The state a
 * sim that reached its target ends in is scanned once (one read of its
 * populations) and reported MCLBM_STOPPED_DIVERGED if it is bad: the steps
 * themselves flag only the states they read. */
mclbm_status mclbm_batch_status(mclbm_batch *b, int32_t *status, int64_t *steps);

/* Release the batch (synchronises).  The sims stay valid and receive their
 * step counters and current buffers, as from mclbm_batch_status. */
mclbm_status mclbm_batch_destroy(mclbm_batch *b);

#ifdef __cplusplus
}
#endif
#endif /* MCLBM_H */
