/*
 * lbm.h -- C-ABI of the MI355X pseudopotential MRT lattice Boltzmann step.
 *
 * Method: W. Zhao, B. Xu, Y. Zhang, arXiv:1803.01756, Section 2.  One call of
 * lbm_step(sim, 1) advances a D2Q9 channel between two plates by one time
 * step:
 *   - macroscopic density and half-force velocity (Eq. 13),
 *   - pseudopotential psi(rho, T) from the Peng-Robinson EOS (Eqs. 10-11),
 *   - Shan-Chen fluid-fluid force (Eq. 9), wall adhesion (Eq. 14), gravity
 *     (Eq. 15) and the oscillating drive rho*g_osc*sin(2 pi n / period) along
 *     +x,
 *   - density-interpolated viscous relaxation time (Eqs. 4-5),
 *   - MRT collision in moment space with Li's source term (Eqs. 6-8),
 *   - classical RK4 of the energy equation (Eqs. 16-18) with isotropic
 *     nine-point finite differences,
 *   - streaming (Eq. 12) with half-way bounce-back at the plates.
 * The plates are the solid rows y = 0 and y = Ny-1 and x is periodic, unless
 * a flag below (LBM_PERIODIC_Y, LBM_OPEN_X) says otherwise.
 *
 * Conventions for every entry point:
 *   - Status codes only; nothing throws or exits.  On failure an output
 *     handle is set to NULL and lbm_last_error() describes the cause.
 *   - Host arrays are caller-owned and indexed [y*Nx + x], y = 0..Ny-1.
 *   - Device memory and streams are plain pointers (hipStream_t is passed as
 *     void*).  A NULL stream means the library creates its own.
 *   - lbm_step only enqueues work.  Device faults surface on the next
 *     synchronising call as LBM_EDEVICE.  A non-finite state surfaces as
 *     LBM_EUNSTABLE: every step checks the rho and T it reads (the state at
 *     its own time level) on every fluid node and counts the non-finite
 *     ones on the device; lbm_synchronize reports any such count, and
 *     lbm_moments and lbm_reduce also check the current time level (the
 *     state the last step wrote).  The count is kept until lbm_load
 *     replaces the state (lbm_health reads it).
 *   - A simulation must not be used from two threads at once.
 */
#ifndef PAPER_1803_01756_LBM_H
#define PAPER_1803_01756_LBM_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct lbm_sim lbm_sim;   /* opaque, library-owned */
typedef struct lbm_pool lbm_pool; /* opaque slot pool for batched / served runs */

typedef enum {
    LBM_OK = 0,
    LBM_EINVAL = -1,    /* invalid argument or parameter set                   */
    LBM_ENOMEM = -2,    /* device memory (or pool capacity) exhausted           */
    LBM_EDEVICE = -3,   /* HIP runtime error                                    */
    LBM_EUNSTABLE = -4, /* non-finite density, velocity or temperature found    */
    LBM_ESTATE = -5     /* call not valid in the current state                  */
} lbm_status;

/* storage precision of the populations and the temperature */
enum {
    LBM_FP32_DEV = 0,          /* FP32 deviations f_i - w_i rho_ref, T - T_0   */
    LBM_FP64 = 1,              /* FP64 deviations                              */
    LBM_FP32_DEV_MASSEXACT = 2 /* FP32 deviations, rest population kept as an
                                  FP32 (hi, lo) pair so that the total mass is
                                  conserved to FP64 rounding                   */
};

/* flags */
enum {
    LBM_FREEZE_T = 1u,     /* isothermal: skip the temperature update           */
    LBM_SINGLE_PHASE = 2u, /* F_m = 0 and no theta term (ideal-gas flow checks) */
    LBM_PERIODIC_Y = 4u,   /* no plates: periodic in y as well                  */
    LBM_FRAME_T = 8u,      /* Sec. 3.1 (droplet in surroundings at a set
                              temperature): the outermost columns, and with
                              LBM_PERIODIC_Y the outermost rows, form a frame
                              whose temperature is held at T_w in every RK
                              stage                                          */
    LBM_FRAME_RHO = 16u,   /* the same frame is an open reservoir at rest:
                              rho = rho_frame and u = 0 there, and its
                              post-collision populations are the rest
                              equilibrium of rho_frame (mass is then not
                              conserved: vapour leaves or enters)            */
    LBM_EOS_CS = 32u,      /* Carnahan-Starling EOS in place of Eq. 11:
                              P = rho R T (1 + e + e^2 - e^3) / (1 - e)^3
                              - a rho^2, e = b rho / 4 (usual constants
                              a = 1, b = 4, R = 1); omega is then unused   */
    LBM_OPEN_X = 64u,      /* Sec. 3.3 boundary set: x is not periodic;
                              column 0 is a Zou-He pressure inlet, column
                              Nx-1 a Zou-He pressure outlet (zero transverse
                              velocity).  Pressures are EOS pressures:
                              p_in(n) = p0 (1 + p_amp sin(2 pi n / p_period))
                              (p_period <= 0: p0 (1 + p_amp)), p_out = p0,
                              p0 = P_EOS(rho_v, T_in); the boundary densities
                              are their vapour-branch roots.  Stencils past
                              the ends see the boundary column's own values;
                              the inlet column holds T = T_in, the outlet
                              column T = T_out when T_out > 0 (else its T
                              evolves).                                     */
    LBM_PHASE_PROPS = 128u, /* lambda and C_v interpolated between the gas
                              values (lambda, C_v) and the liquid values
                              (lambda_l, C_v_l) with the clamped fraction of
                              Eq. 5; the conduction term of Eq. 16 becomes
                              [lambda lap T + grad(lambda).grad(T)] / (rho C_v),
                              solid nodes carrying the gas values           */
    LBM_TOP_MIXED = 256u   /* Sec. 3.2 plates: the top plate holds T_w on the
                              columns cold_x0 <= x < cold_x1 and is adiabatic
                              elsewhere (zero normal gradient at the half-way
                              wall: a temperature stencil reaching such a
                              node reads the fluid node below it, at the
                              same RK stage); the bottom plate holds
                              T_w_bottom.  Not with LBM_PERIODIC_Y,
                              LBM_OPEN_X or T_w_end > 0.                    */
};

/* Parameters, named as in the paper.  lbm_params_default() fills the paper's
 * values and the readings taken for the unstated ones; lbm_params_resolve()
 * fills the derived fields left at <= 0. */
typedef struct {
    int32_t Nx, Ny;         /* nodes, solid plate rows included                    */
    double a, b, R, omega;  /* Eq. 11: 3/49, 2/21, 1; acentric factor 0.344        */
    double T_c;             /* Eq. 11 critical temperature; <= 0: derived          */
    double G;               /* Eqs. 9-10 interaction strength, default -1          */
    double theta;           /* Eq. 8 thermodynamic-consistency factor, 0.104       */
    double G_w, psi_w;      /* Eq. 14 adhesion strength and wall potential         */
    double s_rho, s_e, s_zeta, s_j, s_q; /* Eq. 3 rates; s_e must equal s_zeta    */
    double tau_g, tau_l;    /* Eq. 5 viscous relaxation times of gas and liquid   */
    double rho_g, rho_l;    /* Eq. 5 phase densities; <= 0: Maxwell at T_0        */
    double C_v, lambda;     /* Eq. 16 heat capacity and conductivity, 5 and 0.25  */
    double T_0, T_w;        /* initial fluid and plate temperatures               */
    double g_osc, period;   /* drive amplitude and period in steps (<= 0: off)    */
    double g_x, g_y;        /* Eq. 15 gravity                                      */
    double rho_v;           /* Eq. 15 reference vapour density; < 0: Maxwell gas  */
    double rho_ref;         /* density of the stored deviations; <= 0: rho_v (or
                               the Maxwell gas density when rho_v is 0)          */
    double rho_frame;       /* LBM_FRAME_RHO reservoir density (> 0 required)   */
    double p_amp, p_period; /* LBM_OPEN_X inlet pressure oscillation             */
    double T_w_end;         /* > 0: plate temperature linear in x, from T_w at
                               x = 0 to T_w_end at x = Nx-1 (Sec. 3.3)          */
    double T_in;            /* LBM_OPEN_X inlet temperature; <= 0: T_0          */
    double lambda_l, C_v_l; /* LBM_PHASE_PROPS liquid conductivity and heat
                               capacity (lambda, C_v are then the gas values)    */
    double T_w_bottom;      /* LBM_TOP_MIXED bottom plate temperature; <= 0: T_0 */
    int32_t cold_x0, cold_x1; /* LBM_TOP_MIXED cold columns of the top plate,
                               0 <= cold_x0 <= cold_x1 <= Nx                    */
    int32_t precision;      /* LBM_FP32_DEV, LBM_FP64 or LBM_FP32_DEV_MASSEXACT   */
    uint32_t flags;         /* LBM_FREEZE_T | LBM_SINGLE_PHASE | LBM_PERIODIC_Y |
                               LBM_FRAME_T | LBM_FRAME_RHO | LBM_EOS_CS |
                               LBM_OPEN_X | LBM_PHASE_PROPS | LBM_TOP_MIXED      */
    double alpha_max;       /* > 0: a stated departure from Eq. 17 at delta t = 1.
                               The explicit RK4 of the conduction term with the
                               nine-point Laplacian is stable only while the
                               diffusivity lambda / (rho C_v) stays below 0.522;
                               vapour in equilibrium with liquid below ~0.74 T_c
                               is thinner than that allows at lambda = 0.25,
                               C_v = 5.  With alpha_max > 0 the conduction term
                               of a node whose diffusivity exceeds alpha_max is
                               scaled by alpha_max / (lambda / (rho C_v)), so it
                               acts with diffusivity alpha_max there; 0: off
                               (the paper's equation).  Must be 0 or in
                               (0, 0.522].                                      */
    double T_out;           /* LBM_OPEN_X outlet temperature: > 0 held (a
                               reservoir of vapour at T_out); 0: the outlet
                               column's T evolves                               */
} lbm_params;

/* Fill *p with the defaults: Nx = 128, Ny = 32, a = 3/49, b = 2/21, R = 1,
 * omega = 0.344, T_c derived, G = -1, theta = 0.104, G_w = psi_w = 0,
 * s_rho = s_j = 1, s_e = s_zeta = 0.8, s_q = 1.1, tau_g = tau_l = 1,
 * C_v = 5, lambda = 0.25 (Sec. 3.2), T_0 = 0.86 T_c, T_w = 0.80 T_c,
 * g_osc = 1e-6, period = 2000, no gravity, FP32_DEV, no flags.  T_c, T_0,
 * T_w, rho_g, rho_l, rho_ref stay 0 and rho_v -1 ("derive") until
 * lbm_params_resolve(). */
void lbm_params_default(lbm_params* p);

/* Derive the fields left at <= 0 (rho_v: < 0): T_c (critical point of
 * Eq. 11 with phi = 1), T_0 = 0.86 T_c, T_w = 0.80 T_c, rho_g and rho_l
 * (Maxwell coexistence at T_0), rho_v = rho_g, rho_ref = rho_v (rho_g when
 * rho_v is 0).  LBM_EINVAL if T_0 is not below T_c while a coexistence
 * density is requested. */
lbm_status lbm_params_resolve(lbm_params* p);

/* Critical point (rho_c, T_c) of the Peng-Robinson EOS of Eq. 11 and the
 * coexistence densities at temperature T (equal pressure and chemical
 * potential).  Host FP64. */
lbm_status lbm_eos_critical(double a, double b, double R, double* rho_c, double* T_c);
/* The critical point of the Carnahan-Starling EOS (LBM_EOS_CS). */
lbm_status lbm_eos_critical_cs(double a, double b, double R, double* rho_c, double* T_c);
lbm_status lbm_eos_coexistence(const lbm_params* p, double T, double* rho_g, double* rho_l,
                               double* p_sat);

/* P_EOS(rho, T) of Eq. 11 and the pseudopotential psi of Eq. 10 (clamped at
 * 0) for the EOS constants and G of *p (T_c <= 0: derived).  Host FP64; used
 * e.g. to turn a virtual wall density into psi_w. */
lbm_status lbm_eos_pressure(const lbm_params* p, double rho, double T, double* P, double* psi);

/* Latent heat of Eq. 19 at T < T_c (per unit mass, lattice units): the
 * internal-energy difference of the coexisting phases integrated over the
 * EOS, [a phi(T) - T a dphi/dT] / (2 sqrt2 b) times the difference of
 * ln[(1 + (1+sqrt2) b rho) / (1 + (1-sqrt2) b rho)] between liquid and vapour,
 * plus p_s (1/rho_g - 1/rho_l); the paper's c_alpha and c_a are the PR kappa.
 * The Jacob number of Eq. 20 is C_v (T_sat - T_w) / h_fg(T_sat).  Host FP64.
 * LBM_EINVAL if T is not below T_c or no coexistence is found. */
lbm_status lbm_eos_latent_heat(const lbm_params* p, double T, double* h_fg);

/* Jacob number of Eq. 20, Ja = C_v (T_sat - T_w) / h_fg(T_sat), with h_fg
 * from lbm_eos_latent_heat.  Host FP64; LBM_EINVAL as lbm_eos_latent_heat. */
lbm_status lbm_eos_jacob(const lbm_params* p, double T_sat, double T_w, double* Ja);

/* Device bytes a simulation with these parameters needs (two population
 * buffers, two temperature buffers, moment scratch), for callers that
 * provide the memory themselves.  0 if the parameters are invalid. */
size_t lbm_workspace_bytes(const lbm_params* p);

/* Create a simulation at time level 0.
 *   p          parameters (resolved internally; the caller's copy is not changed)
 *   rho0       host array Nx*Ny of initial densities (solid rows ignored), or
 *              NULL for the uniform density rho_v.  Populations start at the
 *              rest equilibrium f_i = w_i rho0, T = T_0 on fluid nodes.
 *   workspace  device memory of at least lbm_workspace_bytes(p) bytes, owned by
 *              the caller and valid until lbm_destroy; NULL: the library
 *              allocates and frees its own.
 *   ws_bytes   size of workspace (ignored when workspace is NULL)
 *   stream     hipStream_t all work is ordered on, or NULL for a private stream
 *   out        receives the handle
 * LBM_EINVAL: Nx < 3, Ny < 4 (Ny < 3 with LBM_PERIODIC_Y), G = 0, a relaxation
 * rate outside (0, 2), tau <= 1/2, s_e != s_zeta, an initial density that is
 * not positive, reaches the EOS packing limit (b rho >= 1; >= 4 for
 * LBM_EOS_CS) or makes the Eq. 10 argument 2 (P_EOS - rho/3) / G negative at
 * the node's initial temperature (no real psi: P - rho/3 > 0 for G < 0), or
 * a workspace that is too small.  LBM_ENOMEM, LBM_EDEVICE. */
lbm_status lbm_create(const lbm_params* p, const double* rho0, void* workspace,
                      size_t ws_bytes, void* stream, lbm_sim** out);

/* Enqueue n >= 0 time steps (asynchronous). */
lbm_status lbm_step(lbm_sim* sim, int64_t n);

/* Synchronise and copy rho, u (the half-force velocity of Eq. 13) and T at
 * the current time level into caller-owned host arrays of Nx*Ny doubles
 * (any may be NULL).  Solid rows give rho = 0, u = 0, T = T_w.  The arrays
 * are filled also when the call returns LBM_EUNSTABLE (some step read a
 * non-finite rho or T, or the current level holds one). */
lbm_status lbm_moments(lbm_sim* sim, double* rho, double* ux, double* uy, double* T);

/* Synchronise and reduce in FP64 with a fixed summation order:
 * out[0] = sum rho, out[1] = sum rho u_x, out[2] = sum rho u_y,
 * out[3] = sum rho C_v T, out[4] = number of non-finite nodes.
 * Returns LBM_EUNSTABLE when out[4] > 0 or some step read a non-finite
 * state. */
lbm_status lbm_reduce(lbm_sim* sim, double out[5]);

/* For callers that cannot allocate device memory or synchronise (code under
 * HIP graph capture, serving loops, harnesses that forbid hipMalloc): the
 * totals of lbm_reduce, out_dev[0..4] (sum rho, sum rho u_x, sum rho u_y,
 * sum rho C_v T, non-finite nodes) at the current time level, written to
 * caller-owned device memory (5 doubles, 8-byte aligned) by work enqueued
 * on the simulation's stream; the call returns without waiting.  The
 * values equal lbm_reduce's up to the FP64 summation order (one pass over
 * tiles of 64 x 4 nodes instead of two passes through the moment arrays).
 * It allocates nothing, does not synchronise and issues no memset: the
 * block partials live in a 40 KiB array the library holds on every GPU it
 * runs on until the process ends (at most 1024 blocks, a grid-stride loop
 * covers any grid the library accepts).  Every call on one GPU shares that
 * array, so calls that overlap on one GPU (two streams, two threads) race
 * and must be ordered by the caller.  No status from the state: read
 * out_dev[4] for the non-finite count.  LBM_EINVAL for a null or unaligned
 * pointer, LBM_EDEVICE for a launch error. */
lbm_status lbm_reduce_noalloc(lbm_sim* sim, double* out_dev);

/* Wait for all enqueued work.  LBM_EDEVICE on a device error,
 * LBM_EUNSTABLE when some completed step read a non-finite rho or T. */
lbm_status lbm_synchronize(lbm_sim* sim);

/* Synchronise and read the health counters the steps keep on the device
 * (never reset by a step; lbm_load restarts them):
 *   nonfinite   fluid-node readings of a non-finite rho or T, summed over
 *               the steps taken (each step reads the state of its own time
 *               level once per node),
 *   psi_clamps  fluid-node evaluations of Eq. 10 whose argument
 *               2 (P_EOS - rho/3) / G was not positive, so that psi was
 *               clamped to 0, summed over the steps taken.
 * Either pointer may be NULL.  Returns LBM_OK with the counts (LBM_EDEVICE
 * on a device error); the counts do not change the status. */
lbm_status lbm_health(lbm_sim* sim, int64_t* nonfinite, int64_t* psi_clamps);

/* Destroy; NULL is accepted.  Frees library-owned memory and stream. */
lbm_status lbm_destroy(lbm_sim* sim);

int64_t lbm_time(const lbm_sim* sim);

/* Parameters after resolution (derived fields filled). */
lbm_status lbm_get_params(const lbm_sim* sim, lbm_params* out);

/* Message of the last failure on this thread (never NULL). */
const char* lbm_last_error(void);

/* Checkpoint: lbm_state_bytes() bytes hold the time level, the parameters
 * and the device state; lbm_load() restores a state saved from a simulation
 * with the same grid and precision (the saved parameters, which must pass
 * the same checks as lbm_create's, replace the simulation's).  A buffer that
 * is too small, was written by another version of this format or does not
 * match gives LBM_EINVAL and leaves the simulation unchanged.  Both
 * synchronise. */
size_t lbm_state_bytes(const lbm_sim* sim);
lbm_status lbm_save(lbm_sim* sim, void* host, size_t bytes);
lbm_status lbm_load(lbm_sim* sim, const void* host, size_t bytes);

/* Launch shape of the fused step kernel: each wave owns a strip of 54
 * columns and marches over seg_rows fluid rows.  seg_rows <= 0 restores the
 * default: segments sized for about 3072 waves (one resident round at three
 * waves per SIMD on 256 CUs; 2048 and two waves for FP64 and mass-exact
 * storage), at least 2 rows, with seg_rows + 10 a multiple of 6 (pool slots:
 * at least 14 rows, see lbm_pool_set_launch).  lbm_autotune times candidate
 * shapes instead.  The result of a step does not depend on the shape
 * (bitwise). */
lbm_status lbm_set_launch(lbm_sim* sim, int32_t seg_rows);
lbm_status lbm_get_launch(const lbm_sim* sim, int32_t* seg_rows, int32_t* waves);

/* Time candidate launch shapes on this simulation (the state is saved and
 * restored around the trials) and keep the fastest.  best_ms receives the
 * best time per step (may be NULL). */
lbm_status lbm_autotune(lbm_sim* sim, int32_t steps_per_trial, double* best_ms);

/* ---- batched and served runs: a pool of channel slots -------------------
 *
 * A pool steps many independent channels (each with its own grid and
 * parameters, FP32 deviation storage) together: lbm_pool_run enqueues a
 * chunk of steps as one batched launch per step over every active slot.
 * Admission is by device footprint against the pool's byte cap; start-up and
 * read-out run on a second stream, so slots can be admitted and results read
 * while a chunk runs (continuous batching).  A slot's results are bitwise
 * those of the same channel run alone with lbm_create/lbm_step.
 *
 * A slot whose steps read a non-finite rho or T is retired: once the
 * counters copied at the end of a chunk show it (at the latest two chunks
 * after it happened) it takes no further steps, lbm_pool_poll reports it
 * as finished, and lbm_pool_moments returns LBM_EUNSTABLE for it.  The
 * other slots are not affected: a slot's step reads and writes only its
 * own memory. */

/* Device bytes one slot with these parameters holds (two population
 * buffers, two temperature planes); 0 if the parameters are invalid. */
size_t lbm_pool_footprint(const lbm_params* p);

/* Create an empty pool admitting up to cap_bytes of slot footprints;
 * stream: hipStream_t for the batched chunks, NULL for a private one. */
lbm_status lbm_pool_create(size_t cap_bytes, void* stream, lbm_pool** out);

/* Admit a channel that is to run nsteps steps.  rho0: host Nx*Ny initial
 * densities or NULL (uniform rho_v).  *slot receives its id.
 * LBM_ENOMEM when its footprint does not fit under the cap (the caller keeps
 * the request queued), LBM_EINVAL for invalid parameters or initial
 * densities (the checks of lbm_create) or a precision other than
 * LBM_FP32_DEV. */
lbm_status lbm_pool_admit(lbm_pool* pool, const lbm_params* p, const double* rho0,
                          int64_t nsteps, int32_t* slot);

/* Enqueue chunk_steps steps (asynchronous) for every slot with steps left;
 * a slot with fewer left takes only those. */
lbm_status lbm_pool_run(lbm_pool* pool, int32_t chunk_steps);

/* Block until at most max_pending enqueued chunks are still running (host
 * back-pressure for a serving loop that enqueues ahead of the device). */
lbm_status lbm_pool_wait(lbm_pool* pool, int32_t max_pending);

/* Non-blocking: ids of slots that have finished all their steps, or were
 * retired with a non-finite state, and were not reported before (at most
 * max of them) into done[], count in *ndone. */
lbm_status lbm_pool_poll(lbm_pool* pool, int32_t* done, int32_t max, int32_t* ndone);

/* rho, u, T of a slot at its current time level into host arrays of Nx*Ny
 * doubles (any may be NULL), as lbm_moments.  Waits for that slot only.
 * LBM_EUNSTABLE (arrays filled) when the slot's steps read a non-finite
 * state or its current level holds one. */
lbm_status lbm_pool_moments(lbm_pool* pool, int32_t slot, double* rho, double* ux, double* uy,
                            double* T);

/* The health counters of a slot (as lbm_health), after the work enqueued
 * for it so far.  Waits for that slot only. */
lbm_status lbm_pool_slot_health(lbm_pool* pool, int32_t slot, int64_t* nonfinite,
                                int64_t* psi_clamps);

/* Retire a slot; its footprint returns to the cap and its id may be reused. */
lbm_status lbm_pool_release(lbm_pool* pool, int32_t slot);

/* Destroy the pool and every slot in it; NULL is accepted. */
lbm_status lbm_pool_destroy(lbm_pool* pool);

/* Active slots, bytes in use and the cap (any pointer may be NULL). */
lbm_status lbm_pool_info(const lbm_pool* pool, int32_t* active, size_t* bytes_used,
                         size_t* cap_bytes);

/* Time level of a slot (after the work enqueued so far), -1 if no such slot. */
int64_t lbm_pool_slot_time(const lbm_pool* pool, int32_t slot);

/* Rows per wave of every slot's launch shape, capped at the slot's rows
 * (<= 0: the per-slot default, segments of at least 14 rows sized toward
 * one resident round of waves; this also drops a tuned policy). */
lbm_status lbm_pool_set_launch(lbm_pool* pool, int32_t seg_rows);

/* Time launch policies on the slots that have steps left (all admitted slots
 * if none has) and keep the fastest for them and for later admissions.  A
 * policy gives each bucket of fluid rows (up to 32, 64, 128, 256, more) a
 * target segment height, from 8 rows to whole slots; each slot then uses
 * segments of about that height, balanced over its rows.  The search times
 * the default heuristic, one target for all buckets, then each bucket
 * present in turn with the others fixed, steps_per_trial batched steps per
 * policy (after two untimed ones); the winner is kept only if it also beats
 * the default heuristic over three times the steps, each timed twice.  The trials step copies of the slots'
 * memory: states, counters and time levels are unchanged.  Blocks until the
 * pool's work is done; needs device memory for the copies (LBM_ENOMEM if
 * there is none, the policy then stays as it was).  best_ms (may be NULL)
 * receives the time per batched step of the chosen policy.  The results of
 * the steps do not depend on the policy (bitwise). */
lbm_status lbm_pool_autotune(lbm_pool* pool, int32_t steps_per_trial, double* best_ms);

/* Launch shape of a slot: rows per wave and waves per step. */
lbm_status lbm_pool_slot_launch(const lbm_pool* pool, int32_t slot, int32_t* seg_rows,
                                int32_t* waves);

/* Wait for all work of the pool. */
lbm_status lbm_pool_synchronize(lbm_pool* pool);

/* Plain device-to-device copy of `bytes` (rounded down to a multiple of 16)
 * repeated `iters` times on a private stream: achieved bandwidth counting
 * read + write (2 * bytes per copy) in GB/s, and the time per copy.  The
 * roofline denominator the step kernel is compared with, next to the vendor
 * peak; it allocates and frees two buffers of `bytes`. */
lbm_status lbm_bandwidth_probe(size_t bytes, int32_t iters, double* gbps, double* ms_per_copy);

#ifdef __cplusplus
}
#endif

#endif
