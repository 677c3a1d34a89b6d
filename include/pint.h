/*
 * pint.h -- C ABI of the MI355X spherical-harmonic shallow-water propagator
 * and its parallel-in-time drivers (arXiv 2306.09497).
 *
 * The library computes, on one AMD Instinct MI355X (gfx950), the IMEX time
 * step of the rotating shallow-water equations in vorticity/divergence/
 * geopotential form (Sec. 2.1, eq. swe_sphere), discretised with spherical
 * harmonics under triangular truncation on a Gauss grid (Sec. 2.2), and runs
 * it batched over many time slices inside Parareal (Sec. 3.1) and two- and
 * three-level MGRIT (Sec. 3.2).  Around that path: a server that runs many
 * such solves at once, the error norms and kinetic-energy spectrum of
 * Sec. 5 and the stability maps of Sec. 4, all on the device.
 *
 * Conventions shared by every entry point
 * ---------------------------------------
 * Spectral coefficients: Y_{m,n} = Pbar_n^m(mu) exp(i m lambda), mu = sin(lat),
 *   Pbar normalised to 1/2 int Pbar^2 dmu = 1, no Condon-Shortley phase; real
 *   fields keep m >= 0.  Packed m-major: idx(m,n) = m(2M+3-m)/2 + (n-m),
 *   0 <= m <= n <= M; ncoef = (M+1)(M+2)/2.  Each coefficient is complex,
 *   stored as two doubles (re, im).
 * State: three fields ordered (Phi, xi, delta) -- geopotential (in full: its
 *   (0,0) coefficient is the area mean), vorticity, divergence.  A batch of B
 *   states is [B][3][ncoef][2] doubles, batch-major.
 * Grid: lambda_k = 2 pi k / nlon; Gauss latitudes ordered north to south.  A
 *   batch of B grid fields is [B][nlat][nlon] doubles.
 * Memory: every state/grid pointer is DEVICE memory owned by the caller
 *   (e.g. a torch tensor's data_ptr); sizes are element counts as stated.
 *   Arrays passed to one call must not overlap unless said otherwise.
 * Streams: `stream` is a hipStream_t (NULL = the null stream).  All work is
 *   enqueued on it and the call returns without waiting, except where a call
 *   says it synchronises.
 * Errors: every call returns a pint_status and never aborts; a message for
 *   the calling thread is available from pint_last_error().  A plan is not
 *   thread-safe; distinct plans may be used from distinct threads.
 */
#ifndef PINT_H
#define PINT_H

#include <stddef.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  PINT_OK = 0,
  PINT_E_INVAL = -1,    /* invalid argument: message says which            */
  PINT_E_NOMEM = -2,    /* device allocation failed                         */
  PINT_E_HIP = -3,      /* a HIP runtime call failed                        */
  PINT_E_DIVERGED = -4, /* NaN/Inf or blow-up detected in a PinT iteration  */
  PINT_E_NOTCONV = -5   /* tolerance not reached within max_iter            */
} pint_status;

/* Operator switches (tests only; production uses PINT_T_ALL). */
enum {
  PINT_T_LG = 1,    /* linear gravity  L_G = (-Phibar delta, 0, -lap Phi)   */
  PINT_T_LC = 2,    /* linear Coriolis L_C = (0, -div(fV), k.curl(fV))      */
  PINT_T_NL = 4,    /* nonlinear N = N_A + N_R                              */
  PINT_T_VISC = 8,  /* backward-Euler (hyper)viscosity                      */
  PINT_T_ALL = 15
};

/* Arithmetic of the transforms (pint_config.precision).
 * PINT_FP64: every stage in FP64.
 * PINT_LEG_FP32: the Legendre GEMMs (FP32 operands on the FP32 matrix cores,
 *   FP32 accumulation), the Fourier intermediates and the ring FFTs with the
 *   pointwise tendencies run in FP32; the spectral state, the Crank-Nicolson
 *   solve, viscosity, the RK combine, table generation, the Parareal/MGRIT
 *   corrections and the norms stay FP64.
 * PINT_LEG_BF16X3: as PINT_LEG_FP32, except that each Legendre GEMM product
 *   runs on the BF16 matrix cores with both FP32 operands split into a BF16
 *   pair x = hi + lo and three products lo*hi + hi*lo + hi*hi accumulated in
 *   FP32 (relative rounding near 2^-16 per product).
 * The public scalar transforms (pint_synthesis, pint_analysis) stay FP64 in
 * every mode.  Every mode is deterministic and batch invariant.  */
enum { PINT_FP64 = 0, PINT_LEG_FP32 = 1, PINT_LEG_BF16X3 = 2 };

/* Truncation, grid and planet.  Requires M >= 1, nlat even, nlat >= M+2,
 * nlon >= 2M+2, nlon = 2^a 3^b 5^c <= 1024; the 3/2 rule (nlon >= 3M+3,
 * nlat >= (3M+3)/2) makes the quadratic terms alias-free (Sec. 2.2).
 * phibar is the constant mean geopotential Phibar of L_G (Sec. 2.1).
 * max_batch bounds the number of states one internal launch processes; the
 * plan's workspace is sized for it (larger calls are split into chunks).
 * precision is PINT_FP64, PINT_LEG_FP32 or PINT_LEG_BF16X3.  */
typedef struct {
  int M, nlon, nlat;
  double a, omega, g, phibar;
  int max_batch;
  int precision;
} pint_config;

/* One time stepper: IMEX step of size dt (Sec. 2.3.1, eq. IMEX), followed by
 * backward-Euler viscosity of even order q >= 2 and coefficient nu >= 0
 * (App. A; nu = 0 disables it).  `terms` is a PINT_T_* mask.  */
typedef struct {
  double dt;
  int visc_order;
  double visc_nu;
  unsigned terms;
} pint_stepper;

/* One semi-Lagrangian semi-implicit SETTLS stepper (Sec. 2.3.2): step size
 * dt, traj_iters fixed-point iterations of the departure-point estimate (eq.
 * SETTLS_trajectories; 2 is the usual choice, 0 leaves the departure points
 * at the arrival points), then backward-Euler viscosity of even order
 * visc_order >= 2 and coefficient visc_nu >= 0 (Sec. 2.3).  */
typedef struct {
  double dt;
  int traj_iters;
  int visc_order;
  double visc_nu;
} pint_sl_stepper;

typedef struct pint_plan pint_plan;

typedef struct {
  int M, nlon, nlat, ncoef, max_batch;
  size_t state_doubles;        /* 3 * ncoef * 2: doubles per state           */
  size_t workspace_bytes;      /* device memory the plan holds now           */
  long long allocations;       /* device allocations the plan made after its
                                  creation (driver scratch and factor sets)  */
  int gemm_shape[2][2];        /* Legendre GEMM launch shape in use, [synthesis,
                                  analysis][launches of few states, of many]:
                                  few states: 0 = k-slabs of 16, 1 = of 32;
                                  many, synthesis: 0 = 64-column tiles,
                                  1 = 128; many, analysis: 0 = 64 columns,
                                  1 = 64 with k-slabs of 32, 2 = 128 columns */
  double gemm_us[2][2];        /* the autotuner's time per launch of that shape
                                  (0 = not tuned)                            */
  int ring_threads[2];         /* ring kernel workgroup size for launches of
                                  one or two states, of more                 */
  double ring_us[2];           /* the autotuner's time per launch (0 = not
                                  tuned)                                     */
} pint_info;

/* Create a plan: Gauss nodes and weights (Newton iteration), normalised
 * associated Legendre tables and FFT twiddles are generated on the device in
 * FP64 (Sec. 2.2), and workspace for max_batch states is allocated.  The call
 * synchronises `stream` before returning.  On error *out is NULL.  */
pint_status pint_plan_create(const pint_config* cfg, void* stream, pint_plan** out);
pint_status pint_plan_destroy(pint_plan* plan);
pint_status pint_plan_info(const pint_plan* plan, pint_info* info);

/* Copy the Gauss latitudes to HOST memory: mu[nlat] (sin of latitude, north
 * to south) and w[nlat] (weights, sum 2).  Synchronises `stream`.  */
pint_status pint_grid_coords(pint_plan* plan, double* mu_host, double* w_host, void* stream);

/* Scalar spherical-harmonic transforms of B fields (Sec. 2.2: FFT in
 * longitude, Legendre transform in latitude).
 * synthesis: spec[B][ncoef][2] -> grid[B][nlat][nlon]
 * analysis:  grid[B][nlat][nlon] -> spec[B][ncoef][2]
 *            s_{m,n} = 1/2 sum_j w_j Pbar_n^m(mu_j) (1/nlon) sum_k s_jk e^{-i m lambda_k}  */
pint_status pint_synthesis(pint_plan* plan, const double* spec, double* grid, int B, void* stream);
pint_status pint_analysis(pint_plan* plan, const double* grid, double* spec, int B, void* stream);

/* Nonlinear tendencies N(U) = N_A(U) + N_R(U) (Sec. 2.1) of B states,
 * pseudospectral on the plan's grid (Sec. 2.2): u[B][3][ncoef][2] ->
 * n_out[B][3][ncoef][2].  The (0,0) coefficients of N_xi and N_delta are 0.  */
pint_status pint_tendency(pint_plan* plan, const double* u, double* n_out, int B, void* stream);

/* Crank-Nicolson half step of the linear terms (Sec. 2.3.1, eq.
 * IMEX_implicit): solves (I - dt/4 L) x = (I + dt/4 L) u, L = L_G + L_C
 * restricted by st->terms, with the Coriolis term implicit (per zonal
 * wavenumber two tridiagonal chains); then, if st->terms has PINT_T_VISC,
 * applies the viscosity factor 1/(1 + dt nu (n(n+1)/a^2)^(q/2)).
 * u and x are [B][3][ncoef][2]; x may alias u.  */
pint_status pint_implicit(pint_plan* plan, const pint_stepper* st, const double* u, double* x,
                          int B, void* stream);

/* The fine/coarse propagator, the hot path: nsteps IMEX steps (eq. IMEX,
 * CN half step, Heun explicit stage, CN half step, viscosity) applied
 * independently to each of B states (time slices).  u_in and u_out are
 * [B][3][ncoef][2]; u_out may alias u_in.  Results for a state do not depend
 * on B, on the other states or on how the steps are split between calls
 * (n steps in one call equal n one-step calls), bitwise.  */
pint_status pint_step(pint_plan* plan, const pint_stepper* st, const double* u_in, double* u_out,
                      int B, int nsteps, void* stream);

/* pint_step for callers that cannot allocate device memory (code under
 * HIP graph capture, tight serving loops, harnesses that forbid hipMalloc):
 * the same computation and the same results, bitwise, with every buffer
 * beyond u_in, u_out and the plan's tables -- the Crank-Nicolson factors of
 * st (made by a kernel in each call) and the transform workspace -- taken
 * from one static device array of the library, 64 MiB per device, held
 * until the process ends.  The call allocates and frees nothing and reads no
 * plan cache.  Its states are processed in chunks of the largest count, at
 * most max_batch, whose workspace fits the array; a state that does not fit
 * alone (26 MiB for one state at T255 with its factors, 46 MiB at T340; a
 * truncation above about T430 needs more than 64 MiB) is refused with
 * PINT_E_INVAL.
 * Every call on a device shares that device's array, so calls that overlap
 * in time on one device (different streams, or threads) race: order them.
 * The plan must have been created on the current device.  Arguments,
 * layouts and errors otherwise as pint_step.  */
pint_status pint_step_noalloc(pint_plan* plan, const pint_stepper* st, const double* u_in,
                              double* u_out, int B, int nsteps, void* stream);

/* nsteps SL-SI-SETTLS steps (Sec. 2.3.2, eqs. SETTLS_trajectories and
 * SL_SI_SETTLS) of B independent states.  Each step traces the trajectories
 * arriving at the Gauss grid points back to their departure points (in 3-D,
 * with the velocity 2 V^n - V^{n-1} extrapolated to t_{n+1/2}), interpolates
 * R_Phi = Phi' - dt/2 Phibar delta + dt/2 (2 N_R^n - N_R^{n-1}) and the wind
 * R_V = V - dt/2 (grad Phi' + f k x V) there (bicubic on the Gauss grid,
 * rows mirrored across the poles, vectors by Cartesian components turned into
 * the arrival frame), adds dt/2 N_R^n at the arrival points and solves
 * (I - dt/2 L) U^{n+1} = (R_Phi*, curl R_V*, div R_V*) per zonal
 * wavenumber; N_R = -Phi' delta.
 * u_prev = NULL: the first step is the one-step variant of Sec. 3.2.4 (U^{n-1}
 * replaced by U^n); otherwise u_prev holds U^{n-1}.  Later steps use the
 * two-step scheme.  out receives U^{n+nsteps}, and out_prev (if not NULL)
 * U^{n+nsteps-1}, so that a later call can continue the two-step scheme.
 * All state arrays are [B][3][ncoef][2] device memory; out and out_prev may
 * alias u but not each other.  The plan must be PINT_FP64 with
 * max_batch >= 2 (two states per trajectory are transformed together);
 * larger B is processed in chunks of max_batch / 2.  Results for a state do
 * not depend on B or the other states.  PINT_E_INVAL for bad arguments.  */
pint_status pint_sl_steps(pint_plan* plan, const pint_sl_stepper* st, const double* u_prev,
                          const double* u, double* out, double* out_prev, int B, int nsteps,
                          void* stream);

/* Parareal (Sec. 3.1) with the fine IMEX propagator (fine_steps steps of
 * `fine` per slice, on `plan`) and an SL-SI-SETTLS coarse propagator
 * (coarse_steps steps of `coarse` per slice, on coarse_plan, or on `plan`
 * when coarse_plan is NULL; a coarse plan of lower truncation works on the
 * truncated states and pads its results with zeros), for n_inst independent
 * instances (initial states) at once.  The serial coarse sweep is the
 * coarsest level, where the two-step scheme runs in every step (Sec. 3.2.4):
 * with restart = 0 each slice's coarse run starts from the corrected slice
 * state and the last-but-one coarse state of the previous slice's run, and
 * only the first step of the horizon takes the one-step variant; restart = 1
 * takes the one-step variant at every slice start (as on a level whose
 * slices belong to different processors).
 * n_iter iterations; iteration k recomputes slices k..N-1 only (slice k's
 * input is converged).  u0 is [n_inst][3][ncoef][2]; u_slices is
 * [n_slices + 1][n_inst][3][ncoef][2] and receives the slice-boundary
 * states, u_slices[0] = u0.  Results of an instance do not depend on the
 * others.  Runs on `stream` alone; the coarse plan must be PINT_FP64 with
 * max_batch >= 2 and share the planet and Phibar of `plan`.  The driver's
 * scratch is kept in the plan and grown on first use.  */
pint_status pint_parareal_sl(pint_plan* plan, const pint_stepper* fine, int fine_steps,
                             pint_plan* coarse_plan, const pint_sl_stepper* coarse,
                             int coarse_steps, int n_slices, int n_inst, int n_iter, int restart,
                             const double* u0, double* u_slices, void* stream);

/* Parallel-in-time solve of dU/dt = L U + N(U) on [0, n_intervals * DT].
 * method 0 = Parareal (Sec. 3.1): slices of length DT = fine.dt *
 *   fine_steps = coarse.dt * coarse_steps; fine propagator = fine_steps
 *   fine steps, coarse propagator = coarse_steps coarse steps.
 * method 1 = MGRIT with F(CF)^nrelax relaxation and FAS (Sec. 3.2):
 *   fine level = fine.dt, cfactor = fine_steps fine steps per C-interval,
 *   level 1 = coarse_steps coarse steps per C-interval.
 *   levels = 2 (or 0): the level-1 problem is solved by a serial sweep.
 *     With nrelax = 0 it is identical to Parareal.
 *   levels = 3 (multilevel recursion, Sec. 3.2): the level-1 problem (the
 *     level-1 propagator plus the FAS forcing) is solved approximately by
 *     cycles1 two-level MGRIT iterations on levels 1 and 2, starting from
 *     the injected C-points: F(CF)^nrelax relaxation of level 1, level-2
 *     points every cfactor1 level-1 points (n_intervals divisible by
 *     cfactor1), level-2 propagator = coarse2_steps steps of coarse2
 *     spanning cfactor1 level-1 intervals, serial level-2 solve, then an
 *     F-relaxation of level 1.  cycles1 = 1 is a V-cycle; the paper's
 *     F-cycle followed by a post V-cycle reads as cycles1 = 2.  Every update
 *     is formed difference first, (Phi(w) - Phi(v)) + F, so exact slices
 *     stay bitwise exact (finite termination as with two levels).
 * Iterates until the largest relative L2 increment of a slice state is
 * <= tol, or max_iter iterations (tol = 0: exactly max_iter).  The increment
 * of a slice is the larger of the relative changes of Phi' (Phi without its
 * mean) and of the wind (vorticity and divergence through the velocity they
 * induce), both area-weighted L2 norms (see pint_rel_diff).  u_slices[(n_intervals+1)][3][ncoef][2] receives the
 * states at the slice (C-point) boundaries; u0 is its initial state.
 * Synchronises `stream` once per iteration (to read the increment).  The
 * plan keeps the drivers' scratch (about 3 n_intervals + 2 states, more with
 * three levels) between calls and grows it only when a call needs more.  */
typedef struct {
  int method;             /* 0 Parareal, 1 MGRIT two-level                    */
  int n_intervals;        /* N slices / C-intervals                           */
  pint_stepper fine;      /* fine propagator step                             */
  int fine_steps;         /* fine steps per slice (= MGRIT cfactor)            */
  pint_stepper coarse;    /* coarse propagator step                           */
  int coarse_steps;       /* coarse steps per slice                           */
  int nrelax;             /* MGRIT F(CF)^nrelax; ignored by Parareal          */
  int max_iter;
  double tol;
  int resume;             /* 1: u_slices already holds an iterate (all
                             n_intervals+1 states, e.g. a checkpoint); skip
                             the initial coarse sweep and continue from it  */
  int levels;             /* MGRIT levels: 0 or 2 (two-level), 3          */
  int cfactor1;           /* levels 3: level-1 points per level-2 interval */
  pint_stepper coarse2;   /* levels 3: level-2 propagator step             */
  int coarse2_steps;      /* levels 3: coarse2 steps per level-2 interval  */
  int cycles1;            /* levels 3: cycles on levels (1, 2) per
                             iteration, >= 1                              */
  pint_plan* coarse_plan; /* NULL: coarse levels at the plan's truncation.
                             Otherwise spatial coarsening (Sec. 5): every
                             coarse-level step runs on this plan (truncation
                             Mc <= M, same planet and Phibar) as
                             pad(step(truncate(u))): coefficients with
                             n > Mc are dropped before and zero after it.
                             The difference-first updates then keep the
                             fine values of those coefficients exactly.
                             A coarse plan at the fine truncation (Mc = M)
                             runs the coarse levels directly on it, e.g. in
                             a reduced transform precision while the fine
                             propagator stays FP64 (the converged iterate
                             is still the FP64 fine solution); one of the
                             plan's own truncation and precision adds
                             nothing and is ignored (the coarse levels run
                             on the plan itself).
                             Not thread-safe with other calls on either
                             plan.                                         */
  const pint_sl_stepper* coarse_sl; /* NULL: coarse level IMEX (`coarse`).
                             Otherwise two-level MGRIT (method 1, levels 2)
                             with an SL-SI-SETTLS coarse level (Sec. 2.3.2)
                             of one step of this stepper per C-interval
                             (coarse_steps = 1, coarse_sl->dt = fine.dt *
                             fine_steps; `coarse` is not used), on the plan
                             itself (coarse_plan NULL; PINT_FP64 plan with
                             max_batch >= 2).  The coarse level is the
                             coarsest, so every coarse step is the two-step
                             scheme (Sec. 3.2.4): its history is the
                             previous point of the coarse sequence it
                             continues (the relaxed C-point i-1 for the
                             coarse value of C-point i, the corrected point
                             i-1 in the serial solve), and only the first
                             point of the horizon takes the one-step
                             variant.  A converged prefix then stays exact
                             (finite termination holds).  The iteration
                             runs on `stream` alone (no overlap of the
                             sweep with the fine propagation).             */
} pint_pint_params;

typedef struct {
  int iters;                     /* iterations performed                      */
  double incr[128];              /* max relative increment per iteration (the
                                    stopping measure: Phi' and the wind)      */
  double incr_field[128][4];     /* per iteration, the largest relative
                                    increment over slices of Phi', xi, delta
                                    and the wind, each on its own             */
  double seconds[128];           /* host wall time per iteration              */
  double fine_seconds[128];      /* device time from the iteration's start to
                                    the end of its batched fine propagation
                                    (relaxation included)                     */
  double coarse_seconds[128];    /* device time from the iteration's start to
                                    the end of its serial coarse part (the
                                    correction sweep, or the level-1 cycles
                                    with three levels); it runs beside the
                                    fine propagation, so the iteration takes
                                    about the larger of the two.  For an
                                    iteration replayed from a graph both hold
                                    the graph's device time                  */
  long long fine_slice_steps;    /* fine IMEX steps executed (sum over slices)*/
  long long coarse_steps;        /* coarse IMEX steps executed (all coarse
                                    levels, single-state and batched)        */
  int graph_iters;               /* iterations replayed from a HIP graph: an
                                    iteration that repeats the launches of the
                                    one before (MGRIT, or Parareal resumed,
                                    which recompute every slice) is captured
                                    once and replayed, bitwise the same       */
} pint_report;

pint_status pint_solve(pint_plan* plan, const pint_pint_params* p, const double* u0,
                       double* u_slices, pint_report* report, void* stream);

/* Device footprint of a workload on a plan, and its reservation (the problem
 * statement of Sec. 3: slices, fine and coarse propagators, levels).
 * pint_plan_workspace_bytes writes to *bytes the device memory the plan
 * holds once it is ready for
 *   - pint_solve with parameters q (q may be NULL): its driver scratch
 *     (about 3 n_intervals + 2 states, more with three levels or spatial
 *     coarsening) and the Crank-Nicolson factors of its steppers -- those of
 *     the coarse levels counted even when they live on q->coarse_plan; and
 *     pint_step / pint_implicit with q->fine or q->coarse;
 *   - pint_sl_steps with stepper sl (may be NULL): grid scratch for
 *     max_batch / 2 state pairs and the (I - dt/2 L) factors,
 * plus the tables and workspace made at creation.  It is a pure function of
 * the plan's configuration and the arguments.  pint_plan_reserve allocates
 * exactly that (enqueueing the factor kernels on `stream`) and then tunes the
 * plan's Legendre GEMM launch shapes for the workload: it times every shape
 * of each transform at one state per launch (the serial sweep's launches)
 * and at min(n_intervals, max_batch) states (max_batch without q), keeps the
 * fastest (on the coarse plan too) -- likewise the ring kernel's workgroup
 * size -- and synchronises `stream`.  The shapes
 * give bitwise the same results, so tuning never changes an answer;
 * pint_info.gemm_us reports the tuned times.  Afterwards those
 * calls allocate and free no device memory and copy nothing to or from the
 * host, and on a plan that had reserved nothing else
 * pint_info.workspace_bytes equals the query.  Reserving is optional: the
 * calls otherwise grow the same buffers on first use.  A server admits a
 * request by the same footprint (its driver scratch plus the slice states).
 * PINT_E_INVAL for invalid parameters, PINT_E_NOMEM if allocation fails.  */
pint_status pint_plan_workspace_bytes(const pint_plan* plan, const pint_pint_params* q,
                                      const pint_sl_stepper* sl, size_t* bytes);
pint_status pint_plan_reserve(pint_plan* plan, const pint_pint_params* q,
                              const pint_sl_stepper* sl, void* stream);

/* Relative L2 differences used by the stopping test: for each of B state
 * pairs, out[b] = { ||dPhi'||/||Phi'||, ||dxi||/||xi||, ||ddelta||/||delta||,
 * ||dV||/||V|| } of a_b against c_b (d = a - c, norms of a), with the
 * area-weighted spectral norm (Parseval; Phi without its (0,0) coefficient)
 * and the wind norm ||V||^2 = sum_{n>=1} w a^2/(n(n+1)) (|xi|^2 + |delta|^2),
 * w = 1 for m = 0, 2 for m > 0.  a, c are device [B][3][ncoef][2]; out is
 * HOST [B][4].  Synchronises `stream`.  */
pint_status pint_rel_diff(pint_plan* plan, const double* a, const double* c, double* out_host,
                          int B, void* stream);

/* Kinetic-energy spectrum of a triangular truncation (Sec. 5.1, Gaussian bumps
 * test case, after Koshyk and Hamilton): for each of B states
 *   e[b][n] = a^2 / (4 n (n+1)) * sum_{m=-n..n} (|xi_{m,n}|^2 + |delta_{m,n}|^2),
 * n = 0..M, e[b][0] = 0; the m < 0 coefficients of a real field are the
 * conjugates of the stored m > 0 ones.  u: device [B][3][ncoef][2]; e: device
 * [B][M+1].  Asynchronous on `stream`.  */
pint_status pint_ke_spectrum(pint_plan* plan, const double* u, double* e, int B, void* stream);

/* Spectral max-norm errors (Sec. 5, eq. error_definition) of B states u
 * against B references ref, for psi = Phi' (Phi - phibar), xi, delta and
 * every resolution R = 0..M at once:
 *   e[b][f][R] = max_{0<=m<=n<=R} |u - ref| / max_{0<=m<=n<=R} |ref|,
 * 0 where difference and reference are both zero, +inf for a nonzero
 * difference on a zero reference.  u, ref: device [B][3][ncoef][2]; e: device
 * [B][3][M+1].  Needs M <= 511 (PINT_E_INVAL otherwise).  Asynchronous.  */
pint_status pint_spectral_errors(pint_plan* plan, const double* u, const double* ref, double* e,
                                 int B, void* stream);

/* Physical-space relative L2 errors (Sec. 5, the equation after
 * error_definition): for psi = Phi' (Phi - phibar), xi, delta,
 *   out[b][f] = sqrt( sum_nodes (psi - psi_ref)^2 / sum_nodes psi_ref^2 ),
 * the unweighted sums over the nodes of the plan's Gauss grid (the grid
 * means of the printed formula, whose 1/(nlat nlon) cancels); 0 / 0 gives 0
 * and x / 0 gives +inf.  u, ref: device [B][3][ncoef][2]; out: HOST [B][3].
 * Uses the plan's transform workspace (do not overlap with other calls on
 * the plan); synchronises `stream`.  */
pint_status pint_grid_l2_errors(pint_plan* plan, const double* u, const double* ref,
                                double* out_host, int B, void* stream);

/* Stability maps (Sec. 4): max |A| over a grid of xi_N = lambda_N dt for the
 * scalar test equation u' = (lambda_L + lambda_N) u, written to out (device,
 * [nim][nre], row r at Im xi_N = im0 + r (im1 - im0)/(nim - 1), column c at
 * Re xi_N = re0 + c (re1 - re0)/(nre - 1)).
 *   kind 0: the coarse scheme alone, one step: IMEX (Sec. 4.1.1, Heun
 *     keeping U*), or SL-SI-SETTLS: both roots of eq.
 *     stability_SL_SI_SETTLS for ks = 2 pi j / n_ks, j = 0..n_ks;
 *   kind 1: two-level MGRIT with F(CF)^nrelax relaxation (nrelax = 0 is
 *     Parareal) after k iterations at slice n: the closed form of the
 *     recurrence eq. parareal_FCF_nrelax_B, sum_{i<=k} C(n - i nu, i) S^i
 *     R^(n - i(nu+1)), S = F^nu (F - R), with an IMEX fine propagator
 *     F = A_IMEX(xi/cfactor)^(cfactor n_c) and the coarse scheme
 *     R = A_c^(n_c); for SL-SI-SETTLS the maximum over both roots and all
 *     ks.
 * xi_L and xi_N are on the coarse step.  Asynchronous; no plan needed.  */
typedef struct {
  int kind;                  /* 0 scheme alone, 1 two-level MGRIT / Parareal   */
  int coarse;                /* 0 IMEX, 1 SL-SI-SETTLS                         */
  double xl_re, xl_im;       /* xi_L                                           */
  double re0, re1;           /* Re xi_N range                                  */
  int nre;                   /* >= 1 columns                                   */
  double im0, im1;           /* Im xi_N range                                  */
  int nim;                   /* 1..65535 rows; nre nim <= 2^28                 */
  int n, k;                  /* slice n >= 0, iterations 0 <= k <= 64         */
  int cfactor, n_c;          /* >= 1: fine steps per coarse step, coarse steps */
  int nrelax;                /* 0..8                                           */
  int n_ks;                  /* >= 1 phases for SL-SI-SETTLS                   */
} pint_stability_cfg;

pint_status pint_stability_map(const pint_stability_cfg* cfg, double* out, void* stream);

/* ---- Serving with continuous batching ------------------------------------
 * A server runs many Parareal / two-level MGRIT solves (Sec. 3, the
 * iteration of pint_solve) at once: plan 0's work on the stream given at
 * creation, each other plan's on a stream the server creates.  Each tick advances every
 * running request's pending propagation by one chunk of at most
 * steps_per_tick IMEX steps, and all chunks of one plan with the same
 * stepper and length run as one batched propagation: fine propagations of
 * different requests share launches, and so do the serial coarse sweeps of
 * different requests.  A request's chunks depend only on its own step
 * counts and the propagator is batch invariant, so its result is bitwise
 * the same alone and in any mix.  Request state (the pint_solve driver
 * scratch that pint_plan_workspace_bytes counts for its parameters, plus its
 * n_intervals + 1 slice states: 4 n_intervals + 3 states)
 * lives in a device arena of arena_bytes allocated at creation; requests are
 * admitted first in first out when their state fits, and nothing is
 * allocated while serving.  The plans are borrowed: they must outlive the
 * server and must not be used by other calls while it runs.  Not thread
 * safe.  Errors as for the other entry points; a request larger than the
 * arena is refused at submission with PINT_E_NOMEM.  */
typedef struct pint_server pint_server;

typedef struct {
  int n_plans;               /* plans (truncations) requests may use          */
  pint_plan* const* plans;   /* [n_plans], borrowed                           */
  size_t arena_bytes;        /* device bytes for request state                */
  int steps_per_tick;        /* >= 1: IMEX steps per chunk                    */
  int stage_states;          /* >= 1: per-plan staging buffer (states) for
                                merged launches                               */
} pint_server_config;

typedef struct {
  int plan;                  /* index into pint_server_config.plans           */
  pint_pint_params params;   /* method 0 or 1, levels 2, no coarse_plan,
                                resume 0                                       */
  const double* u0;          /* device [3][ncoef][2]; read at admission, so it
                                must stay valid until the request runs        */
  double* u_slices;          /* device [(n_intervals+1)][3][ncoef][2], written
                                when the request completes                    */
} pint_request;

enum { PINT_REQ_QUEUED = 0, PINT_REQ_RUNNING = 1, PINT_REQ_DONE = 2, PINT_REQ_FAILED = 3 };

typedef struct {
  int state;                 /* PINT_REQ_*                                    */
  int status;                /* PINT_OK, PINT_E_NOTCONV (tol not reached: the
                                result is still written), PINT_E_DIVERGED
                                (state FAILED)                                 */
  int iters;                 /* iterations performed                          */
  double incr;               /* last stopping increment (as pint_report)      */
  double t_submit, t_start, t_done;  /* seconds on the server clock           */
  long long fine_slice_steps, coarse_steps;
} pint_request_status;

pint_status pint_server_create(const pint_server_config* cfg, void* stream, pint_server** out);
pint_status pint_server_destroy(pint_server* server);
/* Queue a request (validated as pint_solve's parameters); *id identifies it. */
pint_status pint_server_submit(pint_server* server, const pint_request* req, long long* id);
/* Admit what fits, advance every running request by one chunk, finish what
 * completed; *pending = requests queued or running afterwards.  Synchronises
 * the server's streams once (and a plan's stream once per completed
 * iteration, for the increments). */
pint_status pint_server_tick(pint_server* server, int* pending);
pint_status pint_server_status(pint_server* server, long long id, pint_request_status* st);
/* Seconds since the server was created (the clock of the time stamps). */
pint_status pint_server_clock(pint_server* server, double* t);

/* Kernel timing for measurement.  While enabled, every kernel launch of the
 * plan whose kind is in kind_mask (bit 1 << kind) and that processes at least
 * min_batch states is bracketed by HIP events on its stream (kind_mask = 0
 * disables timing); pint_profile_read
 * synchronises `stream`, sums the elapsed times per (kind, batch) and resets
 * the record.  kind: 0 spectral prep, 1 Legendre synthesis GEMM, 2 ring
 * FFT + tendencies, 3 Legendre analysis GEMM, 4 tendency assembly + RK
 * combine, 5 Crank-Nicolson solve, 6 layout conversion, 7 PinT update and
 * norms, 8 scalar-transform and semi-Lagrangian rings, 9 semi-Lagrangian
 * grid-point kernels (trajectories and interpolation).  out has room for cap entries; *n
 * receives the number written.  */
typedef struct {
  int kind;
  int batch;             /* states per launch                                 */
  long long launches;
  double total_ms;
} pint_prof_entry;

pint_status pint_profile_enable(pint_plan* plan, unsigned kind_mask, int min_batch);
pint_status pint_profile_read(pint_plan* plan, pint_prof_entry* out, int cap, int* n,
                              void* stream);

const char* pint_last_error(void);

#ifdef __cplusplus
}
#endif
#endif /* PINT_H */
