/*
 * hrlb.h -- C ABI of the MI355X half-range lattice Boltzmann solver for planar Couette flow
 * (Ambrus, Sharipov, Sofonea, arXiv:1810.07803).
 *
 * The library advances the reduced Shakhov equations (Sec. II, equation boltz_red) for the two
 * reduced distributions phi and chi on a mixed velocity set HHLB(Nx;Qx) x HLB(Ny;Qy)
 * (Sec. III): half-range Gauss-Hermite on the wall-normal axis p_x, full-range Gauss-Hermite on
 * p_y.  Space: WENO-5 finite differences on the stretched grid of equation (stretch), over the
 * full channel x in [-1/2, 1/2] or, using the point symmetry of Sec. II, its right half [0, 1/2]
 * (hrlb_case_params.half_channel).  Time: third-order TVD (SSP) Runge-Kutta, optionally with
 * local time steps for steady states (local_dt_cap).  Walls: diffuse reflection, equations
 * (diffuse) and (diffuse_nw); the left wall moves with -u_w, the right one with +u_w, both at T_w.
 *
 * Units: m = K_B = L = 1, average density n_ref = 1, reference momentum p0 = 1.  With these,
 * the relaxation time of equation (tau) with mu ~ T^omega is
 *     tau = (T/T_w)^(omega-1) / (n delta sqrt(2)) / sqrt(T_w),
 * and with the tabulated law of equations (mun), (interp) mu(T)/mu(T_w) replaces (T/T_w)^omega.
 *
 * Velocity ordering (also used by every host array below):
 *     v = (h*Qx + i)*Qy + j,  p_x = +z_i (h = 0) or -z_i (h = 1),  p_y = y_j ascending,
 * where z_i are the positive half-range nodes (ascending) and y_j the full-range nodes.
 * Host population arrays are [2][Nv][n_cells] doubles: phi first, then chi, cells contiguous.
 *
 * Conventions for every call:
 *   - No exception crosses the ABI.  Every call returns an hrlb_status; negative values are
 *     errors, HRLB_NOT_CONVERGED (positive) leaves the case valid.  hrlb_last_error() returns
 *     a thread-local message describing the last failure on the calling thread.
 *   - The caller owns every buffer it passes in (host arrays, the device workspace and the
 *     stream).  The library never frees caller memory.  Objects returned through "out"
 *     pointers are owned by the library and released by the matching hrlb_free_* call.
 *   - A case is bound to the stream given at creation and is not thread-safe; calls on one case
 *     must not overlap.  Different cases may be used from different threads.
 *   - Device work is enqueued asynchronously on the case's stream unless stated otherwise.
 */
#ifndef HRLB_H
#define HRLB_H

#include <stddef.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    HRLB_OK = 0,
    HRLB_NOT_CONVERGED = 1, /* run_to_steady hit max_steps; state valid and readable     */
    HRLB_E_INVALID = -1,    /* an argument is out of range or inconsistent             */
    HRLB_E_NOMEM = -2,      /* workspace too small, or host allocation failed          */
    HRLB_E_DEVICE = -3,     /* a HIP runtime call failed                               */
    HRLB_E_DIVERGED = -4,   /* NaN/Inf in the residual; the state is not meaningful      */
    HRLB_E_RANGE = -5       /* a cell left the band in which the truncated equilibrium of eq. (gx) is
                             * evaluated to 2e-13 (0.3 <= T/T_w <= 2.4, |u_x| <= sqrt(T_w)); the state
                             * stays readable, but its accuracy is no longer the stated one        */
} hrlb_status;

/* bits of hrlb_case_flags */
enum { HRLB_FLAG_NONFINITE = 1u, HRLB_FLAG_RANGE = 2u };

enum { HRLB_FP64 = 0, HRLB_FP32_STORE_FP64_MOM = 1 };
enum { HRLB_ROUND_NEAREST = 0, HRLB_ROUND_STOCHASTIC = 1 };
enum { HRLB_STOP_RESIDUAL = 0, HRLB_STOP_PXY = 1, HRLB_STOP_PXY_ERR = 2 };
enum { HRLB_PATH_AUTO = 0, HRLB_PATH_TILED = 1, HRLB_PATH_SMALL = 2 };

typedef struct hrlb_quad hrlb_quad;   /* immutable velocity set; may be shared by many cases */
typedef struct hrlb_case hrlb_case;   /* one Couette problem resident in a device workspace */
typedef struct hrlb_batch hrlb_batch; /* several cases advanced by the same kernel launches */

/* Velocity set HHLB(Nx_order;Qx) x HLB(Ny_order;Qy) (Sec. III, model naming after eq. gy).
 * Qx: half-range order (nodes per semi-axis), 3 <= Qx <= 128; Qy: full-range order, 3..64.
 * Nx_order, Ny_order: expansion orders of the equilibrium truncations (eq. gx and eq. gy),
 * 2 <= Nx_order <= min(Qx-1, 16), 2 <= Ny_order <= Qy-1.  p0 must be 1 (the units above).
 * Host-only: computes the nodes and weights in extended precision, no device work.
 * *out receives a library-owned object; release with hrlb_free_quadrature after every case
 * using it has been freed. */
hrlb_status hrlb_init_quadrature(int Qx, int Nx_order, int Qy, int Ny_order, double p0, hrlb_quad **out);

/* Copies the velocity set to caller host buffers: px, wx [2*Qx] (p_x values and half-range
 * weights in h-major order), py, wy [Qy].  Any pointer may be NULL. */
hrlb_status hrlb_quadrature_nodes(const hrlb_quad *q, double *px, double *wx, double *py, double *wy);

typedef struct {
    double delta;     /* rarefaction parameter, eq. (delta); 0 selects collisionless flow      */
    double u_w;       /* wall speed along y (left wall -u_w, right wall +u_w), |u_w| <= 2 sqrt(T_w) */
    double T_w;       /* wall temperature (> 0) in the units of p0^2/(m K_B): the velocity set is  */
                      /* fixed by p0 = 1, and eq. (gx) is evaluated with an auxiliary rule scaled */
                      /* to T_w, verified for cells with 0.3 <= T/T_w <= 2.4 and |u_x| <= sqrt(T_w) */
                      /* (HRLB_E_RANGE / HRLB_FLAG_RANGE outside)                                  */
    double Pr;        /* Prandtl number of the Shakhov model, > 0                             */
    double omega;     /* viscosity index of eq. (mu): mu ~ T^omega                             */
    int n_cells;      /* cells across the channel (its right half when half_channel is set):    */
                      /* a multiple of 4, 8 <= n_cells <= 65536                                 */
    double stretch_A; /* grid stretching of eq. (stretch), 0 <= A < 1 (0 = uniform)           */
    int precision;    /* HRLB_FP64 or HRLB_FP32_STORE_FP64_MOM                                 */
    int rounding;     /* FP32 storage only: HRLB_ROUND_NEAREST or HRLB_ROUND_STOCHASTIC        */
    double cfl;       /* used when dt <= 0: dt = min(cfl min(J deta)/max|p_x|, tau_w/2)       */
    double dt;        /* time step; <= 0 selects the rule above                               */
    unsigned seed;    /* key of the counter-based generator used by stochastic rounding       */
    int tile_vpt;     /* velocities per thread row of the stage kernel: a divisor of Qy up to  */
                      /* 16; 0 = automatic (largest divisor <= 8 that fills a tile's 16 rows). */
                      /* The choice fixes the summation order of the moments, so a case gives  */
                      /* bitwise the same numbers alone and in any batch for a given tile_vpt. */
    int cell_lanes;   /* lanes per cell of the per-cell kernel: 1, 2, 4, 8 or 16; 0 = automatic */
                      /* (2).  Also part of the plan that fixes the summation order.            */
    int half_channel; /* 0: full channel [-1/2, 1/2] with two diffuse walls.  1: the right half   */
                      /* [0, 1/2] only, using the point symmetry of Sec. II (phi and chi are     */
                      /* unchanged by x, p_x, p_y -> -x, -p_x, -p_y): the ghost cells left of    */
                      /* x = 0 hold the mirrored velocities of the first cells, one diffuse wall */
                      /* at x = 1/2, and the grid of eq. (stretch) on eta in [0, artanh A] as in */
                      /* Sec. III.  Same flow as the full channel with 2 n_cells cells, half the */
                      /* work per step.                                                          */
    /* Transport law.  visc_table_n = 0: eq. (mu) with omega above and the constant Pr.
     * visc_table_n in [2, 256]: the tabulated law of eqs. (mun) and (interp), Sec. II.  Rows
     * (visc_T[k], visc_mu[k], visc_Pr[k]): temperatures in the units of T_w, strictly increasing and
     * positive; viscosities in any unit (only ratios enter); Prandtl numbers Pr_k = c_p mu_k / kappa_k
     * from the tabulated heat conductivity.  Between consecutive rows mu is the power law through
     * both values; below the second row the first interval's law and above the last row the last
     * interval's law are extended.  Pr is Pr_k on [T_k, T_{k+1}), the first value below the second
     * row and the last value from the last row on.  eq. (tau) then uses mu(T)/mu(T_w) and the
     * Shakhov factor Pr(T) per cell; omega and Pr are ignored.  The arrays are host memory, copied
     * by hrlb_init_case (and by hrlb_server_submit); the caller keeps ownership. */
    int visc_table_n;
    const double *visc_T, *visc_mu, *visc_Pr;
    /* Steady-state acceleration (not in the paper).  0 (or 1): every cell advances with dt.  > 1: local
     * time steps, cell s advancing with dt_s = dt max(1, min(J_s/min J, local_dt_cap, tau_w/(2 dt)))
     * (J_s deta the cell width, tau_w = tau(n = 1, T_w), no tau term when collisionless), so every
     * cell runs at the Courant number of the smallest one.  The transient is then not time-accurate
     * and does not conserve mass: every checked step (hrlb_run_to_steady, hrlb_batch_step with check,
     * the server's rounds) rescales the populations to the rest-state mass sum_s J_s deta and
     * recomputes the moments.  The residual becomes ||(f_new - f_old)/dt_s|| / ||f_old||.  The
     * fixed point R(f) = 0, and so the steady state, is the one of the global step.  At most 1e6. */
    double local_dt_cap;
    /* Kernels that advance the case.  HRLB_PATH_TILED: two launches per Runge-Kutta stage over tiles of
     * 64 cells x 16 velocity rows (every case, any size).  HRLB_PATH_SMALL: one launch per block of steps
     * in which one workgroup holds the whole case (populations, stage buffers, tables) in its LDS (as
     * much as the device gives a workgroup: 160 KB on MI355X), for cases of a few thousand cell-velocity
     * units whose tiled steps are bound by launch latency;
     * HRLB_E_INVALID if the case does not fit.  HRLB_PATH_AUTO (0): the small path when the case fits.
     * The two paths sum the moments in different orders; a case takes its path alone and in any batch,
     * so it keeps its bits there. */
    int kernel_path;
} hrlb_case_params;

/* Device workspace size (bytes) needed by a case with these parameters. */
hrlb_status hrlb_case_workspace_bytes(const hrlb_quad *q, const hrlb_case_params *p, size_t *bytes);

/* Creates a case inside the caller's device workspace (at least the size reported above,
 * 256-byte aligned) on the caller's HIP stream (hipStream_t passed as void*, NULL = default
 * stream).  The state starts at the rest equilibrium n = 1, u = 0, T = T_w.  The workspace
 * must stay allocated and untouched until hrlb_free_case.  Enqueues uploads on the stream. */
hrlb_status hrlb_init_case(const hrlb_quad *q, const hrlb_case_params *p, void *dev_workspace,
                           size_t ws_bytes, void *hip_stream, hrlb_case **out);

/* For callers that cannot allocate device memory (code under HIP graph capture, tight serving
 * loops, harnesses that forbid allocation): a case like hrlb_init_case's whose caller passes device
 * memory for the populations only.  dev_state (256-byte aligned, at least hrlb_case_state_bytes;
 * caller-owned, untouched until the case is freed) holds the three state buffers f^0, f^1, f^2,
 * each [2][Nv][n_cells] in the storage precision (phi then chi).  Everything else of the case -- its
 * descriptor, tables, per-cell tables, fields, moment and residual partial sums, work lists and
 * counters -- lives in the library's static scratch: one 32 MiB array per device, held until the
 * process ends.  Allocates no device memory (no hipMalloc, hipFree or allocating routine; it uploads
 * the tables and clears the counters in the scratch, which keeps the last contents otherwise).
 * Every call on a device shares that device's scratch: one such case per device at a time.  Creating
 * another one on the same device replaces the first, whose calls then return HRLB_E_INVALID; work of
 * the first still in flight on a stream when the second is created races with the second's set-up.
 * HRLB_E_INVALID also when the case's auxiliary data exceed the scratch (larger cases use
 * hrlb_init_case).  The case works with every call that takes a case, batches included. */
hrlb_status hrlb_case_state_bytes(const hrlb_quad *q, const hrlb_case_params *p, size_t *bytes);
hrlb_status hrlb_init_case_static(const hrlb_quad *q, const hrlb_case_params *p, void *dev_state,
                                  size_t state_bytes, void *hip_stream, hrlb_case **out);

/* Enqueues n_steps >= 0 full SSP-RK3 steps (three stages each) on the case's stream. */
hrlb_status hrlb_step(hrlb_case *c, long n_steps);

typedef struct {
    long steps;        /* steps taken by this call                                          */
    double residual;   /* last residual: ||f_new - f_old||/(dt ||f_old||), J-weighted L2     */
    double pxy_drift;  /* last |dPxy_mean/dt| / |Pxy_mean| over one check window             */
    double sim_time;   /* total simulated time of the case                                   */
    double wall_s;     /* wall-clock seconds spent in this call                              */
    double mass_drift; /* (mass - initial mass)/initial mass, mass = sum_s J_s deta n_s      */
    double pxy_err;    /* estimated remaining relative error of the mean P_xy (-1 before 9 checks, +inf with none) */
} hrlb_steady_info;

/* Autotuner of the kernel plan of one case: a coordinate search, first over tile_vpt (divisors
 * of Qy up to 16) with the given cell_lanes, then over cell_lanes (1, 2, 4, 8, 16) with the best
 * tile_vpt.  Each candidate is created in the caller's workspace (size from
 * hrlb_tune_workspace_bytes) and timed over n_steps steps with HIP events after one warm-up step.
 * Returns the fastest plan and its ms/step; the workspace contents are scratch afterwards.
 * Synchronous. */
hrlb_status hrlb_tune_workspace_bytes(const hrlb_quad *q, const hrlb_case_params *p, size_t *bytes);
hrlb_status hrlb_tune_plan(const hrlb_quad *q, const hrlb_case_params *p, void *dev_workspace, size_t ws_bytes,
                           void *hip_stream, int n_steps, int *best_vpt, int *best_lanes, double *best_ms_per_step);

/* Runs blocks of check_every steps until the stop criterion drops below tol
 * (HRLB_STOP_RESIDUAL: the residual above; HRLB_STOP_PXY: the relative drift rate of the
 * J-weighted mean P_xy between checks; HRLB_STOP_PXY_ERR: the estimated remaining relative error of
 * that mean below tol on two consecutive checks -- the differences d of the last 9 checked means taken
 * as decaying geometrically, their rate r < 1 per check fitted by least squares to log|d|, and the
 * error bounded by max of the last two |d| times r/(1 - r); no estimate before the 9th check or while
 * r >= 1), NaN/Inf appears (HRLB_E_DIVERGED), a cell leaves the
 * verified band of eq. (gx) (HRLB_E_RANGE, checked at every check) or max_steps is reached
 * (HRLB_NOT_CONVERGED).  Synchronous: returns when the decision is made. */
hrlb_status hrlb_run_to_steady(hrlb_case *c, double tol, long max_steps, int check_every, int stop_rule,
                               hrlb_steady_info *info);

/* Synchronous copy of the current macroscopic state to caller host buffers:
 *   fields [10][n_cells]: n, u_x, u_y, T, P_xx, P_xy, P_yy, T_zz, q_x, q_y (moment definitions
 *                         of Sec. II, accumulated in FP64 for both precisions),
 *   x [n_cells]: cell centres,  Pi: equation (Pi) with the J-weighted channel mean of P_xy,
 *   wall_shear [2]: y-momentum flux sum_v p_x p_y F through the left and right wall faces
 *                   (half channel: the wall at x = 1/2 in both, its mirror image being the same).
 * Any pointer may be NULL. */
hrlb_status hrlb_moments(hrlb_case *c, double *fields, double *x, double *Pi, double *wall_shear);

/* Time averages of the fields over completed steps (post-processing of a steady state whose FP32
 * stochastic rounding keeps it fluctuating around the fixed point).  start: clears the running sums
 * and adds the fields of every step completed from then on (asynchronous, on the case's stream;
 * works alone and inside batches); stop: no further steps are added.  read: synchronous; fields
 * [10][n_cells] as hrlb_moments, Pi from the averaged P_xy, *steps the number of steps averaged;
 * HRLB_E_INVALID if no step was averaged.  Any output pointer may be NULL. */
hrlb_status hrlb_average_start(hrlb_case *c);
hrlb_status hrlb_average_stop(hrlb_case *c);
hrlb_status hrlb_average_read(hrlb_case *c, double *fields, double *Pi, long *steps);

/* Synchronous copies of the populations to/from host [2][Nv][n_cells] doubles (phi, chi).
 * set_state rounds to the storage precision and recomputes the moments; it is how a caller
 * resumes from a checkpoint or starts from a given state. */
hrlb_status hrlb_get_state(hrlb_case *c, double *host_state);
hrlb_status hrlb_set_state(hrlb_case *c, const double *host_state);

/* Synchronous: the sticky condition bits of the case (HRLB_FLAG_NONFINITE: a non-finite value met at
 * a check; HRLB_FLAG_RANGE: since its creation some cell's temperature or normal velocity left the
 * band 0.3 <= T/T_w <= 2.4, |u_x| <= sqrt(T_w) in which eq. (gx) is evaluated to 2e-13; the per-cell
 * kernel sets it at every stage, so it covers steps taken with hrlb_step too). */
hrlb_status hrlb_case_flags(hrlb_case *c, unsigned *flags);

/* The kernels that advance the case: HRLB_PATH_TILED or HRLB_PATH_SMALL (see kernel_path). */
hrlb_status hrlb_case_kernel_path(const hrlb_case *c, int *path);

/* Time step in use and the number of velocities / cells of the case. */
hrlb_status hrlb_case_info(const hrlb_case *c, double *dt, int *n_vel, int *n_cells, long *steps_done);

void hrlb_free_case(hrlb_case *c);
void hrlb_free_quadrature(hrlb_quad *q);
const char *hrlb_last_error(void);

/* The estimate behind HRLB_STOP_PXY_ERR (not a step of the paper's method; the stop rule of the
 * serving metric, a fixed error of the channel-mean P_xy): means[count] are successive checked values
 * of the mean P_xy (count >= 3; hrlb_run_to_steady and the server use the last 9).  The count - 1
 * differences d are taken as decaying geometrically with a rate r per check fitted by least squares
 * to log|d|; *estimate = max(|d_last|, |d_prev|) r/(1 - r) / |means[count - 1]|, 0 when the last two
 * differences are exactly zero, +inf while r >= 1 or another difference is exactly zero.  Host
 * only.  HRLB_E_INVALID for count < 3 or a NULL pointer. */
hrlb_status hrlb_pxy_error_estimate(const double *means, int count, double *estimate);

/* ---- batching: several cases, possibly of different sizes and velocity sets, advanced by shared
 * kernel launches.  The cases of the tiled path are split into parts of about equal work (velocities x
 * cells); each part is advanced by one persistent launch per stage and kernel on a stream of its own,
 * forked from and joined back into the cases' stream, so that one part's per-cell kernel overlaps
 * another part's stage kernel.  Three parts by default for batches of at least 2e7 cell-velocity
 * units, one part below (measured faster on MI355X).  The cases of the small path (kernel_path) form
 * one more part, one block per case and one launch per block of steps.  Each case keeps its own
 * workspace and results; a case's numbers are the same alone, in any batch and in any split.  All
 * cases must share one stream and one precision.  The batch needs its own device workspace for
 * descriptors and tile lists (sized for any split into 1 to 4 parts). */
hrlb_status hrlb_batch_workspace_bytes(hrlb_case *const *cases, int n_cases, size_t *bytes);
hrlb_status hrlb_batch_create(hrlb_case *const *cases, int n_cases, void *dev_workspace, size_t ws_bytes,
                              hrlb_batch **out);
/* Enqueues n_steps steps for every case of the batch; if check is nonzero the last step also
 * computes each case's residual and P_xy mean (read them with hrlb_batch_poll). */
hrlb_status hrlb_batch_step(hrlb_batch *b, long n_steps, int check);
/* Synchronous: residual[i], pxy_mean[i] of case i from the last checked step (NULL allowed). */
hrlb_status hrlb_batch_poll(hrlb_batch *b, double *residual, double *pxy_mean);
void hrlb_batch_free(hrlb_batch *b);
/* Splits the batch's tiled cases into n_streams parts (1..4), each on its own stream (the small-path
 * cases keep their own part); synchronous (waits for the batch's stream, then re-uploads the launch
 * tables). */
hrlb_status hrlb_batch_set_streams(hrlb_batch *b, int n_streams);

/* Step blocks of this many steps are captured once as a HIP graph (on a library-private stream)
 * and replayed on the case's or batch's stream; 0 or 1 launches every kernel directly (default:
 * direct launches measured faster than graph replay on MI355X with ROCm 7).
 * The graph holds the launch arguments of the case/batch, so it stays valid until it is freed. */
hrlb_status hrlb_case_set_graph_steps(hrlb_case *c, int steps_per_graph);
hrlb_status hrlb_batch_set_graph_steps(hrlb_batch *b, int steps_per_graph);

/* Profiling: runs n_steps steps of the batch like hrlb_batch_step, with a HIP event pair recorded
 * on the batch's stream around every kernel launch of the tiled path, then waits and returns the mean
 * duration (ms) of one launch of the stage kernel and of the per-cell kernel (cases on the small path
 * take the same steps, untimed).  Synchronous. */
hrlb_status hrlb_batch_profile(hrlb_batch *b, long n_steps, double *stage_kernel_ms, double *cell_kernel_ms);

/* ---- serving: a request loop with continuous batching.  Couette solves (any velocity set, grid,
 * delta, wall speed, wall temperature and viscosity index) are submitted as they arrive.  Each
 * scheduling round (hrlb_server_pump) retires the solves that have stopped, admits waiting ones as
 * slots and device memory allow, advances every resident solve by check_every steps with shared
 * launches, and applies each solve's stop rule.  A solve's populations stay in device memory from
 * admission until it stops.  Device memory comes from one caller-owned arena that the server
 * sub-allocates (first fit, 256-byte blocks); a request is admitted only when its workspace and
 * the batch's launch tables fit.  Admission follows arrival order; a later request may pass one
 * that does not fit until that one has been passed max_bypass times.
 * Every solve runs exactly the steps and checks that hrlb_run_to_steady(tol, max_steps,
 * check_every, stop_rule) runs on the same case alone, so its results are the same bit for bit
 * whatever else is resident.  Times are seconds on the server's monotonic clock.
 * Not thread-safe: one thread drives a server. */
typedef struct hrlb_server hrlb_server;

typedef struct {
    int max_active;   /* slots: solves resident and stepped together, >= 1                   */
    int check_every;  /* steps per scheduling round (and between stop-rule checks), >= 1      */
    int max_bypass;   /* backfill limit of the admission order, >= 0 (0 = strict FIFO)       */
    int precision;    /* HRLB_FP64 or HRLB_FP32_STORE_FP64_MOM, the same for every request   */
} hrlb_server_config;

typedef struct {
    int Qx, Nx_order, Qy, Ny_order; /* velocity set, as hrlb_init_quadrature (p0 = 1)             */
    hrlb_case_params params;        /* as hrlb_init_case; params.precision = the server's        */
    double tol;                     /* stop rule and tolerance, as hrlb_run_to_steady            */
    int stop_rule;
    long max_steps;                 /* a positive multiple of check_every                         */
    double arrival_s;               /* arrival time on the server clock; < 0 means now           */
} hrlb_solve_request;

enum { HRLB_REQ_WAITING = 0, HRLB_REQ_ACTIVE = 1, HRLB_REQ_DONE = 2, HRLB_REQ_FAILED = 3 };

typedef struct {
    int state;          /* HRLB_REQ_*                                                         */
    int status;         /* DONE: HRLB_OK (stop rule met) or HRLB_NOT_CONVERGED (max_steps);    */
                        /* FAILED: the error (HRLB_E_DIVERGED, HRLB_E_RANGE, HRLB_E_DEVICE...) */
    long steps;         /* steps taken                                                         */
    double residual, pxy_drift, Pi, sim_time, mass_drift;  /* as hrlb_steady_info/hrlb_moments */
    double pxy_err;                                         /* as hrlb_steady_info               */
    double t_arrival, t_admit, t_done;                      /* server clock; -1 if not reached */
    int n_cells, n_vel;
    size_t bytes;       /* device workspace of the solve                                       */
} hrlb_request_info;

typedef struct {
    int waiting, active, done, failed; /* counts after the round                               */
    int admitted, retired;             /* in this round                                        */
    long steps;                        /* steps per resident solve in this round (0 if idle)   */
    double units;                      /* cell-velocity updates in this round                  */
    double round_s;                    /* wall time of the round                               */
    size_t arena_used, arena_largest_free;
} hrlb_server_stats;

/* Creates a server over the caller's device arena (256-byte aligned; it must stay allocated until
 * hrlb_server_free) on the caller's stream.  Host-only apart from remembering the pointers. */
hrlb_status hrlb_server_create(const hrlb_server_config *cfg, void *dev_arena, size_t arena_bytes, void *hip_stream,
                               hrlb_server **out);
/* Seconds since the server was created (monotonic clock). */
double hrlb_server_clock(const hrlb_server *s);
/* Queues a solve; *id receives its handle.  Validates everything hrlb_init_case would and
 * rejects with HRLB_E_NOMEM a solve whose workspace can never fit the arena. */
hrlb_status hrlb_server_submit(hrlb_server *s, const hrlb_solve_request *r, long *id);
/* One scheduling round as described above.  Synchronous.  Returns HRLB_OK also when a solve
 * failed (its request reports the error); a negative status means the server itself failed. */
hrlb_status hrlb_server_pump(hrlb_server *s, hrlb_server_stats *stats);
/* State and result of a request.  fields [10][n_cells] and x [n_cells] (as hrlb_moments) are
 * written once the request is DONE; either may be NULL.  release != 0 forgets a DONE or FAILED
 * request after the copy (its id becomes invalid). */
hrlb_status hrlb_server_request(hrlb_server *s, long id, hrlb_request_info *info, double *fields, double *x,
                                int release);
/* Frees every resident solve, the cached velocity sets and the server.  The arena is the caller's. */
void hrlb_server_free(hrlb_server *s);

#ifdef __cplusplus
}
#endif
#endif /* HRLB_H */
