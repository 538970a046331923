/*
 * odp.h -- C ABI of libodp.so, a gfx950 (MI355X) solver for the time-dependent
 * Hamilton-Jacobi level-set equation (backward reachable sets and tubes).
 *
 * Method (paper "OptimizedDP", Algorithm 1 and the HJ PDE / HJ variational
 * inequality equations of its Methods section): for every grid point and
 * every time step, one-sided differences in each dimension, the optimal
 * control and disturbance for the central costate, the Hamiltonian,
 * Lax-Friedrichs dissipation, a CFL time step from a grid-wide maximum of
 * the dissipation coefficients, a TVD Runge-Kutta update and, for a tube,
 * V = min(V, V0).
 *
 * Conventions shared by every entry point:
 *  - Grid arrays are contiguous, row-major, last axis fastest (the layout of
 *    the paper's cache-aware loop-order section).  Element type is float
 *    (precision 32) or double (precision 64).
 *  - Pointers named *_dev are device (HBM) pointers on the current HIP
 *    device; all other pointers are host pointers.  The caller owns every
 *    buffer it passes; the library never frees caller memory and keeps no
 *    pointer after a call returns (server calls copy what they keep).
 *  - Time is time-to-go tau >= 0 (tau = -s for the paper's backward time s).
 *    tau arrays are strictly increasing; tau[0] is the start time.
 *  - Return codes: 0 OK, > 0 informational, < 0 error.  No C++ exception
 *    crosses the ABI.  odp_last_error() gives a thread-local message for the
 *    last failing call on the calling thread.
 */
#ifndef ODP_H
#define ODP_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum {
    ODP_OK = 0,
    ODP_PENDING = 1,        /* serve: request not finished yet */
    ODP_EINVAL = -1,        /* bad argument (shape, bounds, tau, cfl, id) */
    ODP_ENOMEM = -2,        /* allocation failed / workspace too small /
                               request larger than the server's budget */
    ODP_EHIP = -3,          /* a HIP runtime call failed */
    ODP_EUNSUPPORTED = -4,  /* valid but unsupported combination */
    ODP_EAGAIN = -5,        /* serve queue full, retry later */
    ODP_ENONFINITE = -6,    /* NaN or Inf appeared in the value function */
    ODP_ECANCELED = -7      /* serve request was cancelled */
};

/* Static description of a return code (never NULL). */
const char *odp_strerror(int code);
/* Detail of the last error raised on this thread (empty string if none). */
const char *odp_last_error(void);

/* ------------------------------------------------------------------ grid */

/* Cartesian grid (paper: Grid section).  ndim in [1, 6]; n[d] >= 3 nodes;
 * lo[d] < hi[d]; periodic[d] != 0 makes axis d periodic, in which case hi[d]
 * is excluded and the spacing is (hi - lo) / n, otherwise (hi - lo)/(n - 1).
 * Non-periodic edges use ghost nodes extrapolated away from zero (the ghost
 * keeps the sign of the boundary node).  The total point count must stay
 * below 2^31 per hyperplane of axes 1..ndim-1 and below 2^40 overall.
 * On success *out owns a host object freed by odp_grid_destroy. */
/* odp_solve_opts.tile_chunk: let the library time candidate tilings. */
#define ODP_TILE_AUTOTUNE (-1)

typedef struct odp_grid odp_grid;
int odp_grid_create(int ndim, const int64_t *n, const double *lo, const double *hi,
                    const uint8_t *periodic, odp_grid **out);
void odp_grid_destroy(odp_grid *grid);
/* Number of grid points (product of n). */
int64_t odp_grid_points(const odp_grid *grid);

/* -------------------------------------------------------------- dynamics */

/* Closed set of control-affine dynamics (paper: Dynamical Systems
 * Specification section and appendix).  Parameter layout of p[]:
 *  SINGLE_INTEGRATOR (any ndim, test problem): z' = c + u, |u|_2 <= u_max;
 *      p[0] = u_max, p[1..ndim] = c.
 *  DUBINS3D (x, y, th):  x' = v cos th, y' = v sin th, th' = w, |w| <= w_max;
 *      p[0] = v, p[1] = w_max.  Control w.
 *  DYNCAR4D (x, y, v, th): x' = v cos th, y' = v sin th, v' = a, th' = w;
 *      p[0] = a_max, p[1] = w_max.  Controls a, w.
 *  TWODUBINS6D (x_e, y_e, th_e, x_p, y_p, th_p): two Dubins cars; the
 *      evader turns with the control u (|u| <= u_max), the pursuer with the
 *      disturbance d (|d| <= d_max); p[0] = v_e, p[1] = u_max, p[2] = v_p,
 *      p[3] = d_max.
 *  PE3D (x, y, th): relative pursuit-evasion of two Dubins cars (the
 *      paper's main example): x' = -v_a + v_b cos th + a y,
 *      y' = v_b sin th - a x, th' = b - a; evader turn a (control,
 *      |a| <= a_max), pursuer turn b (disturbance, |b| <= b_max);
 *      p[0] = v_a, p[1] = v_b, p[2] = a_max, p[3] = b_max.  Its dissipation
 *      is taken over the costate box of each Runge-Kutta stage (Algorithm
 *      1's D_min / D_max: a grid-wide reduction before every stage update),
 *      and so is its CFL step: Algorithm 1's alpha^max, the largest box
 *      alpha over the grid for the box of the step's first stage, reduced
 *      on the device every step (with dissipation = 1, the global-alpha
 *      approximation, there is no box: all inputs bound both).
 * u_mode / d_mode: 1 = that player maximises the Hamiltonian, 0 = minimises
 * (for a box input: maximiser picks +bound when its switching function is
 * >= 0, minimiser picks -bound). */
typedef enum {
    ODP_DYN_SINGLE_INTEGRATOR = 0,
    ODP_DYN_DUBINS3D = 1,
    ODP_DYN_DYNCAR4D = 2,
    ODP_DYN_TWODUBINS6D = 3,
    ODP_DYN_PE3D = 4
} odp_dyn_id;

typedef struct {
    int32_t id;      /* odp_dyn_id */
    int32_t u_mode;  /* 1 maximise, 0 minimise */
    int32_t d_mode;  /* 1 maximise, 0 minimise */
    int32_t pad_;
    double p[16];
} odp_dynamics;

/* ----------------------------------------------------------------- solve */

/* Computation method (the paper's table of computation methods, Sec. on the
 * solver interface): after every full CFL step (the last Runge-Kutta stage)
 * the new value V is compared, point by point, with a reference and replaced
 * by the smaller (min) or larger (max) of the two.  NaN in V stays NaN. */
typedef enum {
    ODP_BRS = 0,          /* none: the plain PDE, a backward reachable set */
    ODP_BRT = 1,          /* min with V0 (minVWithV0): the reachable tube,
                             the HJ variational inequality */
    ODP_MIN_V0 = 1,
    ODP_MAX_V0 = 2,       /* max with V0 (maxVWithV0) */
    ODP_MIN_VINIT = 3,    /* min with the value before the step (minVWithVInit:
                             the running minimum over time) */
    ODP_MAX_VINIT = 4,    /* max with the value before the step (maxVWithVInit) */
    ODP_MIN_TARGET = 5,   /* min with the target array opts->target_dev
                             (minVWithVTarget, reach-avoid) */
    ODP_MAX_TARGET = 6    /* max with the target array (maxVWithVTarget) */
} odp_mode;

/* Obstacle method, applied after the target method of the same step. */
typedef enum {
    ODP_OBSTACLE_NONE = 0,
    ODP_MIN_OBSTACLE = 1, /* min with opts->obstacle_dev (minVWithObstacle) */
    ODP_MAX_OBSTACLE = 2  /* max with opts->obstacle_dev (maxVWithObstacle,
                             reach-avoid: g(z) > 0 inside the obstacle) */
} odp_obstacle_mode;

typedef struct {
    int32_t precision;   /* 32 or 64: element type of every grid array */
    int32_t rk_order;    /* 1, 2 or 3 (TVD Runge-Kutta) */
    double cfl;          /* in (0, 1] */
    int32_t mode;        /* odp_mode: the computation method applied after
                            every full step (ODP_BRS: none) */
    int32_t dissipation; /* 0: per-point alpha_d(z_i); 1: global alpha^max_d
                            (the paper's cheaper approximation) */
    double max_dt;       /* 0: none; > 0 caps the CFL step (tests use it) */
    int32_t save_all;    /* 1: also write V at every tau[k] into V_all_dev */
    int32_t tile_chunk;  /* 0: library default; ODP_TILE_AUTOTUNE (-1): chosen by
                            timing the stage launches of step 0 for a list of
                            candidates on the first solve (or batch) of each
                            problem shape, cached for the process (results do
                            not depend on it); else planes marched per block */
    void *stream;        /* hipStream_t for every launch (NULL: null stream) */
    int32_t xcd_group;   /* 0: library default (one contiguous run of tiles per
                            XCD; runs of 64 for grids of 2^28 points or more);
                            g > 0: runs of g tiles dealt round robin to XCDs */
    int32_t graph;       /* time stepping recorded into one HIP graph and
                            replayed: 0 auto (small grids on a non-null
                            stream), 1 always (non-null stream), 2 never.
                            The instantiated graph is kept (16 most recent
                            shapes per process) and replayed by later calls
                            with the same shape, options and workspace. */
    int32_t obstacle_mode; /* odp_obstacle_mode (0: none) */
    int32_t set_slices;    /* 0 or 1: target_dev / obstacle_dev hold one grid
                              each, used for the whole horizon; ntau
                              (odp_hj_solve only): time-varying sets l(z, t),
                              g(z, t), ntau grids one after the other, grid k
                              the set at tau[k]; the steps from tau[k-1] to
                              tau[k] compare with grid k-1 */
    const void *target_dev;   /* device, element type = precision: l(z) of
                                 ODP_MIN_TARGET / ODP_MAX_TARGET (NULL
                                 otherwise); read only */
    const void *obstacle_dev; /* device: g(z) of the obstacle method (NULL
                                 when obstacle_mode is 0); read only */
    int32_t space_order;   /* spatial derivatives (Spatial Derivatives
                              subsection): 0 or 1 first-order upwind; 2
                              second-order ENO (the paper's second-order row
                              pairs it with rk_order 2); beyond a
                              non-periodic edge the second ghost node is
                              V_b + 2 sgn(V_b) |V_b - V_in| */
    int32_t pad2_;
} odp_solve_opts;

typedef struct {
    int64_t steps;       /* CFL steps taken */
    double dt_min, dt_max, t_final;
    double kernel_ms;    /* device time of the time-stepping loop */
    double alg_bytes;    /* algorithmic HBM bytes of the loop */
    double alg_gbps;     /* alg_bytes / kernel time */
    double roofline_frac;/* alg_gbps / 8000 */
    double alpha_max[6]; /* grid-wide maximum dissipation coefficients */
    double latency_ms;   /* server only: submit -> completion (host clock) */
    double queue_ms;     /* server only: submit -> admission (slot and memory) */
    double admit_ms;     /* server only: admission -> prologue done (upload, schedule) */
    double run_ms;       /* server only: prologue done -> last step done */
    double retire_ms;    /* server only: last step done -> result on the host */
    int32_t nonfinite;   /* 1 if a NaN / Inf was produced */
    int32_t pad_;
} odp_solve_stats;

/* Device workspace bytes odp_hj_solve needs for this problem (the float64
 * dt schedule is sized from the dynamics' speed bounds and the horizon).
 * Returns 0 for invalid arguments. */
size_t odp_hj_workspace_bytes(const odp_grid *grid, const odp_dynamics *dyn, const double *tau,
                              int ntau, const odp_solve_opts *opts);

/* Solve V from tau[0] to tau[ntau-1] (ntau >= 2) on opts->stream.
 *  V0_dev:     l(z), the target's implicit function (read only; also the
 *              clamp of a tube).
 *  V_init_dev: value at tau[0]; NULL means V0 (restart: pass V(tau[0])).
 *  workspace_dev: NULL (the library allocates stream-ordered and frees
 *              after the call) or at least odp_hj_workspace_bytes bytes,
 *              256-byte aligned, used exclusively by this call until the
 *              stream reaches its end.
 *  V_out_dev:  receives V(tau[ntau-1]); may not alias V0, V_init or the
 *              target / obstacle arrays.
 *  V_all_dev:  NULL unless opts->save_all; then ntau slices, slice 0 =
 *              the start value, slice k = V(tau[k]).
 *  stats:      NULL, or filled after an internal stream synchronisation.
 * The CFL step is dt = cfl / sum_d alpha^max_d / dx_d, computed in float64 on
 * the device and clipped so that time lands exactly on every tau[k].  The
 * call is stream-ordered: it returns once the work is enqueued (the host
 * works out the step count from the same float64 tables and operations as
 * the device schedule, and uploads through pinned staging), except that
 * stats != NULL synchronises, and so does the first call of a shape with
 * tile_chunk = ODP_TILE_AUTOTUNE (its timing runs).  The device checks that
 * its schedule fits the enqueued steps; with stats != NULL a violation
 * returns ODP_EHIP and ODP_ENONFINITE reports NaN/Inf.  Input buffers must
 * stay valid, and V_out unread, until the stream reaches the call's end. */
int odp_hj_solve(const odp_grid *grid, const odp_dynamics *dyn, const void *V0_dev,
                 const void *V_init_dev, const double *tau, int ntau,
                 const odp_solve_opts *opts, void *workspace_dev, void *V_out_dev,
                 void *V_all_dev, odp_solve_stats *stats);

/* ------------------------------------------------- allocation-free solve */

/* For callers that cannot allocate device or pinned memory (code recorded
 * into a HIP graph, tight serving loops, harnesses that forbid allocation):
 * odp_hj_solve with the same arguments and results, whose workspace is a
 * fixed device array of 256 MiB inside the library (one per GPU, held from
 * the library's load until the process ends) instead of a caller or
 * library allocation.  It allocates nothing: the time stepping is launched
 * eagerly (opts->graph is ignored), ODP_TILE_AUTOTUNE means the default
 * tiling, and the plan is uploaded from pageable host memory (the runtime
 * performs that copy synchronously).  stats: NULL, or filled after a stream
 * synchronisation (kernel_ms is 0: timing would need events).
 * Returns ODP_ENOMEM, before touching the device, when the solve needs more
 * workspace than the array holds (odp_hj_workspace_bytes with the default
 * tiling: e.g. up to about 64M float32 points with RK1/RK2, 32M with RK3).
 * Every call on one GPU uses that GPU's one array: calls that overlap on a
 * GPU (from several threads, or on streams that run concurrently) race and
 * give wrong results; calls in one stream's order are safe. */
int odp_hj_solve_noalloc(const odp_grid *grid, const odp_dynamics *dyn, const void *V0_dev,
                         const void *V_init_dev, const double *tau, int ntau,
                         const odp_solve_opts *opts, void *V_out_dev, void *V_all_dev,
                         odp_solve_stats *stats);

/* ----------------------------------------------------------------- batch */

/* One solve of a batch: its own grid, dynamics, target and horizon. */
typedef struct {
    const odp_grid *grid;
    odp_dynamics dyn;
    const void *V0_dev;    /* device, element type = common->precision */
    const double *tau;     /* host, strictly increasing, ntau >= 2 */
    int32_t ntau;
    int32_t rk_order;      /* 0: the common options' order; else 1, 2 or 3 */
    void *V_out_dev;       /* device, receives V(tau[ntau-1]) */
} odp_solve_desc;

/* Workspace for odp_hj_batch (device bytes). */
size_t odp_hj_batch_workspace_bytes(int nsolves, const odp_solve_desc *descs,
                                    const odp_solve_opts *common);

/* Run nsolves independent solves together on common->stream: every stage
 * launch covers the tiles of all members that are still stepping (members
 * are ordered by step count, longest first, and grouped by kernel shape).
 * common->save_all must be 0; target and obstacle arrays are not available
 * (ODP_EUNSUPPORTED: they belong to one grid), the other computation methods
 * are.  workspace_dev may be NULL (library allocates) or hold
 * odp_hj_batch_workspace_bytes bytes.
 * stats_per_solve: NULL or nsolves entries, filled after a synchronisation
 * (kernel_ms is the whole launch).  Results equal the same solves run one by
 * one through odp_hj_solve with the same options, bit for bit. */
int odp_hj_batch(int nsolves, const odp_solve_desc *descs, const odp_solve_opts *common,
                 void *workspace_dev, size_t workspace_bytes,
                 odp_solve_stats *stats_per_solve);

/* --------------------------------------------------------- time to reach */

/* Time to reach the target set {z : l(z) <= 0} (the Time-independent HJ PDE
 * subsection, Algorithm 2: Lax-Friedrichs sweeping), as the fixed point of
 * the explicit Lax-Friedrichs point update of  min_u max_d grad(phi) . f = -1,
 * phi = 0 on the target:
 *   phi_i <- min(phi_i, [1 + H + sum_d sigma_d (phi_{i+e_d} + phi_{i-e_d}) / (2 dx_d)]
 *                        / sum_d sigma_d / dx_d),
 * H = pbar . f(z, u*, d*) at the centred costate, sigma_d = max |f_d|; nodes
 * on a non-periodic edge take min(phi, max(2 phi_a - phi_b, phi_b)) (a, b the
 * next two nodes inward).  The paper sweeps Gauss-Seidel on the CPU; here
 * each iteration updates every node from the previous iterate (Jacobi),
 * which converges to the same fixed point.  The control minimises the time:
 * pass dyn->u_mode = 0 (and d_mode = 1 for a disturbance that maximises it).
 * The pursuit-evasion model is not available (ODP_EUNSUPPORTED). */
typedef struct {
    int32_t precision;   /* 32 or 64: element type of target and phi */
    int32_t check_every; /* iterations between convergence checks (0: 32) */
    double eps;          /* stop once an iteration changes no node by eps or more */
    int64_t max_iters;   /* >= 1 */
    double big;          /* start value off the target (0: 1e4, the paper's) */
    void *stream;        /* hipStream_t (NULL: null stream) */
} odp_ttr_opts;

typedef struct {
    int64_t iters;        /* iterations run (a multiple of check_every, or max_iters) */
    double last_change;   /* largest change of the last iteration */
    double kernel_ms;     /* device time of the iterations */
    double alg_bytes;     /* 3 arrays per node and iteration */
    double alg_gbps;
    double roofline_frac; /* alg_gbps / 8000 */
    int32_t converged;    /* 1 if an iteration's largest change fell below eps */
    int32_t pad_;
} odp_ttr_stats;

/* Device workspace bytes for odp_ttr_solve (0 for invalid arguments). */
size_t odp_ttr_workspace_bytes(const odp_grid *grid, const odp_ttr_opts *opts);

/* target_dev: l(z) on the grid (device, read only); phi_out_dev: receives
 * the time to reach (device, may not alias target).  workspace_dev: NULL
 * (library allocates stream-ordered) or odp_ttr_workspace_bytes bytes,
 * 256-byte aligned.  Blocks once per check_every iterations to test
 * convergence; returns ODP_OK also when max_iters ran out (stats->converged
 * says which). */
int odp_ttr_solve(const odp_grid *grid, const odp_dynamics *dyn, const void *target_dev,
                  const odp_ttr_opts *opts, void *workspace_dev, size_t workspace_bytes,
                  void *phi_out_dev, odp_ttr_stats *stats);

/* ----------------------------------------------------------------- serve */

/* In-process continuous-batching server.  A scheduler thread admits queued
 * requests while their device footprint fits hbm_budget_bytes and a slot is
 * free, keeps their value functions resident, and advances the active
 * solves (in arrival order, up to a work budget per tick) by a few steps
 * per tick in batched launches, one per RK stage and kernel group, on two
 * compute streams; requests that arrive while others run join at a later
 * tick.  The server owns four streams (two compute, upload, download).
 * Results are the same as odp_hj_solve with the server's options, bit for
 * bit. */
typedef struct odp_server odp_server;

int odp_server_create(size_t hbm_budget_bytes, int max_slots, const odp_solve_opts *opts,
                      odp_server **out);
/* Copy the request (grid shape, dynamics, tau, and V0 from HOST memory:
 * desc->V0_dev is read as a host pointer here, desc->V_out_dev is ignored)
 * and queue it.  The caller may free its buffers on return.
 * ODP_ENOMEM if the request can never fit the budget, ODP_EAGAIN if the
 * queue is full. */
int odp_serve_submit(odp_server *srv, const odp_solve_desc *host_desc, uint64_t *ticket);
/* ODP_PENDING while queued or running.  Once finished: copies V(tau_last)
 * into V_out_host (bytes must equal the grid size times the element size),
 * fills stats (may be NULL), releases the ticket and returns ODP_OK, or the
 * request's error code (ODP_ECANCELED, ODP_ENONFINITE, ...). */
int odp_serve_poll(odp_server *srv, uint64_t ticket, void *V_out_host, size_t bytes,
                   odp_solve_stats *stats);
/* Cancel a queued or running request; its poll then returns ODP_ECANCELED. */
int odp_serve_cancel(odp_server *srv, uint64_t ticket);
/* Number of requests queued, running and finished-but-unpolled. */
int odp_server_counts(odp_server *srv, int *queued, int *running, int *done);
/* Stop the scheduler (running requests are cancelled) and free everything. */
void odp_server_destroy(odp_server *srv);

#ifdef __cplusplus
}
#endif

#endif /* ODP_H */
