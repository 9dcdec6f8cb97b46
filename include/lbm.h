/*
 * lbm.h -- C ABI of the MI355X (gfx950) D2Q9 lattice-BGK lid-driven cavity
 * library.
 *
 * The method is that of Xiang & Shi, "Flow Simulation of Lid-Driven
 * Rectangular Cavity by Using Lattice Boltzmann Method" (arXiv 2211.05009):
 *   - Sec. 2.1 Eq. 1: BGK evolution, collide then stream, one lattice link
 *     per step;
 *   - Sec. 2.1 Eq. 2: second-order equilibrium, c_s^2 = 1/3, D2Q9 weights
 *     4/9, 1/9, 1/36;
 *   - Sec. 2.1 Eq. 3: rho and rho u as moments of the populations;
 *   - Sec. 2.1 Eq. 5 with Sec. 1's Re = U L / nu (L = cavity width):
 *     tau = 3 U Nx / Re + 1/2 in lattice units (dx = dt = c = 1, Sec. 3);
 *   - Sec. 2.2 (i): start from rest, rho = 1, f = f^eq;
 *   - Sec. 2.2 (iii) Eq. 6: relative L2 change of u over 100 steps;
 *   - Sec. 3.3: velocity at observing points, positions in units of L.
 * Walls (default): half-way bounce-back on the three resting walls and the
 * moving-wall bounce-back term -6 w rho_w (c . u_w), rho_w = 1, on the lid.
 * Links through the two top corners belong to the lid.  The paper's own
 * scheme, non-equilibrium extrapolation on on-node walls (Sec. 2.2 (ii)),
 * is selected with lbm_create_wall.
 *
 * Lattice: Nx sites along the lid, Ny sites up; site (x, y), y = 0 at the
 * bottom.  Host arrays exchanged through this ABI are row-major [ny][nx]
 * doubles (populations: [9][ny][nx]), velocity order
 *   0:(0,0) 1:(1,0) 2:(0,1) 3:(-1,0) 4:(0,-1) 5:(1,1) 6:(-1,1) 7:(-1,-1)
 *   8:(1,-1).
 *
 * Conventions for every function:
 *   - returns LBM_OK (0) or a negative error code, never aborts or throws;
 *     lbm_last_error() then holds a message (thread-local);
 *   - a handle is used by one host thread at a time; distinct handles are
 *     independent;
 *   - pointers named *_host are caller-owned host memory, *_dev caller-owned
 *     device memory on the handle's device; the library keeps no reference
 *     to them after the call returns;
 *   - work is issued on the handle's HIP stream (its own by default, see
 *     lbm_set_stream); every function that returns data to the host
 *     synchronises that stream before returning.
 *
 * Run log: when the environment variable LBM_LOG names a file at the first
 * lbm_step / lbm_batch_step call, each such call appends one JSON line to it
 * (kind, handle, lattice, steps of the call, step count, mass, last Eq. 6
 * residual, wall seconds, MLUPS; batches: active cavities before and after,
 * largest residual of the active ones).  Unset: nothing is written.
 */
#ifndef LBM_H
#define LBM_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum {
  LBM_OK = 0,
  LBM_EINVAL = -1,     /* bad argument (the message names it) */
  LBM_ENOMEM = -2,     /* device or host allocation failed */
  LBM_EDEVICE = -3,    /* a HIP runtime call failed */
  LBM_EUNSTABLE = -4,  /* a monitor went non-finite; state kept for inspection */
  LBM_EIO = -5,        /* checkpoint file could not be read or written */
  LBM_ESTATE = -6      /* checkpoint does not match the handle */
};

/* Storage precision of the populations. */
enum {
  LBM_F64 = 0,          /* f stored and collided in FP64 */
  LBM_F32_SHIFTED = 1   /* g = f - w stored and collided in FP32; moments,
                           mass, residual, probes, Psi reduced in FP64 */
};

/* Wall schemes. */
enum {
  LBM_WALL_BOUNCE_BACK = 0,  /* half-way bounce-back; walls half a link outside the sites */
  LBM_WALL_NEE = 1           /* non-equilibrium extrapolation on on-node walls */
};

typedef struct lbm_cavity *lbm_t;

typedef struct {
  int nx, ny;           /* sites along the lid / up */
  int pitch;            /* elements per stored row (nx rounded up to 64) */
  int dtype;            /* LBM_F64 or LBM_F32_SHIFTED */
  double re, u_lid;     /* Reynolds number, lid speed */
  double tau, omega;    /* relaxation time (Eq. 5) and 1/tau */
  int64_t steps_done;   /* applications of Eq. 1 since the last (re)start */
  size_t device_bytes;  /* device memory held by the handle */
  int wall;             /* LBM_WALL_BOUNCE_BACK or LBM_WALL_NEE */
} lbm_info_t;

/* Message of the last failed call on this thread ("" if none). */
const char *lbm_last_error(void);

/* Library version string. */
const char *lbm_version(void);

/*
 * Create a cavity of nx x ny sites at Reynolds number re (Sec. 1 definition,
 * L = nx) with lid speed u_lid, at rest (Sec. 2.2 (i)): rho = 1, u = 0.
 * tau = 3 u_lid nx / re + 1/2 (Eq. 5).
 * Errors: LBM_EINVAL if nx or ny < 2, nx > 65536, ny > 65536, re <= 0 or not
 * finite, tau <= 1/2, |u_lid| >= 1/sqrt(3), out == NULL, unknown dtype;
 * LBM_ENOMEM / LBM_EDEVICE on device failure.  The handle owns its device
 * memory until lbm_destroy.
 */
int lbm_create(int nx, int ny, double re, double u_lid, int dtype, lbm_t *out);

/* Same, with tau given directly (tau > 1/2).  re is reported as
 * 3 u_lid nx / (tau - 1/2) (infinite if u_lid = 0). */
int lbm_create_tau(int nx, int ny, double tau, double u_lid, int dtype,
                   lbm_t *out);

/*
 * Create a cavity with a chosen wall scheme.  LBM_WALL_BOUNCE_BACK is
 * lbm_create.  LBM_WALL_NEE is the paper's scheme (Sec. 2.2 (ii)): nx x ny
 * nodes whose outermost rows and columns are the walls, so L = nx - 1 and
 * tau = 3 u_lid (nx - 1) / re + 1/2.  Each step, wall node (x, y) stores
 *   f*_b = f^eq(rho_r, u_w) + (1 - 1/tau) (f_r - f^eq(rho_r, u_r)),
 * f_r being the streamed populations of its reference node
 * r = (clamp(x, 1, nx-2), clamp(y, 1, ny-2)); u_w = (u_lid, 0) on the top
 * row, corners included, and 0 on the other wall nodes.  Initial state
 * (Sec. 2.2 (i)): f = f^eq(1, u0), u0 = (u_lid, 0) on the top row, 0
 * elsewhere.  Mass, Eq. 6 and moments cover all nodes; probes, Psi and
 * vortex positions use node positions x / (nx - 1) in units of L, and Psi
 * is the trapezoid rule up each column from Psi = 0 on the bottom row.  NEE
 * handles have LBM_OPT_NUM_VARIANTS = 8 tile shapes: 0-3 take one step per
 * launch (64 x {4, 8} nodes), 4-7 take K steps per launch on a tile kept
 * in LDS (16 x 16, K = 4; 32 x 16, K = 5, FP64 16 x 16; 32 x 32, K = 4,
 * FP64 16 x 32; 32 x 32, K = 5, FP64 16 x 32 with K = 2).  Every shape
 * gives the same bits.
 * Errors: as lbm_create; LBM_EINVAL for an unknown wall, or NEE with nx or
 * ny < 3.
 */
int lbm_create_wall(int nx, int ny, double re, double u_lid, int dtype, int wall,
                    lbm_t *out);

/* Free the handle and its device memory.  NULL is a no-op. */
int lbm_destroy(lbm_t h);

/* Issue all further work of h on hip_stream (a hipStream_t, e.g. the
 * current stream of the caller's framework); NULL returns to the handle's
 * own stream.  The caller's stream stays caller-owned and must outlive its
 * use by h.  Pending work of h is finished before the switch. */
int lbm_set_stream(lbm_t h, void *hip_stream);

/* Handle parameters. */
int lbm_info(lbm_t h, lbm_info_t *info);

/*
 * Execution options (do not change results):
 *   LBM_OPT_USE_GRAPH     1 (default): aligned 100-step chunks are replayed
 *                         from a captured HIP graph; 0: launched one by one.
 *   LBM_OPT_STEP_VARIANT  index of the step kernel's tile shape, in
 *                         [0, LBM_OPT_NUM_VARIANTS); picked by lbm_autotune.
 *   LBM_OPT_NUM_VARIANTS  read-only: number of tile shapes.
 *   LBM_OPT_STEPS_PER_LAUNCH  read-only: steps of Eq. 1 one launch of the
 *                         current shape applies (1, or K for the shapes that
 *                         keep a tile in LDS for K steps).
 *   LBM_OPT_TILE_X, LBM_OPT_TILE_Y  read-only: sites along x and y that one
 *                         block of the current shape updates (a K-step
 *                         shape reads a region K sites wider on every side).
 *   LBM_OPT_SYNC          1 (default): lbm_step returns after its work has
 *                         finished; 0: a call that reaches no monitor point
 *                         returns once its launches are issued on the
 *                         handle's stream, like an asynchronous GPU library
 *                         call (the caller synchronises the stream before
 *                         reading results through other APIs; a fault of
 *                         that work surfaces at the next synchronising
 *                         call).  Calls that reach a monitor point still
 *                         finish before returning.
 * LBM_EINVAL for an unknown option or an out-of-range value.
 */
enum {
  LBM_OPT_USE_GRAPH = 1,
  LBM_OPT_STEP_VARIANT = 2,
  LBM_OPT_NUM_VARIANTS = 3,
  LBM_OPT_GRAPH_STEPS = 4, /* batches only: steps per captured graph, a
                              multiple of 100 in [100, 100000] (default 1000) */
  LBM_OPT_STEPS_PER_LAUNCH = 5,
  LBM_OPT_TILE_X = 6,
  LBM_OPT_TILE_Y = 7,
  LBM_OPT_SYNC = 8
};
int lbm_set_option(lbm_t h, int option, int64_t value);
int lbm_get_option(lbm_t h, int option, int64_t *value);

/*
 * Tile-shape autotuner: time every step-kernel tile shape over `chunks`
 * 100-step chunks (1 <= chunks <= 10000) with HIP events on the handle's
 * stream, keep the fastest (LBM_OPT_STEP_VARIANT) and leave the state, step
 * counter and monitors exactly as before the call.  Must be called at a
 * multiple of 100 steps.  If use_cache is non-zero and the file named by the
 * environment variable LBM_TUNE_CACHE holds an entry for this device,
 * storage type and lattice, that entry is applied without timing
 * (*ms_per_step = NaN); a timed result is appended to that file.  Outputs
 * may be NULL.  The shapes give bit-identical results.
 */
int lbm_autotune(lbm_t h, int chunks, int use_cache, int *best_variant,
                 double *ms_per_step);

/*
 * Advance n >= 0 steps of Eq. 1 with the wall treatment above.  At every
 * step count t that is a multiple of 100 the monitors run: total mass and
 * the Eq. 6 residual against the velocity field of step t - 100 (with the
 * multi-step shapes the monitor of step t runs inside the first two launches
 * of the next 100 steps, or in a separate pass before further steps or at
 * the end of the call).  If probes are configured (lbm_probe_config) they
 * are recorded every `every` steps.
 * Execution (results do not depend on it): 100-step chunks starting at a
 * multiple of 100 are replayed from a captured graph; steps off that grid
 * run as launches of the current shape's K steps while t is a multiple of K
 * and K steps remain, and as one-step launches otherwise (a multi-step
 * shape is used only if its K divides a probe cadence of at most 100).
 * Returns after the work has finished (with LBM_OPT_SYNC 0 and no monitor
 * point in the call: once it is issued); LBM_EUNSTABLE if the last monitor
 * (or the final state's mass) is not finite.
 */
int lbm_step(lbm_t h, int64_t n);

/*
 * What the last lbm_step call on h launched, counting the launches inside
 * replayed graphs, so that a timing of the call can be attributed to the
 * kernels that ran.  Shapes are LBM_OPT_STEP_VARIANT indices.  A call that
 * failed leaves the counts of what was issued before the failure.
 * Not a passage of the paper: execution bookkeeping only.
 */
typedef struct {
  int64_t steps;                  /* steps of Eq. 1 the call applied */
  int multi_variant;              /* shape of the K-step launches; -1: none */
  int steps_per_launch;           /* K of that shape; 0: none */
  int64_t multi_launches;         /* K-step launches */
  int64_t multi_monitor_launches; /* of those, launches that also took the
                                     Eq. 6 monitor sums (two per fused chunk) */
  int single_variant;             /* shape of the one-step launches; -1: none */
  int64_t single_launches;        /* one-step launches */
  int64_t graph_replays;          /* 100-step chunks replayed from a graph */
  int64_t monitor_passes;         /* separate monitor passes (mass, Eq. 6) */
  int64_t probe_launches;         /* probe records written */
} lbm_launch_record_t;
int lbm_last_launches(lbm_t h, lbm_launch_record_t *out);

/* Number of steps applied since creation or the last lbm_set_populations /
 * lbm_init_fields / lbm_load. */
int lbm_steps_done(lbm_t h, int64_t *t);

/*
 * Density and velocity (Eq. 3) at the current step, each [ny][nx] doubles.
 * A NULL output is skipped.  _host writes host memory, _dev device memory.
 */
int lbm_moments(lbm_t h, double *rho_host, double *ux_host, double *uy_host);
int lbm_moments_device(lbm_t h, double *rho_dev, double *ux_dev,
                       double *uy_dev);

/*
 * (rho, u_x, u_y) at npts observing points (Sec. 3.3) now.  xy_host holds
 * npts pairs (x, y) in units of the cavity width L; each is interpolated
 * bilinearly between site centres ((i + 1/2)/nx, (j + 1/2)/nx) and clamped
 * to the outermost centres.  out_host receives npts triples.
 * LBM_EINVAL if npts < 1 or npts > 4096, or a coordinate is not finite.
 */
int lbm_probe(lbm_t h, int npts, const double *xy_host, double *out_host);

/*
 * Record a probe time series on the device: from the next step on, every
 * `every` steps (a divisor or a multiple of 100), write (rho, u_x, u_y) at
 * the npts points into a ring of `capacity` records.  npts = 0 stops
 * recording.  Reconfiguring clears the ring.
 */
int lbm_probe_config(lbm_t h, int npts, const double *xy_host, int every,
                     int64_t capacity);

/*
 * Copy the recorded series, oldest first, into buf_host (room for
 * max_records records of 1 + 3 npts doubles: the step number, then the
 * npts triples).  *n_records receives the number copied (at most
 * min(max_records, capacity) of the most recent ones).
 */
int lbm_probe_read(lbm_t h, double *buf_host, int64_t max_records,
                   int64_t *n_records);

/*
 * Flow state of time series (Sec. 3.3: stable, periodic, or aperiodic and
 * unstable, judged from the velocity at an observing point over a late
 * window; Table 3: periods).  The paper judges from plots; this library's
 * definition, computed on the device in FP64:
 *   amplitude A = max - min over the window; LBM_FLOW_STEADY if
 *   A <= steady_tol;
 *   D(T) = mean_{k < n-T} (u[k+T] - u[k])^2 / sigma^2 (sigma: standard
 *   deviation over the window) for lags T in [min_lag, max_lag]
 *   (max_lag <= 0: n / 3; capped at n - 2);
 *   a candidate is a lag with D(T-1) > D(T) <= D(T+1), min_lag < T <
 *   max_lag, reached after D exceeded 1 at a smaller lag; the parabola
 *   through D at T-1, T, T+1 gives the period (its vertex, in samples) and
 *   the mismatch sqrt(max(vertex value, 0));
 *   LBM_FLOW_PERIODIC at the first candidate with mismatch <= periodic_tol;
 *   LBM_FLOW_DRIFT if there is no candidate (the series never returns
 *   towards an earlier value within the window: a monotone approach, e.g.
 *   to a steady state, or a period longer than max_lag; mismatch = +inf);
 *   LBM_FLOW_APERIODIC otherwise (mismatch = the smallest over candidates).
 * A period should span a dozen or more samples; a shorter one can come out
 * as a multiple of itself.
 */
enum {
  LBM_FLOW_TOO_SHORT = -1,  /* batches: fewer records than the window */
  LBM_FLOW_STEADY = 0,
  LBM_FLOW_PERIODIC = 1,
  LBM_FLOW_APERIODIC = 2,
  LBM_FLOW_DRIFT = 3
};
typedef struct {
  int state;          /* LBM_FLOW_* */
  int lag;            /* integer lag of the period (periodic only) */
  double period;      /* refined period in samples; 0 unless periodic */
  double amplitude;   /* max - min over the window */
  double mean, std;   /* over the window */
  double mismatch;    /* see above; 0 when steady */
  double cycle;       /* dominant cycle: the refined lag of the first
                         candidate whatever its mismatch (samples; 0 if none);
                         a modulated oscillation repeats exactly (period)
                         only after several cycles */
  double cycle_mismatch;  /* the mismatch at that candidate (+inf if none) */
} lbm_flow_state_t;

/*
 * Classify nseries device series: sample k of series s at
 * series_dev[s * ld + k] (caller-owned device memory, n >= 8 samples,
 * ld >= n).  1 <= min_lag; the lag range must hold at least 3 lags.
 * out_host: nseries records (caller-owned host).  Work runs on hip_stream
 * (NULL: the default stream); the call allocates and frees its device
 * scratch and returns after the work has finished.
 * Errors: LBM_EINVAL for bad sizes, lags or NULL pointers.
 */
int lbm_classify_series(const double *series_dev, int nseries, int64_t n, int64_t ld,
                        double steady_tol, double periodic_tol, int min_lag, int max_lag,
                        lbm_flow_state_t *out_host, void *hip_stream);

/*
 * lbm_classify_series for callers that cannot allocate device memory (code
 * under HIP graph capture, tight serving loops, harnesses that forbid
 * hipMalloc).  Same inputs, definition and results, bit for bit; but:
 *   - out_dev: nseries records in caller-owned DEVICE memory, written by
 *     the kernel;
 *   - asynchronous: the work is only issued on hip_stream (NULL: the
 *     default stream) of the current device; read out_dev after that stream
 *     has finished.  No allocation, no host copy, no synchronisation.
 *   - its work memory is a fixed 32 MiB array per device (held from the
 *     library's load until the process ends): nseries * (2 n + 8) doubles
 *     must not exceed 4 Mi (4,194,304) doubles, e.g. 209 series of 10,000
 *     samples; LBM_EINVAL otherwise, checked before anything is issued;
 *   - every call on a device shares that device's array: calls that overlap
 *     in time on one device (on different streams, or from several host
 *     threads) race and give undefined results; calls issued one after
 *     another on one stream are safe.  Nothing in the array needs clearing
 *     between calls (each call writes every value it reads).
 * Errors: as lbm_classify_series; LBM_EDEVICE if the array's device address
 * cannot be obtained or the launch fails.
 */
int lbm_classify_series_noalloc(const double *series_dev, int nseries, int64_t n, int64_t ld,
                                double steady_tol, double periodic_tol, int min_lag,
                                int max_lag, lbm_flow_state_t *out_dev, void *hip_stream);

/*
 * Classify the recorded probe series of h (lbm_probe_config) directly on
 * the device: for each probe point, component c (0: rho, 1: u_x, 2: u_y)
 * over the most recent `window` records, one record per `every` steps (so
 * a period in steps is period * every).  window must not exceed the
 * records held (min(recorded, capacity)).  out_host: npts records.
 */
int lbm_probe_classify(lbm_t h, int component, int64_t window, double steady_tol,
                       double periodic_tol, int min_lag, int max_lag,
                       lbm_flow_state_t *out_host);

/* Total mass sum_x rho(x) now, rho the zeroth moment of Eq. 3 (Sec. 2.1),
 * accumulated in FP64 (a fixed-order reduction on the device). */
int lbm_mass(lbm_t h, double *mass);

/*
 * Eq. 6 residual from the most recent monitor: sqrt(sum |u(t) - u(t-100)|^2
 * / sum |u(t-100)|^2).  *at_step receives t (-1 if no monitor has run).
 * The residual is +inf when the denominator is zero or when the reference
 * field was not taken exactly 100 steps before t.
 */
int lbm_residual(lbm_t h, double *residual, int64_t *at_step);

/*
 * Stream function Psi [ny][nx] (lattice units, host): Psi = 0 on the bottom
 * wall, dPsi/dy = -u_x, midpoint rule on site centres, so the clockwise
 * primary vortex has Psi > 0 (the sign of Tables 1-2).  Divide by
 * u_lid * nx for the normalisation of Table 1.
 */
int lbm_stream_function(lbm_t h, double *psi_host);

/*
 * A vortex of the stream function Psi above (Tables 1-2: the primary vortex,
 * its maximum of Psi and centre; the corner vortices; the bottom vortices).
 */
typedef struct {
  double psi;   /* Psi at the centre site, lattice units (as lbm_stream_function) */
  double x, y;  /* the site's centre in units of the width L: ((ix + 1/2)/nx, (iy + 1/2)/nx) */
  int ix, iy;   /* site indices, y = 0 at the bottom */
  int kind;     /* +1: local maximum of Psi, -1: local minimum */
  int reserved;
} lbm_vortex_t;

/*
 * Primary and bottom corner vortices of the current state (Table 1's three
 * column groups), computed on the device in FP64:
 *   out[0] = the site of maximal Psi over the lattice (the primary vortex),
 *   out[1] = the site of minimal Psi with x < nx/2, y < min(ny, nx/2)
 *            (lower-left vortex),
 *   out[2] = likewise with x >= nx/2 (lower-right vortex).
 * Ties go to the smaller linear index y nx + x.  out[1] and out[2] are
 * the minima of those regions even where no corner vortex exists (then
 * their Psi is >= 0).  out is a caller-owned host array of 3 records.
 * Errors: LBM_EINVAL for NULL arguments or nx < 2 (no lower-right region).
 */
int lbm_vortex_extrema(lbm_t h, lbm_vortex_t *out);

/*
 * Vortex centres of the current state: every site with
 * 1 <= ix <= nx-2 and 1 <= iy <= ny-2 where Psi is strictly greater (kind
 * +1) or strictly smaller (kind -1) than at all eight neighbouring sites,
 * with |Psi| >= min_abs_psi (lattice units; 0 keeps all).  *count receives
 * the number of centres; the first min(count, cap) of them in row-major
 * order (by iy, then ix) are written to out (caller-owned host array of cap
 * records; may be NULL when cap = 0).
 * Errors: LBM_EINVAL for cap < 0, a NULL count, or out NULL with cap > 0.
 */
int lbm_vortex_centres(lbm_t h, double min_abs_psi, int cap, lbm_vortex_t *out,
                       int *count);

/*
 * Number of bottom vortices (Table 2's last column): the vortex centres of
 * lbm_vortex_centres (same min_abs_psi) that lie strictly below the primary
 * vortex's row (iy < out[0].iy of lbm_vortex_extrema).
 */
int lbm_bottom_vortex_count(lbm_t h, double min_abs_psi, int *count);

/*
 * Replace the state by the populations f(t) [9][ny][nx] (host, the
 * distribution before the collision of Eq. 1).  The step counter restarts
 * at 0 and the residual reference is reset.  For LBM_F32_SHIFTED the stored
 * value is f - w rounded to FP32.
 */
int lbm_set_populations(lbm_t h, const double *f_host);

/*
 * Read the stored post-collision populations f*(t) = f - (f - f^eq)/tau
 * (the right-hand side of Eq. 1 at step t), [9][ny][nx] doubles (host).
 * Their moments rho, rho u equal those of f(t).
 */
int lbm_get_populations(lbm_t h, double *fstar_host);

/*
 * Warm start: f = f^eq(rho, u) from fields [ny][nx] (host; NULL rho = 1,
 * NULL velocity = 0).  Flags:
 *   LBM_INIT_RENORMALISE_MASS  scale rho so the total mass is nx * ny (that
 *                              of the rest state);
 *   LBM_INIT_ZERO_STAGGERED    remove the two staggered momenta
 *                              P_x = sum (-1)^x rho u_x and
 *                              P_y = sum (-1)^y rho u_y by subtracting a
 *                              uniform (-1)^x (or (-1)^y) momentum.
 * Why the second flag: collision conserves each site's momentum and every
 * link or wall reflection moves a population with c_x != 0 to the other
 * column parity or reverses it, so P_y(t+1) = -P_y(t) and P_x(t+1) =
 * -P_x(t) (+ u_lid/3 if nx is odd) hold exactly for the whole nonlinear
 * update.  A start from rest has P = 0; a general start keeps a
 * non-decaying two-step oscillation that Eq. 6 (which compares states 100
 * steps apart, of equal parity) cannot see, and converges to a different
 * state.  With the flag, the start lies on the rest state's invariant set.
 * Step counter restarts at 0.
 */
enum { LBM_INIT_RENORMALISE_MASS = 1, LBM_INIT_ZERO_STAGGERED = 2 };
int lbm_init_fields(lbm_t h, const double *rho_host, const double *ux_host,
                    const double *uy_host, int flags);

/* As lbm_init_fields with caller-owned *device* arrays (e.g. torch tensors). */
int lbm_init_fields_device(lbm_t h, const double *rho_dev, const double *ux_dev,
                           const double *uy_dev, int flags);

/*
 * Checkpoint: write / read a header (magic, version, nx, ny, dtype, steps,
 * tau, u_lid) followed by the raw stored populations.  Restoring gives a
 * bitwise-identical continuation.  LBM_EIO on file errors, LBM_ESTATE if
 * the file's lattice or dtype differs from the handle's.
 */
int lbm_save(lbm_t h, const char *path);
int lbm_load(lbm_t h, const char *path);

/* ------------------------------------------------------------------------
 * Batched sweep: many cavities of uneven size advanced by one launch per
 * step (the Re x Ar sweep of Sec. 3.3 / Fig. 17 as one job).
 *
 * All cavities share the lid speed and storage type; cavity k has its own
 * nx[k] x ny[k] lattice and Reynolds number re[k] (tau_k = 3 u nx_k / re_k
 * + 1/2).  Each cavity evolves exactly as a single cavity created with the
 * same arguments (bit for bit: the per-site arithmetic is the same).
 * Steps are applied to the *active* cavities; inactive ones keep their state
 * and step count.  Monitors (mass, Eq. 6) run per cavity every 100 batch
 * steps; aligned runs of LBM_OPT_GRAPH_STEPS steps replay a HIP graph.
 * Cavity indices k are 0-based; out-of-range k gives LBM_EINVAL.
 * ---------------------------------------------------------------------- */
typedef struct lbm_batch *lbm_batch_t;

/* Errors as lbm_create, per cavity; 1 <= n <= 4096; the total storage must
 * stay below 2^31 elements per buffer. */
int lbm_batch_create(int n, const int *nx, const int *ny, const double *re,
                     double u_lid, int dtype, lbm_batch_t *out);
int lbm_batch_destroy(lbm_batch_t b);
int lbm_batch_set_stream(lbm_batch_t b, void *hip_stream);
int lbm_batch_set_option(lbm_batch_t b, int option, int64_t value);
int lbm_batch_get_option(lbm_batch_t b, int option, int64_t *value);

/* Advance every active cavity n >= 0 steps.  With a threshold set, a cavity
 * whose Eq. 6 residual is below it at a monitor becomes inactive at the next
 * multiple of 100 steps (checked after each captured chunk).  Stops early
 * when no cavity is active.  LBM_EUNSTABLE if a monitor is not finite. */
int lbm_batch_step(lbm_batch_t b, int64_t n);

/* Residual threshold for automatic deactivation (0 = off, the default). */
int lbm_batch_set_threshold(lbm_batch_t b, double residual);

/* Switch cavity k on or off; only at a multiple of 100 batch steps. */
int lbm_batch_set_active(lbm_batch_t b, int k, int active);

/* The last Eq. 6 residual of every cavity, residuals_host[n] (+inf where
 * none or not valid); the values lbm_batch_status reports one by one. */
int lbm_batch_residuals(lbm_batch_t b, double *residuals_host);

/* Per-cavity state: steps applied to it, last Eq. 6 residual (+inf if none
 * or not valid), the step of that monitor (-1 if none), active flag.
 * NULL outputs are skipped. */
int lbm_batch_status(lbm_batch_t b, int k, int64_t *steps_done,
                     double *residual, int64_t *residual_step, int *active);

/* As the single-cavity calls, for cavity k (host buffers [ny_k][nx_k] or
 * [9][ny_k][nx_k] doubles). */
int lbm_batch_mass(lbm_batch_t b, int k, double *mass);
int lbm_batch_moments(lbm_batch_t b, int k, double *rho_host, double *ux_host,
                      double *uy_host);
int lbm_batch_get_populations(lbm_batch_t b, int k, double *fstar_host);
int lbm_batch_set_populations(lbm_batch_t b, int k, const double *f_host);
int lbm_batch_init_fields(lbm_batch_t b, int k, const double *rho_host,
                          const double *ux_host, const double *uy_host, int flags);

/* As lbm_batch_init_fields with caller-owned device arrays. */
int lbm_batch_init_fields_device(lbm_batch_t b, int k, const double *rho_dev,
                                 const double *ux_dev, const double *uy_dev, int flags);

/* Training target of the warm-start network from cavity k's current state:
 * the 256 x 128 canvas of include/lbm.h's surrogate section, pixel (x, y)
 * (y < round(128 ny/nx)) = bilinear probe at ((x + 1/2)/128, (y + 1/2)/128)
 * in units of L; target_dev FP32 [256][128][3] = (100 (rho - 1),
 * u_x/u_lid, u_y/u_lid), mask_dev FP32 [256][128] (1 inside, 0 outside).
 * LBM_EINVAL if round(128 ny/nx) is not in [1, 256]. */
int lbm_batch_canvas(lbm_batch_t b, int k, float *target_dev, float *mask_dev);

/*
 * Probe time series of a batch (the observing points of Sec. 3.3, one set
 * per cavity): npts points per cavity, xy_host [n][npts][2] in units of L
 * (bilinear over site centres as lbm_probe), recorded at every monitor of
 * an active cavity -- every 100 of its steps -- into a ring of `capacity`
 * records per cavity.  npts = 0 removes the probes.  Recording starts at
 * the next monitor; reconfiguring drops earlier records.
 * Errors: LBM_EINVAL for npts outside [0, 4096], capacity < 1, NULL xy, or
 * rings above 64 GB; LBM_ENOMEM.
 */
int lbm_batch_probe_config(lbm_batch_t b, int npts, const double *xy_host, int64_t capacity);

/*
 * The most recent min(max_records, held) records of cavity k, oldest first,
 * each 3 npts doubles (rho, u_x, u_y per point), into buf_host.
 * *first_step receives the cavity's step count at the first returned record
 * (records are 100 of its steps apart); -1 if none.
 */
int lbm_batch_probe_read(lbm_batch_t b, int k, double *buf_host, int64_t max_records,
                         int64_t *n_records, int64_t *first_step);

/*
 * Flow state (lbm_classify_series' definition) of component c (0: rho,
 * 1: u_x, 2: u_y) of every probe point of every cavity over its most recent
 * `window` records (window <= capacity), on the device.  out_host: [n][npts]
 * records; cavities with fewer records than the window get
 * LBM_FLOW_TOO_SHORT.  Periods are in records (100 steps each).
 */
int lbm_batch_probe_classify(lbm_batch_t b, int component, int64_t window, double steady_tol,
                             double periodic_tol, int min_lag, int max_lag,
                             lbm_flow_state_t *out_host);

/* Lattice, Reynolds number and lid speed of cavity k (NULL outputs skipped). */
int lbm_batch_cavity(lbm_batch_t b, int k, int *nx, int *ny, double *re,
                     double *u_lid);

/* Number of cavities, total sites, batch steps applied, device bytes held. */
int lbm_batch_info(lbm_batch_t b, int *n, int64_t *total_sites,
                   int64_t *steps_done, size_t *device_bytes);

/* Autotuner of the batch kernel's tile shape; as lbm_autotune with `chunks`
 * captured graphs of LBM_OPT_GRAPH_STEPS steps per shape (1..1000).  Must be
 * called at a multiple of 100 steps; the cavities' states are restored.
 * The batch has its own list of LBM_OPT_NUM_VARIANTS shapes (one-step,
 * vector and multi-step shapes); steps off the 100-step grid always use
 * the one-step shape 0. */
int lbm_batch_autotune(lbm_batch_t b, int chunks, int use_cache,
                       int *best_variant, double *ms_per_step);

/* ------------------------------------------------------------------------
 * Learned warm start (an extension of the method; no counterpart in the paper).
 *
 * A convolutional surrogate maps (Re, Ar) to the steady field of the cavity
 * so the lattice can start near its steady state instead of at rest
 * (Sec. 2.2 (i)); the solver then converges by Eq. 1 as usual and the
 * converged state does not depend on the start.
 *
 * Network: 4-level U-Net on a 256 (y) x 128 (x) canvas, NHWC bfloat16
 * activations, FP32 master weights, FP32 accumulation on the BF16 matrix
 * cores.  Input channels: cavity mask (rows y < round(128 Ar)),
 * (x + 1/2)/128, (y + 1/2)/128, Re/3000, Ar/2.  Output channels:
 * 100 (rho - 1), u_x / u_lid, u_y / u_lid on the 128 x round(128 Ar) cavity
 * pixels (pixel centres at ((x + 1/2)/128, (y + 1/2)/128) in units of L).
 * Convolutions 3 x 3, zero padding, ReLU; 2 x 2 average pooling; nearest 2x
 * upsampling; skip concatenation.  Channel widths 32, 64, 128, 256;
 * 1,964,448 parameters (padding included) stored as, for each of the 15
 * convolutions in order, weights [9][ci][co] (tap = 3 dy + dx) then bias
 * [co], with ci of the first and co of the last layer padded to 32 (padding
 * entries must be zero).
 * ------------------------------------------------------------------------ */
typedef struct lbm_surrogate *lbm_sur_t;

/* A surrogate for batches of up to max_batch (1..256) samples; parameters
 * start at zero (load them with lbm_sur_set_params). */
int lbm_sur_create(int max_batch, lbm_sur_t *out);
int lbm_sur_destroy(lbm_sur_t s);
/* Work is issued on hip_stream (NULL: a stream of the handle's own).  The
 * training step's weight gradients run on a second stream of the handle,
 * ordered after the work on hip_stream that produces their inputs; before
 * the backward pass returns, hip_stream waits for them, so every later
 * operation on hip_stream sees them (both joins are events). */
int lbm_sur_set_stream(lbm_sur_t s, void *hip_stream);
int lbm_sur_num_params(lbm_sur_t s, int64_t *n);

/* Load n FP32 parameters (host, layout above); resets the optimiser. */
int lbm_sur_set_params(lbm_sur_t s, const float *params_host, int64_t n);

/* He-normal initialisation from n standard normal draws (host): weight i of
 * a layer = draw i x sqrt(2 / (9 ci_real)) (ci_real = 5 for the first
 * layer), padding entries and biases zero; resets the optimiser. */
int lbm_sur_init_params(lbm_sur_t s, const float *normals_host, int64_t n);

/* Copy the FP32 parameters and / or the gradients of the last training step
 * to host arrays of lbm_sur_num_params floats (either may be NULL). */
int lbm_sur_get_params(lbm_sur_t s, float *params_host, float *grads_host);

/* Forward pass for n samples (Re, Ar host arrays; 0 < Ar <= 2): out_dev
 * receives FP32 [n][256][128][3] (device). */
int lbm_sur_forward(lbm_sur_t s, int n, const double *re, const double *ar,
                    float *out_dev);

/* One training step on n samples: masked mean-squared error against
 * target_dev (FP32 [n][256][128][3], device) with mask_dev (FP32
 * [n][256][128], 1 on cavity pixels), loss = sum over masked pixels and the
 * three channels / number of masked pixels; backward pass; if apply_update,
 * one Adam step (beta 0.9, 0.999, eps 1e-8) with learning rate lr.  *loss
 * receives the loss before the update.  LBM_EUNSTABLE on a non-finite
 * loss. */
int lbm_sur_train_step(lbm_sur_t s, int n, const double *re, const double *ar,
                       const float *target_dev, const float *mask_dev,
                       double lr, int apply_update, double *loss);

/* Warm start: predict the field for the handle's (Re, Ar = ny/nx), map it
 * bilinearly onto the lattice (site centres in units of L, clamped to the
 * cavity pixels), renormalise the mass to nx ny, remove the staggered
 * momenta and set f = f^eq (lbm_init_fields_device with both flags).  The
 * step counter restarts at 0. */
int lbm_sur_warm_start(lbm_sur_t s, lbm_t h);
int lbm_sur_warm_start_batch(lbm_sur_t s, lbm_batch_t b, int k);

/* Single layer kernels (device pointers, bf16 stored as 16-bit words;
 * tensors NHWC with a channel stride and offset so slices of a
 * concatenation can be read or written; channel counts multiples of 32,
 * the strides and offsets of the tensors read multiples of 8 and the
 * tensors 16-byte aligned; LBM_EINVAL for a bad shape, stride or offset):
 *   mode 0 forward:  out[p, oo+o] = relu?(sum_{t,c} x[p+d_t, xo+c] w[t][c][o]
 *                                   + bias[o])
 *   mode 1 dgrad:    out[p, oo+c] (+)= sum_{t,o} x[p-d_t, xo+o] w[t][c][o]
 *                    (x is the output gradient, accumulate adds)
 *   mode 2 wgrad:    out[t][c][o] += sum_p x[p+d_t, xo+c] g[p, go+o]
 *                    (out FP32 [9][ci][co]; per-chunk partials (a chunk
 *                    of pixels per block chain, sized from the layer's
 *                    shape) added in chunk order, so the result does not
 *                    depend on scheduling; the call allocates the partials,
 *                    synchronises the stream and frees them)
 *   (mode 0 likewise allocates a transposed copy of w for the call,
 *   synchronises the stream and frees it; mode 1 only issues the work)
 * d_t = (dy - 1, dx - 1) for tap t = 3 dy + dx, zero outside the image. */
int lbm_nn_conv3x3(int mode, int n, int h, int w, int ci, int co,
                   const void *x, int xs, int xo, const void *g, int gs, int go,
                   const void *wt, const float *bias, int relu, void *out,
                   int os, int oo, int accumulate, void *stream);
/* gb[o] += sum_p g[p, go+o] over npix pixels; co a multiple of 8 in
 * [8, 256], gs and go multiples of 8 with go + co <= gs, g 16-byte aligned
 * (LBM_EINVAL otherwise); per-chunk partial sums added in chunk order
 * (deterministic; the call allocates the partials, synchronises the stream
 * and frees them). */
int lbm_nn_bias_grad(int npix, int co, const void *g, int gs, int go,
                     float *gb, void *stream);
/* (pooling and upsampling: c, channel strides and offsets multiples of 8,
 * tensors 16-byte aligned; LBM_EINVAL otherwise)
 * 2 x 2 average pooling of an h x w (even) image: forward reads a slice
 * (is, io) and writes dense [n][h/2][w/2][c]; backward reads the dense
 * gradient and writes (or adds into, accumulate) the slice (os, oo). */
int lbm_nn_pool2(int backward, int n, int h, int w, int c, const void *in,
                 int is, int io, void *out, int os, int oo, int accumulate,
                 void *stream);
/* Nearest 2x upsampling of an h x w image: forward reads dense [n][h][w][c]
 * and writes the slice (os, oo) of [n][2h][2w]; backward sums the gradient
 * slice (is, io) of [n][2h][2w] into dense [n][h][w][c]. */
int lbm_nn_up2(int backward, int n, int h, int w, int c, const void *in,
               int is, int io, void *out, int os, int oo, void *stream);

/* ------------------------------------------------------------------------
 * 3-D lid-driven box (D3Q19), the extension Sec. 4 names as future work.
 *
 * The same method on the D3Q19 set (weights 1/3, 1/18, 1/36; c_s^2 = 1/3):
 * nx x ny x nz sites, half-way bounce-back on all six faces, the lid above
 * the top row y = ny - 1 moving with (u_lid, 0, 0) and owning every link
 * through its plane (links 8 = (-1,-1,0) and 9 = (1,-1,0) pick up -/+ u_lid/6),
 * tau = 3 u_lid nx / re + 1/2.  Velocity order:
 *   0 (0,0,0); 1 (1,0,0) 2 (-1,0,0) 3 (0,1,0) 4 (0,-1,0) 5 (0,0,1) 6 (0,0,-1)
 *   7 (1,1,0) 8 (-1,-1,0) 9 (1,-1,0) 10 (-1,1,0) 11 (1,0,1) 12 (-1,0,-1)
 *   13 (1,0,-1) 14 (-1,0,1) 15 (0,1,1) 16 (0,-1,-1) 17 (0,1,-1) 18 (0,-1,1).
 * Host arrays are [nz][ny][nx] doubles (populations [19][nz][ny][nx]).
 * Storage LBM_F64 or LBM_F32_SHIFTED as in two dimensions; monitors (mass,
 * Eq. 6 over the three velocity components) every 100 steps in FP64; aligned
 * 100-step chunks replayed from HIP graphs.  Options LBM_OPT_USE_GRAPH,
 * LBM_OPT_STEP_VARIANT (8 tile shapes: 0-2 one step per launch, 64 x {1,
 * 2, 4} sites of a z plane; 3-7 two steps per launch: 3 a 3-D tile kept in
 * LDS, FP32 32 x 8 x 4, FP64 16 x 6 x 4; 4-7 a column marching through z
 * with three planes of step-1 results in LDS, FP32 64 x 8, 64 x 12,
 * 32 x 16, 32 x 24, FP64 32 x 12, 32 x 8, 16 x 16, 24 x 16; every shape
 * gives the same bits), LBM_OPT_NUM_VARIANTS,
 * LBM_OPT_STEPS_PER_LAUNCH (1 or 2).
 * ------------------------------------------------------------------------ */
typedef struct lbm_cube *lbm3d_t;

/* Create a box at rest.  Errors: LBM_EINVAL for a side outside [2, 4096],
 * re <= 0, tau <= 1/2, |u_lid| >= 1/sqrt(3), unknown dtype, or a box whose
 * 19 planes exceed 2^31 elements; LBM_ENOMEM / LBM_EDEVICE. */
int lbm3d_create(int nx, int ny, int nz, double re, double u_lid, int dtype, lbm3d_t *out);
int lbm3d_destroy(lbm3d_t h);
int lbm3d_set_stream(lbm3d_t h, void *hip_stream);
int lbm3d_set_option(lbm3d_t h, int option, int64_t value);
int lbm3d_get_option(lbm3d_t h, int option, int64_t *value);
/* Advance n >= 0 steps; LBM_EUNSTABLE if a monitor goes non-finite. */
int lbm3d_step(lbm3d_t h, int64_t n);
int lbm3d_steps_done(lbm3d_t h, int64_t *steps);
/* Eq. 6 from the last monitor (+inf if none or not 100 steps apart). */
int lbm3d_residual(lbm3d_t h, double *residual, int64_t *at_step);
/* sum rho over the box, FP64. */
int lbm3d_mass(lbm3d_t h, double *mass);
/* rho, u_x, u_y, u_z [nz][ny][nx] (host; NULL outputs skipped). */
int lbm3d_moments(lbm3d_t h, double *rho_host, double *ux_host, double *uy_host,
                  double *uz_host);
/* Replace the state by f(t) [19][nz][ny][nx] (host, before the collision);
 * the step counter restarts at 0. */
int lbm3d_set_populations(lbm3d_t h, const double *f_host);
/* Stored post-collision populations f*(t) [19][nz][ny][nx] (host). */
int lbm3d_get_populations(lbm3d_t h, double *fstar_host);
/* Time the tile shapes over `chunks` 100-step chunks (1..1000), keep the
 * fastest; state, counters and the Eq. 6 reference are restored. */
int lbm3d_autotune(lbm3d_t h, int chunks, int *best_variant, double *ms_per_step);

#ifdef __cplusplus
}
#endif

#endif /* LBM_H */
