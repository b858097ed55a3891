/*
 * dg2.h - C ABI of the MI355X (gfx950) DG2 flood-model time step.
 *
 * The library advances the 2D shallow water equations with the
 * slope-decoupled second-order discontinuous Galerkin (DG2) method of
 * Ayog, Kesserwani, Shaw, Sharifian & Bau, "Second-order discontinuous
 * Galerkin flood model: comparison with industry-standard finite volume
 * models", Sec. 2.1, on one GPU:
 *
 *   - per-element planar modes (mean, x-slope, y-slope) of h, hu, hv
 *     (Sec. 2.1.1, Eq. 2) on a uniform grid of nx x ny rectangles (Sec. 2);
 *   - face limits, positivity-preserving dummy limits and the wall revision
 *     of the bed, an HLL two-argument flux, dummy modes and the operators
 *     L0, L1x, L1y with the well-balanced bed source (Sec. 2.1.2, Eq. 4-5);
 *   - implicit Manning friction split at the centre and the four Gauss
 *     points before each RK2 step (Sec. 2.1.3, Eq. 1 for C_f);
 *   - optional local slope limiting, DG2-LL (Sec. 2.1.3, Eq. 6-7);
 *   - explicit two-stage RK2 with a Courant-limited global time step
 *     (Sec. 2.1.2).
 *
 * Conventions shared by every call:
 *   - Cells are indexed c = j*nx + i, i west->east, j south->north; the cell
 *     centre is (x0 + (i+0.5) dx, y0 + (j+0.5) dy).
 *   - Corner arrays hold (ny+1)*(nx+1) values, row-major, x fastest.
 *   - A mode state is 9 planes of nx*ny values in the order
 *       h0, h1x, h1y, qx0, qx1x, qx1y, qy0, qy1x, qy1y
 *     (mean and slope coefficients of Eq. 2 for h, hu, hv).
 *   - Host arrays are always double and are copied during the call; the
 *     caller keeps ownership.  FP32 contexts convert on the way in and out.
 *   - Every call returns a dg2_status and never aborts or throws.  The text
 *     of the last failure on a context is returned by dg2_last_error(ctx);
 *     dg2_last_error(NULL) gives the last failure of dg2_create on this
 *     thread.  Invalid sizes or parameters, NaN inputs and negative depths,
 *     discharges or Manning values return DG2_EINVAL and change nothing.
 *   - A NaN found in the state on the device is latched and returned as
 *     DG2_ENUMERIC by the next dg2_sync, dg2_get_state, dg2_read_gauges or
 *     dg2_diagnostics.  Depths are never clipped: a negative mean depth is
 *     reported by dg2_diagnostics (min_h), not as an error.
 *   - Work is queued on the context's HIP stream; calls that return host
 *     data synchronise that stream.  A context must be used from one host
 *     thread at a time.
 */
#ifndef DG2_H
#define DG2_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct dg2_ctx dg2_ctx;

typedef enum {
  DG2_OK = 0,
  DG2_EINVAL = -1,       /* bad argument; nothing was changed            */
  DG2_ENOMEM = -2,       /* device or host allocation failed             */
  DG2_EHIP = -3,         /* a HIP runtime call failed                    */
  DG2_ESTATE = -4,       /* call not valid in the current state          */
  DG2_ENUMERIC = -5,     /* NaN found in the state on the device         */
  DG2_EUNSUPPORTED = -6  /* option not available in this library         */
} dg2_status;

typedef enum { DG2_FP64 = 0, DG2_FP32 = 1 } dg2_prec;
/* DG2_NL: no limiting.  DG2_LL: local limiting of Sec. 2.1.3 (the paper's
 * DG2-LL, also called DG2+minmod). */
typedef enum { DG2_NL = 0, DG2_LL = 1 } dg2_variant;
typedef enum { DG2_WEST = 0, DG2_EAST = 1, DG2_SOUTH = 2, DG2_NORTH = 3 } dg2_side;
/* Boundary segments default to solid walls (mirror ghost cells).  An inflow
 * segment takes a discharge hydrograph (dg2_set_inflow_hydrograph). */
/* Boundary kinds of a segment of one side (the rest of the side is a wall).
 * DG2_BC_INFLOW_Q: prescribed discharge hydrograph (dg2_set_inflow_hydrograph).
 * DG2_BC_LEVEL: prescribed water-level hydrograph (dg2_set_level_hydrograph),
 *   as at the west boundary of the Sec. 3.1.1 benchmark: the outside of each
 *   face is a ghost at depth max(0, eta(t) - z_face) whose normal velocity
 *   keeps the Riemann invariant leaving the domain (an inflow capped at the
 *   critical speed); its tangential velocity is zero where that normal
 *   velocity enters the domain and the inside one where it leaves.
 * DG2_BC_OPEN: transmissive: the ghost holds the inside cell's mean state. */
typedef enum { DG2_BC_WALL = 0, DG2_BC_INFLOW_Q = 1, DG2_BC_LEVEL = 2, DG2_BC_OPEN = 3 } dg2_bc;
/* Two-argument face flux of Sec. 2.1.2.  DG2_FLUX_HLL (default): HLL with
 * two-rarefaction wave-speed estimates and dry-bed front speeds.
 * DG2_FLUX_ROE: Roe's solver, the paper's choice (Roe averages, no entropy
 * fix), with the HLL flux at faces that have a side at or below tol_dry. */
typedef enum { DG2_FLUX_HLL = 0, DG2_FLUX_ROE = 1 } dg2_flux;

typedef struct {
  int32_t nx, ny;         /* cells in x and y, each >= 1                      */
  double dx, dy;          /* element size (m), > 0                            */
  double x0, y0;          /* south-west corner of the domain (m)              */
  int32_t prec;           /* dg2_prec: arithmetic and storage of the state    */
  int32_t variant;        /* dg2_variant                                      */
  double g;               /* gravity (m/s^2), default 9.81                    */
  double cfl;             /* Courant number, default 0.3 (Sec. 2.1.2)         */
  double tol_dry;         /* drying tolerance (m), default 1e-5 (Sec. 2.1.3)  */
  double ll_threshold;    /* shock-detector threshold, default 10 (Eq. 6)     */
  double dt_max;          /* cap on the time step (s), default 1              */
  void *hip_stream;       /* borrowed hipStream_t; NULL: the library makes one */
  int32_t flux;           /* dg2_flux, default DG2_FLUX_HLL                   */
} dg2_config;

/* Fill *cfg with the defaults above for an nx x ny grid of dx x dy cells
 * (FP64, DG2-NL, origin 0, library-owned stream). */
void dg2_config_default(dg2_config *cfg, int32_t nx, int32_t ny, double dx, double dy);

/* Create a context on the current HIP device.  The grid is flat (z = 0),
 * dry, frictionless and closed by walls until the setters below change it.
 * On failure *out is NULL.  Returns DG2_EINVAL, DG2_ENOMEM or DG2_EHIP. */
dg2_status dg2_create(const dg2_config *cfg, dg2_ctx **out);

/* Release every device and host resource the context allocated.  NULL-safe. */
void dg2_destroy(dg2_ctx *ctx);

/* Message of the last failing call on ctx (NULL: last dg2_create failure of
 * this thread).  Valid until the next call on ctx. */
const char *dg2_last_error(const dg2_ctx *ctx);

/* Bed elevation at the (ny+1)*(nx+1) corner nodes (DEM points, Sec. 2.1.1).
 * The bed modes z0, z1x, z1y follow Eq. (3) from face-centre averages of the
 * corners, which makes the bed continuous across faces. */
dg2_status dg2_set_dem_corners(dg2_ctx *ctx, const double *z);

/* Manning coefficient n_M of Eq. (1): per cell (nx*ny values, >= 0) when
 * n_cell is not NULL, otherwise the uniform value n_uniform (>= 0). */
dg2_status dg2_set_manning(dg2_ctx *ctx, const double *n_cell, double n_uniform);

/* Initial condition from corner-node values (Eq. 3): the free surface
 * eta (is_eta != 0) or the depth h (is_eta == 0), and the unit discharges
 * qx, qy (NULL = 0).  From eta, the depth modes are the eta modes minus the
 * bed modes (a discrete lake at rest where eta is flat) and elements with a
 * negative mean depth are set dry.  Uses the current DEM.  Resets t to 0,
 * the step counter and the gauge record, and computes the first time step. */
dg2_status dg2_set_initial_corners(dg2_ctx *ctx, const double *surface, int32_t is_eta,
                                   const double *qx, const double *qy);

/* Replace the state by 9*nx*ny mode values (plane order above) at time t.
 * Depth modes may make face limits negative; mean depths must be >= 0. */
dg2_status dg2_set_state(dg2_ctx *ctx, const double *modes9, double t);

/* Copy the state out (modes9: 9*nx*ny doubles, may be NULL) with its time,
 * completed step count and the last step size (each pointer may be NULL).
 * Synchronises the stream; returns a latched DG2_ENUMERIC after copying. */
dg2_status dg2_get_state(dg2_ctx *ctx, double *modes9, double *t, int64_t *step, double *last_dt);

/* Declare cells first..last (0-based along the side: rows for west/east,
 * columns for south/north) of one side as a wall or an inflow segment.  One
 * inflow segment per side; DG2_BC_WALL on a side removes its segment.  An
 * inflow face carries the prescribed flux [q, q^2/h_b + g h_b^2/2, 0] in the
 * normal direction with q = Q(t)/(segment length) and h_b the larger of the
 * inner dummy depth and the critical depth of q; Q = 0 leaves a wall. */
dg2_status dg2_set_boundary(dg2_ctx *ctx, int32_t side, int32_t bc, int32_t first, int32_t last);

/* Discharge hydrograph Q(t) (m^3/s, >= 0) for the side's inflow segment:
 * n >= 1 samples at increasing times t; linear in between, held constant
 * outside.  Each RK stage uses Q at its own stage time. */
dg2_status dg2_set_inflow_hydrograph(dg2_ctx *ctx, int32_t side, const double *t, const double *Q,
                                     int32_t n);

/* Water-level hydrograph of a DG2_BC_LEVEL segment: free-surface elevation
 * eta (m, finite) at n >= 1 increasing times t; linear in between, held
 * outside.  Each RK stage uses eta at its own stage time. */
dg2_status dg2_set_level_hydrograph(dg2_ctx *ctx, int32_t side, const double *t, const double *eta,
                                    int32_t n);

/* Uniform rainfall of rate (m/s, >= 0) during [t_begin, t_end]: the mean
 * depth of every element gains rate * |[t, t+dt] intersect [t_begin, t_end]|
 * at the start of each step.  rate = 0 switches it off. */
dg2_status dg2_set_rainfall(dg2_ctx *ctx, double rate, double t_begin, double t_end);

/* Gauges at n points (xy: n pairs x, y in m, inside the domain; n <= 64).
 * After each step the planar solution (Eq. 2) is sampled there as
 * h, eta = h + z, u, v into a device record that keeps up to capacity
 * samples (capacity <= 0: 65536).  Clears the record.  n = 0 removes them. */
dg2_status dg2_set_gauges(dg2_ctx *ctx, const double *xy, int32_t n, int32_t capacity);

/* dt > 0: every step uses this step size (still capped by a run-to target).
 * dt <= 0: Courant-limited steps, dt = min(Cr min_c m_c, dt_max) with
 * m_c = min(dx/(|u|+c), dy/(|v|+c)) over wet cell means. */
dg2_status dg2_set_fixed_dt(dg2_ctx *ctx, double dt);

/* Queue nsteps time steps (asynchronous). */
dg2_status dg2_step(dg2_ctx *ctx, int32_t nsteps);

/* Advance until t == T: steps are queued in chunks, the last one shortened to
 * land exactly on T; returns when the stream reaches T.  T <= t is a no-op.
 * Later dg2_step calls are no longer bounded by T. */
dg2_status dg2_run_to(dg2_ctx *ctx, double T);

/* Wait for the queued work; returns DG2_ENUMERIC if a failure was latched. */
dg2_status dg2_sync(dg2_ctx *ctx);

/* Copy the gauge samples recorded since the last read (oldest first) into
 * out[ns][ng][4] (h, eta, u, v) and t[ns], with ns <= max_samples returned
 * in *ns; unread samples beyond max_samples stay queued.  If more than the
 * capacity were recorded since the last read the oldest are lost and the
 * call returns DG2_ESTATE after copying the rest. */
dg2_status dg2_read_gauges(dg2_ctx *ctx, double *out, double *t, int32_t max_samples,
                           int32_t *ns);

/* Domain integrals of the current state, reduced on the device in a fixed
 * order: mass = sum of h0 dx dy (Eq. 11), energy (Eq. 12, 2x2 Gauss rule per
 * element) and the smallest mean depth.  Any pointer may be NULL. */
dg2_status dg2_diagnostics(dg2_ctx *ctx, double *mass, double *energy, double *min_h);

/* The integrals of dg2_diagnostics for callers that cannot allocate device
 * memory (code under HIP graph capture, serving loops): no context, no
 * allocation, no host copy and no synchronisation.  Queues two kernels on
 * hip_stream (NULL: the null stream) and returns.
 *   state: 9 device planes of the modes (plane order above), each of
 *          plane_stride >= nx*ny elements, row-major with x fastest;
 *   bed:   3 device planes z0, z1x, z1y with the same plane stride;
 *   prec:  DG2_FP64 (double planes) or DG2_FP32 (float planes);
 *   out4:  device doubles, written when the kernels run: mass (m^3, Eq. 11),
 *          energy (Eq. 12, as dg2_diagnostics), smallest mean depth, and the
 *          number of NaN mean depths.
 * Buffers are borrowed for the duration of the queued work.  The partial
 * sums live in a static device array of 1024 records of 4 doubles (32 KiB)
 * that each GPU holds until the process ends, for any grid size; every call
 * on one GPU uses the same array, so calls that overlap on one GPU (two
 * streams, two threads) race, and must be ordered by the caller.  Errors:
 * DG2_EINVAL for NULL or misaligned pointers, nx or ny < 1, a stride below
 * nx*ny, a bad prec or non-positive dx, dy, g, tol_dry; DG2_EHIP if a launch
 * fails.  The message is dg2_last_error(NULL). */
dg2_status dg2_diagnostics_noalloc(const void *state, const void *bed, int32_t nx, int32_t ny,
                                   int64_t plane_stride, int32_t prec, double dx, double dy, double g,
                                   double tol_dry, double *out4, void *hip_stream);

/* Time nsteps steps with HIP events on the context's stream, one event pair
 * per kernel: average milliseconds of the stage-1 kernel, the stage-2 kernel
 * and of a whole step (any pointer may be NULL).  When the fused step kernel
 * runs (dg2_set_step_kernel), *ms_stage1 is that kernel's time and
 * *ms_stage2 is 0.  The steps are real steps of the simulation. */
dg2_status dg2_time_kernels(dg2_ctx *ctx, int32_t nsteps, double *ms_stage1, double *ms_stage2,
                            double *ms_step);

/* Launch shape of the step kernels (the per-stage kernels and the fused step
 * kernel alike): rows marched per wavefront (>= 1) and wavefronts per
 * workgroup (1, 2 or 4).  rows <= 0 restores the built-in choice for this
 * grid and kernel (about 34 000 wavefronts and at most 32 rows for the
 * per-stage kernels, about 5 800 wavefronts and at most 48 rows for the
 * fused kernel).  Results do not depend on it. */
dg2_status dg2_set_launch(dg2_ctx *ctx, int32_t rows_per_wave, int32_t waves_per_block);

/* Stage-1 Courant check (an option, off by default).  The step size comes
 * from the Courant bound Cr of Sec. 2.1.2 on the state at the start of the
 * step; on steep banks stage 1 can give a thin film speeds far beyond it, and
 * stage 2 then drives mean depths negative.  With repeats = n > 0, after
 * stage 1 the step is compared with Cr times the Courant minimum of the
 * stage-1 result; while it is larger, stage 1 is repeated (at most n times)
 * with that smaller step, which the time step then takes.  A fixed step size
 * (dg2_set_fixed_dt) is never changed.  Each step queues n repeat launches
 * that return at once when not needed: repeats of stage 1 with the per-stage
 * kernels, trials of the whole step with the fused step kernel (whose result
 * is the same).  Batches refuse members that use it.  repeats: 0..8, else
 * DG2_EINVAL. */
dg2_status dg2_set_stage_check(dg2_ctx *ctx, int32_t repeats);

/* Partly-wet rule (an option, off by default; not part of the paper's
 * method).  The paper flags dry elements by the mean depth alone (Sec.
 * 2.1.3): after each RK stage an element whose mean depth is at or below
 * tol_dry gets zero discharge modes, and nothing else changes.  With on = 1,
 * an element with a wet mean but a face-limit depth h0 - max(|h1x|, |h1y|)
 * at or below tol_dry also drops all six slope modes after each stage
 * (locally first order at a wet/dry front).  Batches refuse members that
 * differ in this setting.  on: 0 or 1, else DG2_EINVAL. */
dg2_status dg2_set_partly_wet_flat(dg2_ctx *ctx, int32_t on);

/* How dg2_step runs the two RK stages of Sec. 2.1.2.  fused = 1 (default):
 * one kernel per step that computes stage 1 a row ahead of stage 2 and keeps
 * the stage-1 result in registers, so a step reads and writes the state once;
 * it applies to DG2-NL (FP32 and FP64) with the state in library memory
 * (otherwise the per-stage kernels run).  fused = 0: one kernel per stage, with the stage-1
 * result in a device buffer.  Results are bitwise the same.  DG2_EINVAL for
 * other values. */
dg2_status dg2_set_step_kernel(dg2_ctx *ctx, int32_t fused);

/* Pick the launch shape (rows marched per wavefront x wavefronts per
 * workgroup) by timing candidates, the built-in shape first, on copies of
 * the current state (the state is restored afterwards); budget_ms bounds
 * the time spent.  With a tune cache (dg2_set_tune_cache) a shape stored for
 * the same key (GPU architecture, precision, variant, flux, fused or
 * per-stage kernels, grid size rounded up to powers of two) is taken without
 * timing; otherwise the chosen shape is stored there.  The chosen
 * rows-per-wave is returned in *rows (may be NULL).  The shape never changes
 * results.  DG2_EINVAL if the cache file cannot be written. */
dg2_status dg2_autotune(dg2_ctx *ctx, double budget_ms, int32_t *rows);

/* File of the autotuner's cache (a small JSON object, created if missing);
 * NULL or "" turns the cache off (the default).  Host arrays are copied. */
dg2_status dg2_set_tune_cache(dg2_ctx *ctx, const char *path);

/* Current launch shape: rows per wavefront, wavefronts per workgroup, and
 * whether the last dg2_autotune took it from the cache (1) or not (0).
 * Any pointer may be NULL. */
dg2_status dg2_get_launch(const dg2_ctx *ctx, int32_t *rows, int32_t *waves, int32_t *from_cache);

/* Bytes of device memory a state needs (9 planes, padded plane stride) and
 * the plane stride in elements; for dg2_bind_device_state. */
dg2_status dg2_state_layout(const dg2_ctx *ctx, size_t *bytes, size_t *plane_stride);

/* Keep the state in caller-owned device memory (e.g. a torch tensor) of at
 * least dg2_state_layout bytes, 256-byte aligned.  The current state is
 * copied in; the buffer is borrowed and must outlive the context or the
 * next dg2_bind_device_state(ctx, NULL, 0), which returns to own memory.
 * With a bound state dg2_step runs the per-stage kernels, which update the
 * state in place (the fused step writes to a second buffer). */
dg2_status dg2_bind_device_state(dg2_ctx *ctx, void *dev_ptr, size_t bytes);

/* ------------------------------------------------------------------------
 * Batched ensemble.  A batch advances many independent scenarios (contexts of
 * any grid size) together: each RK stage is one persistent launch whose
 * wavefronts stride through the (scenario, strip, row-segment) work items of
 * all members, and each scenario keeps its own device-resident time step,
 * time, inflows, rain and Courant minimum, exactly as if it were stepped
 * alone (results are bitwise those of dg2_step on each member).  Steps are
 * replayed from a captured HIP graph.  When every member would step with the
 * fused step kernel (dg2_set_step_kernel) the batch does too: one persistent
 * launch per step over all members.
 * ------------------------------------------------------------------------ */
typedef struct dg2_batch dg2_batch;

/* Build a batch from n >= 1 fully set-up contexts of the same precision,
 * variant, g, tol_dry and ll_threshold.  The contexts stay owned by the
 * caller and must outlive the batch; their parameters are read now (call
 * dg2_batch_refresh after changing them).  While the batch is in use, step
 * members only through it; call dg2_batch_sync before reading a member with
 * dg2_get_state, dg2_read_gauges or dg2_diagnostics.  hip_stream: borrowed
 * stream, or NULL for one owned by the batch.  Errors: DG2_EINVAL (bad or
 * mixed members), DG2_ENOMEM, DG2_EHIP. */
dg2_status dg2_batch_create(dg2_ctx *const *members, int32_t n, void *hip_stream, dg2_batch **out);

/* Release the batch's resources (not the members).  NULL-safe. */
void dg2_batch_destroy(dg2_batch *b);

/* Message of the last failing call on b (NULL: last dg2_batch_create failure). */
const char *dg2_batch_last_error(const dg2_batch *b);

/* Re-read the members' parameters (boundaries, hydrographs, rain, Manning,
 * fixed dt, gauges, bound state buffers).  A member's state buffer is also
 * re-read by itself when it changed (a member stepped alone by the fused
 * step kernel alternates between two buffers). */
dg2_status dg2_batch_refresh(dg2_batch *b);

/* Rows per wavefront (<= 0: built-in choice), wavefronts per workgroup (1, 2
 * or 4) and steps per captured graph (<= 1: no graph, eager launches; with
 * the fused step kernel an odd count is rounded up, since each step switches
 * the members between their two state buffers).  Results do not depend on
 * these. */
dg2_status dg2_batch_set_launch(dg2_batch *b, int32_t rows_per_wave, int32_t waves_per_block,
                                int32_t graph_steps);

/* Time candidate launch shapes on the members' current states (restored
 * afterwards) and keep the fastest: rows per wavefront x wavefronts per
 * workgroup at the current graph length, then graph lengths 8, 16, 32 at the
 * best shape; each candidate is timed over two graph replays.  budget_ms
 * bounds the time spent.  With a tune cache (dg2_batch_set_tune_cache) a
 * stored entry for the same key is taken without timing, else the choice is
 * stored.  The chosen rows-per-wave is returned in *rows (may be NULL). */
dg2_status dg2_batch_autotune(dg2_batch *b, double budget_ms, int32_t *rows);

/* Tune cache of a batch (as dg2_set_tune_cache); the key adds the member
 * count and the total cell count rounded up to a power of two, and an entry
 * holds rows per wavefront, wavefronts per workgroup and the graph length. */
dg2_status dg2_batch_set_tune_cache(dg2_batch *b, const char *path);

/* Current batch launch shape and graph length, and whether the last
 * dg2_batch_autotune took them from the cache.  Any pointer may be NULL. */
dg2_status dg2_batch_get_launch(const dg2_batch *b, int32_t *rows, int32_t *waves, int32_t *graph_steps,
                                int32_t *from_cache);

/* Queue nsteps time steps of every member (asynchronous). */
dg2_status dg2_batch_step(dg2_batch *b, int32_t nsteps);

/* Advance every member to time T (each lands on T exactly); returns when all
 * have arrived.  Later dg2_batch_step calls are no longer bounded by T. */
dg2_status dg2_batch_run_to(dg2_batch *b, double T);

/* Wait for the batch's queued work; DG2_ENUMERIC if a member latched a NaN. */
dg2_status dg2_batch_sync(dg2_batch *b);

/* Run nsteps steps bracketed by HIP events on the batch stream and return
 * the average milliseconds per step (all members). */
dg2_status dg2_batch_time_steps(dg2_batch *b, int32_t nsteps, double *ms_per_step);


/* ------------------------------------------------------------------------
 * Adjoint (reverse mode) of the DG2-NL step.  For a fixed step size, the
 * forward run records the depth h at every gauge after each of `steps`
 * steps; the backward run takes the gradient of any scalar loss with respect
 * to those depths and returns the gradient with respect to the per-cell
 * Manning coefficients n (Sec. 2.1.3 friction) and to the samples Q of one
 * inflow hydrograph (the control side).  The step is differentiated as the
 * library computes it: HLL flux, dummy limits and wall-revised bed of
 * Sec. 2.1.2, RK2 stages, friction split and the end-of-stage wet/dry
 * treatment (which passes no derivative through its decisions).  Where a
 * min/max has equal arguments each receives half; the celerity sqrt(g h) has
 * derivative 0 at h = 0.  Checkpoints of the state are kept every
 * `checkpoint_every` steps; the forward run also keeps every step of its last
 * segment, and the backward run recomputes each other segment once from its
 * checkpoint (with checkpoint_every >= steps nothing is recomputed: the whole
 * trajectory is kept).  Gradients do not depend on the interval.
 * ------------------------------------------------------------------------ */
typedef struct dg2_adj dg2_adj;

/* Bind an adjoint to ctx (FP64, DG2_NL, fixed dt > 0 set, >= 1 gauge).  The
 * context's current state and time are the initial condition U^0; the
 * control side (DG2_WEST..DG2_NORTH, or -1 for none) must have an inflow
 * segment and hydrograph, whose sample times are read now.  ctx must
 * outlive the adjoint; device memory: about (steps/K + 2K + 5) states of
 * 9 nx ny doubles.  Errors: DG2_EINVAL, DG2_EUNSUPPORTED (FP32 or DG2-LL),
 * DG2_ESTATE (no fixed dt, no gauges, no hydrograph), DG2_ENOMEM. */
dg2_status dg2_adj_create(dg2_ctx *ctx, int32_t steps, int32_t checkpoint_every,
                          int32_t control_side, dg2_adj **out);

void dg2_adj_destroy(dg2_adj *adj);

/* Message of the last failing call on adj (NULL: last dg2_adj_create failure). */
const char *dg2_adj_last_error(const dg2_adj *adj);

/* Forward run from U^0.  n_cell (ny*nx, row-major, >= 0; NULL: keep the
 * context's Manning values) and Q (one value per hydrograph sample of the
 * control side, >= 0; NULL: keep) are written into the context first.
 * gauge_h (may be NULL) receives h[steps][ng]: the depth of the planar
 * solution at each gauge after each step.  Returns when done. */
dg2_status dg2_adj_forward(dg2_adj *adj, const double *n_cell, const double *Q, double *gauge_h);

/* Backward run for the last forward run.  dL_dh[steps][ng]: gradient of the
 * loss with respect to gauge_h.  grad_n (ny*nx, may be NULL) receives dL/dn
 * per cell; grad_Q (one per hydrograph sample, may be NULL) dL/dQ.  The
 * state adjoint is reduced in a fixed order: results are reproducible. */
dg2_status dg2_adj_backward(dg2_adj *adj, const double *dL_dh, double *grad_n, double *grad_Q);

/* Device milliseconds of the last forward and backward run (HIP events). */
dg2_status dg2_adj_timing(const dg2_adj *adj, double *ms_forward, double *ms_backward);

#ifdef __cplusplus
}
#endif

#endif /* DG2_H */
