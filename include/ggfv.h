/*
 * ggfv.h -- C ABI of the MI355X (gfx950) library for the explicit finite-volume
 * step of the anisotropic, heterogeneous Gatenby-Gawlinski model.
 *
 * The model (Section 1, eq. (1)) evolves normal cells u, tumour cells v and excess
 * lactic acid w on a rectangle [0,lx] x [0,ly] with Neumann boundaries:
 *   du/dt = u(1-u) - delta1 u w
 *   dv/dt = rho2 v(1-v) + Delta2 div[(1-u) grad v]
 *   dw/dt = rho3 v - delta3 w + div(A grad w),   A = [[a,b],[b,c]] SPD (eq. (2))
 * The paper's symbols map as d = delta1, r = rho2, alpha = Delta2, and its acid
 * term c(v - w) is the case rho3 = delta3 = c.
 *
 * One library step is the fully discrete scheme eq. (3) of Section 2: forward
 * Euler with every right-hand side at the old level, the five-point flux of
 * Table 1 for v, the nine-point flux of Table 2 for w (face coefficients are
 * arithmetic means of the two cells; the cross terms use central tangential
 * differences), and zero total flux through every boundary face; tangential
 * differences in the first/last row or column use the boundary cell itself as the
 * missing neighbour.
 *
 * Grid and layout.  nx by ny cells, dx = lx/nx, dy = ly/ny, cell (i,j) centred at
 * ((i+1/2)dx, (j+1/2)dy).  Every field crossing this ABI is a dense row-major
 * array of nx*ny values, index j*nx + i (x fastest), no padding.  Inside the
 * library fields are structure-of-arrays with each row padded to a multiple of 64
 * values; the padding never crosses the ABI.
 *
 * Precision (ggfv_dtype) is fixed per context and covers both storage and
 * arithmetic:
 *   GGFV_F64   FP64 state, tensor and arithmetic.
 *   GGFV_F32   FP32 state, tensor and arithmetic.
 *   GGFV_F32C  FP32 tensor and arithmetic with a compensated state: each of u, v,
 *              w is held as an unevaluated sum hi + lo of two FP32 words; the
 *              right-hand side is evaluated in FP32 from hi, and the update
 *              x + dt*f is added with an error-free two-sum so that increments
 *              below half an FP32 ulp of x are not lost.
 * Arrays exchanged with the library are FP64 or FP32 as chosen by the io_dtype
 * argument (GGFV_F64 or GGFV_F32), independent of the context precision; the
 * library converts.  Reading an F32C state as FP64 returns hi + lo exactly.
 *
 * Memory and ownership.  `where` says whether a pointer is host memory
 * (GGFV_HOST) or device memory on the context's GPU (GGFV_DEVICE).  The library
 * never keeps a caller pointer past the call: host arrays are copied and the
 * call returns after the copy; device arrays are read or written by work
 * enqueued on the context's stream, so they must stay valid until that stream
 * reaches it.  The context owns all its device memory (state in two buffers,
 * tensor, reduction scratch) and frees it in ggfv_destroy.
 *
 * Streams.  All device work is enqueued on the stream given at creation (or by
 * ggfv_set_stream); NULL means the default stream.  Calls that return data to
 * the host (host reads, ggfv_stable_dt, ggfv_diagnostics) synchronize that
 * stream; ggfv_step does not.
 *
 * Errors.  Every int-returning call returns a ggfv_status.  Invalid arguments are
 * rejected before any device work is enqueued.  The message of the last failure
 * of a context is available from ggfv_last_error.  Nothing aborts or throws
 * across this ABI.  A context is not thread-safe; separate contexts are
 * independent.
 */
#ifndef GGFV_H
#define GGFV_H

#ifdef __cplusplus
extern "C" {
#endif

typedef struct ggfv_ctx ggfv_ctx;

typedef enum {
    GGFV_OK = 0,
    GGFV_EINVAL = 1,     /* bad argument: sizes, pointers, dtype, dt, non-SPD tensor */
    GGFV_ENOMEM = 2,     /* device or host allocation failed */
    GGFV_EHIP = 3,       /* a HIP runtime call failed (message names it) */
    GGFV_ESTATE = 4,     /* call out of order, e.g. stepping before state/tensor are set */
    GGFV_EUNSTABLE = 5   /* diagnostics found non-finite values or cfl > 1 */
} ggfv_status;

typedef enum { GGFV_F32 = 1, GGFV_F64 = 2, GGFV_F32C = 3 } ggfv_dtype;
typedef enum { GGFV_HOST = 0, GGFV_DEVICE = 1 } ggfv_where;

/* Reaction and diffusion parameters of eq. (1) (nondimensional). */
typedef struct {
    double delta1;   /* acid kill rate of normal cells (paper: d) */
    double rho2;     /* tumour growth rate (paper: r) */
    double Delta2;   /* tumour diffusion constant (paper: alpha) */
    double rho3;     /* acid production rate (paper: c) */
    double delta3;   /* acid removal rate (paper: c) */
} ggfv_params;

/* Diagnostics of the current state (Section 2's explicit scheme is limited by its
 * CFL condition; cfl is the per-cell Gershgorin bound of the update,
 *   cfl = dt * max_ij max(2(a idx^2 + c idy^2) + |b| idx idy,
 *                         2 Delta2 |1-u| (idx^2 + idy^2)),
 * idx = 1/dx, idy = 1/dy; the step is stable while cfl <= 1). */
typedef struct {
    double t;              /* simulated time: sum of dt over all steps taken */
    long long steps;       /* steps taken since the state was last set */
    double mass[3];        /* dx*dy*sum of u, v, w */
    double vmin[3];        /* minimum of u, v, w over finite values */
    double vmax[3];        /* maximum of u, v, w over finite values */
    double cfl;            /* see above, for the dt of the last step */
    long long nonfinite;   /* number of non-finite values among u, v, w */
} ggfv_diag;

/* Create a context for an nx-by-ny grid on [0,lx] x [0,ly] with precision dtype
 * on HIP device `device`, enqueuing on `hip_stream` (a hipStream_t or NULL).
 * Allocates all device memory.  EINVAL if nx < 1, ny < 1, lx or ly not > 0, or
 * dtype unknown; ENOMEM if device memory is short; EHIP if the device cannot be
 * selected.  On failure *out is NULL. */
int ggfv_create(ggfv_ctx **out, int nx, int ny, double lx, double ly, int dtype,
                int device, void *hip_stream);

/* Release the context and all its device memory (waits for its stream first).
 * NULL is ignored. */
void ggfv_destroy(ggfv_ctx *ctx);

/* Replace the stream used for all later work of this context. */
int ggfv_set_stream(ggfv_ctx *ctx, void *hip_stream);

/* Set the reaction/diffusion parameters (eq. (1)).  EINVAL if any is not finite
 * or Delta2 < 0. */
int ggfv_set_params(ggfv_ctx *ctx, const ggfv_params *params);

/* Set the per-cell tensor entries a, b, c (eq. (2); piecewise constant per cell,
 * Section 2).  Three arrays of nx*ny io_dtype values.  The tensor is checked for
 * positive definiteness (a > 0 and a*c - b^2 > 0 in every cell, after rounding
 * to the context precision): EINVAL if it fails. */
int ggfv_set_tensor(ggfv_ctx *ctx, const void *a, const void *b, const void *c,
                    int where, int io_dtype);

/* Set the tensor from its eigen-description: A = R(theta) diag(lam1, lam2)
 * R(theta)^T, i.e. a = lam1 cos^2 + lam2 sin^2, c = lam1 sin^2 + lam2 cos^2,
 * b = (lam1 - lam2) sin cos, evaluated on the device.  EINVAL if the result is
 * not positive definite (lam1 or lam2 not > 0). */
int ggfv_set_tensor_eig(ggfv_ctx *ctx, const void *lam1, const void *lam2,
                        const void *theta, int where, int io_dtype);

/* Copy the tensor out (three arrays of nx*ny io_dtype values). */
int ggfv_get_tensor(ggfv_ctx *ctx, void *a, void *b, void *c, int where, int io_dtype);

/* Set the state u, v, w (three arrays of nx*ny io_dtype values); resets the
 * simulated time and the step count to zero. */
int ggfv_set_state(ggfv_ctx *ctx, const void *u, const void *v, const void *w,
                   int where, int io_dtype);

/* Copy the current state out.  For GGFV_F32C read as GGFV_F64 the value is the
 * exact sum hi + lo; read as GGFV_F32 it is hi. */
int ggfv_get_state(ggfv_ctx *ctx, void *u, void *v, void *w, int where, int io_dtype);

/* Largest stable explicit step for the current tensor and parameters:
 *   dt = safety / (2 * max(max_ij lambda_max(A_ij), Delta2) * (idx^2 + idy^2)),
 * lambda_max(A) = (a+c)/2 + sqrt(((a-c)/2)^2 + b^2), reduced on the device in
 * FP64 from the stored tensor.  EINVAL unless 0 < safety. Synchronizes. */
int ggfv_stable_dt(ggfv_ctx *ctx, double safety, double *dt_out);

/* Advance the state by nsteps forward-Euler steps of eq. (3) with step dt
 * (rounded to FP32 for F32 and F32C contexts).  Enqueues the work and returns.
 * EINVAL if dt is not finite and > 0 or nsteps < 0; ESTATE if the state, tensor
 * or parameters were never set.  nsteps == 0 is a no-op. */
int ggfv_step(ggfv_ctx *ctx, double dt, long long nsteps);

/* Advance nsteps steps of eq. (3) with the step size recomputed before every
 * step, as the time discretization of Section 2 does (a new step size after each
 * iteration, chosen for stability).  The paper prints no rule; this one takes
 * the largest step whose per-cell Gershgorin number (the cfl of ggfv_diag) on
 * the state the step starts from equals `safety`:
 *   dt_k = safety / max_ij max( 2(a idx^2 + c idy^2) + |b| idx idy,
 *                               2 Delta2 |1 - u_ij^k| (idx^2 + idy^2) ),
 * evaluated in FP64 (u = hi + lo for the compensated state).  Everything runs
 * on the device: each step kernel reduces max |1-u| of the state it writes, and
 * the next step derives its size from it, so there is no host round trip
 * between steps.  Single-step launches (the step size may change every step).
 * dt_log: NULL or device memory for nsteps doubles, receiving dt_0 .. dt_{n-1}.
 * Synchronizes once at the end, to update the context's time and last step.
 * EINVAL on safety <= 0 or not finite, nsteps < 0; ESTATE before state, tensor
 * and parameters are set; ENOMEM if the 64-byte control block cannot be
 * allocated (once per context). */
int ggfv_step_adaptive(ggfv_ctx *ctx, double safety, long long nsteps, double *dt_log);

/* Fronts of the current state for fronts that advance towards +x: the
 * propagating tumour front and the hypocellular interstitial gap ahead of it
 * (Section 2's homogeneous and heterogeneous invasion).  The paper prints no
 * definition; per row j:
 *   tumour front xv_j: the last cell i with v >= theta_v, moved to the crossing
 *     by linear interpolation towards cell i+1 (x_i + (v_i - theta_v)/(v_i -
 *     v_i+1) dx when cell i+1 exists);
 *   tissue front xu_j: the first cell i beyond it with u >= theta_u, moved back
 *     to the crossing when u_i-1 < theta_u (x_i - (u_i - theta_u)/(u_i -
 *     u_i-1) dx);
 *   gap g_j = xu_j - xv_j;
 * with cell centres x_i = (i + 1/2) lx/nx and u, v as FP64 (hi + lo for the
 * compensated state).  out (host, 11 doubles): mean, min, max of xv over rows
 * with a tumour front; mean, min, max of xu and of g over rows with both
 * fronts; the two row counts.  Means of no rows are 0, their min/max +inf /
 * -inf.  Synchronizes.  EINVAL on NULL out or non-finite thresholds, ESTATE
 * without a state, ENOMEM if the (4 ny + 16)-double buffer cannot be allocated
 * (once per context). */
int ggfv_front_diagnostics(ggfv_ctx *ctx, double theta_u, double theta_v, double *out);
/* Space-averaged front speed (LeVeque and Yee, cited in Section 2) from the mass
 * of one population at two times (ggfv_diagnostics): a transition from density
 * `behind` to density `ahead` moving at speed s across a domain of height ly
 * changes the mass at the rate ly (behind - ahead) s.  Pure arithmetic. */
double ggfv_front_speed(double mass0, double mass1, double t0, double t1, double ly, double behind, double ahead);

/* Diagnostics of the current state (FP64 accumulation in a fixed order, so the
 * result is reproducible).  Synchronizes.  Returns GGFV_EUNSTABLE (with *out
 * filled) if nonfinite > 0 or cfl > 1. */
int ggfv_diagnostics(ggfv_ctx *ctx, ggfv_diag *out);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): the
 * diagnostics of ggfv_diagnostics for a state and tensor held in caller device
 * arrays, with no context, no allocation, no host copy and no
 * synchronization.  u, v, w, a, b, c: dense row-major device arrays of nx*ny
 * io_dtype values (GGFV_F64 or GGFV_F32) on `device`; for a compensated state
 * pass hi + lo as FP64.  Delta2 is the tumour-cell diffusion of eq. (1), dt
 * the step the cfl refers to.  out: 11 doubles of device memory, written by
 * work enqueued on hip_stream (NULL: the null stream):
 *   out[0..2] masses of u, v, w (dx*dy times the sum of the finite values),
 *   out[3..5] minima, out[6..8] maxima (over finite values),
 *   out[9]    cfl = dt * max over cells of max(2(a idx^2 + c idy^2) + |b| idx idy,
 *             2 Delta2 |1-u| (idx^2 + idy^2)),
 *   out[10]   the number of non-finite values among u, v, w,
 * the same values, bit for bit, as ggfv_diagnostics on a context holding this
 * state, tensor and Delta2 after steps of size dt.  The reduction's per-block
 * partials live in a static device array of the library: at most 1024 blocks
 * x 12 doubles (96 KiB per device, held until the process ends), enough for
 * every grid the library accepts; every block rewrites its own partials, so
 * nothing needs clearing between calls.  Calls on one device share that array:
 * calls that overlap on one device (different streams or threads) race and
 * give wrong results.  EINVAL (before any device work) for nx or ny < 1, more
 * than 2^34 cells, non-finite or non-positive lx, ly, a bad io_dtype, a NULL
 * pointer, a negative or non-finite Delta2 or dt, or a device out of range;
 * EHIP if the array's device address cannot be obtained or the launch fails.
 * ggfv_last_error(NULL) reports why on the calling thread. */
int ggfv_diagnostics_noalloc(int nx, int ny, double lx, double ly, int io_dtype, const void *u, const void *v,
                             const void *w, const void *a, const void *b, const void *c, double Delta2,
                             double dt, double *out, int device, void *hip_stream);

/* ---- gradients ------------------------------------------------------------
 *
 * The adjoint of the explicit step: for a loss L of the state after N steps,
 * lam^k = dL/dx^k satisfies lam^k = (dF/dx)^T lam^{k+1} with F one step of
 * eq. (3) (dt fixed), and the gradients with respect to the tensor (a, b, c) and
 * the five parameters are sums over steps of (dF/dA)^T lam^{k+1} and
 * (dF/dp)^T lam^{k+1}.  F is differentiated exactly as implemented (the
 * discrete adjoint), including the zero-flux faces and the mirrored tangential
 * differences of the boundary rule.  The arithmetic is in the context precision
 * (for GGFV_F32C the adjoint reads the hi word of the state); the five scalar
 * gradients are accumulated in FP64 in a fixed order. */

/* Bytes of one stored state (all fields, padded rows): the unit of checkpoint and
 * work buffers below. */
long long ggfv_state_bytes(const ggfv_ctx *ctx);

/* Like ggfv_step, and also copies the state before steps 0, every, 2*every, ...
 * into the caller's device buffer ckpt (slot k at byte offset k*state_bytes),
 * i.e. ceil(nsteps/every) slots.  EINVAL if every < 1, nsteps < 1 or ckpt_bytes
 * is too small.  Asynchronous on the context's stream. */
int ggfv_step_checkpointed(ggfv_ctx *ctx, double dt, long long nsteps, long long every,
                           void *ckpt, long long ckpt_bytes);

/* One adjoint step at the state x = (u, v, w): lam_out = (dF/dx)^T lam_in;
 * (g_a, g_b, g_c) += (dF/dA)^T lam_in (in place); g_params[0..4] (host, FP64,
 * order delta1, rho2, Delta2, rho3, delta3) += (dF/dp)^T lam_in.  All arrays are
 * nx*ny io_dtype values at `where`.  Uses the context's tensor and parameters;
 * does not touch its state.  Synchronizes. */
int ggfv_adjoint_step(ggfv_ctx *ctx, double dt, const void *u, const void *v, const void *w,
                      const void *lam_u, const void *lam_v, const void *lam_w, void *out_u,
                      void *out_v, void *out_w, void *g_a, void *g_b, void *g_c,
                      double *g_params, int where, int io_dtype);

/* Reverse sweep over nsteps steps with the checkpoints written by
 * ggfv_step_checkpointed(dt, nsteps, every): for each segment of `every` steps,
 * last to first, the states of the segment are recomputed from its checkpoint
 * into the caller's device buffer work (at least max(1, every-1) states) and the
 * adjoint steps run backwards through them.  Memory is ceil(N/every) + every
 * states; every ~ sqrt(N) gives 2 sqrt(N).
 * lam_u, lam_v, lam_w: on entry dL/dx^N, on exit dL/dx^0.  g_a, g_b, g_c and
 * g_params[5] (host) are overwritten with the gradients.  Arrays at `where` in
 * io_dtype; ckpt and work are device memory.  Uses the context's tensor and
 * parameters; does not touch its state.  Synchronizes. */
int ggfv_adjoint_run(ggfv_ctx *ctx, double dt, long long nsteps, long long every,
                     const void *ckpt, long long ckpt_bytes, void *work, long long work_bytes,
                     void *lam_u, void *lam_v, void *lam_w, void *g_a, void *g_b, void *g_c,
                     double *g_params, int where, int io_dtype);

/* Chain rule of the tensor map of ggfv_set_tensor_eig: from (g_a, g_b, g_c) and
 * (lam1, lam2, theta) to the gradients with respect to lam1, lam2 and theta:
 *   g_l1 = g_a cos^2 + g_c sin^2 + g_b sin cos
 *   g_l2 = g_a sin^2 + g_c cos^2 - g_b sin cos
 *   g_th = (lam1 - lam2)((g_c - g_a) sin 2theta + g_b cos 2theta)
 * (FP64 arithmetic).  Nine arrays of nx*ny io_dtype values at `where`.
 * Synchronizes for host arrays. */
int ggfv_eig_backward(ggfv_ctx *ctx, const void *lam1, const void *lam2, const void *theta,
                      const void *g_a, const void *g_b, const void *g_c, void *g_l1, void *g_l2,
                      void *g_th, int where, int io_dtype);

/* Launch shape of the step.  rows_per_strip is the number of grid rows one
 * workgroup sweeps (0 = chosen from the grid size; for the lane-shift kernels,
 * the tallest strips whose workgroups fill the device's resident slots once,
 * from the kernel's occupancy and the number of compute units).
 * lane_shift = 0 selects the single-step kernel (one step per launch, threads
 * = its workgroup width, 64, 128 or 256, 0 = chosen from the grid size).
 * lane_shift = 1 selects the one-wave kernels that keep the rows of every time
 * level in registers and exchange x-neighbours by lane shifts (threads is then
 * ignored); lane_shift = 2 the same kernels with wide lanes, 16 bytes of
 * columns per lane (two FP64 or four FP32 columns: half the lane shifts and
 * halo columns per cell, twice the registers; not for GGFV_F32C).
 * fused_steps (1..4, 0 = 1; above 1 only with lane_shift 1 or 2) is the number
 * of time steps computed per launch: the old state is read from HBM once, the
 * intermediate levels stay on chip, and only the last level is written, so HBM
 * traffic per step falls by that factor; a run of n steps uses n / fused_steps
 * fused launches and single steps for the remainder.
 * A new context starts with the shape measured fastest on MI355X for its grid
 * size, from h4 = ny * ceil(nx / W) / (8 * compute units) (W = 248 columns for
 * GGFV_F32, 120 otherwise: the strip height at which the 4-step lane-shift
 * kernel's one-wave strips fill the device once): h4 >= 8 gives rows_per_strip
 * 0, fused_steps 4, lane_shift 2 (1 for GGFV_F32C); 3 <= h4 < 8 the same with
 * fused_steps 2; smaller grids the single-step kernel (fused_steps 1,
 * lane_shift 0, threads 0).  On MI355X 4096^2 and 2048^2 get four steps per
 * launch, 1024^2 two, 512^2 one.
 * Every shape gives the same results bit for bit.  EINVAL for values outside
 * these sets. */
typedef struct {
    int rows_per_strip;
    int threads;
    int fused_steps;
    int lane_shift;
} ggfv_tuning;

int ggfv_set_tuning(ggfv_ctx *ctx, const ggfv_tuning *tuning);
int ggfv_get_tuning(const ggfv_ctx *ctx, ggfv_tuning *tuning);

/* Time `trial_steps` steps for each candidate shape (the single-step kernel at
 * widths 64, 128, 256; the lane-shift kernels, narrow and wide, at fused depths
 * 1..4; strip heights 2, 4, 8, 16, 24, 32, 48, 64, 128, the default, and for
 * the lane-shift kernels the heights that fill the resident slots half a
 * round, 1.5 and 2 rounds over) on the
 * context's own data, keep the fastest per step as the context's tuning and
 * return it (with the height it ran).  The state, simulated time and step count are restored
 * afterwards.  Needs state, tensor and parameters.  Synchronizes. */
int ggfv_autotune(ggfv_ctx *ctx, double dt, int trial_steps, ggfv_tuning *best);

/* ---- ensembles ---------------------------------------------------------------
 *
 * A batch holds n independent instances (each its own grid size, parameters,
 * tensor, state and dt) that advance together: one launch of a batched kernel
 * moves every instance by one step of eq. (3) (single-step kernel) or by K steps
 * (lane-shift kernel, ggfv_batch_set_fused_steps), and runs of many steps are
 * captured once into a HIP graph and replayed.  Each instance is an ordinary
 * context owned by the batch: set its parameters, tensor and state, read its
 * state and diagnostics with the ggfv_* calls above through
 * ggfv_batch_instance (never ggfv_destroy it).  All instances share one stream
 * and precision. */
typedef struct ggfv_batch ggfv_batch;

/* n instances, instance i an nx[i]-by-ny[i] grid on [0,lx] x [0,ly].  With
 * hip_stream NULL the batch creates its own (default-priority) stream, because
 * graph capture needs a stream other than the null stream; that stream is a
 * blocking one, so its work is ordered with work on the null stream both ways
 * (device arrays written or read there need no extra synchronization).  EINVAL on bad sizes
 * or dtype; ENOMEM / EHIP as ggfv_create.  On failure *out is NULL and
 * ggfv_batch_last_error(NULL) reports why. */
int ggfv_batch_create(ggfv_batch **out, int n, const int *nx, const int *ny, double lx, double ly,
                      int dtype, int device, void *hip_stream);
void ggfv_batch_destroy(ggfv_batch *b);
/* The context of instance i (owned by the batch), or NULL if i is out of range. */
ggfv_ctx *ggfv_batch_instance(ggfv_batch *b, int i);
/* Step size of instance i (rounded to FP32 for FP32 batches).  EINVAL unless finite and > 0. */
int ggfv_batch_set_dt(ggfv_batch *b, int i, double dt);
/* Instance i in one call: parameters (eq. (1)), the tensor (a, b, c) of eq. (2)
 * as in ggfv_set_tensor, the state as in ggfv_set_state (which resets the
 * instance's time and step count) and its step size as in ggfv_batch_set_dt.
 * Arrays of nx[i]*ny[i] values, host or device (where), FP32 or FP64
 * (io_dtype), read during the call.  EINVAL for i out of range or a bad dt
 * (nothing changed), otherwise the status of the first setter that fails. */
int ggfv_batch_set(ggfv_batch *b, int i, const ggfv_params *params, double dt, const void *a, const void *bb,
                   const void *c, const void *u, const void *v, const void *w, int where, int io_dtype);
/* Copy the state of instance i out, as ggfv_get_state does (host outputs
 * synchronize).  EINVAL for i out of range; ESTATE before its state is set. */
int ggfv_batch_get_state(ggfv_batch *b, int i, void *u, void *v, void *w, int where, int io_dtype);
/* Advance every instance by nsteps steps (each with its own dt).  Enqueues and
 * returns.  ESTATE if an instance lacks state, tensor, parameters or dt. */
int ggfv_batch_run(ggfv_batch *b, long long nsteps);
/* Launch shape of the batched kernels: workgroup width of the single-step kernel
 * (64 or 256), strip height (0 = 16 rows, or per instance via ggfv_set_tuning on
 * the instance), and about how many steps a graph holds (it holds an even number
 * of launches, at least two; 0 = no graph).  Results are identical for every
 * shape. */
int ggfv_batch_set_tuning(ggfv_batch *b, int threads, int rows_per_strip, int graph_steps);
/* Steps per launch: 1 = the single-step kernel; 2..4 = the lane-shift kernel with
 * that many time levels per launch (a run whose step count is not a multiple
 * finishes with single steps).  Results are identical bit for bit.  EINVAL
 * outside 1..4. */
int ggfv_batch_set_fused_steps(ggfv_batch *b, int fused_steps);
/* The current launch shape (any output pointer may be NULL). */
int ggfv_batch_get_tuning(const ggfv_batch *b, int *threads, int *rows_per_strip, int *graph_steps,
                          int *fused_steps);
/* Time about trial_steps batched steps for each candidate (single-step kernel at
 * widths 64 and 256, lane-shift kernel at 2..4 steps per launch) and strip height
 * (4..64), keep the fastest per step and report its width and height (the steps
 * per launch through ggfv_batch_get_tuning); instance states, times and step
 * counts are restored afterwards.  Synchronizes. */
int ggfv_batch_autotune(ggfv_batch *b, int trial_steps, int *best_threads, int *best_rows);
const char *ggfv_batch_last_error(const ggfv_batch *b);

/* Message describing the last failure of this context ("" if none).  With
 * ctx == NULL: the message of the last failed ggfv_create or
 * ggfv_diagnostics_noalloc on the calling thread. */
const char *ggfv_last_error(const ggfv_ctx *ctx);

/* Static name of a status code. */
const char *ggfv_status_string(int status);

#ifdef __cplusplus
}
#endif

#endif /* GGFV_H */
