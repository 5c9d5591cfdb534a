/*
 * ggfv3.h -- C ABI of the three-dimensional form of the explicit finite-volume
 * step (the scheme of Section 2, eq. (3), with the same flux form in three
 * directions; the model of Section 1 is stated for dimension 2 or 3).
 *
 * The acid diffuses with a symmetric tensor per cell
 *   A = [[axx, axy, axz], [axy, ayy, ayz], [axz, ayz, azz]]
 * through face fluxes
 *   FX(i+1/2) = (axx_l + axx_r)/2 (W_r - W_l) idx + (axy_l ty_l + axy_r ty_r)/2
 *             + (axz_l tz_l + axz_r tz_r)/2,    FY and FZ alike,
 * with central tangential differences tx, ty, tz (the boundary cell as its own
 * missing neighbour): a 19-point stencil.  The tumour cells diffuse with the
 * face mobility 1 - (U_l + U_r)/2 over the six faces; the reactions and the
 * forward-Euler update are the 2D scheme's.  Boundary faces carry zero flux.
 *
 * Fields are arrays of nz*ny*nx values, x fastest then y then z (index
 * (k*ny + j)*nx + i).  Storage precision GGFV_F64 or GGFV_F32 (the arithmetic
 * precision too); io arrays FP64 or FP32, host or device, as in ggfv.h.  Status
 * codes, ggfv_params and the dtype / where constants are those of ggfv.h.
 */
#ifndef GGFV3_H
#define GGFV3_H

#include "ggfv.h"

#ifdef __cplusplus
extern "C" {
#endif

typedef struct ggfv3_ctx ggfv3_ctx;

/* An nx-by-ny-by-nz grid on [0,lx] x [0,ly] x [0,lz].  dtype GGFV_F64 or
 * GGFV_F32.  hip_stream: the stream every call enqueues on (NULL: the null
 * stream).  EINVAL on bad sizes or dtype, ENOMEM when device memory runs out
 * (two state buffers of 3 fields and 6 tensor fields, rows padded to 64
 * values), EHIP on runtime errors.  On failure *out is NULL and
 * ggfv3_last_error(NULL) says why. */
int ggfv3_create(ggfv3_ctx **out, int nx, int ny, int nz, double lx, double ly, double lz, int dtype,
                 int device, void *hip_stream);
void ggfv3_destroy(ggfv3_ctx *ctx);
/* Parameters of eq. (1) (delta1, rho2, Delta2, rho3, delta3).  EINVAL if not finite. */
int ggfv3_set_params(ggfv3_ctx *ctx, const ggfv_params *p);
/* The six tensor fields (read, not kept).  EINVAL on NULL pointers or bad
 * where / io_dtype, and EINVAL if the tensor is not positive definite in some
 * cell (Section 1 asks for a positive definite tensor; checked by Sylvester's
 * criterion, axx > 0, axx*ayy - axy^2 > 0 and det > 0, in FP64 on the entries
 * after rounding to the context precision).  Synchronizes.  After a failed call
 * the context has no tensor (ESTATE for step and stable_dt) until a valid one
 * is set. */
int ggfv3_set_tensor(ggfv3_ctx *ctx, const void *axx, const void *ayy, const void *azz, const void *axy,
                     const void *axz, const void *ayz, int where, int io_dtype);
/* The state (u, v, w); resets the time and the step count. */
int ggfv3_set_state(ggfv3_ctx *ctx, const void *u, const void *v, const void *w, int where, int io_dtype);
/* Copy the current state out (synchronizes for host outputs).  ESTATE before a state is set. */
int ggfv3_get_state(ggfv3_ctx *ctx, void *u, void *v, void *w, int where, int io_dtype);
/* Explicit step bound: the largest eigenvalue of each cell's tensor is bounded
 * by its largest absolute row sum G (Gershgorin), so
 *   dt = safety / (2 max(max_cells G, Delta2) (idx^2 + idy^2 + idz^2)).
 * Synchronizes.  ESTATE before tensor and parameters are set; EINVAL on
 * safety <= 0 or when no diffusion is positive. */
int ggfv3_stable_dt(ggfv3_ctx *ctx, double safety, double *dt);
/* nsteps forward-Euler steps of size dt (enqueued; rounded to FP32 for FP32
 * contexts).  EINVAL on dt <= 0 or nsteps < 0; ESTATE before state, tensor and
 * parameters are set. */
int ggfv3_step(ggfv3_ctx *ctx, double dt, long long nsteps);
/* Masses dx dy dz sum(f) of u, v, w (FP64 accumulation in a fixed order, so
 * repeated calls give the same bits).  Synchronizes. */
int ggfv3_mass(ggfv3_ctx *ctx, double *mass3);
/* Simulated time and step count of the context. */
int ggfv3_time(const ggfv3_ctx *ctx, double *t, long long *steps);
/* Launch shape: the number of planes each wave marches through, the number of
 * rows each wave holds (1, 2 or 4), and the waves of one workgroup along x and
 * y (which march in step); 0 leaves the library's choice.  Results are
 * identical for every shape.  EINVAL on negative values, other row counts or
 * more than 8 waves per workgroup. */
int ggfv3_set_tuning(ggfv3_ctx *ctx, int z_per_strip, int rows_per_wave, int waves_x, int waves_y);
/* The launch shape the next step uses, defaults resolved, and the number of
 * workgroups a step launches (any pointer may be NULL).  EINVAL on a NULL
 * context. */
int ggfv3_get_tuning(const ggfv3_ctx *ctx, int *z_per_strip, int *rows_per_wave, int *waves_x, int *waves_y,
                     long long *workgroups);
/* Last failure message of ctx ("" if none); ctx == NULL: the last failed
 * ggfv3_create on the calling thread. */
const char *ggfv3_last_error(const ggfv3_ctx *ctx);

#ifdef __cplusplus
}
#endif

#endif /* GGFV3_H */
