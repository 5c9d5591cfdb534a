// ggfv_aux.hip -- data movement and reductions around the step kernel:
//   * dense io arrays <-> padded storage planes (with the hi/lo split of the
//     compensated FP32 state),
//   * the tensor from its eigen-description, A = R(theta) diag(l1, l2) R(theta)^T
//     (eq. (2)),
//   * the positive-definiteness check of the tensor (Sylvester's criterion),
//   * the largest eigenvalue of A over the grid, which sets the explicit step
//     bound of the CFL condition (Section 2),
//   * diagnostics: masses, extrema, non-finite count and the cfl number.
//
// Reductions are two-pass and deterministic: each block folds a fixed
// grid-stride slice of cells in a fixed order, reduces across its wave64s with
// xor-butterflies and LDS, writes one partial; a single block then folds the
// partials in index order.  All accumulation is FP64.

#include <cmath>
#include <mutex>

#include "ggfv_internal.hpp"

namespace ggfv {
namespace {

// ---------------------------------------------------------------------------
// packing

template <typename S, typename T>
__global__ void pack_kernel(const S *__restrict__ s0, const S *__restrict__ s1,
                            const S *__restrict__ s2, T *__restrict__ dst, size_t plane,
                            int nx, int ny, int pitch, bool split_lo)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    const int j = blockIdx.y;
    if (i >= pitch || j >= ny) return;
    const size_t o = (size_t)j * pitch + i;
    const S *src[3] = {s0, s1, s2};
#pragma unroll
    for (int p = 0; p < 3; ++p) {
        T hi = T(0), lo = T(0);
        if (i < nx) {
            const S x = src[p][(size_t)j * nx + i];
            hi = T(x);
            if (split_lo) lo = T(double(x) - double(hi));
        }
        dst[p * plane + o] = hi;
        if (split_lo) dst[(3 + p) * plane + o] = lo;
    }
}

template <typename T, typename D>
__global__ void unpack_kernel(const T *__restrict__ src, size_t plane, bool has_lo,
                              D *__restrict__ d0, D *__restrict__ d1, D *__restrict__ d2,
                              int nx, int ny, int pitch)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    const int j = blockIdx.y;
    if (i >= nx || j >= ny) return;
    const size_t o = (size_t)j * pitch + i;
    D *dst[3] = {d0, d1, d2};
#pragma unroll
    for (int p = 0; p < 3; ++p) {
        double x = double(src[p * plane + o]);
        if (has_lo && sizeof(D) == 8) x = x + double(src[(3 + p) * plane + o]);
        dst[p][(size_t)j * nx + i] = D(x);
    }
}

template <typename S, typename T>
__global__ void tensor_eig_kernel(const S *__restrict__ l1, const S *__restrict__ l2,
                                  const S *__restrict__ th, T *__restrict__ abc, size_t plane,
                                  int nx, int ny, int pitch)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    const int j = blockIdx.y;
    if (i >= pitch || j >= ny) return;
    const size_t o = (size_t)j * pitch + i;
    double a = 0.0, b = 0.0, c = 0.0;
    if (i < nx) {
        const size_t k = (size_t)j * nx + i;
        const double L1 = double(l1[k]), L2 = double(l2[k]), TH = double(th[k]);
        const double cs = cos(TH), sn = sin(TH);
        a = L1 * (cs * cs) + L2 * (sn * sn);
        c = L1 * (sn * sn) + L2 * (cs * cs);
        b = (L1 - L2) * (sn * cs);
    }
    abc[o] = T(a);
    abc[plane + o] = T(b);
    abc[2 * plane + o] = T(c);
}

// ---------------------------------------------------------------------------
// reductions

enum class Op { Sum, Min, Max };

__device__ __forceinline__ double combine(Op op, double x, double y)
{
    if (op == Op::Sum) return x + y;
    if (op == Op::Min) return fmin(x, y);
    return fmax(x, y);
}

__device__ __forceinline__ double identity(Op op)
{
    if (op == Op::Sum) return 0.0;
    if (op == Op::Min) return INFINITY;
    return -INFINITY;
}

// Block-wide reduction of NS slots with per-slot operators; result valid in
// thread 0.  Wave64 xor-butterfly then a fixed-order pass over the four waves.
template <int NS>
__device__ void block_reduce(double (&x)[NS], const Op (&ops)[NS])
{
    __shared__ double sm[kReduceThreads / 64][NS];
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
#pragma unroll
    for (int s = 0; s < NS; ++s) {
#pragma unroll
        for (int off = 32; off >= 1; off >>= 1) x[s] = combine(ops[s], x[s], __shfl_xor(x[s], off, 64));
    }
    if (lane == 0) {
#pragma unroll
        for (int s = 0; s < NS; ++s) sm[wv][s] = x[s];
    }
    __syncthreads();
    if (threadIdx.x == 0) {
#pragma unroll
        for (int s = 0; s < NS; ++s) {
            double r = sm[0][s];
            for (int w = 1; w < kReduceThreads / 64; ++w) r = combine(ops[s], r, sm[w][s]);
            x[s] = r;
        }
    }
}

// Final pass: fold nparts partials of NS slots (row-major [part][slot]).
template <int NS>
__global__ __launch_bounds__(kReduceThreads) void final_kernel(const double *__restrict__ parts,
                                                               int nparts, double *__restrict__ out,
                                                               Op o0, Op o1, Op o2, int nsum3)
{
    // slot operators: o0 for slots [0, nsum3), o1 for [nsum3, 2*nsum3), o2 for the rest
    Op ops[NS];
#pragma unroll
    for (int s = 0; s < NS; ++s) ops[s] = s < nsum3 ? o0 : (s < 2 * nsum3 ? o1 : o2);
    double x[NS];
#pragma unroll
    for (int s = 0; s < NS; ++s) x[s] = identity(ops[s]);
    for (int p = threadIdx.x; p < nparts; p += kReduceThreads) {
#pragma unroll
        for (int s = 0; s < NS; ++s) x[s] = combine(ops[s], x[s], parts[(size_t)p * NS + s]);
    }
    block_reduce<NS>(x, ops);
    if (threadIdx.x == 0) {
#pragma unroll
        for (int s = 0; s < NS; ++s) out[s] = x[s];
    }
}

template <typename T>
__global__ __launch_bounds__(kReduceThreads) void spd_kernel(const T *__restrict__ abc, size_t plane,
                                                             int nx, int ny, int pitch,
                                                             double *__restrict__ parts)
{
    const Op ops[2] = {Op::Sum, Op::Max};
    double x[2] = {0.0, -INFINITY};
    const long n = (long)nx * ny;
    for (long k = blockIdx.x * (long)kReduceThreads + threadIdx.x; k < n;
         k += (long)gridDim.x * kReduceThreads) {
        const int j = (int)(k / nx), i = (int)(k - (long)j * nx);
        const size_t o = (size_t)j * pitch + i;
        const double a = abc[o], b = abc[plane + o], c = abc[2 * plane + o];
        const double det = a * c - b * b;
        const bool ok = (a > 0.0) && (det > 0.0) && isfinite(a) && isfinite(b) && isfinite(c);
        if (!ok) x[0] += 1.0;
        // largest eigenvalue (a+c)/2 + sqrt(((a-c)/2)^2 + b^2)
        const double m = 0.5 * (a + c), d = 0.5 * (a - c);
        const double lm = m + sqrt(d * d + b * b);
        if (ok) x[1] = fmax(x[1], lm);
    }
    block_reduce<2>(x, ops);
    if (threadIdx.x == 0) {
        parts[blockIdx.x * 2 + 0] = x[0];
        parts[blockIdx.x * 2 + 1] = x[1];
    }
}

// Fields of the diagnostics: u, v, w (and their low words for the compensated
// state, else null) and the tensor a, b, c, each a row-major plane with rows
// `pitch` values apart.
template <typename T>
struct DiagFields {
    const T *f[3];
    const T *lo[3];
    const T *a, *b, *c;
};

// Diagnostics partial: slots 0-2 sums, 3-5 minima, 6-8 maxima, 9 cfl max,
// 10 non-finite count, 11 unused (kept zero).  Cell k of the grid goes to
// thread k mod (blocks * threads) whatever the row pitch, so dense and padded
// planes of the same values give the same partials.
template <typename T>
__global__ __launch_bounds__(kReduceThreads) void diag_kernel(DiagFields<T> F, bool has_lo, int nx,
                                                              int ny, int pitch, double idx2,
                                                              double idy2, double idxy, double D2,
                                                              double *__restrict__ parts)
{
    const Op ops[kDiagSlots] = {Op::Sum, Op::Sum, Op::Sum, Op::Min, Op::Min, Op::Min,
                                Op::Max, Op::Max, Op::Max, Op::Max, Op::Sum, Op::Sum};
    double x[kDiagSlots];
#pragma unroll
    for (int s = 0; s < kDiagSlots; ++s) x[s] = identity(ops[s]);
    x[9] = 0.0;
    const long n = (long)nx * ny;
    for (long k = blockIdx.x * (long)kReduceThreads + threadIdx.x; k < n;
         k += (long)gridDim.x * kReduceThreads) {
        const int j = (int)(k / nx), i = (int)(k - (long)j * nx);
        const size_t o = (size_t)j * pitch + i;
        double f[3];
#pragma unroll
        for (int p = 0; p < 3; ++p) {
            f[p] = double(F.f[p][o]);
            if (has_lo) f[p] = f[p] + double(F.lo[p][o]);
            if (!isfinite(f[p])) {
                x[10] += 1.0;
            } else {
                x[p] += f[p];
                x[3 + p] = fmin(x[3 + p], f[p]);
                x[6 + p] = fmax(x[6 + p], f[p]);
            }
        }
        const double a = F.a[o], b = F.b[o], c = F.c[o];
        const double cw = 2.0 * (a * idx2 + c * idy2) + fabs(b) * idxy;
        const double cv = 2.0 * D2 * fabs(1.0 - f[0]) * (idx2 + idy2);
        x[9] = fmax(x[9], fmax(cw, cv));
    }
    block_reduce<kDiagSlots>(x, ops);
    if (threadIdx.x == 0) {
#pragma unroll
        for (int s = 0; s < kDiagSlots; ++s) parts[(size_t)blockIdx.x * kDiagSlots + s] = x[s];
    }
}

// Adaptive stepping: reset the control block.
__global__ void adapt_reset_kernel(AdaptCtl *ctl, double t0)
{
    if (threadIdx.x == 0 && blockIdx.x == 0) {
        ctl->m[0] = ctl->m[1] = ctl->m[2] = 0ull;
        ctl->t = t0;
        ctl->tensor_max = 0.0;
        ctl->last_dt = 0.0;
    }
}

// Adaptive stepping: max over cells of the tensor term 2(a idx^2 + c idy^2) +
// |b| idx idy (at least 0) and of |1 - u| (u = hi + lo in FP64 for the
// compensated state), as unsigned atomic maxima of the non-negative doubles'
// bits into the control block.
template <typename T>
__global__ __launch_bounds__(kReduceThreads) void adapt_init_kernel(const T *__restrict__ st, size_t plane,
                                                                    bool has_lo, const T *__restrict__ abc,
                                                                    int nx, int ny, int pitch, double idx2,
                                                                    double idy2, double idxy, AdaptCtl *ctl)
{
    const Op ops[2] = {Op::Max, Op::Max};
    double x[2] = {0.0, 0.0};
    const long n = (long)nx * ny;
    for (long k = blockIdx.x * (long)kReduceThreads + threadIdx.x; k < n;
         k += (long)gridDim.x * kReduceThreads) {
        const int j = (int)(k / nx), i = (int)(k - (long)j * nx);
        const size_t o = (size_t)j * pitch + i;
        const double a = abc[o], b = abc[plane + o], c = abc[2 * plane + o];
        const double cw = 2.0 * (a * idx2 + c * idy2) + fabs(b) * idxy;
        double u = double(st[o]);
        if (has_lo) u = u + double(st[3 * plane + o]);
        x[0] = fmax(x[0], cw);
        x[1] = fmax(x[1], fabs(1.0 - u));
    }
    block_reduce<2>(x, ops);
    if (threadIdx.x == 0) {
        atomicMax(reinterpret_cast<unsigned long long *>(&ctl->tensor_max),
                  (unsigned long long)__double_as_longlong(x[0]));
        atomicMax(&ctl->m[0], (unsigned long long)__double_as_longlong(x[1]));
    }
}

// Front diagnostics, per row (one wave per row): the tumour front is the last
// cell with v >= theta_v, moved to the crossing by linear interpolation towards
// the next cell; the tissue front is the first cell beyond it with u >=
// theta_u, moved back to the crossing when the previous cell lies below the
// threshold.  Writes (xv, xu, xu - xv, flags) per row; flags bit 0: tumour
// front, bit 1: tissue front (gap).  Values are u, v (hi + lo in FP64 for the
// compensated state); positions are cell centres (i + 1/2) dx.
template <typename T>
__device__ __forceinline__ double field_at(const T *__restrict__ hi, const T *__restrict__ lo, int i)
{
    return lo ? double(hi[i]) + double(lo[i]) : double(hi[i]);
}

template <typename T>
__global__ __launch_bounds__(64) void front_row_kernel(const T *__restrict__ st, size_t plane, bool has_lo, int nx,
                                                       int pitch, double dx, double theta_u, double theta_v,
                                                       double *__restrict__ rows)
{
    const int j = blockIdx.x, lane = threadIdx.x;
    const T *u = st + (size_t)j * pitch;
    const T *v = st + plane + (size_t)j * pitch;
    const T *ul = has_lo ? st + 3 * plane + (size_t)j * pitch : nullptr;
    const T *vl = has_lo ? st + 4 * plane + (size_t)j * pitch : nullptr;
    int iv = -1;
    for (int i = lane; i < nx; i += 64)
        if (field_at(v, vl, i) >= theta_v) iv = i;
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) iv = max(iv, __shfl_xor(iv, off, 64));
    int iu = nx;
    if (iv >= 0) {
        for (int i = iv + 1 + lane; i < nx; i += 64)
            if (field_at(u, ul, i) >= theta_u) {
                iu = i;
                break;
            }
    }
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) iu = min(iu, __shfl_xor(iu, off, 64));
    if (lane == 0) {
        double xv = 0.0, xu = 0.0, flags = 0.0;
        if (iv >= 0) {
            xv = (iv + 0.5) * dx;
            if (iv + 1 < nx) {
                const double a = field_at(v, vl, iv), b = field_at(v, vl, iv + 1);
                xv = xv + (a - theta_v) / (a - b) * dx;
            }
            flags = 1.0;
            if (iu < nx) {
                xu = (iu + 0.5) * dx;
                const double c = field_at(u, ul, iu), d = field_at(u, ul, iu - 1);
                if (d < theta_u) xu = xu - (c - theta_u) / (c - d) * dx;
                flags = 3.0;
            }
        }
        rows[4 * (size_t)j + 0] = xv;
        rows[4 * (size_t)j + 1] = xu;
        rows[4 * (size_t)j + 2] = xu - xv;
        rows[4 * (size_t)j + 3] = flags;
    }
}

// Front diagnostics over rows: sums, minima and maxima of the per-row values
// (each thread a fixed contiguous range of rows, then the fixed-order block
// reduction), and the counts; out holds the 11 results of
// ggfv_front_diagnostics in the order include/ggfv.h documents.
__global__ __launch_bounds__(kReduceThreads) void front_final_kernel(const double *__restrict__ rows, int ny,
                                                                     double *__restrict__ out)
{
    const Op ops[11] = {Op::Sum, Op::Min, Op::Max, Op::Sum, Op::Min, Op::Max,
                        Op::Sum, Op::Min, Op::Max, Op::Sum, Op::Sum};
    double x[11];
#pragma unroll
    for (int s = 0; s < 11; ++s) x[s] = identity(ops[s]);
    const int per = (ny + kReduceThreads - 1) / kReduceThreads;
    const int j0 = threadIdx.x * per, j1 = min(ny, j0 + per);
    for (int j = j0; j < j1; ++j) {
        const double f = rows[4 * (size_t)j + 3];
        if (f >= 1.0) {
            const double xv = rows[4 * (size_t)j];
            x[0] += xv;
            x[1] = fmin(x[1], xv);
            x[2] = fmax(x[2], xv);
            x[9] += 1.0;
        }
        if (f >= 3.0) {
            const double xu = rows[4 * (size_t)j + 1], g = rows[4 * (size_t)j + 2];
            x[3] += xu;
            x[4] = fmin(x[4], xu);
            x[5] = fmax(x[5], xu);
            x[6] += g;
            x[7] = fmin(x[7], g);
            x[8] = fmax(x[8], g);
            x[10] += 1.0;
        }
    }
    block_reduce<11>(x, ops);
    if (threadIdx.x == 0) {
        out[0] = x[9] > 0.0 ? x[0] / x[9] : 0.0;
        out[3] = x[10] > 0.0 ? x[3] / x[10] : 0.0;
        out[6] = x[10] > 0.0 ? x[6] / x[10] : 0.0;
        out[1] = x[1];
        out[2] = x[2];
        out[4] = x[4];
        out[5] = x[5];
        out[7] = x[7];
        out[8] = x[8];
        out[9] = x[9];
        out[10] = x[10];
    }
}

// Diagnostics final pass (fixed operators per slot) into the first nout slots
// of out; the sums of slots 0-2 are multiplied by `area` and the maximum of
// slot 9 by `dt` (1 and 1 leave them as they are).
__global__ __launch_bounds__(kReduceThreads) void diag_final_kernel(const double *__restrict__ parts,
                                                                    int nparts, double area, double dt,
                                                                    int nout, double *__restrict__ out)
{
    const Op ops[kDiagSlots] = {Op::Sum, Op::Sum, Op::Sum, Op::Min, Op::Min, Op::Min,
                                Op::Max, Op::Max, Op::Max, Op::Max, Op::Sum, Op::Sum};
    double x[kDiagSlots];
#pragma unroll
    for (int s = 0; s < kDiagSlots; ++s) x[s] = identity(ops[s]);
    for (int p = threadIdx.x; p < nparts; p += kReduceThreads) {
#pragma unroll
        for (int s = 0; s < kDiagSlots; ++s) x[s] = combine(ops[s], x[s], parts[(size_t)p * kDiagSlots + s]);
    }
    block_reduce<kDiagSlots>(x, ops);
    if (threadIdx.x == 0) {
#pragma unroll
        for (int s = 0; s < 3; ++s) x[s] = area * x[s];
        x[9] = dt * x[9];
#pragma unroll
        for (int s = 0; s < kDiagSlots; ++s)
            if (s < nout) out[s] = x[s];
    }
}

// Partial blocks of the reductions over an nx*ny grid: about four cells per
// thread, at most kMaxPartialBlocks.
int reduce_blocks_of(long n)
{
    long b = (n + 4L * kReduceThreads - 1) / (4L * kReduceThreads);
    if (b < 1) b = 1;
    if (b > kMaxPartialBlocks) b = kMaxPartialBlocks;
    return (int)b;
}

int reduce_blocks(const ggfv_ctx *ctx) { return reduce_blocks_of((long)ctx->nx * ctx->ny); }

double *parts_of(ggfv_ctx *ctx) { return static_cast<double *>(ctx->scratch); }
double *result_of(ggfv_ctx *ctx)
{
    return static_cast<double *>(ctx->scratch) + (size_t)kMaxPartialBlocks * kDiagSlots;
}

}  // namespace

hipError_t launch_pack3(ggfv_ctx *ctx, const void *s0, const void *s1, const void *s2,
                        bool src_is_f64, void *dst_base, int nplanes_dst, bool split_lo)
{
    (void)nplanes_dst;
    dim3 blk(256), grd((ctx->pitch + 255) / 256, ctx->ny);
    const bool dst_f64 = (ctx->dtype == GGFV_F64);
    if (src_is_f64 && dst_f64)
        hipLaunchKernelGGL((pack_kernel<double, double>), grd, blk, 0, ctx->stream,
                           (const double *)s0, (const double *)s1, (const double *)s2,
                           (double *)dst_base, ctx->plane, ctx->nx, ctx->ny, ctx->pitch, false);
    else if (src_is_f64 && !dst_f64)
        hipLaunchKernelGGL((pack_kernel<double, float>), grd, blk, 0, ctx->stream,
                           (const double *)s0, (const double *)s1, (const double *)s2,
                           (float *)dst_base, ctx->plane, ctx->nx, ctx->ny, ctx->pitch, split_lo);
    else if (!src_is_f64 && dst_f64)
        hipLaunchKernelGGL((pack_kernel<float, double>), grd, blk, 0, ctx->stream,
                           (const float *)s0, (const float *)s1, (const float *)s2,
                           (double *)dst_base, ctx->plane, ctx->nx, ctx->ny, ctx->pitch, false);
    else
        hipLaunchKernelGGL((pack_kernel<float, float>), grd, blk, 0, ctx->stream,
                           (const float *)s0, (const float *)s1, (const float *)s2,
                           (float *)dst_base, ctx->plane, ctx->nx, ctx->ny, ctx->pitch, split_lo);
    return hipGetLastError();
}

hipError_t launch_unpack3(ggfv_ctx *ctx, const void *src_base, bool has_lo, void *d0, void *d1,
                          void *d2, bool dst_is_f64)
{
    dim3 blk(256), grd((ctx->nx + 255) / 256, ctx->ny);
    const bool src_f64 = (ctx->dtype == GGFV_F64);
    if (src_f64 && dst_is_f64)
        hipLaunchKernelGGL((unpack_kernel<double, double>), grd, blk, 0, ctx->stream,
                           (const double *)src_base, ctx->plane, false, (double *)d0,
                           (double *)d1, (double *)d2, ctx->nx, ctx->ny, ctx->pitch);
    else if (src_f64 && !dst_is_f64)
        hipLaunchKernelGGL((unpack_kernel<double, float>), grd, blk, 0, ctx->stream,
                           (const double *)src_base, ctx->plane, false, (float *)d0,
                           (float *)d1, (float *)d2, ctx->nx, ctx->ny, ctx->pitch);
    else if (!src_f64 && dst_is_f64)
        hipLaunchKernelGGL((unpack_kernel<float, double>), grd, blk, 0, ctx->stream,
                           (const float *)src_base, ctx->plane, has_lo, (double *)d0,
                           (double *)d1, (double *)d2, ctx->nx, ctx->ny, ctx->pitch);
    else
        hipLaunchKernelGGL((unpack_kernel<float, float>), grd, blk, 0, ctx->stream,
                           (const float *)src_base, ctx->plane, false, (float *)d0,
                           (float *)d1, (float *)d2, ctx->nx, ctx->ny, ctx->pitch);
    return hipGetLastError();
}

hipError_t launch_tensor_eig(ggfv_ctx *ctx, const void *l1, const void *l2, const void *th,
                             bool src_is_f64)
{
    dim3 blk(256), grd((ctx->pitch + 255) / 256, ctx->ny);
    const bool dst_f64 = (ctx->dtype == GGFV_F64);
#define GGFV_EIG(S, T)                                                                         \
    hipLaunchKernelGGL((tensor_eig_kernel<S, T>), grd, blk, 0, ctx->stream, (const S *)l1,       \
                       (const S *)l2, (const S *)th, (T *)ctx->tensor, ctx->plane, ctx->nx,      \
                       ctx->ny, ctx->pitch)
    if (src_is_f64 && dst_f64) GGFV_EIG(double, double);
    else if (src_is_f64) GGFV_EIG(double, float);
    else if (dst_f64) GGFV_EIG(float, double);
    else GGFV_EIG(float, float);
#undef GGFV_EIG
    return hipGetLastError();
}

// Writes (count of non-SPD cells, max lambda_max over SPD cells) to result[0..1].
hipError_t launch_spd_count(ggfv_ctx *ctx)
{
    const int nb = reduce_blocks(ctx);
    if (ctx->dtype == GGFV_F64)
        hipLaunchKernelGGL((spd_kernel<double>), dim3(nb), dim3(kReduceThreads), 0, ctx->stream,
                           (const double *)ctx->tensor, ctx->plane, ctx->nx, ctx->ny, ctx->pitch,
                           parts_of(ctx));
    else
        hipLaunchKernelGGL((spd_kernel<float>), dim3(nb), dim3(kReduceThreads), 0, ctx->stream,
                           (const float *)ctx->tensor, ctx->plane, ctx->nx, ctx->ny, ctx->pitch,
                           parts_of(ctx));
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL((final_kernel<2>), dim3(1), dim3(kReduceThreads), 0, ctx->stream,
                       parts_of(ctx), nb, result_of(ctx), Op::Sum, Op::Max, Op::Max, 1);
    return hipGetLastError();
}

hipError_t launch_lambda_max(ggfv_ctx *ctx) { return launch_spd_count(ctx); }

hipError_t launch_adapt_init(ggfv_ctx *ctx, AdaptCtl *ctl, double t0)
{
    hipLaunchKernelGGL(adapt_reset_kernel, dim3(1), dim3(64), 0, ctx->stream, ctl, t0);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    const int nb = reduce_blocks(ctx);
    const double idx = ctx->nx / ctx->lx, idy = ctx->ny / ctx->ly;
    const bool lo = (ctx->dtype == GGFV_F32C);
    if (ctx->dtype == GGFV_F64)
        hipLaunchKernelGGL((adapt_init_kernel<double>), dim3(nb), dim3(kReduceThreads), 0, ctx->stream,
                           (const double *)ctx->state[ctx->cur], ctx->plane, false, (const double *)ctx->tensor,
                           ctx->nx, ctx->ny, ctx->pitch, idx * idx, idy * idy, idx * idy, ctl);
    else
        hipLaunchKernelGGL((adapt_init_kernel<float>), dim3(nb), dim3(kReduceThreads), 0, ctx->stream,
                           (const float *)ctx->state[ctx->cur], ctx->plane, lo, (const float *)ctx->tensor,
                           ctx->nx, ctx->ny, ctx->pitch, idx * idx, idy * idy, idx * idy, ctl);
    return hipGetLastError();
}

hipError_t launch_front_diagnostics(ggfv_ctx *ctx, double theta_u, double theta_v, double *rows, double *out)
{
    const double dx = ctx->lx / ctx->nx;
    const bool lo = (ctx->dtype == GGFV_F32C);
    if (ctx->dtype == GGFV_F64)
        hipLaunchKernelGGL((front_row_kernel<double>), dim3(ctx->ny), dim3(64), 0, ctx->stream,
                           (const double *)ctx->state[ctx->cur], ctx->plane, false, ctx->nx, ctx->pitch, dx,
                           theta_u, theta_v, rows);
    else
        hipLaunchKernelGGL((front_row_kernel<float>), dim3(ctx->ny), dim3(64), 0, ctx->stream,
                           (const float *)ctx->state[ctx->cur], ctx->plane, lo, ctx->nx, ctx->pitch, dx, theta_u,
                           theta_v, rows);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(front_final_kernel, dim3(1), dim3(kReduceThreads), 0, ctx->stream, rows, ctx->ny, out);
    return hipGetLastError();
}

template <typename T>
DiagFields<T> ctx_fields(ggfv_ctx *ctx)
{
    const T *st = static_cast<const T *>(ctx->state[ctx->cur]);
    const T *ab = static_cast<const T *>(ctx->tensor);
    const size_t P = ctx->plane;
    const bool lo = (ctx->dtype == GGFV_F32C);
    DiagFields<T> F;
    for (int p = 0; p < 3; ++p) {
        F.f[p] = st + p * P;
        F.lo[p] = lo ? st + (3 + p) * P : nullptr;
    }
    F.a = ab;
    F.b = ab + P;
    F.c = ab + 2 * P;
    return F;
}

hipError_t launch_diagnostics(ggfv_ctx *ctx, double dt)
{
    (void)dt;
    const int nb = reduce_blocks(ctx);
    const double idx = ctx->nx / ctx->lx, idy = ctx->ny / ctx->ly;
    const bool lo = (ctx->dtype == GGFV_F32C);
    if (ctx->dtype == GGFV_F64)
        hipLaunchKernelGGL((diag_kernel<double>), dim3(nb), dim3(kReduceThreads), 0, ctx->stream,
                           ctx_fields<double>(ctx), false, ctx->nx, ctx->ny, ctx->pitch, idx * idx,
                           idy * idy, idx * idy, ctx->prm.Delta2, parts_of(ctx));
    else
        hipLaunchKernelGGL((diag_kernel<float>), dim3(nb), dim3(kReduceThreads), 0, ctx->stream,
                           ctx_fields<float>(ctx), lo, ctx->nx, ctx->ny, ctx->pitch, idx * idx,
                           idy * idy, idx * idy, ctx->prm.Delta2, parts_of(ctx));
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(diag_final_kernel, dim3(1), dim3(kReduceThreads), 0, ctx->stream,
                       parts_of(ctx), nb, 1.0, 1.0, kDiagSlots, result_of(ctx));
    return hipGetLastError();
}

// ---- diagnostics without allocation ------------------------------------------
//
// ggfv_diagnostics_noalloc keeps its per-block partials in this array instead
// of memory the library allocates: kMaxPartialBlocks x kDiagSlots doubles (96
// KiB), which covers every grid (the reduction uses at most kMaxPartialBlocks
// blocks, whatever the grid size).  Each device the library runs on holds its
// own copy until the process ends.  Host code never uses the array's name as an
// address: its device address, per device, comes from hipGetSymbolAddress.
static __device__ __align__(256) double scratch[kMaxPartialBlocks * kDiagSlots];

namespace {

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
double *g_scratch_ptr[kMaxDevices] = {};

}  // namespace

hipError_t noalloc_scratch(int device, double **out)
{
    if (device < 0 || device >= kMaxDevices) return hipErrorInvalidDevice;
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_ptr[device]) {
        void *p = nullptr;
        const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return e;
        g_scratch_ptr[device] = static_cast<double *>(p);
    }
    *out = g_scratch_ptr[device];
    return hipSuccess;
}

hipError_t launch_diagnostics_dense(int nx, int ny, double lx, double ly, bool f64, const void *u,
                                    const void *v, const void *w, const void *a, const void *b,
                                    const void *c, double Delta2, double dt, double *parts, double *out,
                                    hipStream_t stream)
{
    const int nb = reduce_blocks_of((long)nx * ny);
    const double idx = nx / lx, idy = ny / ly;
    if (f64) {
        DiagFields<double> F{{static_cast<const double *>(u), static_cast<const double *>(v),
                              static_cast<const double *>(w)},
                             {nullptr, nullptr, nullptr}, static_cast<const double *>(a),
                             static_cast<const double *>(b), static_cast<const double *>(c)};
        hipLaunchKernelGGL((diag_kernel<double>), dim3(nb), dim3(kReduceThreads), 0, stream, F, false, nx, ny,
                           nx, idx * idx, idy * idy, idx * idy, Delta2, parts);
    } else {
        DiagFields<float> F{{static_cast<const float *>(u), static_cast<const float *>(v),
                             static_cast<const float *>(w)},
                            {nullptr, nullptr, nullptr}, static_cast<const float *>(a),
                            static_cast<const float *>(b), static_cast<const float *>(c)};
        hipLaunchKernelGGL((diag_kernel<float>), dim3(nb), dim3(kReduceThreads), 0, stream, F, false, nx, ny,
                           nx, idx * idx, idy * idy, idx * idy, Delta2, parts);
    }
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    const double dx = lx / nx, dy = ly / ny;
    hipLaunchKernelGGL(diag_final_kernel, dim3(1), dim3(kReduceThreads), 0, stream, parts, nb, dx * dy, dt,
                       kDiagSlots - 1, out);
    return hipGetLastError();
}

}  // namespace ggfv
