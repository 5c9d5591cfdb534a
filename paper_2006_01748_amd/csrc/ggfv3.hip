// ggfv3.hip -- the three-dimensional form of the explicit finite-volume step.
//
// The scheme of Section 2 (eq. (3)) with the same flux form in three
// directions: acid faces with the full symmetric tensor (19-point stencil),
// tumour-cell faces with the mobility 1 - (U_l + U_r)/2 (7 points), the
// reactions and the forward-Euler update of the 2D scheme, zero flux through
// boundary faces and the boundary cell as its own missing neighbour in the
// tangential differences.
//
// Layout: every field is nz*ny rows of `pitch` values (nx rounded up to 64),
// x fastest, then y, then z.  Two state buffers (u, v, w) alternate; the tensor
// holds axx, ayy, azz, axy, axz, ayz.
//
// Step kernel: a workgroup of 64 x 4 threads owns 64 x 4 (x, y) columns and a
// strip of zs planes; each thread marches up its column.  The cell's own values
// of the planes below and above stay in registers as the column advances, and
// the flux through the bottom face of a plane is the top face of the plane
// below (computed once, so both cells see the same bits).  The x and y faces are
// evaluated by both neighbouring cells from identical operands in identical
// order, and neighbour values come through the caches.  The arithmetic order is
//   FX(i+1/2) = 0.5*(axx_l + axx_r)*((W_r - W_l)*idx)
//             + 0.5*(axy_l*ty_l + axy_r*ty_r) + 0.5*(axz_l*tz_l + axz_r*tz_r)
//   (FY, FZ alike), GX = (1 - 0.5*(U_l + U_r))*((V_r - V_l)*idx),
//   divW = ((FX_e - FX_w)*idx + (FY_n - FY_s)*idy) + (FZ_t - FZ_b)*idz,
// with no contraction into FMA, so FP64 results equal a plain CPU loop's.

#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <new>
#include <string>

#include "ggfv3.h"
#include "ggfv_internal.hpp"

struct ggfv3_ctx {
    int nx = 0, ny = 0, nz = 0, pitch = 0;
    double lx = 1.0, ly = 1.0, lz = 1.0;
    int dtype = 0, device = 0;
    hipStream_t stream = nullptr;
    size_t field = 0;              // values per field (nz * ny * pitch)
    size_t elem = 0;               // bytes per value
    void *state[2] = {nullptr, nullptr};
    int cur = 0;
    void *tensor = nullptr;        // 6 fields
    void *staging = nullptr;       // dense io arrays (FP64-sized)
    size_t staging_bytes = 0;
    double *scratch = nullptr;     // reduction partials and results
    ggfv_params prm{};
    bool has_params = false, has_tensor = false, has_state = false;
    double t = 0.0;
    long long steps = 0;
    int zs = 0;                    // planes per strip (0: default)
    std::string err;
};

namespace {

thread_local std::string g3_create_error;
constexpr int kRed3 = 256;         // reduction workgroup
constexpr int kRed3Blocks = 512;   // reduction partial blocks

int fail3(ggfv3_ctx *ctx, int code, const char *fmt, ...) __attribute__((format(printf, 3, 4)));

int fail3(ggfv3_ctx *ctx, int code, const char *fmt, ...)
{
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    if (ctx)
        ctx->err = buf;
    else
        g3_create_error = buf;
    return code;
}

#define GGFV3_HIP(ctx, call)                                                                 \
    do {                                                                                     \
        hipError_t e_ = (call);                                                              \
        if (e_ != hipSuccess)                                                                \
            return fail3((ctx), GGFV_EHIP, "%s failed: %s", #call, hipGetErrorString(e_));   \
    } while (0)

struct Guard3 {
    int prev = -1;
    explicit Guard3(int dev)
    {
        (void)hipGetDevice(&prev);
        (void)hipSetDevice(dev);
    }
    ~Guard3()
    {
        if (prev >= 0) (void)hipSetDevice(prev);
    }
};

template <typename T>
struct Step3Args {
    const T *u, *v, *w;
    T *un, *vn, *wn;
    const T *axx, *ayy, *azz, *axy, *axz, *ayz;
    int nx, ny, nz, pitch, zs;
    T idx, idy, idz, hx, hy, hz, dt;
    T d1, r2, D2, r3, d3;
};

template <typename T>
struct Grid3 {
    const Step3Args<T> &A;
    __device__ __forceinline__ size_t at(int i, int j, int k) const
    {
        return ((size_t)k * A.ny + j) * A.pitch + i;
    }
    __device__ __forceinline__ int cx(int i) const { return i < 0 ? 0 : (i >= A.nx ? A.nx - 1 : i); }
    __device__ __forceinline__ int cy(int j) const { return j < 0 ? 0 : (j >= A.ny ? A.ny - 1 : j); }
    __device__ __forceinline__ int cz(int k) const { return k < 0 ? 0 : (k >= A.nz ? A.nz - 1 : k); }
    __device__ __forceinline__ T tx(int i, int j, int k) const
    {
        return (A.w[at(cx(i + 1), j, k)] - A.w[at(cx(i - 1), j, k)]) * A.hx;
    }
    __device__ __forceinline__ T ty(int i, int j, int k) const
    {
        return (A.w[at(i, cy(j + 1), k)] - A.w[at(i, cy(j - 1), k)]) * A.hy;
    }
    __device__ __forceinline__ T tz(int i, int j, int k) const
    {
        return (A.w[at(i, j, cz(k + 1))] - A.w[at(i, j, cz(k - 1))]) * A.hz;
    }
    // acid flux through the face between cell (i,j,k) and its +x / +y / +z neighbour
    __device__ __forceinline__ T fx(int i, int j, int k) const
    {
        const size_t l = at(i, j, k), r = at(i + 1, j, k);
        const T half = T(0.5);
        const T tyl = ty(i, j, k), tyr = ty(i + 1, j, k);
        const T tzl = tz(i, j, k), tzr = tz(i + 1, j, k);
        return half * (A.axx[l] + A.axx[r]) * ((A.w[r] - A.w[l]) * A.idx) + half * (A.axy[l] * tyl + A.axy[r] * tyr) +
               half * (A.axz[l] * tzl + A.axz[r] * tzr);
    }
    __device__ __forceinline__ T fy(int i, int j, int k) const
    {
        const size_t l = at(i, j, k), r = at(i, j + 1, k);
        const T half = T(0.5);
        const T txl = tx(i, j, k), txr = tx(i, j + 1, k);
        const T tzl = tz(i, j, k), tzr = tz(i, j + 1, k);
        return half * (A.ayy[l] + A.ayy[r]) * ((A.w[r] - A.w[l]) * A.idy) + half * (A.axy[l] * txl + A.axy[r] * txr) +
               half * (A.ayz[l] * tzl + A.ayz[r] * tzr);
    }
    __device__ __forceinline__ T fz(int i, int j, int k) const
    {
        const size_t l = at(i, j, k), r = at(i, j, k + 1);
        const T half = T(0.5);
        const T txl = tx(i, j, k), txr = tx(i, j, k + 1);
        const T tyl = ty(i, j, k), tyr = ty(i, j, k + 1);
        return half * (A.azz[l] + A.azz[r]) * ((A.w[r] - A.w[l]) * A.idz) + half * (A.axz[l] * txl + A.axz[r] * txr) +
               half * (A.ayz[l] * tyl + A.ayz[r] * tyr);
    }
    // tumour-cell flux through the face between l and r (spacing factor id)
    __device__ __forceinline__ T g(size_t l, size_t r, T id) const
    {
        return (T(1) - T(0.5) * (A.u[l] + A.u[r])) * ((A.v[r] - A.v[l]) * id);
    }
};

template <typename T>
__global__ __launch_bounds__(256) void step3_kernel(Step3Args<T> A)
{
    const int i = blockIdx.x * 64 + threadIdx.x;
    const int j = blockIdx.y * 4 + threadIdx.y;
    if (i >= A.nx || j >= A.ny) return;            // no barriers below
    const int k0 = blockIdx.z * A.zs, k1 = min(A.nz, k0 + A.zs);
    const Grid3<T> G{A};
    const bool has_e = i + 1 < A.nx, has_w = i > 0, has_n = j + 1 < A.ny, has_s = j > 0;
    const T one = T(1);
    // bottom faces of the first plane of the strip
    T FZb = k0 > 0 ? G.fz(i, j, k0 - 1) : T(0);
    T GZb = k0 > 0 ? G.g(G.at(i, j, k0 - 1), G.at(i, j, k0), A.idz) : T(0);
    for (int k = k0; k < k1; ++k) {
        const size_t c = G.at(i, j, k);
        const bool has_t = k + 1 < A.nz;
        const T FXe = has_e ? G.fx(i, j, k) : T(0);
        const T FXw = has_w ? G.fx(i - 1, j, k) : T(0);
        const T FYn = has_n ? G.fy(i, j, k) : T(0);
        const T FYs = has_s ? G.fy(i, j - 1, k) : T(0);
        const T FZt = has_t ? G.fz(i, j, k) : T(0);
        const T GXe = has_e ? G.g(c, G.at(i + 1, j, k), A.idx) : T(0);
        const T GXw = has_w ? G.g(G.at(i - 1, j, k), c, A.idx) : T(0);
        const T GYn = has_n ? G.g(c, G.at(i, j + 1, k), A.idy) : T(0);
        const T GYs = has_s ? G.g(G.at(i, j - 1, k), c, A.idy) : T(0);
        const T GZt = has_t ? G.g(c, G.at(i, j, k + 1), A.idz) : T(0);
        const T divW = ((FXe - FXw) * A.idx + (FYn - FYs) * A.idy) + (FZt - FZb) * A.idz;
        const T divV = ((GXe - GXw) * A.idx + (GYn - GYs) * A.idy) + (GZt - GZb) * A.idz;
        const T U = A.u[c], V = A.v[c], W = A.w[c];
        A.un[c] = U + A.dt * (U * (one - U) - (A.d1 * U) * W);
        A.vn[c] = V + A.dt * ((A.r2 * V) * (one - V) + A.D2 * divV);
        A.wn[c] = W + A.dt * ((A.r3 * V - A.d3 * W) + divW);
        FZb = FZt;
        GZb = GZt;
    }
}

// dense (nz*ny rows of nx) io array -> padded field
template <typename S, typename T>
__global__ void pack3_kernel(const S *__restrict__ src, T *__restrict__ dst, int nx, long rows, int pitch)
{
    const long n = (long)nx * rows;
    for (long q = blockIdx.x * (long)blockDim.x + threadIdx.x; q < n; q += (long)gridDim.x * blockDim.x) {
        const long r = q / nx;
        const int i = (int)(q - r * nx);
        dst[(size_t)r * pitch + i] = T(src[q]);
    }
}

template <typename T, typename D>
__global__ void unpack3_kernel(const T *__restrict__ src, D *__restrict__ dst, int nx, long rows, int pitch)
{
    const long n = (long)nx * rows;
    for (long q = blockIdx.x * (long)blockDim.x + threadIdx.x; q < n; q += (long)gridDim.x * blockDim.x) {
        const long r = q / nx;
        const int i = (int)(q - r * nx);
        dst[q] = D(src[(size_t)r * pitch + i]);
    }
}

__device__ __forceinline__ double wave_sum(double x)
{
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) x += __shfl_xor(x, off, 64);
    return x;
}

__device__ __forceinline__ double wave_max(double x)
{
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) x = fmax(x, __shfl_xor(x, off, 64));
    return x;
}

// Per-block partial sums of the three state fields (fixed partition and order),
// and of the Gershgorin bound of the tensor (max), written to parts[block*4 + q].
template <typename T>
__global__ __launch_bounds__(kRed3) void reduce3_kernel(const T *__restrict__ st, const T *__restrict__ ten,
                                                       size_t field, int nx, long rows, int pitch,
                                                       double *__restrict__ parts)
{
    __shared__ double sm[kRed3 / 64][4];
    double x[4] = {0.0, 0.0, 0.0, 0.0};
    const long n = (long)nx * rows;
    for (long q = blockIdx.x * (long)kRed3 + threadIdx.x; q < n; q += (long)gridDim.x * kRed3) {
        const long r = q / nx;
        const size_t o = (size_t)r * pitch + (q - r * nx);
        if (st) {
#pragma unroll
            for (int f = 0; f < 3; ++f) x[f] += double(st[f * field + o]);
        }
        if (ten) {
            const double axx = ten[o], ayy = ten[field + o], azz = ten[2 * field + o];
            const double axy = ten[3 * field + o], axz = ten[4 * field + o], ayz = ten[5 * field + o];
            const double r0 = fabs(axx) + fabs(axy) + fabs(axz);
            const double r1 = fabs(axy) + fabs(ayy) + fabs(ayz);
            const double r2 = fabs(axz) + fabs(ayz) + fabs(azz);
            x[3] = fmax(x[3], fmax(r0, fmax(r1, r2)));
        }
    }
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
#pragma unroll
    for (int f = 0; f < 3; ++f) x[f] = wave_sum(x[f]);
    x[3] = wave_max(x[3]);
    if (lane == 0) {
#pragma unroll
        for (int f = 0; f < 4; ++f) sm[wv][f] = x[f];
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        double s[4] = {sm[0][0], sm[0][1], sm[0][2], sm[0][3]};
        for (int w = 1; w < kRed3 / 64; ++w) {
            for (int f = 0; f < 3; ++f) s[f] += sm[w][f];
            s[3] = fmax(s[3], sm[w][3]);
        }
        for (int f = 0; f < 4; ++f) parts[(size_t)blockIdx.x * 4 + f] = s[f];
    }
}

// Fold the partials in block order (one thread: a fixed order).
__global__ void reduce3_final_kernel(const double *__restrict__ parts, int nb, double *__restrict__ out)
{
    if (threadIdx.x != 0 || blockIdx.x != 0) return;
    double s[4] = {0.0, 0.0, 0.0, 0.0};
    for (int b = 0; b < nb; ++b) {
        for (int f = 0; f < 3; ++f) s[f] += parts[(size_t)b * 4 + f];
        s[3] = fmax(s[3], parts[(size_t)b * 4 + 3]);
    }
    for (int f = 0; f < 4; ++f) out[f] = s[f];
}

size_t io_bytes(int io) { return io == GGFV_F64 ? 8 : 4; }

int check_io(ggfv3_ctx *ctx, int where, int io)
{
    if (where != GGFV_HOST && where != GGFV_DEVICE) return fail3(ctx, GGFV_EINVAL, "where must be HOST or DEVICE");
    if (io != GGFV_F64 && io != GGFV_F32) return fail3(ctx, GGFV_EINVAL, "io dtype must be F64 or F32");
    return GGFV_OK;
}

long rows_of(const ggfv3_ctx *ctx) { return (long)ctx->ny * ctx->nz; }

int ensure_staging3(ggfv3_ctx *ctx, int narrays)
{
    const size_t need = (size_t)narrays * ctx->nx * rows_of(ctx) * sizeof(double);
    if (ctx->staging && ctx->staging_bytes >= need) return GGFV_OK;
    if (ctx->staging) {
        (void)hipStreamSynchronize(ctx->stream);
        (void)hipFree(ctx->staging);
        ctx->staging = nullptr;
    }
    if (hipMalloc(&ctx->staging, need) != hipSuccess) {
        ctx->staging = nullptr;
        return fail3(ctx, GGFV_ENOMEM, "cannot allocate %zu bytes of staging memory", need);
    }
    ctx->staging_bytes = need;
    return GGFV_OK;
}

// Pack n dense io arrays (host or device) into consecutive fields at dst.
int pack_fields(ggfv3_ctx *ctx, const void *const *src, int n, int where, int io, void *dst)
{
    const size_t count = (size_t)ctx->nx * rows_of(ctx);
    const void *d[6];
    if (where == GGFV_HOST) {
        int rc = ensure_staging3(ctx, n);
        if (rc) return rc;
        for (int p = 0; p < n; ++p) {
            char *s = static_cast<char *>(ctx->staging) + p * count * io_bytes(io);
            GGFV3_HIP(ctx, hipMemcpyAsync(s, src[p], count * io_bytes(io), hipMemcpyHostToDevice, ctx->stream));
            d[p] = s;
        }
    } else {
        for (int p = 0; p < n; ++p) d[p] = src[p];
    }
    const int blocks = 1024;
    for (int p = 0; p < n; ++p) {
        char *out = static_cast<char *>(dst) + p * ctx->field * ctx->elem;
        if (ctx->dtype == GGFV_F64 && io == GGFV_F64)
            hipLaunchKernelGGL((pack3_kernel<double, double>), dim3(blocks), dim3(256), 0, ctx->stream,
                               (const double *)d[p], (double *)out, ctx->nx, rows_of(ctx), ctx->pitch);
        else if (ctx->dtype == GGFV_F64)
            hipLaunchKernelGGL((pack3_kernel<float, double>), dim3(blocks), dim3(256), 0, ctx->stream,
                               (const float *)d[p], (double *)out, ctx->nx, rows_of(ctx), ctx->pitch);
        else if (io == GGFV_F64)
            hipLaunchKernelGGL((pack3_kernel<double, float>), dim3(blocks), dim3(256), 0, ctx->stream,
                               (const double *)d[p], (float *)out, ctx->nx, rows_of(ctx), ctx->pitch);
        else
            hipLaunchKernelGGL((pack3_kernel<float, float>), dim3(blocks), dim3(256), 0, ctx->stream,
                               (const float *)d[p], (float *)out, ctx->nx, rows_of(ctx), ctx->pitch);
        GGFV3_HIP(ctx, hipGetLastError());
    }
    // the host staging area is reused by the next call
    if (where == GGFV_HOST) GGFV3_HIP(ctx, hipStreamSynchronize(ctx->stream));
    return GGFV_OK;
}

int reduce3(ggfv3_ctx *ctx, bool state, bool tensor, double *host4)
{
    double *parts = ctx->scratch, *res = ctx->scratch + (size_t)kRed3Blocks * 4;
    const void *st = state ? ctx->state[ctx->cur] : nullptr;
    const void *tn = tensor ? ctx->tensor : nullptr;
    if (ctx->dtype == GGFV_F64)
        hipLaunchKernelGGL((reduce3_kernel<double>), dim3(kRed3Blocks), dim3(kRed3), 0, ctx->stream,
                           (const double *)st, (const double *)tn, ctx->field, ctx->nx, rows_of(ctx), ctx->pitch,
                           parts);
    else
        hipLaunchKernelGGL((reduce3_kernel<float>), dim3(kRed3Blocks), dim3(kRed3), 0, ctx->stream,
                           (const float *)st, (const float *)tn, ctx->field, ctx->nx, rows_of(ctx), ctx->pitch,
                           parts);
    GGFV3_HIP(ctx, hipGetLastError());
    hipLaunchKernelGGL(reduce3_final_kernel, dim3(1), dim3(64), 0, ctx->stream, parts, kRed3Blocks, res);
    GGFV3_HIP(ctx, hipGetLastError());
    GGFV3_HIP(ctx, hipMemcpyAsync(host4, res, 4 * sizeof(double), hipMemcpyDeviceToHost, ctx->stream));
    GGFV3_HIP(ctx, hipStreamSynchronize(ctx->stream));
    return GGFV_OK;
}

template <typename T>
Step3Args<T> args3(const ggfv3_ctx *ctx, double dt)
{
    Step3Args<T> A{};
    const T *in = static_cast<const T *>(ctx->state[ctx->cur]);
    T *out = static_cast<T *>(ctx->state[1 - ctx->cur]);
    const T *tn = static_cast<const T *>(ctx->tensor);
    const size_t F = ctx->field;
    A.u = in;
    A.v = in + F;
    A.w = in + 2 * F;
    A.un = out;
    A.vn = out + F;
    A.wn = out + 2 * F;
    A.axx = tn;
    A.ayy = tn + F;
    A.azz = tn + 2 * F;
    A.axy = tn + 3 * F;
    A.axz = tn + 4 * F;
    A.ayz = tn + 5 * F;
    A.nx = ctx->nx;
    A.ny = ctx->ny;
    A.nz = ctx->nz;
    A.pitch = ctx->pitch;
    const double idx = ctx->nx / ctx->lx, idy = ctx->ny / ctx->ly, idz = ctx->nz / ctx->lz;
    A.idx = T(idx);
    A.idy = T(idy);
    A.idz = T(idz);
    A.hx = T(0.5 * idx);
    A.hy = T(0.5 * idy);
    A.hz = T(0.5 * idz);
    A.dt = T(dt);
    A.d1 = T(ctx->prm.delta1);
    A.r2 = T(ctx->prm.rho2);
    A.D2 = T(ctx->prm.Delta2);
    A.r3 = T(ctx->prm.rho3);
    A.d3 = T(ctx->prm.delta3);
    // strips of z: about four workgroups per CU on 256 CUs
    int zs = ctx->zs;
    if (zs <= 0) {
        const long cols = (long)((ctx->nx + 63) / 64) * ((ctx->ny + 3) / 4);
        const long target = 1024;
        long nzb = (target + cols - 1) / cols;
        if (nzb < 1) nzb = 1;
        zs = (int)((ctx->nz + nzb - 1) / nzb);
        if (zs < 4) zs = 4;
    }
    A.zs = zs > ctx->nz ? ctx->nz : zs;
    return A;
}

template <typename T>
hipError_t launch3(ggfv3_ctx *ctx, double dt)
{
    const Step3Args<T> A = args3<T>(ctx, dt);
    const dim3 grid((ctx->nx + 63) / 64, (ctx->ny + 3) / 4, (ctx->nz + A.zs - 1) / A.zs);
    hipLaunchKernelGGL((step3_kernel<T>), grid, dim3(64, 4), 0, ctx->stream, A);
    return hipGetLastError();
}

}  // namespace

extern "C" {

int ggfv3_create(ggfv3_ctx **out, int nx, int ny, int nz, double lx, double ly, double lz, int dtype,
                 int device, void *hip_stream)
{
    if (!out) return fail3(nullptr, GGFV_EINVAL, "null output pointer");
    *out = nullptr;
    if (nx < 1 || ny < 1 || nz < 1) return fail3(nullptr, GGFV_EINVAL, "sizes must be >= 1");
    if ((long long)nx * ny * nz > (1LL << 31))
        return fail3(nullptr, GGFV_EINVAL, "grid of %lld cells is too large", (long long)nx * ny * nz);
    if (!(lx > 0.0) || !(ly > 0.0) || !(lz > 0.0) || !std::isfinite(lx) || !std::isfinite(ly) || !std::isfinite(lz))
        return fail3(nullptr, GGFV_EINVAL, "domain lengths must be finite and > 0");
    if (dtype != GGFV_F64 && dtype != GGFV_F32) return fail3(nullptr, GGFV_EINVAL, "dtype must be F64 or F32");
    int ndev = 0;
    hipError_t he = hipGetDeviceCount(&ndev);
    if (he != hipSuccess) return fail3(nullptr, GGFV_EHIP, "hipGetDeviceCount failed: %s", hipGetErrorString(he));
    if (device < 0 || device >= ndev) return fail3(nullptr, GGFV_EINVAL, "device %d out of range [0, %d)", device, ndev);
    ggfv3_ctx *c = new (std::nothrow) ggfv3_ctx;
    if (!c) return fail3(nullptr, GGFV_ENOMEM, "out of host memory");
    c->nx = nx;
    c->ny = ny;
    c->nz = nz;
    c->lx = lx;
    c->ly = ly;
    c->lz = lz;
    c->dtype = dtype;
    c->device = device;
    c->stream = static_cast<hipStream_t>(hip_stream);
    c->pitch = ggfv::round_up(nx, ggfv::kRowAlign);
    c->field = (size_t)nz * ny * c->pitch;
    c->elem = dtype == GGFV_F64 ? 8 : 4;
    Guard3 g(device);
    bool ok = hipMalloc(&c->state[0], 3 * c->field * c->elem) == hipSuccess &&
              hipMalloc(&c->state[1], 3 * c->field * c->elem) == hipSuccess &&
              hipMalloc(&c->tensor, 6 * c->field * c->elem) == hipSuccess &&
              hipMalloc(reinterpret_cast<void **>(&c->scratch), ((size_t)kRed3Blocks * 4 + 8) * sizeof(double)) ==
                  hipSuccess;
    if (ok) ok = hipMemset(c->state[0], 0, 3 * c->field * c->elem) == hipSuccess &&
                 hipMemset(c->state[1], 0, 3 * c->field * c->elem) == hipSuccess &&
                 hipMemset(c->tensor, 0, 6 * c->field * c->elem) == hipSuccess;
    if (!ok) {
        ggfv3_destroy(c);
        return fail3(nullptr, GGFV_ENOMEM, "cannot allocate device memory for a %dx%dx%d grid", nx, ny, nz);
    }
    *out = c;
    return GGFV_OK;
}

void ggfv3_destroy(ggfv3_ctx *ctx)
{
    if (!ctx) return;
    {
        Guard3 g(ctx->device);
        (void)hipStreamSynchronize(ctx->stream);
        for (void *p : {ctx->state[0], ctx->state[1], ctx->tensor, ctx->staging, static_cast<void *>(ctx->scratch)})
            if (p) (void)hipFree(p);
    }
    delete ctx;
}

int ggfv3_set_params(ggfv3_ctx *ctx, const ggfv_params *p)
{
    if (!ctx) return GGFV_EINVAL;
    if (!p) return fail3(ctx, GGFV_EINVAL, "null params");
    const double v[5] = {p->delta1, p->rho2, p->Delta2, p->rho3, p->delta3};
    for (double x : v)
        if (!std::isfinite(x)) return fail3(ctx, GGFV_EINVAL, "parameters must be finite");
    ctx->prm = *p;
    ctx->has_params = true;
    return GGFV_OK;
}

int ggfv3_set_tensor(ggfv3_ctx *ctx, const void *axx, const void *ayy, const void *azz, const void *axy,
                     const void *axz, const void *ayz, int where, int io)
{
    if (!ctx) return GGFV_EINVAL;
    int rc = check_io(ctx, where, io);
    if (rc) return rc;
    const void *src[6] = {axx, ayy, azz, axy, axz, ayz};
    for (const void *p : src)
        if (!p) return fail3(ctx, GGFV_EINVAL, "null tensor field");
    Guard3 g(ctx->device);
    if ((rc = pack_fields(ctx, src, 6, where, io, ctx->tensor))) return rc;
    ctx->has_tensor = true;
    return GGFV_OK;
}

int ggfv3_set_state(ggfv3_ctx *ctx, const void *u, const void *v, const void *w, int where, int io)
{
    if (!ctx) return GGFV_EINVAL;
    int rc = check_io(ctx, where, io);
    if (rc) return rc;
    if (!u || !v || !w) return fail3(ctx, GGFV_EINVAL, "null state field");
    Guard3 g(ctx->device);
    const void *src[3] = {u, v, w};
    if ((rc = pack_fields(ctx, src, 3, where, io, ctx->state[ctx->cur]))) return rc;
    ctx->has_state = true;
    ctx->t = 0.0;
    ctx->steps = 0;
    return GGFV_OK;
}

int ggfv3_get_state(ggfv3_ctx *ctx, void *u, void *v, void *w, int where, int io)
{
    if (!ctx) return GGFV_EINVAL;
    int rc = check_io(ctx, where, io);
    if (rc) return rc;
    if (!u || !v || !w) return fail3(ctx, GGFV_EINVAL, "null output field");
    if (!ctx->has_state) return fail3(ctx, GGFV_ESTATE, "state not set");
    Guard3 g(ctx->device);
    const size_t count = (size_t)ctx->nx * rows_of(ctx);
    void *dst[3] = {u, v, w};
    if (where == GGFV_HOST && (rc = ensure_staging3(ctx, 3))) return rc;
    for (int p = 0; p < 3; ++p) {
        const char *src = static_cast<const char *>(ctx->state[ctx->cur]) + p * ctx->field * ctx->elem;
        void *d = where == GGFV_HOST ? static_cast<char *>(ctx->staging) + p * count * io_bytes(io) : dst[p];
        if (ctx->dtype == GGFV_F64 && io == GGFV_F64)
            hipLaunchKernelGGL((unpack3_kernel<double, double>), dim3(1024), dim3(256), 0, ctx->stream,
                               (const double *)src, (double *)d, ctx->nx, rows_of(ctx), ctx->pitch);
        else if (ctx->dtype == GGFV_F64)
            hipLaunchKernelGGL((unpack3_kernel<double, float>), dim3(1024), dim3(256), 0, ctx->stream,
                               (const double *)src, (float *)d, ctx->nx, rows_of(ctx), ctx->pitch);
        else if (io == GGFV_F64)
            hipLaunchKernelGGL((unpack3_kernel<float, double>), dim3(1024), dim3(256), 0, ctx->stream,
                               (const float *)src, (double *)d, ctx->nx, rows_of(ctx), ctx->pitch);
        else
            hipLaunchKernelGGL((unpack3_kernel<float, float>), dim3(1024), dim3(256), 0, ctx->stream,
                               (const float *)src, (float *)d, ctx->nx, rows_of(ctx), ctx->pitch);
        GGFV3_HIP(ctx, hipGetLastError());
        if (where == GGFV_HOST)
            GGFV3_HIP(ctx, hipMemcpyAsync(dst[p], d, count * io_bytes(io), hipMemcpyDeviceToHost, ctx->stream));
    }
    if (where == GGFV_HOST) GGFV3_HIP(ctx, hipStreamSynchronize(ctx->stream));
    return GGFV_OK;
}

int ggfv3_stable_dt(ggfv3_ctx *ctx, double safety, double *dt)
{
    if (!ctx) return GGFV_EINVAL;
    if (!dt) return fail3(ctx, GGFV_EINVAL, "null dt");
    if (!(safety > 0.0) || !std::isfinite(safety)) return fail3(ctx, GGFV_EINVAL, "safety must be > 0");
    if (!ctx->has_tensor || !ctx->has_params) return fail3(ctx, GGFV_ESTATE, "tensor and parameters must be set");
    Guard3 g(ctx->device);
    double r[4];
    int rc = reduce3(ctx, false, true, r);
    if (rc) return rc;
    double gmax = ctx->prm.Delta2;
    if (r[3] > gmax) gmax = r[3];
    if (!(gmax > 0.0)) return fail3(ctx, GGFV_EINVAL, "no positive diffusion: step bound undefined");
    const double idx = ctx->nx / ctx->lx, idy = ctx->ny / ctx->ly, idz = ctx->nz / ctx->lz;
    *dt = safety / (2.0 * gmax * (idx * idx + idy * idy + idz * idz));
    return GGFV_OK;
}

int ggfv3_step(ggfv3_ctx *ctx, double dt, long long nsteps)
{
    if (!ctx) return GGFV_EINVAL;
    if (!(dt > 0.0) || !std::isfinite(dt)) return fail3(ctx, GGFV_EINVAL, "dt must be finite and > 0");
    if (nsteps < 0) return fail3(ctx, GGFV_EINVAL, "nsteps must be >= 0");
    if (!ctx->has_state || !ctx->has_tensor || !ctx->has_params)
        return fail3(ctx, GGFV_ESTATE, "state, tensor and parameters must be set before stepping");
    Guard3 g(ctx->device);
    for (long long s = 0; s < nsteps; ++s) {
        GGFV3_HIP(ctx, ctx->dtype == GGFV_F64 ? launch3<double>(ctx, dt) : launch3<float>(ctx, dt));
        ctx->cur ^= 1;
    }
    const double dt_used = ctx->dtype == GGFV_F64 ? dt : (double)(float)dt;
    ctx->t += dt_used * (double)nsteps;
    ctx->steps += nsteps;
    return GGFV_OK;
}

int ggfv3_mass(ggfv3_ctx *ctx, double *mass3)
{
    if (!ctx) return GGFV_EINVAL;
    if (!mass3) return fail3(ctx, GGFV_EINVAL, "null output");
    if (!ctx->has_state) return fail3(ctx, GGFV_ESTATE, "state not set");
    Guard3 g(ctx->device);
    double r[4];
    int rc = reduce3(ctx, true, false, r);
    if (rc) return rc;
    const double vol = (ctx->lx / ctx->nx) * (ctx->ly / ctx->ny) * (ctx->lz / ctx->nz);
    for (int f = 0; f < 3; ++f) mass3[f] = vol * r[f];
    return GGFV_OK;
}

int ggfv3_time(const ggfv3_ctx *ctx, double *t, long long *steps)
{
    if (!ctx) return GGFV_EINVAL;
    if (t) *t = ctx->t;
    if (steps) *steps = ctx->steps;
    return GGFV_OK;
}

int ggfv3_set_tuning(ggfv3_ctx *ctx, int z_per_strip)
{
    if (!ctx) return GGFV_EINVAL;
    if (z_per_strip < 0) return fail3(ctx, GGFV_EINVAL, "z_per_strip must be >= 0");
    ctx->zs = z_per_strip;
    return GGFV_OK;
}

const char *ggfv3_last_error(const ggfv3_ctx *ctx) { return ctx ? ctx->err.c_str() : g3_create_error.c_str(); }

}  // extern "C"
