// ggfv_api.hip -- the C ABI declared in include/ggfv.h: context lifetime, device
// buffers, host/device transfers, argument checking and the step loop.

#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <new>

#include "ggfv_internal.hpp"

using namespace ggfv;

namespace {

// Message of the last failed ggfv_create on this thread (there is no context to
// hold it); reported by ggfv_last_error(NULL).
thread_local std::string g_create_error;

int fail(ggfv_ctx *ctx, int code, const char *fmt, ...) __attribute__((format(printf, 3, 4)));

int fail(ggfv_ctx *ctx, int code, const char *fmt, ...)
{
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    if (ctx)
        ctx->err = buf;
    else
        g_create_error = buf;
    return code;
}

// Makes the context's device current for the scope of an API call.
struct DeviceGuard {
    int prev = -1;
    hipError_t status = hipSuccess;
    explicit DeviceGuard(int dev)
    {
        if (hipGetDevice(&prev) != hipSuccess) prev = -1;
        if (prev != dev) status = hipSetDevice(dev);
    }
    ~DeviceGuard()
    {
        int now = -1;
        if (prev >= 0 && hipGetDevice(&now) == hipSuccess && now != prev) (void)hipSetDevice(prev);
    }
};

#define GGFV_HIP(ctx, call)                                                                  \
    do {                                                                                     \
        hipError_t e_ = (call);                                                              \
        if (e_ != hipSuccess)                                                                \
            return fail((ctx), GGFV_EHIP, "%s failed: %s", #call, hipGetErrorString(e_));    \
    } while (0)

bool valid_io(int io) { return io == GGFV_F32 || io == GGFV_F64; }
size_t io_size(int io) { return io == GGFV_F64 ? 8 : 4; }

int check_ptrs(ggfv_ctx *ctx, const void *p0, const void *p1, const void *p2, int where, int io)
{
    if (!ctx) return GGFV_EINVAL;
    if (!p0 || !p1 || !p2) return fail(ctx, GGFV_EINVAL, "null array pointer");
    if (where != GGFV_HOST && where != GGFV_DEVICE)
        return fail(ctx, GGFV_EINVAL, "where must be GGFV_HOST or GGFV_DEVICE (got %d)", where);
    if (!valid_io(io))
        return fail(ctx, GGFV_EINVAL, "io_dtype must be GGFV_F32 or GGFV_F64 (got %d)", io);
    return GGFV_OK;
}

int ensure_staging(ggfv_ctx *ctx, int narrays = 3)
{
    const size_t need = (size_t)narrays * ctx->nx * ctx->ny * sizeof(double);
    if (ctx->staging && ctx->staging_bytes >= need) return GGFV_OK;
    if (ctx->staging) {
        (void)hipStreamSynchronize(ctx->stream);
        (void)hipFree(ctx->staging);
        ctx->staging = nullptr;
    }
    if (hipMalloc(&ctx->staging, need) != hipSuccess) {
        ctx->staging = nullptr;
        return fail(ctx, GGFV_ENOMEM, "cannot allocate %zu bytes of staging memory", need);
    }
    ctx->staging_bytes = need;
    return GGFV_OK;
}

// Default launch shape, from h4 = ny * (column strips of the 4-step lane-shift
// kernel) / (8 * compute units): the strip height at which those one-wave
// strips fill the device's wave slots once at two waves per SIMD (wide lanes
// except for the compensated state).  Every level of a strip repeats a
// pipeline fill of about 2K+2 rows, so fused launches pay only on strips that
// are tall enough.  Measured on MI355X (FP64 / compensated FP32,
// Gcell-updates/s: single step, 2 and 4 steps per launch): 512^2 (h4 = 1.3)
// 39 / 23 / 15 and 31 / 23 / 15; 1024^2 (h4 = 4.5) 58 / 73 / 54 and 61 / 84 /
// 58; 1536^2 (h4 = 9.8) 60 / 118 / 115 and 76 / 151 / 123; 2048^2 (h4 = 18)
// 72 / 141 / 134 and 71 / 170 / 185; 4096^2 (h4 = 70) 71 / 127 / 230 and 80 /
// 136 / 279.  Hence: h4 >= 8, four steps per launch; 3 <= h4 < 8, two;
// otherwise the single-step kernel.
void set_default_shape(ggfv_ctx *ctx)
{
    ctx->rows_per_strip = 0;
    ctx->threads = 0;
    ctx->fused_steps = 4;
    ctx->lane_shift = (ctx->dtype == GGFV_F32C) ? 1 : 2;
    const int outw = (ctx->dtype == GGFV_F32) ? 248 : 120;     // output columns of one wave, K = 4
    const double h4 = (double)ctx->ny * ((ctx->nx + outw - 1) / outw) / (8.0 * (ctx->cus > 0 ? ctx->cus : 256));
    if (h4 >= 8.0) return;
    if (h4 >= 3.0) {
        ctx->fused_steps = 2;
        return;
    }
    ctx->fused_steps = 1;
    ctx->lane_shift = 0;
}

// Copy three dense host arrays into the staging area; returns device pointers.
int stage_in(ggfv_ctx *ctx, const void *h0, const void *h1, const void *h2, int io,
             const void *(&d)[3])
{
    int rc = ensure_staging(ctx);
    if (rc) return rc;
    const size_t bytes = (size_t)ctx->nx * ctx->ny * io_size(io);
    const void *h[3] = {h0, h1, h2};
    for (int p = 0; p < 3; ++p) {
        char *dst = static_cast<char *>(ctx->staging) + p * bytes;
        GGFV_HIP(ctx, hipMemcpyAsync(dst, h[p], bytes, hipMemcpyHostToDevice, ctx->stream));
        d[p] = dst;
    }
    return GGFV_OK;
}

int read_result(ggfv_ctx *ctx, double *host, int count)
{
    const double *res = static_cast<const double *>(ctx->scratch) + (size_t)kMaxPartialBlocks * kDiagSlots;
    GGFV_HIP(ctx, hipMemcpyAsync(host, res, count * sizeof(double), hipMemcpyDeviceToHost, ctx->stream));
    GGFV_HIP(ctx, hipStreamSynchronize(ctx->stream));
    return GGFV_OK;
}

// Adjoint buffers (context precision planes, then FP64 slots):
//   planes 0-2: a state x for a single adjoint step; 3-5 and 6-8: adjoint state
//   ping-pong; 9-11: tensor gradient; then adjoint_blocks()*5 partial-sum slots
//   and 8 result doubles.
int ensure_adjoint(ggfv_ctx *ctx)
{
    const size_t planes = 12 * ctx->plane * ctx->elem;
    const size_t slots = ((size_t)adjoint_blocks(ctx) * 5 + 8) * sizeof(double);
    const size_t need = planes + slots;
    if (ctx->adj && ctx->adj_bytes >= need) return GGFV_OK;
    if (ctx->adj) {
        (void)hipStreamSynchronize(ctx->stream);
        (void)hipFree(ctx->adj);
        ctx->adj = nullptr;
    }
    if (hipMalloc(&ctx->adj, need) != hipSuccess) {
        ctx->adj = nullptr;
        return fail(ctx, GGFV_ENOMEM, "cannot allocate %zu bytes for the adjoint", need);
    }
    ctx->adj_bytes = need;
    return GGFV_OK;
}

void *adj_planes(ggfv_ctx *ctx, int first)
{
    return static_cast<char *>(ctx->adj) + (size_t)first * ctx->plane * ctx->elem;
}

double *adj_slots(ggfv_ctx *ctx)
{
    return reinterpret_cast<double *>(static_cast<char *>(ctx->adj) + 12 * ctx->plane * ctx->elem);
}

double *adj_result(ggfv_ctx *ctx) { return adj_slots(ctx) + (size_t)adjoint_blocks(ctx) * 5; }

// Pack three caller arrays (host or device) into three storage planes.
int pack_in(ggfv_ctx *ctx, const void *p0, const void *p1, const void *p2, int where, int io, void *dst)
{
    const void *d[3] = {p0, p1, p2};
    int rc;
    if (where == GGFV_HOST && (rc = stage_in(ctx, p0, p1, p2, io, d))) return rc;
    GGFV_HIP(ctx, launch_pack3(ctx, d[0], d[1], d[2], io == GGFV_F64, dst, 3, false));
    return GGFV_OK;
}

}  // namespace

extern "C" {

const char *ggfv_status_string(int s)
{
    switch (s) {
    case GGFV_OK: return "GGFV_OK";
    case GGFV_EINVAL: return "GGFV_EINVAL";
    case GGFV_ENOMEM: return "GGFV_ENOMEM";
    case GGFV_EHIP: return "GGFV_EHIP";
    case GGFV_ESTATE: return "GGFV_ESTATE";
    case GGFV_EUNSTABLE: return "GGFV_EUNSTABLE";
    default: return "GGFV_UNKNOWN";
    }
}

const char *ggfv_last_error(const ggfv_ctx *ctx) { return ctx ? ctx->err.c_str() : g_create_error.c_str(); }

int ggfv_create(ggfv_ctx **out, int nx, int ny, double lx, double ly, int dtype, int device,
                void *hip_stream)
{
    if (!out) return fail(nullptr, GGFV_EINVAL, "null output pointer");
    *out = nullptr;
    if (nx < 1 || ny < 1) return fail(nullptr, GGFV_EINVAL, "grid must be at least 1x1 (got %dx%d)", nx, ny);
    if ((long long)nx * ny > (1LL << 34)) return fail(nullptr, GGFV_EINVAL, "grid too large (%dx%d)", nx, ny);
    if (!(lx > 0.0) || !(ly > 0.0) || !std::isfinite(lx) || !std::isfinite(ly))
        return fail(nullptr, GGFV_EINVAL, "domain sides must be finite and > 0");
    if (dtype != GGFV_F32 && dtype != GGFV_F64 && dtype != GGFV_F32C)
        return fail(nullptr, GGFV_EINVAL, "unknown dtype %d", dtype);
    int ndev = 0;
    hipError_t he = hipGetDeviceCount(&ndev);
    if (he != hipSuccess) return fail(nullptr, GGFV_EHIP, "hipGetDeviceCount failed: %s", hipGetErrorString(he));
    if (device < 0 || device >= ndev)
        return fail(nullptr, GGFV_EHIP, "device %d out of range (%d devices)", device, ndev);

    int cus = 0;
    he = hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, device);
    if (he != hipSuccess || cus < 1)
        return fail(nullptr, GGFV_EHIP, "cannot query the compute units of device %d", device);

    ggfv_ctx *ctx = new (std::nothrow) ggfv_ctx;
    if (!ctx) return GGFV_ENOMEM;
    ctx->cus = cus;
    ctx->nx = nx;
    ctx->ny = ny;
    ctx->lx = lx;
    ctx->ly = ly;
    ctx->dtype = dtype;
    ctx->device = device;
    ctx->stream = static_cast<hipStream_t>(hip_stream);
    ctx->pitch = round_up(nx, kRowAlign);
    ctx->plane = (size_t)ctx->pitch * ny;
    ctx->elem = (dtype == GGFV_F64) ? 8 : 4;
    ctx->nfields = (dtype == GGFV_F32C) ? 6 : 3;

    DeviceGuard g(device);
    if (g.status != hipSuccess) {
        delete ctx;
        return fail(nullptr, GGFV_EHIP, "hipSetDevice(%d) failed: %s", device, hipGetErrorString(g.status));
    }
    set_default_shape(ctx);
    const size_t sbytes = ctx->nfields * ctx->plane * ctx->elem;
    const size_t tbytes = 3 * ctx->plane * ctx->elem;
    ctx->scratch_bytes = ((size_t)kMaxPartialBlocks * kDiagSlots + 64) * sizeof(double);
    bool ok = hipMalloc(&ctx->state[0], sbytes) == hipSuccess &&
              hipMalloc(&ctx->state[1], sbytes) == hipSuccess &&
              hipMalloc(&ctx->tensor, tbytes) == hipSuccess &&
              hipMalloc(&ctx->scratch, ctx->scratch_bytes) == hipSuccess;
    if (ok) {
        // zero padding columns once; every kernel keeps them zero afterwards
        ok = hipMemset(ctx->state[0], 0, sbytes) == hipSuccess &&
             hipMemset(ctx->state[1], 0, sbytes) == hipSuccess &&
             hipMemset(ctx->tensor, 0, tbytes) == hipSuccess &&
             hipMemset(ctx->scratch, 0, ctx->scratch_bytes) == hipSuccess;
    }
    if (!ok) {
        (void)hipGetLastError();
        ggfv_destroy(ctx);
        return fail(nullptr, GGFV_ENOMEM, "cannot allocate %zu bytes of device memory",
                    2 * sbytes + tbytes);
    }
    *out = ctx;
    return GGFV_OK;
}

void ggfv_destroy(ggfv_ctx *ctx)
{
    if (!ctx) return;
    {
        DeviceGuard g(ctx->device);
        (void)hipStreamSynchronize(ctx->stream);
        for (void *p : {ctx->state[0], ctx->state[1], ctx->tensor, ctx->scratch, ctx->staging, ctx->adj,
                        static_cast<void *>(ctx->adapt), static_cast<void *>(ctx->front)})
            if (p) (void)hipFree(p);
    }
    delete ctx;
}

int ggfv_set_stream(ggfv_ctx *ctx, void *hip_stream)
{
    if (!ctx) return GGFV_EINVAL;
    ctx->stream = static_cast<hipStream_t>(hip_stream);
    return GGFV_OK;
}

int ggfv_set_params(ggfv_ctx *ctx, const ggfv_params *p)
{
    if (!ctx) return GGFV_EINVAL;
    if (!p) return fail(ctx, GGFV_EINVAL, "null params");
    const double v[5] = {p->delta1, p->rho2, p->Delta2, p->rho3, p->delta3};
    for (double x : v)
        if (!std::isfinite(x)) return fail(ctx, GGFV_EINVAL, "parameters must be finite");
    if (p->Delta2 < 0.0) return fail(ctx, GGFV_EINVAL, "Delta2 must be >= 0 (got %g)", p->Delta2);
    ctx->prm = *p;
    ctx->has_params = true;
    return GGFV_OK;
}

static int check_spd(ggfv_ctx *ctx)
{
    GGFV_HIP(ctx, launch_spd_count(ctx));
    double r[2];
    int rc = read_result(ctx, r, 2);
    if (rc) return rc;
    if (r[0] > 0.0) {
        ctx->has_tensor = false;
        return fail(ctx, GGFV_EINVAL,
                    "tensor is not positive definite in %.0f cells (need a > 0 and a*c - b^2 > 0)", r[0]);
    }
    ctx->has_tensor = true;
    return GGFV_OK;
}

int ggfv_set_tensor(ggfv_ctx *ctx, const void *a, const void *b, const void *c, int where, int io)
{
    int rc = check_ptrs(ctx, a, b, c, where, io);
    if (rc) return rc;
    DeviceGuard g(ctx->device);
    const void *d[3] = {a, b, c};
    if (where == GGFV_HOST && (rc = stage_in(ctx, a, b, c, io, d))) return rc;
    GGFV_HIP(ctx, launch_pack3(ctx, d[0], d[1], d[2], io == GGFV_F64, ctx->tensor, 3, false));
    return check_spd(ctx);
}

int ggfv_set_tensor_eig(ggfv_ctx *ctx, const void *l1, const void *l2, const void *th, int where, int io)
{
    int rc = check_ptrs(ctx, l1, l2, th, where, io);
    if (rc) return rc;
    DeviceGuard g(ctx->device);
    const void *d[3] = {l1, l2, th};
    if (where == GGFV_HOST && (rc = stage_in(ctx, l1, l2, th, io, d))) return rc;
    GGFV_HIP(ctx, launch_tensor_eig(ctx, d[0], d[1], d[2], io == GGFV_F64));
    return check_spd(ctx);
}

static int copy_out(ggfv_ctx *ctx, const void *src_base, bool has_lo, void *o0, void *o1, void *o2,
                    int where, int io);

static int check9(ggfv_ctx *ctx, const void *const *p, int where, int io)
{
    for (int k = 0; k < 9; k += 3) {
        int rc = check_ptrs(ctx, p[k], p[k + 1], p[k + 2], where, io);
        if (rc) return rc;
    }
    return GGFV_OK;
}

long long ggfv_state_bytes(const ggfv_ctx *ctx)
{
    if (!ctx) return 0;
    return (long long)(ctx->nfields * ctx->plane * ctx->elem);
}

int ggfv_step_checkpointed(ggfv_ctx *ctx, double dt, long long nsteps, long long every, void *ckpt,
                           long long ckpt_bytes)
{
    if (!ctx) return GGFV_EINVAL;
    if (!(dt > 0.0) || !std::isfinite(dt)) return fail(ctx, GGFV_EINVAL, "dt must be finite and > 0 (got %g)", dt);
    if (nsteps < 1 || every < 1) return fail(ctx, GGFV_EINVAL, "need nsteps >= 1 and every >= 1");
    if (!ckpt) return fail(ctx, GGFV_EINVAL, "null checkpoint buffer");
    if (!ctx->has_state || !ctx->has_tensor || !ctx->has_params)
        return fail(ctx, GGFV_ESTATE, "state, tensor and parameters must be set before stepping");
    const long long sb = ggfv_state_bytes(ctx);
    const long long nck = (nsteps + every - 1) / every;
    if (ckpt_bytes < nck * sb)
        return fail(ctx, GGFV_EINVAL, "checkpoint buffer holds %lld bytes, %lld needed", ckpt_bytes, nck * sb);
    DeviceGuard g(ctx->device);
    const double dt_used = (ctx->dtype == GGFV_F64) ? dt : (double)(float)dt;
    for (long long s = 0; s < nsteps; s += every) {
        GGFV_HIP(ctx, hipMemcpyAsync(static_cast<char *>(ckpt) + (s / every) * sb, ctx->state[ctx->cur], sb,
                                     hipMemcpyDeviceToDevice, ctx->stream));
        const long long n = (nsteps - s < every) ? nsteps - s : every;
        GGFV_HIP(ctx, advance_steps(ctx, dt, n));
    }
    ctx->t += dt_used * (double)nsteps;
    ctx->steps += nsteps;
    ctx->last_dt = dt_used;
    return GGFV_OK;
}

int ggfv_adjoint_step(ggfv_ctx *ctx, double dt, const void *u, const void *v, const void *w,
                      const void *lam_u, const void *lam_v, const void *lam_w, void *out_u, void *out_v,
                      void *out_w, void *g_a, void *g_b, void *g_c, double *g_params, int where, int io)
{
    if (!ctx) return GGFV_EINVAL;
    const void *ins[9] = {u, v, w, lam_u, lam_v, lam_w, g_a, g_b, g_c};
    int rc = check9(ctx, ins, where, io);
    if (rc) return rc;
    if ((rc = check_ptrs(ctx, out_u, out_v, out_w, where, io))) return rc;
    if (!g_params) return fail(ctx, GGFV_EINVAL, "null g_params");
    if (!(dt > 0.0) || !std::isfinite(dt)) return fail(ctx, GGFV_EINVAL, "dt must be finite and > 0");
    if (!ctx->has_tensor || !ctx->has_params) return fail(ctx, GGFV_ESTATE, "tensor and parameters must be set");
    DeviceGuard g(ctx->device);
    if ((rc = ensure_adjoint(ctx))) return rc;
    void *X = adj_planes(ctx, 0), *LA = adj_planes(ctx, 3), *LB = adj_planes(ctx, 6), *G = adj_planes(ctx, 9);
    if ((rc = pack_in(ctx, u, v, w, where, io, X))) return rc;
    if ((rc = pack_in(ctx, lam_u, lam_v, lam_w, where, io, LA))) return rc;
    if ((rc = pack_in(ctx, g_a, g_b, g_c, where, io, G))) return rc;
    const int nb = adjoint_blocks(ctx);
    GGFV_HIP(ctx, launch_zero(ctx, adj_slots(ctx), (size_t)nb * 5 * sizeof(double)));
    GGFV_HIP(ctx, launch_adjoint_step(ctx, X, LA, LB, G, adj_slots(ctx), dt));
    GGFV_HIP(ctx, launch_slots_reduce(ctx, adj_slots(ctx), nb, adj_result(ctx)));
    if ((rc = copy_out(ctx, LB, false, out_u, out_v, out_w, where, io))) return rc;
    if ((rc = copy_out(ctx, G, false, g_a, g_b, g_c, where, io))) return rc;
    double gp[5];
    GGFV_HIP(ctx, hipMemcpyAsync(gp, adj_result(ctx), sizeof gp, hipMemcpyDeviceToHost, ctx->stream));
    GGFV_HIP(ctx, hipStreamSynchronize(ctx->stream));
    for (int k = 0; k < 5; ++k) g_params[k] += gp[k];
    return GGFV_OK;
}

int ggfv_adjoint_run(ggfv_ctx *ctx, double dt, long long nsteps, long long every, const void *ckpt,
                     long long ckpt_bytes, void *work, long long work_bytes, void *lam_u, void *lam_v,
                     void *lam_w, void *g_a, void *g_b, void *g_c, double *g_params, int where, int io)
{
    if (!ctx) return GGFV_EINVAL;
    int rc = check_ptrs(ctx, lam_u, lam_v, lam_w, where, io);
    if (rc) return rc;
    if ((rc = check_ptrs(ctx, g_a, g_b, g_c, where, io))) return rc;
    if (!g_params || !ckpt || !work) return fail(ctx, GGFV_EINVAL, "null checkpoint, work or g_params");
    if (!(dt > 0.0) || !std::isfinite(dt)) return fail(ctx, GGFV_EINVAL, "dt must be finite and > 0");
    if (nsteps < 1 || every < 1) return fail(ctx, GGFV_EINVAL, "need nsteps >= 1 and every >= 1");
    if (!ctx->has_tensor || !ctx->has_params) return fail(ctx, GGFV_ESTATE, "tensor and parameters must be set");
    const long long sb = ggfv_state_bytes(ctx);
    const long long nck = (nsteps + every - 1) / every;
    const long long nwork = every > 1 ? every - 1 : 1;
    if (ckpt_bytes < nck * sb) return fail(ctx, GGFV_EINVAL, "checkpoint buffer too small");
    if (work_bytes < nwork * sb) return fail(ctx, GGFV_EINVAL, "work buffer too small (%lld < %lld)", work_bytes, nwork * sb);
    DeviceGuard g(ctx->device);
    if ((rc = ensure_adjoint(ctx))) return rc;
    void *L[2] = {adj_planes(ctx, 3), adj_planes(ctx, 6)};
    void *G = adj_planes(ctx, 9);
    if ((rc = pack_in(ctx, lam_u, lam_v, lam_w, where, io, L[0]))) return rc;
    const int nb = adjoint_blocks(ctx);
    GGFV_HIP(ctx, launch_zero(ctx, G, 3 * ctx->plane * ctx->elem));
    GGFV_HIP(ctx, launch_zero(ctx, adj_slots(ctx), (size_t)nb * 5 * sizeof(double)));
    int cur = 0;
    const char *ck = static_cast<const char *>(ckpt);
    char *wk = static_cast<char *>(work);
    for (long long c = nck - 1; c >= 0; --c) {
        const long long s0 = c * every;
        const long long len = (nsteps - s0 < every) ? nsteps - s0 : every;
        auto state = [&](long long t) -> const void * {
            return t == 0 ? static_cast<const void *>(ck + c * sb) : static_cast<const void *>(wk + (t - 1) * sb);
        };
        for (long long t = 0; t + 1 < len; ++t)
            GGFV_HIP(ctx, launch_step_planes(ctx, state(t), wk + t * sb, dt));
        for (long long t = len - 1; t >= 0; --t) {
            GGFV_HIP(ctx, launch_adjoint_step(ctx, state(t), L[cur], L[1 - cur], G, adj_slots(ctx), dt));
            cur ^= 1;
        }
    }
    GGFV_HIP(ctx, launch_slots_reduce(ctx, adj_slots(ctx), nb, adj_result(ctx)));
    if ((rc = copy_out(ctx, L[cur], false, lam_u, lam_v, lam_w, where, io))) return rc;
    if ((rc = copy_out(ctx, G, false, g_a, g_b, g_c, where, io))) return rc;
    GGFV_HIP(ctx, hipMemcpyAsync(g_params, adj_result(ctx), 5 * sizeof(double), hipMemcpyDeviceToHost, ctx->stream));
    GGFV_HIP(ctx, hipStreamSynchronize(ctx->stream));
    return GGFV_OK;
}

int ggfv_eig_backward(ggfv_ctx *ctx, const void *lam1, const void *lam2, const void *theta, const void *g_a,
                      const void *g_b, const void *g_c, void *g_l1, void *g_l2, void *g_th, int where, int io)
{
    if (!ctx) return GGFV_EINVAL;
    const void *ins[9] = {lam1, lam2, theta, g_a, g_b, g_c, g_l1, g_l2, g_th};
    int rc = check9(ctx, ins, where, io);
    if (rc) return rc;
    DeviceGuard g(ctx->device);
    const bool f64 = io == GGFV_F64;
    if (where == GGFV_DEVICE) {
        GGFV_HIP(ctx, launch_eig_backward(ctx, lam1, lam2, theta, g_a, g_b, g_c, g_l1, g_l2, g_th, f64));
        return GGFV_OK;
    }
    if ((rc = ensure_staging(ctx, 9))) return rc;
    const size_t bytes = (size_t)ctx->nx * ctx->ny * io_size(io);
    char *s = static_cast<char *>(ctx->staging);
    for (int k = 0; k < 6; ++k)
        GGFV_HIP(ctx, hipMemcpyAsync(s + k * bytes, ins[k], bytes, hipMemcpyHostToDevice, ctx->stream));
    GGFV_HIP(ctx, launch_eig_backward(ctx, s, s + bytes, s + 2 * bytes, s + 3 * bytes, s + 4 * bytes,
                                      s + 5 * bytes, s + 6 * bytes, s + 7 * bytes, s + 8 * bytes, f64));
    void *outs[3] = {g_l1, g_l2, g_th};
    for (int k = 0; k < 3; ++k)
        GGFV_HIP(ctx, hipMemcpyAsync(outs[k], s + (6 + k) * bytes, bytes, hipMemcpyDeviceToHost, ctx->stream));
    GGFV_HIP(ctx, hipStreamSynchronize(ctx->stream));
    return GGFV_OK;
}

static int copy_out(ggfv_ctx *ctx, const void *src_base, bool has_lo, void *o0, void *o1, void *o2,
                    int where, int io)
{
    if (where == GGFV_DEVICE) {
        GGFV_HIP(ctx, launch_unpack3(ctx, src_base, has_lo, o0, o1, o2, io == GGFV_F64));
        return GGFV_OK;
    }
    int rc = ensure_staging(ctx);
    if (rc) return rc;
    const size_t bytes = (size_t)ctx->nx * ctx->ny * io_size(io);
    char *s = static_cast<char *>(ctx->staging);
    GGFV_HIP(ctx, launch_unpack3(ctx, src_base, has_lo, s, s + bytes, s + 2 * bytes, io == GGFV_F64));
    void *o[3] = {o0, o1, o2};
    for (int p = 0; p < 3; ++p)
        GGFV_HIP(ctx, hipMemcpyAsync(o[p], s + p * bytes, bytes, hipMemcpyDeviceToHost, ctx->stream));
    GGFV_HIP(ctx, hipStreamSynchronize(ctx->stream));
    return GGFV_OK;
}

int ggfv_get_tensor(ggfv_ctx *ctx, void *a, void *b, void *c, int where, int io)
{
    int rc = check_ptrs(ctx, a, b, c, where, io);
    if (rc) return rc;
    if (!ctx->has_tensor) return fail(ctx, GGFV_ESTATE, "tensor not set");
    DeviceGuard g(ctx->device);
    return copy_out(ctx, ctx->tensor, false, a, b, c, where, io);
}

int ggfv_set_state(ggfv_ctx *ctx, const void *u, const void *v, const void *w, int where, int io)
{
    int rc = check_ptrs(ctx, u, v, w, where, io);
    if (rc) return rc;
    DeviceGuard g(ctx->device);
    const void *d[3] = {u, v, w};
    if (where == GGFV_HOST && (rc = stage_in(ctx, u, v, w, io, d))) return rc;
    GGFV_HIP(ctx, launch_pack3(ctx, d[0], d[1], d[2], io == GGFV_F64, ctx->state[ctx->cur],
                               ctx->nfields, ctx->dtype == GGFV_F32C));
    if (where == GGFV_HOST) GGFV_HIP(ctx, hipStreamSynchronize(ctx->stream));
    ctx->has_state = true;
    ctx->t = 0.0;
    ctx->steps = 0;
    return GGFV_OK;
}

int ggfv_get_state(ggfv_ctx *ctx, void *u, void *v, void *w, int where, int io)
{
    int rc = check_ptrs(ctx, u, v, w, where, io);
    if (rc) return rc;
    if (!ctx->has_state) return fail(ctx, GGFV_ESTATE, "state not set");
    DeviceGuard g(ctx->device);
    return copy_out(ctx, ctx->state[ctx->cur], ctx->dtype == GGFV_F32C, u, v, w, where, io);
}

int ggfv_stable_dt(ggfv_ctx *ctx, double safety, double *dt_out)
{
    if (!ctx) return GGFV_EINVAL;
    if (!dt_out) return fail(ctx, GGFV_EINVAL, "null dt_out");
    if (!(safety > 0.0) || !std::isfinite(safety)) return fail(ctx, GGFV_EINVAL, "safety must be > 0");
    if (!ctx->has_tensor || !ctx->has_params) return fail(ctx, GGFV_ESTATE, "tensor and parameters must be set");
    DeviceGuard g(ctx->device);
    GGFV_HIP(ctx, launch_lambda_max(ctx));
    double r[2];
    int rc = read_result(ctx, r, 2);
    if (rc) return rc;
    double lm = ctx->prm.Delta2;
    if (r[1] > lm) lm = r[1];
    if (!(lm > 0.0)) return fail(ctx, GGFV_EINVAL, "no positive diffusion: step bound undefined");
    const double idx = ctx->nx / ctx->lx, idy = ctx->ny / ctx->ly;
    *dt_out = safety / (2.0 * lm * (idx * idx + idy * idy));
    return GGFV_OK;
}

int ggfv_step(ggfv_ctx *ctx, double dt, long long nsteps)
{
    if (!ctx) return GGFV_EINVAL;
    if (!(dt > 0.0) || !std::isfinite(dt)) return fail(ctx, GGFV_EINVAL, "dt must be finite and > 0 (got %g)", dt);
    if (nsteps < 0) return fail(ctx, GGFV_EINVAL, "nsteps must be >= 0 (got %lld)", nsteps);
    if (!ctx->has_state || !ctx->has_tensor || !ctx->has_params)
        return fail(ctx, GGFV_ESTATE, "state, tensor and parameters must be set before stepping");
    if (nsteps == 0) return GGFV_OK;
    DeviceGuard g(ctx->device);
    const double dt_used = (ctx->dtype == GGFV_F64) ? dt : (double)(float)dt;
    GGFV_HIP(ctx, advance_steps(ctx, dt, nsteps));
    ctx->t += dt_used * (double)nsteps;
    ctx->steps += nsteps;
    ctx->last_dt = dt_used;
    return GGFV_OK;
}

int ggfv_step_adaptive(ggfv_ctx *ctx, double safety, long long nsteps, double *dt_log)
{
    if (!ctx) return GGFV_EINVAL;
    if (!(safety > 0.0) || !std::isfinite(safety))
        return fail(ctx, GGFV_EINVAL, "safety must be finite and > 0 (got %g)", safety);
    if (nsteps < 0) return fail(ctx, GGFV_EINVAL, "nsteps must be >= 0 (got %lld)", nsteps);
    if (!ctx->has_state || !ctx->has_tensor || !ctx->has_params)
        return fail(ctx, GGFV_ESTATE, "state, tensor and parameters must be set before stepping");
    if (nsteps == 0) return GGFV_OK;
    DeviceGuard g(ctx->device);
    if (!ctx->adapt && hipMalloc(reinterpret_cast<void **>(&ctx->adapt), sizeof(AdaptCtl)) != hipSuccess) {
        ctx->adapt = nullptr;
        return fail(ctx, GGFV_ENOMEM, "cannot allocate the adaptive-step control block");
    }
    GGFV_HIP(ctx, launch_adapt_init(ctx, ctx->adapt, ctx->t));
    AdaptArgs ad;
    ad.ctl = ctx->adapt;
    ad.dt_log = dt_log;
    ad.safety = safety;
    ad.twoD2 = 2.0 * ctx->prm.Delta2;
    const double idx = ctx->nx / ctx->lx, idy = ctx->ny / ctx->ly;
    ad.q = idx * idx + idy * idy;
    for (long long k = 0; k < nsteps; ++k) {
        ad.k = k;
        GGFV_HIP(ctx, launch_step_adaptive(ctx, ctx->state[ctx->cur], ctx->state[1 - ctx->cur], ad));
        ctx->cur ^= 1;
    }
    AdaptCtl host;
    GGFV_HIP(ctx, hipMemcpyAsync(&host, ctx->adapt, sizeof host, hipMemcpyDeviceToHost, ctx->stream));
    GGFV_HIP(ctx, hipStreamSynchronize(ctx->stream));
    ctx->t = host.t;
    ctx->steps += nsteps;
    ctx->last_dt = host.last_dt;
    return GGFV_OK;
}

int ggfv_front_diagnostics(ggfv_ctx *ctx, double theta_u, double theta_v, double *out)
{
    if (!ctx) return GGFV_EINVAL;
    if (!out) return fail(ctx, GGFV_EINVAL, "null output");
    if (!std::isfinite(theta_u) || !std::isfinite(theta_v))
        return fail(ctx, GGFV_EINVAL, "thresholds must be finite");
    if (!ctx->has_state) return fail(ctx, GGFV_ESTATE, "no state set");
    DeviceGuard g(ctx->device);
    const size_t n = 4 * (size_t)ctx->ny + 16;
    if (!ctx->front && hipMalloc(reinterpret_cast<void **>(&ctx->front), n * sizeof(double)) != hipSuccess) {
        ctx->front = nullptr;
        return fail(ctx, GGFV_ENOMEM, "cannot allocate the front-diagnostics buffer");
    }
    double *res = ctx->front + 4 * (size_t)ctx->ny;
    GGFV_HIP(ctx, launch_front_diagnostics(ctx, theta_u, theta_v, ctx->front, res));
    GGFV_HIP(ctx, hipMemcpyAsync(out, res, 11 * sizeof(double), hipMemcpyDeviceToHost, ctx->stream));
    GGFV_HIP(ctx, hipStreamSynchronize(ctx->stream));
    return GGFV_OK;
}

double ggfv_front_speed(double mass0, double mass1, double t0, double t1, double ly, double behind, double ahead)
{
    return (mass1 - mass0) / ((t1 - t0) * ly * (behind - ahead));
}

int ggfv_set_tuning(ggfv_ctx *ctx, const ggfv_tuning *tn)
{
    if (!ctx) return GGFV_EINVAL;
    if (!tn) return fail(ctx, GGFV_EINVAL, "null tuning");
    if (tn->rows_per_strip < 0) return fail(ctx, GGFV_EINVAL, "rows_per_strip must be >= 0");
    if (tn->threads != 0 && tn->threads != 64 && tn->threads != 128 && tn->threads != 256)
        return fail(ctx, GGFV_EINVAL, "threads must be 0, 64, 128 or 256 (got %d)", tn->threads);
    if (tn->fused_steps < 0 || tn->fused_steps > 4)
        return fail(ctx, GGFV_EINVAL, "fused_steps must be 0..4 (got %d)", tn->fused_steps);
    if (tn->lane_shift < 0 || tn->lane_shift > 2)
        return fail(ctx, GGFV_EINVAL, "lane_shift must be 0, 1 or 2 (got %d)", tn->lane_shift);
    if (tn->lane_shift == 2 && ctx->dtype == GGFV_F32C)
        return fail(ctx, GGFV_EINVAL, "wide lanes (lane_shift 2) are for FP64 and plain FP32 contexts");
    if (tn->fused_steps > 1 && tn->lane_shift == 0)
        return fail(ctx, GGFV_EINVAL, "fused_steps > 1 needs the lane-shift kernels (lane_shift 1 or 2)");
    ctx->rows_per_strip = tn->rows_per_strip;
    ctx->threads = tn->threads;
    ctx->fused_steps = tn->fused_steps < 1 ? 1 : tn->fused_steps;
    ctx->lane_shift = tn->lane_shift;
    return GGFV_OK;
}

int ggfv_get_tuning(const ggfv_ctx *ctx, ggfv_tuning *tn)
{
    if (!ctx || !tn) return GGFV_EINVAL;
    tn->rows_per_strip = ctx->rows_per_strip;
    tn->threads = ctx->threads;
    tn->fused_steps = ctx->fused_steps;
    tn->lane_shift = ctx->lane_shift;
    return GGFV_OK;
}

int ggfv_autotune(ggfv_ctx *ctx, double dt, int trial_steps, ggfv_tuning *best)
{
    if (!ctx) return GGFV_EINVAL;
    if (!best) return fail(ctx, GGFV_EINVAL, "null output");
    if (trial_steps < 1) return fail(ctx, GGFV_EINVAL, "trial_steps must be >= 1");
    if (!(dt > 0.0) || !std::isfinite(dt)) return fail(ctx, GGFV_EINVAL, "dt must be finite and > 0");
    if (!ctx->has_state || !ctx->has_tensor || !ctx->has_params)
        return fail(ctx, GGFV_ESTATE, "state, tensor and parameters must be set before tuning");
    DeviceGuard g(ctx->device);
    const size_t sb = ctx->nfields * ctx->plane * ctx->elem;
    void *save = nullptr;
    if (hipMalloc(&save, sb) != hipSuccess) return fail(ctx, GGFV_ENOMEM, "cannot allocate tuning backup");
    const int cur0 = ctx->cur;
    const double t0 = ctx->t, last0 = ctx->last_dt;
    const long long s0 = ctx->steps;
    const int rows0 = ctx->rows_per_strip, thr0 = ctx->threads, fus0 = ctx->fused_steps, lan0 = ctx->lane_shift;
    hipEvent_t e0 = nullptr, e1 = nullptr;
    int rc = GGFV_OK;
    float best_ms = 0.0f;
    ggfv_tuning bt{rows0, thr0, fus0, lan0};
    auto cleanup = [&]() {
        if (e0) (void)hipEventDestroy(e0);
        if (e1) (void)hipEventDestroy(e1);
        (void)hipFree(save);
    };
    if (hipMemcpyAsync(save, ctx->state[cur0], sb, hipMemcpyDeviceToDevice, ctx->stream) != hipSuccess ||
        hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess) {
        cleanup();
        return fail(ctx, GGFV_EHIP, "autotune setup failed");
    }
    // negative heights (lane-shift kernels only): strips that fill the resident
    // wave slots half a round, 1.5 and 2 rounds over (0 is the one-round fit)
    const int heights[13] = {0, 2, 4, 8, 16, 24, 32, 48, 64, 128, -1, -3, -4};
    const int widths[5] = {64, 128, 256, 0, -1};     // 0: lane-shift kernels; -1: wide lanes
    bool first = true;
    for (int K = 1; K <= 4 && rc == GGFV_OK; ++K)
        for (int wdt : widths)
            for (int h : heights) {
                const bool lanes = wdt <= 0;
                if (wdt < 0 && ctx->dtype == GGFV_F32C) continue;
                if (!lanes && K > 1) continue;                  // several steps per launch: lane-shift kernels
                if (h < 0) {
                    if (!lanes) continue;
                    ctx->lane_shift = wdt < 0 ? 2 : 1;           // the fit depends on the kernel
                    h = ggfv::lane_shift_fit_rows(ctx, K, -h);
                }
                if (h > ctx->ny) continue;
                if (K > 1 && h != 0 && h < 4 * K) continue;
                if (lanes && h != 0 && h < 8) continue;
                ctx->threads = lanes ? 64 : wdt;
                ctx->fused_steps = K;
                ctx->lane_shift = wdt < 0 ? 2 : lanes ? 1 : 0;
                ctx->rows_per_strip = h;
                const long long n = (long long)trial_steps * K;
                hipError_t e = advance_steps(ctx, dt, K);       // warm-up
                if (e == hipSuccess) e = hipEventRecord(e0, ctx->stream);
                if (e == hipSuccess) e = advance_steps(ctx, dt, n);
                if (e == hipSuccess) e = hipEventRecord(e1, ctx->stream);
                if (e == hipSuccess) e = hipEventSynchronize(e1);
                float ms = 0.0f;
                if (e == hipSuccess) e = hipEventElapsedTime(&ms, e0, e1);
                if (e != hipSuccess) {
                    rc = fail(ctx, GGFV_EHIP, "autotune trial failed: %s", hipGetErrorString(e));
                    break;
                }
                const float per_step = ms / (float)n;
                if (first || per_step < best_ms) {
                    best_ms = per_step;
                    bt.rows_per_strip = h;
                    bt.threads = ctx->threads;
                    bt.fused_steps = K;
                    bt.lane_shift = ctx->lane_shift;
                    first = false;
                }
            }
    // restore the state exactly as it was
    ctx->cur = cur0;
    if (hipMemcpyAsync(ctx->state[cur0], save, sb, hipMemcpyDeviceToDevice, ctx->stream) != hipSuccess ||
        hipStreamSynchronize(ctx->stream) != hipSuccess)
        rc = fail(ctx, GGFV_EHIP, "autotune restore failed");
    ctx->t = t0;
    ctx->steps = s0;
    ctx->last_dt = last0;
    cleanup();
    if (rc) {
        ctx->rows_per_strip = rows0;
        ctx->threads = thr0;
        ctx->fused_steps = fus0;
        ctx->lane_shift = lan0;
        return rc;
    }
    ctx->rows_per_strip = bt.rows_per_strip;
    ctx->threads = bt.threads;
    ctx->fused_steps = bt.fused_steps;
    ctx->lane_shift = bt.lane_shift;
    *best = bt;
    return GGFV_OK;
}

int ggfv_diagnostics(ggfv_ctx *ctx, ggfv_diag *out)
{
    if (!ctx) return GGFV_EINVAL;
    if (!out) return fail(ctx, GGFV_EINVAL, "null output");
    if (!ctx->has_state || !ctx->has_tensor) return fail(ctx, GGFV_ESTATE, "state and tensor must be set");
    DeviceGuard g(ctx->device);
    GGFV_HIP(ctx, launch_diagnostics(ctx, ctx->last_dt));
    double r[kDiagSlots];
    int rc = read_result(ctx, r, kDiagSlots);
    if (rc) return rc;
    const double dx = ctx->lx / ctx->nx, dy = ctx->ly / ctx->ny;
    out->t = ctx->t;
    out->steps = ctx->steps;
    for (int q = 0; q < 3; ++q) {
        out->mass[q] = dx * dy * r[q];
        out->vmin[q] = r[3 + q];
        out->vmax[q] = r[6 + q];
    }
    out->cfl = ctx->last_dt * r[9];
    out->nonfinite = (long long)r[10];
    if (out->nonfinite > 0 || out->cfl > 1.0)
        return fail(ctx, GGFV_EUNSTABLE, "unstable state: %lld non-finite values, cfl %.3g",
                    out->nonfinite, out->cfl);
    return GGFV_OK;
}

int ggfv_diagnostics_noalloc(int nx, int ny, double lx, double ly, int io_dtype, const void *u, const void *v,
                             const void *w, const void *a, const void *b, const void *c, double Delta2,
                             double dt, double *out, int device, void *hip_stream)
{
    if (nx < 1 || ny < 1) return fail(nullptr, GGFV_EINVAL, "grid must be at least 1x1 (got %dx%d)", nx, ny);
    if ((long long)nx * ny > (1LL << 34))
        return fail(nullptr, GGFV_EINVAL, "grid too large (%dx%d; at most 2^34 cells)", nx, ny);
    if (!(lx > 0.0) || !(ly > 0.0) || !std::isfinite(lx) || !std::isfinite(ly))
        return fail(nullptr, GGFV_EINVAL, "domain sides must be finite and > 0");
    if (!valid_io(io_dtype))
        return fail(nullptr, GGFV_EINVAL, "io_dtype must be GGFV_F32 or GGFV_F64 (got %d)", io_dtype);
    if (!u || !v || !w || !a || !b || !c || !out) return fail(nullptr, GGFV_EINVAL, "null array pointer");
    if (!(Delta2 >= 0.0) || !std::isfinite(Delta2) || !(dt >= 0.0) || !std::isfinite(dt))
        return fail(nullptr, GGFV_EINVAL, "Delta2 and dt must be finite and >= 0");
    int ndev = 0;
    hipError_t he = hipGetDeviceCount(&ndev);
    if (he != hipSuccess) return fail(nullptr, GGFV_EHIP, "hipGetDeviceCount failed: %s", hipGetErrorString(he));
    if (device < 0 || device >= ndev)
        return fail(nullptr, GGFV_EINVAL, "device %d out of range (%d devices)", device, ndev);
    DeviceGuard g(device);
    if (g.status != hipSuccess)
        return fail(nullptr, GGFV_EHIP, "hipSetDevice(%d) failed: %s", device, hipGetErrorString(g.status));
    double *parts = nullptr;
    he = noalloc_scratch(device, &parts);
    if (he != hipSuccess)
        return fail(nullptr, GGFV_EHIP, "no scratch address on device %d: %s", device, hipGetErrorString(he));
    he = launch_diagnostics_dense(nx, ny, lx, ly, io_dtype == GGFV_F64, u, v, w, a, b, c, Delta2, dt, parts, out,
                                  static_cast<hipStream_t>(hip_stream));
    if (he != hipSuccess) return fail(nullptr, GGFV_EHIP, "diagnostics launch failed: %s", hipGetErrorString(he));
    return GGFV_OK;
}

}  // extern "C"
