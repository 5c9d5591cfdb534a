// ggfv_batch.hip -- ensembles of independent instances stepped together.
//
// Every instance is an ordinary context (own grid, tensor, parameters, state,
// dt).  One launch of a batched kernel advances all of them: the single-step
// kernel by one step, the lane-shift kernel by `fused` steps.  The work items
// are the strips of all instances (instance i owns the items [prefix[i],
// prefix[i+1]) of the kernel's own work table), and each instance's step
// description (planes, sizes, coefficients, dt, strip height) is read from a
// device array.  Two description arrays alternate, because each launch swaps
// every instance's input and output planes.  Runs are captured once into a HIP
// graph of an even number of launches (so the planes are back in place after
// every replay) and replayed.  Only kernel nodes are captured.

#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <new>
#include <string>
#include <vector>

#include "ggfv_internal.hpp"

using namespace ggfv;

struct ggfv_batch {
    int n = 0;
    int dtype = 0;
    int device = 0;
    hipStream_t stream = nullptr;
    bool own_stream = false;
    std::vector<ggfv_ctx *> inst;
    std::vector<double> dt;
    int threads = 64;              // width of the single-step kernel
    int fused = 1;                 // 1: single-step kernel; 2..4: lane-shift kernel, steps per launch
    int rows = 0;                  // 0: 16 rows unless the instance fixes its own
    int graph_steps = 50;
    // host images and device copies of the two description arrays and of the
    // work tables of the single-step (index 0) and lane-shift (index 1) kernels
    std::vector<unsigned char> hdesc[2];
    std::vector<int> hprefix[2];
    void *ddesc[2] = {nullptr, nullptr};
    int *dprefix = nullptr;        // 2 * (n + 1) ints: both work tables
    size_t desc_cap = 0;
    int prefix_cap = 0;
    bool dirty = true;
    std::vector<int> cur_at_build;
    int items[2] = {0, 0};
    hipGraphExec_t exec = nullptr;
    int exec_launches = 0;         // launches in the graph
    int exec_fused = 0;            // steps per launch in the graph
    std::string err;
};

namespace {

thread_local std::string g_batch_create_error;

int bfail(ggfv_batch *b, int code, const char *fmt, ...) __attribute__((format(printf, 3, 4)));

int bfail(ggfv_batch *b, int code, const char *fmt, ...)
{
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    if (b)
        b->err = buf;
    else
        g_batch_create_error = buf;
    return code;
}

#define GGFV_BHIP(b, call)                                                                   \
    do {                                                                                     \
        hipError_t e_ = (call);                                                              \
        if (e_ != hipSuccess)                                                                \
            return bfail((b), GGFV_EHIP, "%s failed: %s", #call, hipGetErrorString(e_));     \
    } while (0)

int rows_of(const ggfv_batch *b, const ggfv_ctx *c)
{
    int r = c->rows_per_strip > 0 ? c->rows_per_strip : (b->rows > 0 ? b->rows : 16);
    return r > c->ny ? c->ny : r;
}

void drop_graph(ggfv_batch *b)
{
    if (b->exec) (void)hipGraphExecDestroy(b->exec);
    b->exec = nullptr;
    b->exec_launches = 0;
    b->exec_fused = 0;
}

// (Re)build both description arrays and the prefix for the instances' current
// planes; copies them to the device synchronously.
int build(ggfv_batch *b)
{
    bool same = !b->dirty && (int)b->cur_at_build.size() == b->n;
    for (int i = 0; same && i < b->n; ++i) same = b->cur_at_build[i] == b->inst[i]->cur;
    if (same) return GGFV_OK;
    const size_t sz = step_args_bytes(b->dtype);
    // columns per workgroup of the single-step and of the lane-shift kernel
    const int cols[2] = {step_columns_per_group(b->dtype, b->threads),
                         lane_shift_columns_per_group(b->dtype, b->fused)};
    for (int p = 0; p < 2; ++p) b->hdesc[p].assign(sz * b->n, 0);
    for (int k = 0; k < 2; ++k) b->hprefix[k].assign(b->n + 1, 0);
    b->cur_at_build.assign(b->n, 0);
    long long items[2] = {0, 0};
    for (int i = 0; i < b->n; ++i) {
        ggfv_ctx *c = b->inst[i];
        const int rows = rows_of(b, c);
        const double dt = b->dtype == GGFV_F64 ? b->dt[i] : (double)(float)b->dt[i];
        fill_step_args(c, c->state[c->cur], c->state[1 - c->cur], dt, rows, &b->hdesc[0][sz * i]);
        fill_step_args(c, c->state[1 - c->cur], c->state[c->cur], dt, rows, &b->hdesc[1][sz * i]);
        for (int k = 0; k < 2; ++k) {
            const long long strips = (long long)((c->nx + cols[k] - 1) / cols[k]) * ((c->ny + rows - 1) / rows);
            b->hprefix[k][i] = (int)items[k];
            items[k] += strips;
        }
        b->cur_at_build[i] = c->cur;
    }
    for (int k = 0; k < 2; ++k) {
        if (items[k] > (1LL << 30)) return bfail(b, GGFV_EINVAL, "too many work items (%lld)", items[k]);
        b->hprefix[k][b->n] = (int)items[k];
        b->items[k] = (int)items[k];
    }
    if (b->desc_cap < sz * b->n || b->prefix_cap < b->n + 1) {
        (void)hipStreamSynchronize(b->stream);
        drop_graph(b);
        for (int p = 0; p < 2; ++p)
            if (b->ddesc[p]) (void)hipFree(b->ddesc[p]);
        if (b->dprefix) (void)hipFree(b->dprefix);
        b->ddesc[0] = b->ddesc[1] = nullptr;
        b->dprefix = nullptr;
        if (hipMalloc(&b->ddesc[0], sz * b->n) != hipSuccess || hipMalloc(&b->ddesc[1], sz * b->n) != hipSuccess ||
            hipMalloc(reinterpret_cast<void **>(&b->dprefix), 2 * sizeof(int) * (b->n + 1)) != hipSuccess)
            return bfail(b, GGFV_ENOMEM, "cannot allocate batch descriptions");
        b->desc_cap = sz * b->n;
        b->prefix_cap = b->n + 1;
    }
    // the previous graph may still be reading the descriptions
    GGFV_BHIP(b, hipStreamSynchronize(b->stream));
    for (int p = 0; p < 2; ++p)
        GGFV_BHIP(b, hipMemcpy(b->ddesc[p], b->hdesc[p].data(), sz * b->n, hipMemcpyHostToDevice));
    for (int k = 0; k < 2; ++k)
        GGFV_BHIP(b, hipMemcpy(b->dprefix + k * (b->n + 1), b->hprefix[k].data(), sizeof(int) * (b->n + 1),
                               hipMemcpyHostToDevice));
    b->dirty = false;
    return GGFV_OK;
}

// One launch: the lane-shift kernel (lanes) or the single-step kernel, reading
// description array `parity`.
hipError_t launch_one(const ggfv_batch *b, bool lanes, int parity)
{
    BatchLaunch L;
    L.dtype = b->dtype;
    L.threads = b->threads;
    L.fused = b->fused;
    L.n = b->n;
    L.items = b->items[lanes ? 1 : 0];
    L.desc = b->ddesc[parity & 1];
    L.prefix = b->dprefix + (lanes ? b->n + 1 : 0);
    return lanes ? launch_step_batch_dpp(L, b->stream) : launch_step_batch(L, b->stream);
}

int ready(ggfv_batch *b)
{
    for (int i = 0; i < b->n; ++i) {
        const ggfv_ctx *c = b->inst[i];
        if (!c->has_state || !c->has_tensor || !c->has_params)
            return bfail(b, GGFV_ESTATE, "instance %d lacks state, tensor or parameters", i);
        if (!(b->dt[i] > 0.0)) return bfail(b, GGFV_ESTATE, "instance %d has no dt", i);
    }
    return GGFV_OK;
}

// Record launches for nsteps steps on the stream: fused launches while at least
// `fused` steps remain, then single steps.  Parity alternates per launch from
// `parity`; the number of launches is added to *launches.
int enqueue(ggfv_batch *b, long long nsteps, long long *launches)
{
    const int K = b->fused;
    long long nl = *launches;
    if (K > 1)
        for (; nsteps >= K; nsteps -= K, ++nl) GGFV_BHIP(b, launch_one(b, true, (int)(nl & 1)));
    for (; nsteps > 0; --nsteps, ++nl) GGFV_BHIP(b, launch_one(b, false, (int)(nl & 1)));
    *launches = nl;
    return GGFV_OK;
}

// nsteps steps done in `launches` launches (each swapped the planes once).
void advance(ggfv_batch *b, long long nsteps, long long launches)
{
    for (int i = 0; i < b->n; ++i) {
        ggfv_ctx *c = b->inst[i];
        const double dt = b->dtype == GGFV_F64 ? b->dt[i] : (double)(float)b->dt[i];
        if (launches & 1) c->cur ^= 1;
        c->t += dt * (double)nsteps;
        c->steps += nsteps;
        c->last_dt = dt;
    }
}

}  // namespace

extern "C" {

int ggfv_batch_create(ggfv_batch **out, int n, const int *nx, const int *ny, double lx, double ly, int dtype,
                      int device, void *hip_stream)
{
    if (!out) return bfail(nullptr, GGFV_EINVAL, "null output pointer");
    *out = nullptr;
    if (n < 1 || !nx || !ny) return bfail(nullptr, GGFV_EINVAL, "need n >= 1 and size arrays");
    if (dtype != GGFV_F32 && dtype != GGFV_F64 && dtype != GGFV_F32C)
        return bfail(nullptr, GGFV_EINVAL, "unknown dtype %d", dtype);
    ggfv_batch *b = new (std::nothrow) ggfv_batch;
    if (!b) return bfail(nullptr, GGFV_ENOMEM, "out of host memory");
    b->n = n;
    b->dtype = dtype;
    b->device = device;
    int prev = -1;
    (void)hipGetDevice(&prev);
    if (hipSetDevice(device) != hipSuccess) {
        delete b;
        return bfail(nullptr, GGFV_EHIP, "hipSetDevice(%d) failed", device);
    }
    if (hip_stream) {
        b->stream = static_cast<hipStream_t>(hip_stream);
    } else {
        // a blocking stream: its work is ordered with the null stream's (the
        // default stream of most callers) both ways, so device arrays that the
        // caller wrote or will read there need no extra synchronization
        if (hipStreamCreateWithFlags(&b->stream, hipStreamDefault) != hipSuccess) {
            delete b;
            if (prev >= 0) (void)hipSetDevice(prev);
            return bfail(nullptr, GGFV_EHIP, "cannot create the batch stream");
        }
        b->own_stream = true;
    }
    b->inst.assign(n, nullptr);
    b->dt.assign(n, 0.0);
    for (int i = 0; i < n; ++i) {
        int rc = ggfv_create(&b->inst[i], nx[i], ny[i], lx, ly, dtype, device, b->stream);
        if (rc != GGFV_OK) {
            char why[600];
            snprintf(why, sizeof why, "instance %d (%dx%d): %s", i, nx[i], ny[i], ggfv_last_error(nullptr));
            ggfv_batch_destroy(b);
            if (prev >= 0) (void)hipSetDevice(prev);
            return bfail(nullptr, rc, "%s", why);
        }
    }
    if (prev >= 0) (void)hipSetDevice(prev);
    *out = b;
    return GGFV_OK;
}

void ggfv_batch_destroy(ggfv_batch *b)
{
    if (!b) return;
    int prev = -1;
    (void)hipGetDevice(&prev);
    (void)hipSetDevice(b->device);
    if (b->stream) (void)hipStreamSynchronize(b->stream);
    drop_graph(b);
    for (int p = 0; p < 2; ++p)
        if (b->ddesc[p]) (void)hipFree(b->ddesc[p]);
    if (b->dprefix) (void)hipFree(b->dprefix);
    for (ggfv_ctx *c : b->inst) ggfv_destroy(c);
    if (b->own_stream) (void)hipStreamDestroy(b->stream);
    if (prev >= 0) (void)hipSetDevice(prev);
    delete b;
}

ggfv_ctx *ggfv_batch_instance(ggfv_batch *b, int i)
{
    if (!b || i < 0 || i >= b->n) return nullptr;
    b->dirty = true;   // the caller may change this instance's tensor, parameters or tuning
    return b->inst[i];
}

int ggfv_batch_set_dt(ggfv_batch *b, int i, double dt)
{
    if (!b) return GGFV_EINVAL;
    if (i < 0 || i >= b->n) return bfail(b, GGFV_EINVAL, "instance %d out of range", i);
    if (!(dt > 0.0) || !std::isfinite(dt)) return bfail(b, GGFV_EINVAL, "dt must be finite and > 0");
    b->dt[i] = dt;
    b->dirty = true;
    return GGFV_OK;
}

int ggfv_batch_set(ggfv_batch *b, int i, const ggfv_params *params, double dt, const void *a, const void *bb,
                   const void *c, const void *u, const void *v, const void *w, int where, int io_dtype)
{
    if (!b) return GGFV_EINVAL;
    if (i < 0 || i >= b->n) return bfail(b, GGFV_EINVAL, "instance %d out of range", i);
    if (!(dt > 0.0) || !std::isfinite(dt)) return bfail(b, GGFV_EINVAL, "dt must be finite and > 0");
    ggfv_ctx *ctx = b->inst[i];
    b->dirty = true;
    int rc = ggfv_set_params(ctx, params);
    if (rc == GGFV_OK) rc = ggfv_set_tensor(ctx, a, bb, c, where, io_dtype);
    if (rc == GGFV_OK) rc = ggfv_set_state(ctx, u, v, w, where, io_dtype);
    if (rc != GGFV_OK) return bfail(b, rc, "instance %d: %s", i, ggfv_last_error(ctx));
    return ggfv_batch_set_dt(b, i, dt);
}

int ggfv_batch_get_state(ggfv_batch *b, int i, void *u, void *v, void *w, int where, int io_dtype)
{
    if (!b) return GGFV_EINVAL;
    if (i < 0 || i >= b->n) return bfail(b, GGFV_EINVAL, "instance %d out of range", i);
    const int rc = ggfv_get_state(b->inst[i], u, v, w, where, io_dtype);
    if (rc != GGFV_OK) return bfail(b, rc, "instance %d: %s", i, ggfv_last_error(b->inst[i]));
    return GGFV_OK;
}

int ggfv_batch_set_tuning(ggfv_batch *b, int threads, int rows_per_strip, int graph_steps)
{
    if (!b) return GGFV_EINVAL;
    if (threads != 64 && threads != 256) return bfail(b, GGFV_EINVAL, "threads must be 64 or 256");
    if (rows_per_strip < 0 || graph_steps < 0) return bfail(b, GGFV_EINVAL, "negative tuning value");
    if (threads != b->threads || rows_per_strip != b->rows) {
        b->dirty = true;
        drop_graph(b);
    }
    b->threads = threads;
    b->rows = rows_per_strip;
    b->graph_steps = graph_steps;
    drop_graph(b);
    return GGFV_OK;
}

int ggfv_batch_set_fused_steps(ggfv_batch *b, int fused_steps)
{
    if (!b) return GGFV_EINVAL;
    if (fused_steps < 1 || fused_steps > 4) return bfail(b, GGFV_EINVAL, "fused_steps must be 1..4");
    if (fused_steps != b->fused) {
        b->dirty = true;
        drop_graph(b);
    }
    b->fused = fused_steps;
    return GGFV_OK;
}

int ggfv_batch_get_tuning(const ggfv_batch *b, int *threads, int *rows_per_strip, int *graph_steps,
                          int *fused_steps)
{
    if (!b) return GGFV_EINVAL;
    if (threads) *threads = b->threads;
    if (rows_per_strip) *rows_per_strip = b->rows;
    if (graph_steps) *graph_steps = b->graph_steps;
    if (fused_steps) *fused_steps = b->fused;
    return GGFV_OK;
}

int ggfv_batch_run(ggfv_batch *b, long long nsteps)
{
    if (!b) return GGFV_EINVAL;
    if (nsteps < 0) return bfail(b, GGFV_EINVAL, "nsteps must be >= 0");
    if (nsteps == 0) return GGFV_OK;
    int rc = ready(b);
    if (rc) return rc;
    int prev = -1;
    (void)hipGetDevice(&prev);
    (void)hipSetDevice(b->device);
    const bool was_dirty = b->dirty;
    if ((rc = build(b))) return rc;
    if (was_dirty) drop_graph(b);
    long long done = 0, launches = 0;
    const int K = b->fused;
    // the graph: an even number of launches of K steps covering about graph_steps steps
    long long GL = b->graph_steps / K;
    GL += GL & 1;
    if (b->graph_steps > 0 && GL > 0 && nsteps >= GL * K) {
        if (!b->exec || b->exec_launches != GL || b->exec_fused != K) {
            drop_graph(b);
            hipGraph_t graph = nullptr;
            GGFV_BHIP(b, hipStreamBeginCapture(b->stream, hipStreamCaptureModeThreadLocal));
            long long nl = 0;
            int erc = enqueue(b, GL * K, &nl);
            hipError_t ee = hipStreamEndCapture(b->stream, &graph);
            if (erc) {
                if (graph) (void)hipGraphDestroy(graph);
                return erc;
            }
            if (ee != hipSuccess) return bfail(b, GGFV_EHIP, "graph capture failed: %s", hipGetErrorString(ee));
            hipError_t ie = hipGraphInstantiate(&b->exec, graph, nullptr, nullptr, 0);
            (void)hipGraphDestroy(graph);
            if (ie != hipSuccess) {
                b->exec = nullptr;
                return bfail(b, GGFV_EHIP, "graph instantiation failed: %s", hipGetErrorString(ie));
            }
            b->exec_launches = (int)GL;
            b->exec_fused = K;
        }
        for (; done + GL * K <= nsteps; done += GL * K, launches += GL)
            GGFV_BHIP(b, hipGraphLaunch(b->exec, b->stream));
    }
    if ((rc = enqueue(b, nsteps - done, &launches))) return rc;
    advance(b, nsteps, launches);
    if (launches & 1) b->dirty = true;     // planes swapped: descriptions rebuilt next run
    if (prev >= 0) (void)hipSetDevice(prev);
    return GGFV_OK;
}

int ggfv_batch_autotune(ggfv_batch *b, int trial_steps, int *best_threads, int *best_rows)
{
    if (!b) return GGFV_EINVAL;
    if (trial_steps < 2 || !best_threads || !best_rows) return bfail(b, GGFV_EINVAL, "bad autotune arguments");
    int rc = ready(b);
    if (rc) return rc;
    (void)hipSetDevice(b->device);
    // keep every instance's state, time and step count
    std::vector<void *> save(b->n, nullptr);
    std::vector<int> cur0(b->n);
    std::vector<double> t0(b->n), last0(b->n);
    std::vector<long long> s0(b->n);
    for (int i = 0; i < b->n; ++i) {
        ggfv_ctx *c = b->inst[i];
        const size_t sb = c->nfields * c->plane * c->elem;
        if (hipMalloc(&save[i], sb) != hipSuccess) {
            for (void *p : save)
                if (p) (void)hipFree(p);
            return bfail(b, GGFV_ENOMEM, "cannot allocate autotune backup");
        }
        (void)hipMemcpyAsync(save[i], c->state[c->cur], sb, hipMemcpyDeviceToDevice, b->stream);
        cur0[i] = c->cur;
        t0[i] = c->t;
        s0[i] = c->steps;
        last0[i] = c->last_dt;
    }
    const int thr0 = b->threads, rows0 = b->rows, fus0 = b->fused;
    hipEvent_t e0 = nullptr, e1 = nullptr;
    (void)hipEventCreate(&e0);
    (void)hipEventCreate(&e1);
    float best_ms = -1.0f;
    int bt = thr0, br = rows0, bk = fus0;
    // candidates: the single-step kernel at widths 64 and 256 (K = 1) and the
    // lane-shift kernel at K = 2..4, each over the strip heights
    const int kinds[5][2] = {{1, 64}, {1, 256}, {2, 64}, {3, 64}, {4, 64}};
    const int heights[5] = {4, 8, 16, 32, 64};
    for (const auto &kd : kinds) {
        for (int h : heights) {
            b->fused = kd[0];
            b->threads = kd[1];
            b->rows = h;
            b->dirty = true;
            drop_graph(b);
            if ((rc = build(b))) break;
            long long nl = 0;
            // warm-up, then an even number of launches keeps the planes in place
            if ((rc = enqueue(b, 2LL * b->fused, &nl))) break;
            (void)hipEventRecord(e0, b->stream);
            const long long lt = 2 * ((trial_steps + 2 * b->fused - 1) / (2 * b->fused));
            nl = 0;
            if ((rc = enqueue(b, lt * b->fused, &nl))) break;
            (void)hipEventRecord(e1, b->stream);
            (void)hipEventSynchronize(e1);
            float ms = 0.0f;
            (void)hipEventElapsedTime(&ms, e0, e1);
            const float per_step = ms / (float)(lt * b->fused);
            if (best_ms < 0.0f || per_step < best_ms) {
                best_ms = per_step;
                bt = kd[1];
                br = h;
                bk = kd[0];
            }
        }
        if (rc) break;
    }
    for (int i = 0; i < b->n; ++i) {
        ggfv_ctx *c = b->inst[i];
        c->cur = cur0[i];
        (void)hipMemcpyAsync(c->state[c->cur], save[i], c->nfields * c->plane * c->elem, hipMemcpyDeviceToDevice,
                             b->stream);
        c->t = t0[i];
        c->steps = s0[i];
        c->last_dt = last0[i];
    }
    (void)hipStreamSynchronize(b->stream);
    for (void *p : save) (void)hipFree(p);
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    b->threads = rc ? thr0 : bt;
    b->rows = rc ? rows0 : br;
    b->fused = rc ? fus0 : bk;
    b->dirty = true;
    drop_graph(b);
    if (rc) return rc;
    *best_threads = bt;
    *best_rows = br;
    return GGFV_OK;
}

const char *ggfv_batch_last_error(const ggfv_batch *b) { return b ? b->err.c_str() : g_batch_create_error.c_str(); }

}  // extern "C"
