// ggfv_batch.hip -- ensembles of independent instances stepped together.
//
// Every instance is an ordinary context (own grid, tensor, parameters, state,
// dt).  One launch of the batched step kernel advances all of them by one step:
// the work items are the strips of all instances (instance i owns the items
// [prefix[i], prefix[i+1])), and each instance's step description (planes, sizes,
// coefficients, dt, strip height) is read from a device array.  Two description
// arrays alternate, because each step swaps every instance's input and output
// planes.  Runs of many steps are captured once into a HIP graph of
// `graph_steps` launches (an even number, so the planes are back in place after
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
    int threads = 64;
    int rows = 0;                  // 0: 16 rows unless the instance fixes its own
    int graph_steps = 50;
    // host images and device copies of the two description arrays and the prefix
    std::vector<unsigned char> hdesc[2];
    std::vector<int> hprefix;
    void *ddesc[2] = {nullptr, nullptr};
    int *dprefix = nullptr;
    size_t desc_cap = 0;
    int prefix_cap = 0;
    bool dirty = true;
    std::vector<int> cur_at_build;
    int items = 0;
    hipGraphExec_t exec = nullptr;
    int exec_steps = 0;
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
    b->exec_steps = 0;
}

// (Re)build both description arrays and the prefix for the instances' current
// planes; copies them to the device synchronously.
int build(ggfv_batch *b)
{
    bool same = !b->dirty && (int)b->cur_at_build.size() == b->n;
    for (int i = 0; same && i < b->n; ++i) same = b->cur_at_build[i] == b->inst[i]->cur;
    if (same) return GGFV_OK;
    const size_t sz = step_args_bytes(b->dtype);
    const int cols = step_columns_per_group(b->dtype, b->threads);
    for (int p = 0; p < 2; ++p) b->hdesc[p].assign(sz * b->n, 0);
    b->hprefix.assign(b->n + 1, 0);
    b->cur_at_build.assign(b->n, 0);
    long long items = 0;
    for (int i = 0; i < b->n; ++i) {
        ggfv_ctx *c = b->inst[i];
        const int rows = rows_of(b, c);
        const double dt = b->dtype == GGFV_F64 ? b->dt[i] : (double)(float)b->dt[i];
        fill_step_args(c, c->state[c->cur], c->state[1 - c->cur], dt, rows, &b->hdesc[0][sz * i]);
        fill_step_args(c, c->state[1 - c->cur], c->state[c->cur], dt, rows, &b->hdesc[1][sz * i]);
        const long long strips = (long long)((c->nx + cols - 1) / cols) * ((c->ny + rows - 1) / rows);
        b->hprefix[i] = (int)items;
        items += strips;
        b->cur_at_build[i] = c->cur;
    }
    if (items > (1LL << 30)) return bfail(b, GGFV_EINVAL, "too many work items (%lld)", items);
    b->hprefix[b->n] = (int)items;
    b->items = (int)items;
    if (b->desc_cap < sz * b->n || b->prefix_cap < b->n + 1) {
        (void)hipStreamSynchronize(b->stream);
        drop_graph(b);
        for (int p = 0; p < 2; ++p)
            if (b->ddesc[p]) (void)hipFree(b->ddesc[p]);
        if (b->dprefix) (void)hipFree(b->dprefix);
        b->ddesc[0] = b->ddesc[1] = nullptr;
        b->dprefix = nullptr;
        if (hipMalloc(&b->ddesc[0], sz * b->n) != hipSuccess || hipMalloc(&b->ddesc[1], sz * b->n) != hipSuccess ||
            hipMalloc(reinterpret_cast<void **>(&b->dprefix), sizeof(int) * (b->n + 1)) != hipSuccess)
            return bfail(b, GGFV_ENOMEM, "cannot allocate batch descriptions");
        b->desc_cap = sz * b->n;
        b->prefix_cap = b->n + 1;
    }
    // the previous graph may still be reading the descriptions
    GGFV_BHIP(b, hipStreamSynchronize(b->stream));
    for (int p = 0; p < 2; ++p)
        GGFV_BHIP(b, hipMemcpy(b->ddesc[p], b->hdesc[p].data(), sz * b->n, hipMemcpyHostToDevice));
    GGFV_BHIP(b, hipMemcpy(b->dprefix, b->hprefix.data(), sizeof(int) * (b->n + 1), hipMemcpyHostToDevice));
    b->dirty = false;
    return GGFV_OK;
}

BatchLaunch launch_of(const ggfv_batch *b, int parity)
{
    BatchLaunch L;
    L.dtype = b->dtype;
    L.threads = b->threads;
    L.n = b->n;
    L.items = b->items;
    L.desc = b->ddesc[parity & 1];
    L.prefix = b->dprefix;
    return L;
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

// Record nsteps batched launches (parity alternates from 0) on the stream.
int enqueue(ggfv_batch *b, long long nsteps)
{
    for (long long s = 0; s < nsteps; ++s) GGFV_BHIP(b, launch_step_batch(launch_of(b, (int)(s & 1)), b->stream));
    return GGFV_OK;
}

void advance(ggfv_batch *b, long long nsteps)
{
    for (int i = 0; i < b->n; ++i) {
        ggfv_ctx *c = b->inst[i];
        const double dt = b->dtype == GGFV_F64 ? b->dt[i] : (double)(float)b->dt[i];
        if (nsteps & 1) c->cur ^= 1;
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
        if (hipStreamCreateWithFlags(&b->stream, hipStreamNonBlocking) != hipSuccess) {
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
    b->graph_steps = graph_steps + (graph_steps & 1);   // even: planes return in place
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
    long long done = 0;
    const int G = b->graph_steps;
    if (G > 0 && nsteps >= G) {
        if (!b->exec || b->exec_steps != G) {
            drop_graph(b);
            hipGraph_t graph = nullptr;
            GGFV_BHIP(b, hipStreamBeginCapture(b->stream, hipStreamCaptureModeThreadLocal));
            int erc = enqueue(b, G);
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
            b->exec_steps = G;
        }
        for (; done + G <= nsteps; done += G) GGFV_BHIP(b, hipGraphLaunch(b->exec, b->stream));
    }
    if ((rc = enqueue(b, nsteps - done))) return rc;
    advance(b, nsteps);
    if (nsteps & 1) b->dirty = true;     // planes swapped: descriptions rebuilt next run
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
    const int thr0 = b->threads, rows0 = b->rows;
    hipEvent_t e0 = nullptr, e1 = nullptr;
    (void)hipEventCreate(&e0);
    (void)hipEventCreate(&e1);
    float best_ms = -1.0f;
    int bt = thr0, br = rows0;
    const int widths[2] = {64, 256};
    const int heights[5] = {4, 8, 16, 32, 64};
    for (int w : widths)
        for (int h : heights) {
            b->threads = w;
            b->rows = h;
            b->dirty = true;
            drop_graph(b);
            if ((rc = build(b))) break;
            // even counts keep the planes in place
            if ((rc = enqueue(b, 2))) break;
            (void)hipEventRecord(e0, b->stream);
            const int steps = trial_steps + (trial_steps & 1);
            if ((rc = enqueue(b, steps))) break;
            (void)hipEventRecord(e1, b->stream);
            (void)hipEventSynchronize(e1);
            float ms = 0.0f;
            (void)hipEventElapsedTime(&ms, e0, e1);
            if (best_ms < 0.0f || ms < best_ms) {
                best_ms = ms;
                bt = w;
                br = h;
            }
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
    b->dirty = true;
    drop_graph(b);
    if (rc) return rc;
    *best_threads = bt;
    *best_rows = br;
    return GGFV_OK;
}

const char *ggfv_batch_last_error(const ggfv_batch *b) { return b ? b->err.c_str() : g_batch_create_error.c_str(); }

}  // extern "C"
