// ggfv_internal.hpp -- context layout and kernel launchers shared by the HIP
// sources of the library.  Not part of the public ABI (include/ggfv.h).
#pragma once

#include <hip/hip_runtime.h>

#include <cstddef>
#include <string>

#include "ggfv.h"

namespace ggfv {

// Every row of every internal field is padded to a multiple of this many values
// so that wide vector loads of a row never straddle into the next row.
constexpr int kRowAlign = 64;

// Workgroup size of the streaming step kernel (four wave64s side by side).
constexpr int kStepThreads = 256;

inline int round_up(int x, int m) { return (x + m - 1) / m * m; }

// Scratch layout (bytes): reduction partials of up to kMaxPartialBlocks blocks,
// a small result area and an integer counter.
constexpr int kReduceThreads = 256;
constexpr int kMaxPartialBlocks = 1024;
constexpr int kDiagSlots = 12;    // per-block partials of the diagnostics reduction

}  // namespace ggfv

namespace ggfv {
// Adaptive stepping (ggfv_step_adaptive): device-resident control block.  m[]
// holds max |1-u| of a state as the bits of a non-negative double (so an
// unsigned 64-bit atomic max orders them); step k reads m[k % 3], accumulates
// the max of its output into m[(k+1) % 3] and clears m[(k+2) % 3].
struct AdaptCtl {
    unsigned long long m[3];
    double t;              // simulated time
    double tensor_max;     // max over cells of 2(a idx^2 + c idy^2) + |b| idx idy (>= 0)
    double last_dt;
    double pad[2];
};
}  // namespace ggfv

struct ggfv_ctx {
    int nx = 0, ny = 0, pitch = 0;
    double lx = 1.0, ly = 1.0;
    int dtype = 0;
    int device = 0;
    hipStream_t stream = nullptr;

    size_t plane = 0;        // pitch * ny values per field
    size_t elem = 0;         // bytes per stored value (4 or 8)
    int nfields = 0;         // stored state fields: 3, or 6 for the compensated state
    void *state[2] = {nullptr, nullptr};
    int cur = 0;             // which of state[0], state[1] holds the current level
    void *tensor = nullptr;  // a, b, c planes
    void *scratch = nullptr; // reduction partials and counters
    size_t scratch_bytes = 0;
    void *staging = nullptr; // dense host<->device staging area (3 * nx*ny doubles)
    size_t staging_bytes = 0;

    ggfv_params prm{};
    bool has_state = false, has_tensor = false, has_params = false;
    double t = 0.0;
    long long steps = 0;
    double last_dt = 0.0;
    int cus = 0;             // compute units of the device
    int rows_per_strip = 0;  // 0: chosen per launch
    int threads = 0;         // workgroup width of the single-step kernel: 64, 128, 256, or 0 (by grid size)
    int fused_steps = 4;     // time steps per launch (1..4; above 1 only with the lane-shift kernels)
    int lane_shift = 2;      // 0: single-step kernel; 1: one-wave register/lane-shift kernels
                             // (ggfv_fused_dpp.hpp); 2: the same with wide lanes (set per dtype at create)
    ggfv::AdaptCtl *adapt = nullptr;   // adaptive-step control block (lazily allocated)
    double *front = nullptr;           // front diagnostics: 4 * ny per-row values + 16 results (lazily)

    void *adj = nullptr;     // adjoint buffers (see ggfv_adjoint.hip), allocated on first use
    size_t adj_bytes = 0;

    std::string err;
};

namespace ggfv {

// Pointers to the planes of one stored state level (lo planes are null unless
// the state is compensated).
template <typename T>
struct StatePlanes {
    T *u, *v, *w, *ulo, *vlo, *wlo;
};

// ---- kernel launchers (each returns the hipError_t of its launch) ----------

// One step of eq. (3) from state[cur] to state[1 - cur].
hipError_t launch_step(ggfv_ctx *ctx, double dt);
// One step from the stored state at `in` (nfields planes) to `out`.
hipError_t launch_step_planes(ggfv_ctx *ctx, const void *in, void *out, double dt);
// K (1..4) steps per launch with rows in registers and lane shifts (ggfv_fused_dpp.hpp;
// FP32 in ggfv_fused_dpp.hip, FP64 in ggfv_fused_dpp_f64.hip).
hipError_t launch_step_fused_dpp(ggfv_ctx *ctx, const void *in, void *out, double dt, int K);
// Strip height at which the lane-shift kernel of depth K fills the device's
// resident wave slots `rounds2 / 2` times over (rounds2 = 1: half a round).
int lane_shift_fit_rows(const ggfv_ctx *ctx, int K, int rounds2);
// n steps of the context's current state with its tuning (fused launches plus
// single steps for the remainder); flips ctx->cur once per launch.
hipError_t advance_steps(ggfv_ctx *ctx, double dt, long long n);

// ---- batched step (all instances of an ensemble advance one step per launch) --
struct AdaptArgs {
    AdaptCtl *ctl = nullptr;
    double *dt_log = nullptr;      // device, one entry per step of the run, or null
    long long k = 0;               // step index within the run
    double safety = 0.0;
    double twoD2 = 0.0;            // 2 * Delta2
    double q = 0.0;                // idx^2 + idy^2
};
hipError_t launch_step_adaptive(ggfv_ctx *ctx, const void *in, void *out, const AdaptArgs &ad);
// Reset the control block (time t0) and reduce the tensor term and max |1-u| of
// the context's current state into it.
hipError_t launch_adapt_init(ggfv_ctx *ctx, AdaptCtl *ctl, double t0);
// Front diagnostics of the current state: per-row values into rows (4 * ny
// doubles), the 11 results into out (device).
hipError_t launch_front_diagnostics(ggfv_ctx *ctx, double theta_u, double theta_v, double *rows, double *out);

struct BatchLaunch {
    int dtype = 0;
    int threads = 64;        // workgroup width of the single-step kernel: 64 or 256
    int fused = 1;           // steps per launch of the lane-shift kernel (launch_step_batch_dpp)
    int n = 0;               // instances
    int items = 0;           // total work items (strips) = prefix[n]
    const void *desc = nullptr;   // device array of n step descriptions
    const int *prefix = nullptr;  // device array of n+1 work-item offsets
};
hipError_t launch_step_batch(const BatchLaunch &b, hipStream_t stream);
// The ensemble form of the lane-shift kernels: b.fused (1..4) steps per launch
// (ggfv_fused_dpp.hip); output columns per workgroup for a precision and depth.
hipError_t launch_step_batch_dpp(const BatchLaunch &b, hipStream_t stream);
int lane_shift_columns_per_group(int dtype, int K);
// The FP64 instances of the lane-shift kernels live in their own source
// (ggfv_fused_dpp_f64.hip, built with the default instruction schedule); the
// three entry points above dispatch FP64 work to these.
int lane_shift_fit_rows_f64(const ggfv_ctx *ctx, int K, int rounds2, bool wide);
hipError_t launch_step_fused_dpp_f64(ggfv_ctx *ctx, const void *in, void *out, double dt, int K, bool wide);
hipError_t launch_step_batch_dpp_f64(const BatchLaunch &b, hipStream_t stream);
// Size of one step description, columns per workgroup, and filling one
// description for a context (input planes, output planes, dt, strip height).
size_t step_args_bytes(int dtype);
int step_columns_per_group(int dtype, int threads);
void fill_step_args(const ggfv_ctx *ctx, const void *in, void *out, double dt, int rows, void *dst);

// ---- adjoint (ggfv_adjoint.hip) ---------------------------------------------
// Buffers of the adjoint, allocated on first use: state planes for a single
// adjoint step (3), adjoint state ping-pong (2 x 3), tensor gradient (3), and one
// slot of five partial sums per adjoint block.
int adjoint_blocks(const ggfv_ctx *ctx);
// lam_out = (dF/dx)^T lam_in at state x (three planes u, v, w of the stored
// precision); g (three planes) += (dF/dA)^T lam_in; per-block partial sums of
// (dF/dp)^T lam_in are added into slots[block][5].
hipError_t launch_adjoint_step(ggfv_ctx *ctx, const void *x, const void *lam_in, void *lam_out,
                               void *g, double *slots, double dt);
// slots[nblocks][5] -> out[5] (fixed order).
hipError_t launch_slots_reduce(ggfv_ctx *ctx, const double *slots, int nblocks, double *out);
// zero `count` doubles (or floats) on the stream (a fill kernel, not a memset).
hipError_t launch_zero(ggfv_ctx *ctx, void *p, size_t bytes);
// Chain rule of the tensor map from dense io arrays to dense io arrays.
hipError_t launch_eig_backward(ggfv_ctx *ctx, const void *l1, const void *l2, const void *th,
                               const void *ga, const void *gb, const void *gc, void *g1,
                               void *g2, void *gt, bool f64);

// Dense io array (float or double, nx*ny) -> padded storage planes (and lo
// planes for the compensated state).  src_is_f64 selects the io type.
hipError_t launch_pack3(ggfv_ctx *ctx, const void *s0, const void *s1, const void *s2,
                        bool src_is_f64, void *dst_base, int nplanes_dst, bool split_lo);
// Padded storage -> dense io arrays.
hipError_t launch_unpack3(ggfv_ctx *ctx, const void *src_base, bool has_lo, void *d0,
                          void *d1, void *d2, bool dst_is_f64);
// (lam1, lam2, theta) dense io arrays -> tensor planes a, b, c.
hipError_t launch_tensor_eig(ggfv_ctx *ctx, const void *l1, const void *l2,
                             const void *th, bool src_is_f64);
// Count of cells whose stored tensor is not SPD -> *(unsigned long long*)scratch.
hipError_t launch_spd_count(ggfv_ctx *ctx);
// max over cells of lambda_max(A) -> *(double*)scratch (FP64).
hipError_t launch_lambda_max(ggfv_ctx *ctx);
// Diagnostics partials and final reduction -> kDiagSlots doubles at scratch.
hipError_t launch_diagnostics(ggfv_ctx *ctx, double dt);
// Diagnostics of dense nx*ny arrays (FP64 or FP32), no context: partials into
// `parts` (kMaxPartialBlocks * kDiagSlots doubles), the 11 results into `out`
// (device), masses times dx*dy and the cfl maximum times dt.
hipError_t launch_diagnostics_dense(int nx, int ny, double lx, double ly, bool f64, const void *u,
                                    const void *v, const void *w, const void *a, const void *b,
                                    const void *c, double Delta2, double dt, double *parts, double *out,
                                    hipStream_t stream);
// Device address of the library's static diagnostics scratch on `device`
// (which must be current); looked up once per device.
hipError_t noalloc_scratch(int device, double **out);

}  // namespace ggfv
