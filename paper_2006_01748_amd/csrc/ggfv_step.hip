// ggfv_step.hip -- the explicit finite-volume step of eq. (3) for gfx950.
//
// One launch advances the whole grid by one forward-Euler step (Section 2): every
// cell reads the old level of u, v, w and the tensor a, b, c, and writes the new
// level of u, v, w into the other state buffer.
//
// Work decomposition.  A workgroup of 256 threads (four wave64s side by side)
// owns a vertical strip of TXW = 256*CPL columns and `rows` rows.  Each thread
// owns CPL adjacent columns and marches up its strip one row at a time
// (a streaming, "2.5D" sweep): the newest row of every field is loaded once from
// HBM with coalesced CPL-wide vector loads, staged in small LDS row rings for the
// x-neighbours, and the y-neighbours are carried in registers from the previous
// rows.  The y-face fluxes are carried too: the north face of row j is the south
// face of row j+1, so each face flux is evaluated once and both cells see
// identical bits (exact telescoping, hence exact conservation up to the sum).
// The x-face fluxes are evaluated by both neighbouring threads from identical
// operands in identical order, so they agree bit for bit as well.
//
// Boundaries (Section 2, Neumann): faces on the domain boundary carry zero flux;
// the tangential differences in the first/last row and column take the boundary
// cell itself as the missing neighbour.  Both are realised by clamping row and
// column indices into the grid and zeroing boundary faces explicitly.
//
// Arithmetic order per cell (the same order as any FP64 reference must use for
// bitwise agreement; no contraction into FMA, the library is built with
// -ffp-contract=off):
//   ty = (W(i,j+1) - W(i,j-1))*hy,  tx = (W(i+1,j) - W(i-1,j))*hx
//   FX(i+1/2) = 0.5*(a_l + a_r)*((W_r - W_l)*idx) + 0.5*(b_l*ty_l + b_r*ty_r)
//   FY(j+1/2) = 0.5*(c_l + c_r)*((W_r - W_l)*idy) + 0.5*(b_l*tx_l + b_r*tx_r)
//   GX, GY    = (1 - 0.5*(U_l + U_r))*((V_r - V_l)*idx or idy)
//   divW = (FX_e - FX_w)*idx + (FY_n - FY_s)*idy, divV alike
//   U' = U + dt*(U*(1-U) - (delta1*U)*W)
//   V' = V + dt*((rho2*V)*(1-V) + Delta2*divV)
//   W' = W + dt*((rho3*V - delta3*W) + divW)
// For the compensated FP32 state the increment dt*f is added to x = hi + lo as
// s = hi + (dt*f + lo) with an error-free two-sum, which keeps the part of the
// increment that falls below half an FP32 ulp of hi.
//
// XCD-aware order: workgroups are dealt round-robin to the eight XCDs, so the
// linear workgroup id is remapped so that each XCD receives one contiguous band of
// strips; horizontally adjacent strips (which re-read each other's edge columns)
// then share one L2.

#include <cstring>

#include "ggfv_step_common.hpp"

namespace ggfv {
namespace {

// Values of one row that a thread needs: its own CPL columns of every field.
template <typename T, bool COMP, int CPL>
struct Row {
    T W[CPL], U[CPL], V[CPL], a[CPL], b[CPL], c[CPL];
    T Ulo[COMP ? CPL : 1], Vlo[COMP ? CPL : 1], Wlo[COMP ? CPL : 1];
    // halo column value (only meaningful in the two halo threads)
    T hW, hU, hV, ha, hb;
};

// Load row `jr` (already clamped into [0, ny)) for the thread's columns starting
// at `col` (clamped so the vector stays inside the padded row), plus the halo
// column `hcol` when hcol >= 0.
template <typename T, bool COMP, int CPL>
__device__ __forceinline__ void load_row(const StepArgs<T> &A, int jr, int col, int hcol,
                                         Row<T, COMP, CPL> &r)
{
    const size_t base = (size_t)jr * A.pitch;
    load_vec<T, CPL>(A.w + base + col, r.W);
    load_vec<T, CPL>(A.u + base + col, r.U);
    load_vec<T, CPL>(A.v + base + col, r.V);
    load_vec<T, CPL>(A.a + base + col, r.a);
    load_vec<T, CPL>(A.b + base + col, r.b);
    load_vec<T, CPL>(A.c + base + col, r.c);
    if constexpr (COMP) {
        load_vec<T, CPL>(A.ulo + base + col, r.Ulo);
        load_vec<T, CPL>(A.vlo + base + col, r.Vlo);
        load_vec<T, CPL>(A.wlo + base + col, r.Wlo);
    }
    if (hcol >= 0) {
        r.hW = A.w[base + hcol];
        r.hU = A.u[base + hcol];
        r.hV = A.v[base + hcol];
        r.ha = A.a[base + hcol];
        r.hb = A.b[base + hcol];
    }
}

// One workgroup's strip (sx, sy): columns [sx*TXW, (sx+1)*TXW), rows
// [sy*rows, (sy+1)*rows), one step from A's input planes to its output planes.
// With TRACK the thread also returns in *umax the largest |1 - u| over the new
// u values it wrote (u = hi + lo in FP64 for the compensated state).
template <typename T, bool COMP, int CPL, int NT, bool TRACK = false>
__device__ __forceinline__ void step_strip(const StepArgs<T> &A, const int sx, const int sy,
                                          double *umax = nullptr)
{
    constexpr int TXW = NT * CPL;          // owned columns per workgroup
    constexpr int LW = TXW + 2 * CPL;      // LDS row: CPL pad, TXW owned, CPL pad
    __shared__ __align__(16) T sW[4][LW];  // W rows j-1, j, j+1 (+1 being filled)
    __shared__ __align__(16) T sU[2][LW];
    __shared__ __align__(16) T sV[2][LW];
    __shared__ __align__(16) T sA[2][LW];
    __shared__ __align__(16) T sB[2][LW];

    const int t = threadIdx.x;
    const int nx = A.nx, ny = A.ny;
    const int i0 = sx * TXW;
    const int j0 = sy * A.rows;
    const int j1 = min(ny, j0 + A.rows);
    const int js = j0 > 0 ? j0 - 1 : j0;   // first row swept (warm-up row for FY_s)

    // Own columns i0 + t*CPL .. +CPL-1; the vector load address is clamped into
    // the padded row (values beyond nx are never used as neighbours).
    const int cbase = i0 + t * CPL;
    const int lcol = min(cbase, A.pitch - CPL);
    // Halo columns: thread 0 loads i0-1, thread NT-1 loads i0+TXW (when inside).
    int hcol = -1;
    if (t == 0 && i0 > 0) hcol = i0 - 1;
    if (t == NT - 1 && i0 + TXW < nx) hcol = i0 + TXW;
    const int hpos = (t == 0) ? CPL - 1 : TXW + CPL;

    auto clampj = [&](int j) { return j < 0 ? 0 : (j >= ny ? ny - 1 : j); };
    // LDS position of a neighbour column, with mirrored (clamped) index.
    auto posof = [&](int i) {
        const int ic = i < 0 ? 0 : (i >= nx ? nx - 1 : i);
        return ic - i0 + CPL;
    };

    Row<T, COMP, CPL> cur, nxt, pre;
    T Wprev[CPL];
    {
        Row<T, COMP, CPL> rp;
        load_row<T, COMP, CPL>(A, clampj(js - 1), lcol, hcol, rp);
#pragma unroll
        for (int k = 0; k < CPL; ++k) Wprev[k] = rp.W[k];
        lds_store_vec<T, CPL>(&sW[(js - 1) & 3][t * CPL + CPL], rp.W);
        if (hcol >= 0) sW[(js - 1) & 3][hpos] = rp.hW;
    }
    load_row<T, COMP, CPL>(A, clampj(js), lcol, hcol, cur);
    lds_store_vec<T, CPL>(&sW[js & 3][t * CPL + CPL], cur.W);
    if (hcol >= 0) sW[js & 3][hpos] = cur.hW;
    load_row<T, COMP, CPL>(A, clampj(js + 1), lcol, hcol, nxt);

    const T half = T(0.5), one = T(1);
    T FYs[CPL], GYs[CPL];
#pragma unroll
    for (int k = 0; k < CPL; ++k) { FYs[k] = T(0); GYs[k] = T(0); }
    double mu = 0.0;

    for (int jj = js; jj < j1; ++jj) {
        // Publish W(jj+1) and U, V, a, b (jj) for the x-neighbours.
        {
            const int s4 = (jj + 1) & 3, s2 = jj & 1;
            lds_store_vec<T, CPL>(&sW[s4][t * CPL + CPL], nxt.W);
            lds_store_vec<T, CPL>(&sU[s2][t * CPL + CPL], cur.U);
            lds_store_vec<T, CPL>(&sV[s2][t * CPL + CPL], cur.V);
            lds_store_vec<T, CPL>(&sA[s2][t * CPL + CPL], cur.a);
            lds_store_vec<T, CPL>(&sB[s2][t * CPL + CPL], cur.b);
            if (hcol >= 0) {
                sW[s4][hpos] = nxt.hW;
                sU[s2][hpos] = cur.hU;
                sV[s2][hpos] = cur.hV;
                sA[s2][hpos] = cur.ha;
                sB[s2][hpos] = cur.hb;
            }
        }
        __syncthreads();
        // Prefetch row jj+2 while this row is computed.
        if (jj + 2 <= j1) load_row<T, COMP, CPL>(A, clampj(jj + 2), lcol, hcol, pre);

        const T *Wm = sW[(jj - 1) & 3];
        const T *W0 = sW[jj & 3];
        const T *Wp = sW[(jj + 1) & 3];
        const T *U0 = sU[jj & 1];
        const T *V0 = sV[jj & 1];
        const T *A0 = sA[jj & 1];
        const T *B0 = sB[jj & 1];
        const bool has_n = (jj + 1 < ny);
        const bool upd = (jj >= j0);

        T ou[CPL], ov[CPL], ow[CPL], oul[CPL], ovl[CPL], owl[CPL];
#pragma unroll
        for (int k = 0; k < CPL; ++k) {
            const int i = cbase + k;
            const int pl = posof(i - 1), pr = posof(i + 1);
            const T Wc = cur.W[k], Wn = nxt.W[k], Ws = Wprev[k];
            const T WL = W0[pl], WR = W0[pr];
            const T WLn = Wp[pl], WRn = Wp[pr];
            const T WLs = Wm[pl], WRs = Wm[pr];
            const T Uc = cur.U[k], Vc = cur.V[k];
            const T UL = U0[pl], UR = U0[pr], VL = V0[pl], VR = V0[pr];
            const T ac = cur.a[k], aL = A0[pl], aR = A0[pr];
            const T bc = cur.b[k], bL = B0[pl], bR = B0[pr];

            const T tyc = (Wn - Ws) * A.hy;
            const T tyL = (WLn - WLs) * A.hy;
            const T tyR = (WRn - WRs) * A.hy;
            const T txc = (WR - WL) * A.hx;
            const T txn = (WRn - WLn) * A.hx;

            const bool has_e = (i + 1 < nx), has_w = (i > 0);
            const T FXe = has_e ? madd<T, COMP>(half * (ac + aR), (WR - Wc) * A.idx, half * (bc * tyc + bR * tyR))
                                : T(0);
            const T FXw = has_w ? madd<T, COMP>(half * (aL + ac), (Wc - WL) * A.idx, half * (bL * tyL + bc * tyc))
                                : T(0);
            const T FYn = has_n ? madd<T, COMP>(half * (cur.c[k] + nxt.c[k]), (Wn - Wc) * A.idy,
                                                half * (bc * txc + nxt.b[k] * txn))
                                : T(0);
            const T GXe = has_e ? madd<T, COMP>(-half, Uc + UR, one) * ((VR - Vc) * A.idx) : T(0);
            const T GXw = has_w ? madd<T, COMP>(-half, UL + Uc, one) * ((Vc - VL) * A.idx) : T(0);
            const T GYn = has_n ? madd<T, COMP>(-half, Uc + nxt.U[k], one) * ((nxt.V[k] - Vc) * A.idy) : T(0);

            const T divW = (FXe - FXw) * A.idx + (FYn - FYs[k]) * A.idy;
            const T divV = (GXe - GXw) * A.idx + (GYn - GYs[k]) * A.idy;
            const T fu = madd<T, COMP>(-(A.d1 * Uc), Wc, Uc * (one - Uc));
            const T fv = madd<T, COMP>(A.D2, divV, (A.r2 * Vc) * (one - Vc));
            const T fw = madd<T, COMP>(A.r3, Vc, -(A.d3 * Wc)) + divW;
            const bool inside = (i < nx);
            if constexpr (COMP) {
                T h, l;
                comp_add(Uc, cur.Ulo[k], A.dt * fu, h, l);
                ou[k] = inside ? h : T(0);
                oul[k] = inside ? l : T(0);
                comp_add(Vc, cur.Vlo[k], A.dt * fv, h, l);
                ov[k] = inside ? h : T(0);
                ovl[k] = inside ? l : T(0);
                comp_add(Wc, cur.Wlo[k], A.dt * fw, h, l);
                ow[k] = inside ? h : T(0);
                owl[k] = inside ? l : T(0);
            } else {
                ou[k] = inside ? madd<T, COMP>(A.dt, fu, Uc) : T(0);
                ov[k] = inside ? madd<T, COMP>(A.dt, fv, Vc) : T(0);
                ow[k] = inside ? madd<T, COMP>(A.dt, fw, Wc) : T(0);
            }
            FYs[k] = FYn;
            GYs[k] = GYn;
        }
        if constexpr (TRACK) {
            if (upd) {
#pragma unroll
                for (int k = 0; k < CPL; ++k) {
                    const double un = COMP ? double(ou[k]) + double(oul[k]) : double(ou[k]);
                    if (cbase + k < nx) mu = fmax(mu, fabs(1.0 - un));
                }
            }
        }
        if (upd && cbase < A.pitch) {
            const size_t o = (size_t)jj * A.pitch + cbase;
            store_vec<T, CPL>(A.un + o, ou);
            store_vec<T, CPL>(A.vn + o, ov);
            store_vec<T, CPL>(A.wn + o, ow);
            if constexpr (COMP) {
                store_vec<T, CPL>(A.unlo + o, oul);
                store_vec<T, CPL>(A.vnlo + o, ovl);
                store_vec<T, CPL>(A.wnlo + o, owl);
            }
        }
#pragma unroll
        for (int k = 0; k < CPL; ++k) Wprev[k] = cur.W[k];
        cur = nxt;
        nxt = pre;
    }
    if constexpr (TRACK) *umax = mu;
}

template <typename T, bool COMP, int CPL, int NT>
__global__ __launch_bounds__(NT) void step_kernel(StepArgs<T> A)
{
    const int nbx = gridDim.x;
    const int lid = xcd_local_id(blockIdx.x + nbx * blockIdx.y, gridDim.x * gridDim.y);
    step_strip<T, COMP, CPL, NT>(A, lid % nbx, lid / nbx);
}

// Adaptive form (Section 2: a new step size after every iteration): the step
// size is computed here, from the control block, as
//   dt_k = safety / max(tensor_max, (2 Delta2 * max|1 - u^k|) * (idx^2 + idy^2))
// in FP64 (max|1 - u^k| was reduced by the previous step, or by the run's
// initial reduction), and the workgroups reduce max|1 - u^{k+1}| of their output
// into the next slot.  Workgroup 0 advances the time, logs dt_k and clears slot
// (k+2) % 3, the one step k+1 accumulates into (step k-1 read it last; nothing
// touches it during step k).
template <typename T, bool COMP, int CPL, int NT>
__global__ __launch_bounds__(NT) void step_adaptive_kernel(StepArgs<T> A, AdaptArgs D)
{
    __shared__ double red[NT / 64];
    const double M = __longlong_as_double((long long)D.ctl->m[D.k % 3]);
    const double cv = (D.twoD2 * M) * D.q;
    double cmax = D.ctl->tensor_max;
    if (cv > cmax) cmax = cv;
    const double dt = D.safety / cmax;
    StepArgs<T> B = A;
    B.dt = T(dt);
    const int nbx = gridDim.x;
    const int bid = blockIdx.x + nbx * blockIdx.y;
    const int lid = xcd_local_id(bid, gridDim.x * gridDim.y);
    double mu = 0.0;
    step_strip<T, COMP, CPL, NT, true>(B, lid % nbx, lid / nbx, &mu);
    // workgroup max of |1 - u|, then one atomic per workgroup
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) mu = fmax(mu, __shfl_xor(mu, off, 64));
    const int wave = threadIdx.x / 64, lane = threadIdx.x % 64;
    if (lane == 0) red[wave] = mu;
    __syncthreads();
    if (threadIdx.x == 0) {
        double m = red[0];
#pragma unroll
        for (int w = 1; w < NT / 64; ++w) m = fmax(m, red[w]);
        atomicMax(&D.ctl->m[(D.k + 1) % 3], (unsigned long long)__double_as_longlong(m));
        if (bid == 0) {
            D.ctl->t = D.ctl->t + dt;
            D.ctl->last_dt = dt;
            D.ctl->m[(D.k + 2) % 3] = 0ull;
            if (D.dt_log) D.dt_log[D.k] = dt;
        }
    }
}

// Batched form: work item k of all instances' strips; instance i owns items
// [prefix[i], prefix[i+1]) and its own step description D[i] (sizes, planes,
// parameters, dt and strip height).
template <typename T, bool COMP, int CPL, int NT>
__global__ __launch_bounds__(NT) void step_batch_kernel(const StepArgs<T> *__restrict__ D,
                                                        const int *__restrict__ prefix, int n)
{
    const int lid = xcd_local_id(blockIdx.x, gridDim.x);
    int lo = 0, hi = n;                    // prefix[lo] <= lid < prefix[hi]
    while (hi - lo > 1) {
        const int mid = (lo + hi) >> 1;
        if (prefix[mid] <= lid) lo = mid;
        else hi = mid;
    }
    const StepArgs<T> A = D[lo];
    constexpr int TXW = NT * CPL;
    const int nbx = (A.nx + TXW - 1) / TXW;
    const int local = lid - prefix[lo];
    step_strip<T, COMP, CPL, NT>(A, local % nbx, local / nbx);
}

// Default launch shape.  Large grids (>= 4M cells) use 256-thread workgroups
// and about four workgroups per CU (256 CUs) with strips of >= 8 rows; smaller
// grids use one-wave workgroups and shorter strips so that ~2048 workgroups
// still cover the chip.  A context may fix either choice (ggfv_set_tuning).
int pick_threads(const ggfv_ctx *ctx)
{
    if (ctx->threads == 64 || ctx->threads == 128 || ctx->threads == 256) return ctx->threads;
    return (long)ctx->nx * ctx->ny >= (1L << 22) ? 256 : 64;
}

int pick_rows(const ggfv_ctx *ctx, int nbx, int threads)
{
    int rows = ctx->rows_per_strip;
    if (rows <= 0) {
        const long target = threads == 64 ? 2048 : 1024;
        const int floor_rows = threads == 64 ? 4 : 8;
        long per = ((long)ctx->ny * nbx + target - 1) / target;
        rows = (int)(per < floor_rows ? floor_rows : per);
    }
    return rows > ctx->ny ? ctx->ny : rows;
}

template <typename T, bool COMP, int CPL, int NT>
hipError_t launch_typed(ggfv_ctx *ctx, const void *in_base, void *out_base, double dt)
{
    constexpr int TXW = NT * CPL;
    const int nbx = (ctx->nx + TXW - 1) / TXW;
    const int rows = pick_rows(ctx, nbx, NT);
    const StepArgs<T> A = make_args<T>(ctx, in_base, out_base, dt, rows);
    const int nby = (ctx->ny + rows - 1) / rows;
    hipLaunchKernelGGL((step_kernel<T, COMP, CPL, NT>), dim3(nbx, nby), dim3(NT), 0, ctx->stream, A);
    return hipGetLastError();
}

template <typename T, bool COMP, int CPL>
hipError_t launch_width(ggfv_ctx *ctx, const void *in, void *out, double dt)
{
    const int w = pick_threads(ctx);
    if (w == 64) return launch_typed<T, COMP, CPL, 64>(ctx, in, out, dt);
    if (w == 128) return launch_typed<T, COMP, CPL, 128>(ctx, in, out, dt);
    return launch_typed<T, COMP, CPL, 256>(ctx, in, out, dt);
}

template <typename T, bool COMP, int CPL, int NT>
hipError_t launch_batch_typed(const BatchLaunch &b, hipStream_t stream)
{
    hipLaunchKernelGGL((step_batch_kernel<T, COMP, CPL, NT>), dim3(b.items), dim3(NT), 0, stream,
                       static_cast<const StepArgs<T> *>(b.desc), b.prefix, b.n);
    return hipGetLastError();
}

}  // namespace

hipError_t launch_step_planes(ggfv_ctx *ctx, const void *in, void *out, double dt)
{
    switch (ctx->dtype) {
    case GGFV_F64: return launch_width<double, false, 1>(ctx, in, out, dt);
    case GGFV_F32: return launch_width<float, false, 2>(ctx, in, out, dt);
    case GGFV_F32C: return launch_width<float, true, 2>(ctx, in, out, dt);
    default: return hipErrorInvalidValue;
    }
}

size_t step_args_bytes(int dtype) { return dtype == GGFV_F64 ? sizeof(StepArgs<double>) : sizeof(StepArgs<float>); }

int step_columns_per_group(int dtype, int threads) { return threads * (dtype == GGFV_F64 ? 1 : 2); }

void fill_step_args(const ggfv_ctx *ctx, const void *in, void *out, double dt, int rows, void *dst)
{
    if (ctx->dtype == GGFV_F64) {
        StepArgs<double> A = make_args<double>(ctx, in, out, dt, rows);
        memcpy(dst, &A, sizeof A);
    } else {
        StepArgs<float> A = make_args<float>(ctx, in, out, dt, rows);
        memcpy(dst, &A, sizeof A);
    }
}

hipError_t launch_step_batch(const BatchLaunch &b, hipStream_t stream)
{
    const bool narrow = b.threads == 64;
    switch (b.dtype) {
    case GGFV_F64:
        return narrow ? launch_batch_typed<double, false, 1, 64>(b, stream)
                      : launch_batch_typed<double, false, 1, 256>(b, stream);
    case GGFV_F32:
        return narrow ? launch_batch_typed<float, false, 2, 64>(b, stream)
                      : launch_batch_typed<float, false, 2, 256>(b, stream);
    case GGFV_F32C:
        return narrow ? launch_batch_typed<float, true, 2, 64>(b, stream)
                      : launch_batch_typed<float, true, 2, 256>(b, stream);
    default: return hipErrorInvalidValue;
    }
}

namespace {
template <typename T, bool COMP, int CPL, int NT>
hipError_t launch_adaptive_typed(ggfv_ctx *ctx, const void *in, void *out, const AdaptArgs &ad)
{
    constexpr int TXW = NT * CPL;
    const int nbx = (ctx->nx + TXW - 1) / TXW;
    const int rows = pick_rows(ctx, nbx, NT);
    const int nby = (ctx->ny + rows - 1) / rows;
    const StepArgs<T> A = make_args<T>(ctx, in, out, 0.0, rows);
    hipLaunchKernelGGL((step_adaptive_kernel<T, COMP, CPL, NT>), dim3(nbx, nby), dim3(NT), 0, ctx->stream, A, ad);
    return hipGetLastError();
}

template <typename T, bool COMP, int CPL>
hipError_t launch_adaptive_width(ggfv_ctx *ctx, const void *in, void *out, const AdaptArgs &ad)
{
    const int w = pick_threads(ctx);
    if (w == 64) return launch_adaptive_typed<T, COMP, CPL, 64>(ctx, in, out, ad);
    if (w == 128) return launch_adaptive_typed<T, COMP, CPL, 128>(ctx, in, out, ad);
    return launch_adaptive_typed<T, COMP, CPL, 256>(ctx, in, out, ad);
}
}  // namespace

hipError_t launch_step_adaptive(ggfv_ctx *ctx, const void *in, void *out, const AdaptArgs &ad)
{
    switch (ctx->dtype) {
    case GGFV_F64: return launch_adaptive_width<double, false, 1>(ctx, in, out, ad);
    case GGFV_F32: return launch_adaptive_width<float, false, 2>(ctx, in, out, ad);
    case GGFV_F32C: return launch_adaptive_width<float, true, 2>(ctx, in, out, ad);
    default: return hipErrorInvalidValue;
    }
}

hipError_t launch_step(ggfv_ctx *ctx, double dt)
{
    return launch_step_planes(ctx, ctx->state[ctx->cur], ctx->state[1 - ctx->cur], dt);
}

hipError_t advance_steps(ggfv_ctx *ctx, double dt, long long n)
{
    const int K = ctx->fused_steps > 1 ? ctx->fused_steps : 1;
    hipError_t e = hipSuccess;
    if (ctx->lane_shift) {
        for (; n >= K && e == hipSuccess; n -= K) {
            e = launch_step_fused_dpp(ctx, ctx->state[ctx->cur], ctx->state[1 - ctx->cur], dt, K);
            ctx->cur ^= 1;
        }
        for (; n > 0 && e == hipSuccess; --n) {
            e = launch_step_fused_dpp(ctx, ctx->state[ctx->cur], ctx->state[1 - ctx->cur], dt, 1);
            ctx->cur ^= 1;
        }
        return e;
    }
    for (; n > 0 && e == hipSuccess; --n) {
        e = launch_step(ctx, dt);
        ctx->cur ^= 1;
    }
    return e;
}

}  // namespace ggfv
