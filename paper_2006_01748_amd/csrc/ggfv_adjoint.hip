// ggfv_adjoint.hip -- the discrete adjoint of one step of eq. (3) and the chain
// rule of the tensor map, for gradients of a loss of the final state with respect
// to the initial state, the reaction parameters and the per-cell tensor.
//
// With F the forward step x^k -> x^{k+1} (dt fixed) and lam' = dL/dx^{k+1}, one
// adjoint step computes, for every cell m,
//   lam(m)   = ((dF/dx)^T lam')(m)
//   g_A(m)  += ((dF/d(a,b,c))^T lam')(m)
//   g_p     += (dF/dp)^T lam'    (p = delta1, rho2, Delta2, rho3, delta3)
// in gather form: each lane owns a cell of the row being swept and collects the
// contributions of every face flux that reads a value of that cell.  Writing s_f for the loss
// sensitivity of a face flux,
//   x-face (l, l+1): s = dt*idx*(lamW_l - lamW_r),  sv = dt*Delta2*idx*(lamV_l - lamV_r)
//   y-face (l, l+1): the same with idy,
// and S_x(i, j) = s(i-1|i) + s(i|i+1) (the sum over the cell's two x-faces, absent
// faces contributing nothing), the contributions to cell m = (i, j) are
//   lamW += s_w*0.5(a_{i-1}+a_i)idx - s_e*0.5(a_i+a_{i+1})idx  (+ y alike with c)
//         + 0.5*hy*[ b(i,j-1) S_x(i,j-1) - b(i,j+1) S_x(i,j+1) ]  (rows that exist)
//         + 0.5*hy*b(i,j) S_x(i,j) * ([j == ny-1] - [j == 0])     (mirrored rows)
//         + the same across x with hx, S_y
//   g_a  += s_w*0.5(W_i - W_{i-1})idx + s_e*0.5(W_{i+1} - W_i)idx,   g_c alike in y
//   g_b  += 0.5*ty(i,j) S_x(i,j) + 0.5*tx(i,j) S_y(i,j)
//   lamV += sv_w*mob_w*idx - sv_e*mob_e*idx (+ y) + lamV(1 + dt rho2 (1-2V)) + dt rho3 lamW
//   lamU += -0.5*sv_w*(V_i - V_{i-1})idx - 0.5*sv_e*(V_{i+1} - V_i)idx (+ y)
//           + lamU(1 + dt(1 - 2U - delta1 W))
// and lamW also gains lamW(1 - dt delta3) - dt delta1 U lamU.
// The mirrored-row terms are the transpose of the boundary rule of the forward
// step (a tangential difference in the first/last row uses the boundary cell
// twice).
//
// Memory: reads x^k (3), lam' (3), a, b, c (3), g (3) and writes lam (3), g (3):
// 18 values per cell-update, each read once per strip (plus a halo row above
// and below the strip and a halo column on each side).  The five scalar partial
// sums are folded per workgroup in a fixed order and added into that
// workgroup's own slot (no atomics), so repeated sweeps give identical bits.

#include <cmath>

#include "ggfv_dpp.hpp"
#include "ggfv_step_common.hpp"

namespace ggfv {
namespace {

constexpr int kAdjCols = 62;      // output columns of a one-wave strip (64 lanes, one halo lane each side)
// Bytes of one adjoint step's arrays above which they no longer fit the
// last-level cache (256 MB on MI355X): streaming stores, taller strips.
constexpr size_t kAdjCacheBytes = size_t(256) << 20;

template <typename T>
struct AdjArgs {
    const T *u, *v, *w;         // state x^k
    const T *lu1, *lv1, *lw1;   // lam^{k+1}
    T *lu, *lv, *lw;            // lam^k
    T *ga, *gb, *gc;            // accumulated tensor gradient
    const T *a, *b, *c;
    double *slots;              // [nblocks][5]
    int nx, ny, pitch;
    T idx, idy, hx, hy, dt;
    T d1, r2, D2, r3, d3;
};

// Streaming sweep: one wave per workgroup owns a strip of 62 columns (lane l
// holds column x0 - 1 + l; lanes 0 and 63 only supply neighbour values) and
// `rows` rows, and marches up it.  At the row-j iteration the lanes hold rows
// j and j+1 of the fields read at y-neighbours (lam_w', lam_v', w, u, v, c, b)
// and row j of the rest (a, lam_u', g); x-neighbours come through DPP lane
// shifts.  Every face quantity is evaluated once, by the cell west of the
// x-face (and handed east by a shift) or south of the y-face (and carried in
// registers to the next row): the face sensitivities of lam_w' and lam_v', the
// face coefficients, the mobility, the differences of w and v, and b times the
// face-sensitivity sums of a row.  The expressions and their operands are those
// of the per-cell formulas above, so lam and g do not depend on the strips.
// OFF32: every plane spans less than 4 GiB, so a cell's byte offset from its
// plane's base fits 32 bits and one offset register serves every field (the
// bases stay scalar).  NT: the step's arrays exceed the last-level cache, so
// the outputs are written with streaming stores (nothing reads them again in
// this step); on cache-resident grids cached stores measured faster.
template <typename T, bool OFF32, bool NT>
__global__ __launch_bounds__(64) void adjoint_kernel(AdjArgs<T> A, int rows, int nsy)
{
    const int lid = xcd_local_id(blockIdx.x, gridDim.x);
    const int sx = lid / nsy, sy = lid - sx * nsy;
    const int lane = threadIdx.x;
    const int nx = A.nx, ny = A.ny;
    const int i = sx * kAdjCols - 1 + lane;
    const int ic = min(max(i, 0), nx - 1);
    const bool out_lane = lane >= 1 && lane <= kAdjCols && i < nx;
    const bool hw = i > 0, he = i + 1 < nx;
    const int j0 = sy * rows, j1 = min(j0 + rows, ny);
    const size_t P = A.pitch;
    const T zero = T(0), half = T(0.5), one = T(1), two = T(2);
    const T dtx = A.dt * A.idx, dty = A.dt * A.idy;
    const T dvx = A.dt * A.D2 * A.idx, dvy = A.dt * A.D2 * A.idy;
    auto at = [&](const T *p, int r) -> const T * {
        if constexpr (OFF32)
            return reinterpret_cast<const T *>(reinterpret_cast<const char *>(p) +
                                               ((unsigned)r * (unsigned)P + (unsigned)ic) * (unsigned)sizeof(T));
        else
            return p + ((size_t)r * P + ic);
    };
    auto ld = [&](const T *p, int r) { return *at(p, r); };
    auto mut = [&](T *p, int r) { return const_cast<T *>(at(p, r)); };

    // east-face sensitivity of lam_w' in a row and the row's sum over both x-faces
    auto xfaces = [&](T L, T &sxw, T &sxe) {
        const T Le = from_right(L);
        const T F = dtx * (L - Le);
        const T Fw = from_left(F);
        sxw = hw ? Fw : zero;
        sxe = he ? F : zero;
    };

    // rows j0-1 (clamped; its faces are masked off at j0 = 0) and j0
    const int jm = max(j0 - 1, 0);
    const T Lm = ld(A.lw1, jm), LVm = ld(A.lv1, jm), Wm0 = ld(A.w, jm), Um = ld(A.u, jm), Vm = ld(A.v, jm);
    const T Cm = ld(A.c, jm), Bm = ld(A.b, jm);
    T L0 = ld(A.lw1, j0), LV0 = ld(A.lv1, j0), W0 = ld(A.w, j0), U0 = ld(A.u, j0), V0 = ld(A.v, j0);
    T C0 = ld(A.c, j0), B0 = ld(A.b, j0);
    T Wm = Wm0;
    T sxw_m, sxe_m, sxw0, sxe0;
    xfaces(Lm, sxw_m, sxe_m);
    xfaces(L0, sxw0, sxe0);
    T Qm = Bm * (sxw_m + sxe_m);
    T Q0 = B0 * (sxw0 + sxe0);
    // the face between the previous row and the current one
    T Fy_s = dty * (Lm - L0);
    T HC_s = half * (Cm + C0) * A.idy;
    T GWy_s = half * (W0 - Wm0) * A.idy;
    T SVy_s = dvy * (LVm - LV0);
    T MN_s = one - half * (Um + U0);
    T DVy_s = V0 - Vm;
    double part[5] = {0.0, 0.0, 0.0, 0.0, 0.0};

    for (int j = j0; j < j1; ++j) {
        const int jp = min(j + 1, ny - 1);
        const bool hs = j > 0, hn = j + 1 < ny;
        const T Ln = ld(A.lw1, jp), LVn = ld(A.lv1, jp), Wn = ld(A.w, jp), Un = ld(A.u, jp), Vn = ld(A.v, jp);
        const T Cn = ld(A.c, jp), Bn = ld(A.b, jp);
        const T a0 = ld(A.a, j), LU = ld(A.lu1, j);
        const T GA0 = ld(A.ga, j), GB0 = ld(A.gb, j), GC0 = ld(A.gc, j);

        // row j: x-neighbours
        const T ae = from_right(a0);
        const T HA = half * (a0 + ae) * A.idx;              // (a_i + a_i+1)/2 idx, east face
        const T HAw = from_left(HA);
        const T We = from_right(W0), Ww = from_left(W0);
        const T GW = half * (We - W0) * A.idx;
        const T GWw = from_left(GW);
        const T Ue = from_right(U0);
        const T me = one - half * (U0 + Ue);
        const T mw = from_left(me);
        const T Ve = from_right(V0);
        const T DV = Ve - V0;
        const T DVw = from_left(DV);
        const T LVe = from_right(LV0);
        const T SV = dvx * (LV0 - LVe);
        const T SVw = from_left(SV);
        const T svw = hw ? SVw : zero;
        const T sve = he ? SV : zero;
        const T GX = me * (DV * A.idx);
        const T GXl = from_left(GX);

        // row j+1: its x-faces; the face between rows j and j+1
        T sxw_n, sxe_n;
        xfaces(Ln, sxw_n, sxe_n);
        const T Qn = Bn * (sxw_n + sxe_n);
        const T Fy_n = dty * (L0 - Ln);
        const T HC_n = half * (C0 + Cn) * A.idy;
        const T GWy_n = half * (Wn - W0) * A.idy;
        const T SVy_n = dvy * (LV0 - LVn);
        const T MN_n = one - half * (U0 + Un);
        const T DVy_n = Vn - V0;

        const T sy_s = hs ? Fy_s : zero, sy_n = hn ? Fy_n : zero;
        const T svs = hs ? SVy_s : zero, svn = hn ? SVy_n : zero;
        const T SX0 = sxw0 + sxe0;
        const T SY0 = sy_s + sy_n;
        const T P0 = B0 * SY0;
        const T Pw = from_left(P0), Pe = from_right(P0);

        // acid
        T lw = L0 * (one - A.dt * A.d3) - A.dt * A.d1 * U0 * LU;
        lw += sxw0 * HAw - sxe0 * HA;
        lw += sy_s * HC_s - sy_n * HC_n;
        T cy = (hs ? Qm : zero) - (hn ? Qn : zero);
        if (j == ny - 1) cy += Q0;
        if (j == 0) cy -= Q0;
        T cx = (hw ? Pw : zero) - (he ? Pe : zero);
        if (i == nx - 1) cx += P0;
        if (i == 0) cx -= P0;
        lw += half * A.hy * cy + half * A.hx * cx;

        // tensor gradients
        const T ty0 = (Wn - Wm) * A.hy, tx0 = (We - Ww) * A.hx;
        const T dga = sxw0 * GWw + sxe0 * GW;
        const T dgc = sy_s * GWy_s + sy_n * GWy_n;
        const T dgb = half * ty0 * SX0 + half * tx0 * SY0;

        // tumour cells
        T lv = LV0 * (one + A.dt * A.r2 * (one - two * V0)) + A.dt * A.r3 * L0;
        lv += svw * mw * A.idx - sve * me * A.idx + svs * MN_s * A.idy - svn * MN_n * A.idy;
        T lu = LU * (one + A.dt * (one - two * U0 - A.d1 * W0));
        lu += svw * (-half * DVw * A.idx) + sve * (-half * DV * A.idx);
        lu += svs * (-half * DVy_s * A.idy) + svn * (-half * DVy_n * A.idy);

        if (out_lane) {
            auto st = [&](T *p, T x) {
                if constexpr (NT) __builtin_nontemporal_store(x, mut(p, j));
                else *mut(p, j) = x;
            };
            st(A.lu, lu);
            st(A.lv, lv);
            st(A.lw, lw);
            st(A.ga, GA0 + dga);
            st(A.gb, GB0 + dgb);
            st(A.gc, GC0 + dgc);
            // scalar gradients (FP64 accumulation); divV at x^k in the forward order
            const T GXe = he ? GX : zero;
            const T GXw = hw ? GXl : zero;
            const T GYn = hn ? MN_n * (DVy_n * A.idy) : zero;
            const T GYs = hs ? MN_s * (DVy_s * A.idy) : zero;
            const T divV = (GXe - GXw) * A.idx + (GYn - GYs) * A.idy;
            const double dt = double(A.dt);
            part[0] += -dt * double(U0) * double(W0) * double(LU);
            part[1] += dt * double(V0) * (1.0 - double(V0)) * double(LV0);
            part[2] += dt * double(divV) * double(LV0);
            part[3] += dt * double(V0) * double(L0);
            part[4] += -dt * double(W0) * double(L0);
        }

        // move up one row
        Wm = W0;
        L0 = Ln; LV0 = LVn; W0 = Wn; U0 = Un; V0 = Vn; C0 = Cn; B0 = Bn;
        sxw0 = sxw_n; sxe0 = sxe_n;
        Qm = Q0; Q0 = Qn;
        Fy_s = Fy_n; HC_s = HC_n; GWy_s = GWy_n; SVy_s = SVy_n; MN_s = MN_n; DVy_s = DVy_n;
    }

    // wave reduction of the five partial sums in a fixed order, into the
    // workgroup's own slot
#pragma unroll
    for (int s = 0; s < 5; ++s)
#pragma unroll
        for (int off = 32; off >= 1; off >>= 1) part[s] += __shfl_xor(part[s], off, 64);
    if (lane < 5) {
        double r = part[0];
#pragma unroll
        for (int s = 1; s < 5; ++s)
            if (lane == s) r = part[s];
        double *slot = A.slots + (size_t)lid * 5;
        slot[lane] = slot[lane] + r;
    }
}

__global__ __launch_bounds__(256) void slots_reduce_kernel(const double *__restrict__ slots, int nblocks,
                                                           double *__restrict__ out)
{
    double x[5] = {0.0, 0.0, 0.0, 0.0, 0.0};
    for (int k = threadIdx.x; k < nblocks; k += 256)
#pragma unroll
        for (int s = 0; s < 5; ++s) x[s] += slots[(size_t)k * 5 + s];
    __shared__ double sm[4][5];
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
#pragma unroll
    for (int s = 0; s < 5; ++s)
#pragma unroll
        for (int off = 32; off >= 1; off >>= 1) x[s] += __shfl_xor(x[s], off, 64);
    if (lane == 0)
#pragma unroll
        for (int s = 0; s < 5; ++s) sm[wv][s] = x[s];
    __syncthreads();
    if (threadIdx.x < 5) out[threadIdx.x] = sm[0][threadIdx.x] + sm[1][threadIdx.x] + sm[2][threadIdx.x] +
                                            sm[3][threadIdx.x];
}

__global__ void zero_kernel(unsigned int *__restrict__ p, size_t nwords)
{
    for (size_t k = blockIdx.x * (size_t)blockDim.x + threadIdx.x; k < nwords;
         k += (size_t)gridDim.x * blockDim.x)
        p[k] = 0u;
}

template <typename S>
__global__ void eig_backward_kernel(const S *__restrict__ l1, const S *__restrict__ l2,
                                    const S *__restrict__ th, const S *__restrict__ ga,
                                    const S *__restrict__ gb, const S *__restrict__ gc,
                                    S *__restrict__ g1, S *__restrict__ g2, S *__restrict__ gt,
                                    size_t n)
{
    for (size_t k = blockIdx.x * (size_t)blockDim.x + threadIdx.x; k < n;
         k += (size_t)gridDim.x * blockDim.x) {
        const double cs = cos(double(th[k])), sn = sin(double(th[k]));
        const double s2 = 2.0 * sn * cs, c2 = cs * cs - sn * sn;
        const double a = ga[k], b = gb[k], c = gc[k];
        g1[k] = S(a * (cs * cs) + c * (sn * sn) + b * (sn * cs));
        g2[k] = S(a * (sn * sn) + c * (cs * cs) - b * (sn * cs));
        gt[k] = S((double(l1[k]) - double(l2[k])) * (-a * s2 + c * s2 + b * c2));
    }
}

// The step's arrays (18 values per cell) exceed the last-level cache.
bool adjoint_big(const ggfv_ctx *ctx) { return 18 * ctx->plane * ctx->elem > kAdjCacheBytes; }

}  // namespace
int adjoint_rows(const ggfv_ctx *ctx);
namespace {

template <typename T>
hipError_t launch_adjoint_typed(ggfv_ctx *ctx, const void *x, const void *lam_in, void *lam_out,
                                void *g, double *slots, double dt)
{
    AdjArgs<T> A{};
    const size_t P = ctx->plane;
    const T *xs = static_cast<const T *>(x);
    const T *li = static_cast<const T *>(lam_in);
    T *lo = static_cast<T *>(lam_out);
    T *gg = static_cast<T *>(g);
    const T *tn = static_cast<const T *>(ctx->tensor);
    A.u = xs;
    A.v = xs + P;
    A.w = xs + 2 * P;
    A.lu1 = li;
    A.lv1 = li + P;
    A.lw1 = li + 2 * P;
    A.lu = lo;
    A.lv = lo + P;
    A.lw = lo + 2 * P;
    A.ga = gg;
    A.gb = gg + P;
    A.gc = gg + 2 * P;
    A.a = tn;
    A.b = tn + P;
    A.c = tn + 2 * P;
    A.slots = slots;
    A.nx = ctx->nx;
    A.ny = ctx->ny;
    A.pitch = ctx->pitch;
    const double idx = ctx->nx / ctx->lx, idy = ctx->ny / ctx->ly;
    A.idx = T(idx);
    A.idy = T(idy);
    A.hx = T(0.5 * idx);
    A.hy = T(0.5 * idy);
    A.dt = T(dt);
    A.d1 = T(ctx->prm.delta1);
    A.r2 = T(ctx->prm.rho2);
    A.D2 = T(ctx->prm.Delta2);
    A.r3 = T(ctx->prm.rho3);
    A.d3 = T(ctx->prm.delta3);
    const int rows = adjoint_rows(ctx);
    const int nsx = (ctx->nx + kAdjCols - 1) / kAdjCols, nsy = (ctx->ny + rows - 1) / rows;
    const bool off32 = ctx->plane * sizeof(T) < (size_t(1) << 32), big = adjoint_big(ctx);
    const dim3 grid(nsx * nsy), block(64);
    if (off32 && big)
        hipLaunchKernelGGL((adjoint_kernel<T, true, true>), grid, block, 0, ctx->stream, A, rows, nsy);
    else if (off32)
        hipLaunchKernelGGL((adjoint_kernel<T, true, false>), grid, block, 0, ctx->stream, A, rows, nsy);
    else
        hipLaunchKernelGGL((adjoint_kernel<T, false, true>), grid, block, 0, ctx->stream, A, rows, nsy);
    return hipGetLastError();
}

}  // namespace

// Strip height of the adjoint sweep: the tallest strips whose one-wave
// workgroups fill the device's resident wave slots (the kernel's occupancy
// times the compute units) at most once, or half of them on grids beyond the
// last-level cache.  Taller strips re-read fewer halo rows; a second, partial
// round of waves would leave most CUs idle at its end.  Measured at 4096^2
// (FP64): 531 us per step at half a round, 552 at one, 676 at 1.35 rounds;
// at 512^2 one round (2-row strips) is the fastest.
int adjoint_rows(const ggfv_ctx *ctx)
{
    const bool off32 = ctx->plane * ctx->elem < (size_t(1) << 32), big = adjoint_big(ctx);
    const void *k;
    if (ctx->dtype == GGFV_F64)
        k = off32 ? (big ? (const void *)adjoint_kernel<double, true, true> : (const void *)adjoint_kernel<double, true, false>)
                  : (const void *)adjoint_kernel<double, false, true>;
    else
        k = off32 ? (big ? (const void *)adjoint_kernel<float, true, true> : (const void *)adjoint_kernel<float, true, false>)
                  : (const void *)adjoint_kernel<float, false, true>;
    int per_cu = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, k, 64, 0) != hipSuccess || per_cu < 1) {
        (void)hipGetLastError();
        per_cu = 8;
    }
    const long nsx = (ctx->nx + kAdjCols - 1) / kAdjCols;
    long slots = (long)per_cu * (ctx->cus > 0 ? ctx->cus : 256);
    if (big) slots /= 2;
    long nsy = slots / nsx;
    if (nsy < 1) nsy = 1;
    long rows = (ctx->ny + nsy - 1) / nsy;
    return (int)(rows < 1 ? 1 : rows);
}

int adjoint_blocks(const ggfv_ctx *ctx)
{
    const int rows = adjoint_rows(ctx);
    return ((ctx->nx + kAdjCols - 1) / kAdjCols) * ((ctx->ny + rows - 1) / rows);
}

hipError_t launch_adjoint_step(ggfv_ctx *ctx, const void *x, const void *lam_in, void *lam_out,
                               void *g, double *slots, double dt)
{
    if (ctx->dtype == GGFV_F64) return launch_adjoint_typed<double>(ctx, x, lam_in, lam_out, g, slots, dt);
    return launch_adjoint_typed<float>(ctx, x, lam_in, lam_out, g, slots, dt);
}

hipError_t launch_slots_reduce(ggfv_ctx *ctx, const double *slots, int nblocks, double *out)
{
    hipLaunchKernelGGL(slots_reduce_kernel, dim3(1), dim3(256), 0, ctx->stream, slots, nblocks, out);
    return hipGetLastError();
}

hipError_t launch_zero(ggfv_ctx *ctx, void *p, size_t bytes)
{
    const size_t words = bytes / 4;
    size_t blocks = (words + 255) / 256;
    if (blocks > 4096) blocks = 4096;
    if (blocks < 1) blocks = 1;
    hipLaunchKernelGGL(zero_kernel, dim3((unsigned)blocks), dim3(256), 0, ctx->stream,
                       static_cast<unsigned int *>(p), words);
    return hipGetLastError();
}

hipError_t launch_eig_backward(ggfv_ctx *ctx, const void *l1, const void *l2, const void *th,
                               const void *ga, const void *gb, const void *gc, void *g1, void *g2,
                               void *gt, bool f64)
{
    const size_t n = (size_t)ctx->nx * ctx->ny;
    size_t blocks = (n + 255) / 256;
    if (blocks > 8192) blocks = 8192;
    if (f64)
        hipLaunchKernelGGL((eig_backward_kernel<double>), dim3((unsigned)blocks), dim3(256), 0,
                           ctx->stream, (const double *)l1, (const double *)l2, (const double *)th,
                           (const double *)ga, (const double *)gb, (const double *)gc, (double *)g1,
                           (double *)g2, (double *)gt, n);
    else
        hipLaunchKernelGGL((eig_backward_kernel<float>), dim3((unsigned)blocks), dim3(256), 0,
                           ctx->stream, (const float *)l1, (const float *)l2, (const float *)th,
                           (const float *)ga, (const float *)gb, (const float *)gc, (float *)g1,
                           (float *)g2, (float *)gt, n);
    return hipGetLastError();
}

}  // namespace ggfv
