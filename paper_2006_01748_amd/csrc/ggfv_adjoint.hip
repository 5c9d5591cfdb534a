// ggfv_adjoint.hip -- the discrete adjoint of one step of eq. (3) and the chain
// rule of the tensor map, for gradients of a loss of the final state with respect
// to the initial state, the reaction parameters and the per-cell tensor.
//
// With F the forward step x^k -> x^{k+1} (dt fixed) and lam' = dL/dx^{k+1}, one
// adjoint step computes, for every cell m,
//   lam(m)   = ((dF/dx)^T lam')(m)
//   g_A(m)  += ((dF/d(a,b,c))^T lam')(m)
//   g_p     += (dF/dp)^T lam'    (p = delta1, rho2, Delta2, rho3, delta3)
// in gather form: each thread owns one cell and collects the contributions of
// every face flux that reads a value of that cell.  Writing s_f for the loss
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
// 18 values per cell-update.  Neighbour reuse goes through L1/L2.  The five
// scalar partial sums are folded per block in a fixed order and added into that
// block's own slot (no atomics), so repeated sweeps give identical bits.

#include <cmath>

#include "ggfv_internal.hpp"

namespace ggfv {
namespace {

constexpr int kAdjBX = 64;
constexpr int kAdjBY = 4;

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

template <typename T>
__global__ __launch_bounds__(kAdjBX *kAdjBY) void adjoint_kernel(AdjArgs<T> A)
{
    const int i = blockIdx.x * kAdjBX + threadIdx.x;
    const int j = blockIdx.y * kAdjBY + threadIdx.y;
    const int nx = A.nx, ny = A.ny;
    const bool inside = (i < nx) && (j < ny);
    double part[5] = {0.0, 0.0, 0.0, 0.0, 0.0};

    if (inside) {
        const int im = max(i - 1, 0), ip = min(i + 1, nx - 1);
        const int jm = max(j - 1, 0), jp = min(j + 1, ny - 1);
        const bool hw = i > 0, he = i + 1 < nx, hs = j > 0, hn = j + 1 < ny;
        const size_t P = A.pitch;
        auto at = [&](const T *p, int ii, int jj) { return p[(size_t)jj * P + ii]; };
        const T zero = T(0), half = T(0.5), one = T(1), two = T(2);

        // adjoint values on the 3x3 neighbourhood (clamped; absent faces are zeroed below)
        const T L00 = at(A.lw1, i, j);
        const T Lw0 = at(A.lw1, im, j), Le0 = at(A.lw1, ip, j);
        const T L0s = at(A.lw1, i, jm), L0n = at(A.lw1, i, jp);
        const T Lws = at(A.lw1, im, jm), Les = at(A.lw1, ip, jm);
        const T Lwn = at(A.lw1, im, jp), Len = at(A.lw1, ip, jp);

        // sums of the loss sensitivities of a cell's two x-faces (row r) and two y-faces (col q)
        auto SXrow = [&](T Lm, T L0, T Lp) {
            return (hw ? A.dt * A.idx * (Lm - L0) : zero) + (he ? A.dt * A.idx * (L0 - Lp) : zero);
        };
        auto SYcol = [&](T Ls, T L0, T Ln) {
            return (hs ? A.dt * A.idy * (Ls - L0) : zero) + (hn ? A.dt * A.idy * (L0 - Ln) : zero);
        };
        const T sx_w = hw ? A.dt * A.idx * (Lw0 - L00) : zero;   // face (i-1, i)
        const T sx_e = he ? A.dt * A.idx * (L00 - Le0) : zero;   // face (i, i+1)
        const T sy_s = hs ? A.dt * A.idy * (L0s - L00) : zero;   // face (j-1, j)
        const T sy_n = hn ? A.dt * A.idy * (L00 - L0n) : zero;   // face (j, j+1)
        const T SX0 = sx_w + sx_e;
        const T SXs = SXrow(Lws, L0s, Les);                       // row j-1 (used only if j > 0)
        const T SXn = SXrow(Lwn, L0n, Len);                       // row j+1 (used only if j+1 < ny)
        const T SY0 = sy_s + sy_n;
        const T SYw = SYcol(Lws, Lw0, Lwn);                       // column i-1 (used only if i > 0)
        const T SYe = SYcol(Les, Le0, Len);                       // column i+1 (used only if i+1 < nx)

        const T W0 = at(A.w, i, j), Ww = at(A.w, im, j), We = at(A.w, ip, j);
        const T Ws = at(A.w, i, jm), Wn = at(A.w, i, jp);
        const T a0 = at(A.a, i, j), aw = at(A.a, im, j), ae = at(A.a, ip, j);
        const T c0 = at(A.c, i, j), cs = at(A.c, i, jm), cn = at(A.c, i, jp);
        const T b0 = at(A.b, i, j), bw = at(A.b, im, j), be = at(A.b, ip, j);
        const T bs = at(A.b, i, jm), bn = at(A.b, i, jp);
        const T U0 = at(A.u, i, j), Uw = at(A.u, im, j), Ue = at(A.u, ip, j);
        const T Us = at(A.u, i, jm), Un = at(A.u, i, jp);
        const T V0 = at(A.v, i, j), Vw = at(A.v, im, j), Ve = at(A.v, ip, j);
        const T Vs = at(A.v, i, jm), Vn = at(A.v, i, jp);
        const T LU = at(A.lu1, i, j);
        const T LV0 = at(A.lv1, i, j), LVw = at(A.lv1, im, j), LVe = at(A.lv1, ip, j);
        const T LVs = at(A.lv1, i, jm), LVn = at(A.lv1, i, jp);

        // acid: diagonal part of the face fluxes
        T lw = L00 * (one - A.dt * A.d3) - A.dt * A.d1 * U0 * LU;
        lw += sx_w * (half * (aw + a0) * A.idx) - sx_e * (half * (a0 + ae) * A.idx);
        lw += sy_s * (half * (cs + c0) * A.idy) - sy_n * (half * (c0 + cn) * A.idy);
        // acid: cross terms through the tangential differences of neighbouring cells
        T cy = (hs ? bs * SXs : zero) - (hn ? bn * SXn : zero);
        if (j == ny - 1) cy += b0 * SX0;
        if (j == 0) cy -= b0 * SX0;
        T cx = (hw ? bw * SYw : zero) - (he ? be * SYe : zero);
        if (i == nx - 1) cx += b0 * SY0;
        if (i == 0) cx -= b0 * SY0;
        lw += half * A.hy * cy + half * A.hx * cx;

        // tensor gradients
        const T ty0 = (Wn - Ws) * A.hy, tx0 = (We - Ww) * A.hx;
        const T dga = sx_w * (half * (W0 - Ww) * A.idx) + sx_e * (half * (We - W0) * A.idx);
        const T dgc = sy_s * (half * (W0 - Ws) * A.idy) + sy_n * (half * (Wn - W0) * A.idy);
        const T dgb = half * ty0 * SX0 + half * tx0 * SY0;

        // tumour cells: mobility fluxes
        const T svw = hw ? A.dt * A.D2 * A.idx * (LVw - LV0) : zero;
        const T sve = he ? A.dt * A.D2 * A.idx * (LV0 - LVe) : zero;
        const T svs = hs ? A.dt * A.D2 * A.idy * (LVs - LV0) : zero;
        const T svn = hn ? A.dt * A.D2 * A.idy * (LV0 - LVn) : zero;
        const T mw = one - half * (Uw + U0), me = one - half * (U0 + Ue);
        const T ms = one - half * (Us + U0), mn = one - half * (U0 + Un);
        T lv = LV0 * (one + A.dt * A.r2 * (one - two * V0)) + A.dt * A.r3 * L00;
        lv += svw * mw * A.idx - sve * me * A.idx + svs * ms * A.idy - svn * mn * A.idy;
        T lu = LU * (one + A.dt * (one - two * U0 - A.d1 * W0));
        lu += svw * (-half * (V0 - Vw) * A.idx) + sve * (-half * (Ve - V0) * A.idx);
        lu += svs * (-half * (V0 - Vs) * A.idy) + svn * (-half * (Vn - V0) * A.idy);

        const size_t o = (size_t)j * P + i;
        A.lu[o] = lu;
        A.lv[o] = lv;
        A.lw[o] = lw;
        A.ga[o] = A.ga[o] + dga;
        A.gb[o] = A.gb[o] + dgb;
        A.gc[o] = A.gc[o] + dgc;

        // scalar gradients (FP64 accumulation); divV at x^k in the forward order
        const T GXe = he ? me * ((Ve - V0) * A.idx) : zero;
        const T GXw = hw ? mw * ((V0 - Vw) * A.idx) : zero;
        const T GYn = hn ? mn * ((Vn - V0) * A.idy) : zero;
        const T GYs = hs ? ms * ((V0 - Vs) * A.idy) : zero;
        const T divV = (GXe - GXw) * A.idx + (GYn - GYs) * A.idy;
        const double dt = double(A.dt);
        part[0] = -dt * double(U0) * double(W0) * double(LU);
        part[1] = dt * double(V0) * (1.0 - double(V0)) * double(LV0);
        part[2] = dt * double(divV) * double(LV0);
        part[3] = dt * double(V0) * double(L00);
        part[4] = -dt * double(W0) * double(L00);
    }

    // block reduction of the five partial sums in a fixed order
    __shared__ double sm[kAdjBX * kAdjBY / 64][5];
    const int tid = threadIdx.y * kAdjBX + threadIdx.x;
    const int lane = tid & 63, wv = tid >> 6;
#pragma unroll
    for (int s = 0; s < 5; ++s)
#pragma unroll
        for (int off = 32; off >= 1; off >>= 1) part[s] += __shfl_xor(part[s], off, 64);
    if (lane == 0)
#pragma unroll
        for (int s = 0; s < 5; ++s) sm[wv][s] = part[s];
    __syncthreads();
    if (tid < 5) {
        double r = 0.0;
        for (int k = 0; k < kAdjBX * kAdjBY / 64; ++k) r += sm[k][tid];
        double *slot = A.slots + ((size_t)blockIdx.y * gridDim.x + blockIdx.x) * 5;
        slot[tid] = slot[tid] + r;
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
    dim3 blk(kAdjBX, kAdjBY), grd((ctx->nx + kAdjBX - 1) / kAdjBX, (ctx->ny + kAdjBY - 1) / kAdjBY);
    hipLaunchKernelGGL(adjoint_kernel<T>, grd, blk, 0, ctx->stream, A);
    return hipGetLastError();
}

}  // namespace

int adjoint_blocks(const ggfv_ctx *ctx)
{
    return ((ctx->nx + kAdjBX - 1) / kAdjBX) * ((ctx->ny + kAdjBY - 1) / kAdjBY);
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
