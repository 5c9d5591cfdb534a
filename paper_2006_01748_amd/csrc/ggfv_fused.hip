// ggfv_fused.hip -- K steps of eq. (3) fused into one launch (temporal blocking).
//
// The single-step kernel reads six fields and writes three per step, so it is
// bound by HBM bandwidth.  This kernel reads the old level once, computes K time
// levels on chip and writes only level K, cutting HBM traffic per step by K.
//
// Schedule.  A workgroup owns a strip of OUTW = NT*CPL - 2H output columns and
// `rows` output rows (H = K rounded up to a multiple of CPL).  It loads the
// extended columns [o0 - H, o0 + OUTW + H) and sweeps upwards.  At sweep
// iteration r, time level s (1..K) computes row q = r - 2(s-1): level 1 reads
// rows r-1, r, r+1 of the old level (row r+1 arrived this iteration), and level
// s > 1 reads rows q-1, q, q+1 of level s-1, which were finished in earlier
// iterations.  The two-row lag between levels therefore needs only one barrier
// per iteration (after the new old-level row is published).  Each level's
// valid column range shrinks by one per level on each side; the halo is
// recomputed redundantly instead of exchanged, so workgroups never wait on each
// other.
//
// Per level s the rows [j0-(K-s), j1+(K-s)) are computed (clipped to the grid),
// preceded by one warm-up row whose only product is the carried south-face flux
// (the north face of the row below).  Rows of every level live in LDS rings:
// W in 4 slots (rows q-1..q+1 read while q+2 is written), U, V and the low
// words of the compensated state in 3 slots, the tensor in 2K+1 slots.
//
// The arithmetic per cell is the single-step kernel's, in the same order, so the
// results equal K single steps bit for bit.

#include "ggfv_step_common.hpp"

namespace ggfv {
namespace {

template <typename T, bool COMP, int CPL>
struct Row0 {
    T W[CPL], U[CPL], V[CPL], a[CPL], b[CPL], c[CPL];
    T Wl[COMP ? CPL : 1], Ul[COMP ? CPL : 1], Vl[COMP ? CPL : 1];
};

template <typename T, bool COMP, int CPL>
__device__ __forceinline__ void load0(const StepArgs<T> &A, int jr, int col, Row0<T, COMP, CPL> &r)
{
    const size_t base = (size_t)jr * A.pitch + col;
    load_vec<T, CPL>(A.w + base, r.W);
    load_vec<T, CPL>(A.u + base, r.U);
    load_vec<T, CPL>(A.v + base, r.V);
    load_vec<T, CPL>(A.a + base, r.a);
    load_vec<T, CPL>(A.b + base, r.b);
    load_vec<T, CPL>(A.c + base, r.c);
    if constexpr (COMP) {
        load_vec<T, CPL>(A.wlo + base, r.Wl);
        load_vec<T, CPL>(A.ulo + base, r.Ul);
        load_vec<T, CPL>(A.vlo + base, r.Vl);
    }
}

template <typename T, bool COMP, int CPL, int NT, int K>
__global__ __launch_bounds__(NT) void fused_kernel(StepArgs<T> A)
{
    constexpr int TXW = NT * CPL;
    constexpr int H = (K + CPL - 1) / CPL * CPL;
    constexpr int OUTW = TXW - 2 * H;
    constexpr int LW = TXW + 2 * CPL;
    constexpr int RT = 2 * K + 1;
    constexpr int NLO = COMP ? K : 1;
    static_assert(OUTW > 0, "strip too narrow for the fused depth");
    __shared__ __align__(16) T sW[K][4][LW];
    __shared__ __align__(16) T sU[K][3][LW];
    __shared__ __align__(16) T sV[K][3][LW];
    __shared__ __align__(16) T sL[NLO][3][3][LW];   // low words of u, v, w (compensated state)
    __shared__ __align__(16) T ta[RT][LW];
    __shared__ __align__(16) T tb[RT][LW];
    __shared__ __align__(16) T tc[RT][LW];

    const int nbx = gridDim.x;
    const int lid = xcd_local_id(blockIdx.x + nbx * blockIdx.y, gridDim.x * gridDim.y);
    const int sx = lid % nbx, sy = lid / nbx;
    const int t = threadIdx.x;
    const int nx = A.nx, ny = A.ny;
    const int o0 = sx * OUTW;
    const int e0 = o0 - H;
    const int j0 = sy * A.rows;
    const int j1 = min(ny, j0 + A.rows);
    const int own = t * CPL + CPL;                  // LDS position of the thread's first column
    const int cbase = e0 + t * CPL;                 // its first global column
    const int lcol = min(max(cbase, 0), A.pitch - CPL);

    auto cl = [&](int j) { return j < 0 ? 0 : (j >= ny ? ny - 1 : j); };
    auto posof = [&](int i) { return (i < 0 ? 0 : (i >= nx ? nx - 1 : i)) - e0 + CPL; };
    auto lo_of = [&](int s) { return max(0, j0 - (K - s) - 1); };   // first row swept by level s
    auto re_of = [&](int s) { return max(0, j0 - (K - s)); };       // first real row of level s
    auto hi_of = [&](int s) { return min(ny, j1 + (K - s)); };      // end of level s

    auto put0 = [&](int row, const Row0<T, COMP, CPL> &r) {
        lds_store_vec<T, CPL>(&sW[0][row & 3][own], r.W);
        lds_store_vec<T, CPL>(&sU[0][row % 3][own], r.U);
        lds_store_vec<T, CPL>(&sV[0][row % 3][own], r.V);
        lds_store_vec<T, CPL>(&ta[row % RT][own], r.a);
        lds_store_vec<T, CPL>(&tb[row % RT][own], r.b);
        lds_store_vec<T, CPL>(&tc[row % RT][own], r.c);
        if constexpr (COMP) {
            lds_store_vec<T, CPL>(&sL[0][0][row % 3][own], r.Ul);
            lds_store_vec<T, CPL>(&sL[0][1][row % 3][own], r.Vl);
            lds_store_vec<T, CPL>(&sL[0][2][row % 3][own], r.Wl);
        }
    };

    const int r_begin = lo_of(1);
    const int r_end = hi_of(K) - 1 + 2 * (K - 1);
    const int last0 = hi_of(1);                     // last old-level row needed (clamped on use)
    {
        Row0<T, COMP, CPL> r0;
        load0<T, COMP, CPL>(A, cl(r_begin - 1), lcol, r0);
        put0(cl(r_begin - 1), r0);
        load0<T, COMP, CPL>(A, cl(r_begin), lcol, r0);
        put0(cl(r_begin), r0);
    }
    Row0<T, COMP, CPL> pre;
    if (r_begin + 1 <= last0) load0<T, COMP, CPL>(A, cl(r_begin + 1), lcol, pre);

    T FYs[K][CPL], GYs[K][CPL];
#pragma unroll
    for (int s = 0; s < K; ++s)
#pragma unroll
        for (int k = 0; k < CPL; ++k) {
            FYs[s][k] = T(0);
            GYs[s][k] = T(0);
        }
    const T half = T(0.5), one = T(1);

    for (int r = r_begin; r <= r_end; ++r) {
        if (r + 1 <= last0) put0(cl(r + 1), pre);
        __syncthreads();
        if (r + 2 <= last0) load0<T, COMP, CPL>(A, cl(r + 2), lcol, pre);

#pragma unroll
        for (int s = 1; s <= K; ++s) {
            const int q = r - 2 * (s - 1);
            if (q < lo_of(s) || q >= hi_of(s)) continue;   // uniform across the workgroup
            const bool real = q >= re_of(s);
            const int src = s - 1;
            const int qm = cl(q - 1), qp = cl(q + 1);
            const bool has_n = q + 1 < ny;
            const T *W0 = sW[src][q & 3];
            const T *Wp = sW[src][qp & 3];
            const T *Wm = sW[src][qm & 3];
            const T *U0 = sU[src][q % 3];
            const T *Up = sU[src][qp % 3];
            const T *V0 = sV[src][q % 3];
            const T *Vp = sV[src][qp % 3];
            const T *A0 = ta[q % RT];
            const T *B0 = tb[q % RT];
            const T *Bp = tb[qp % RT];
            const T *C0 = tc[q % RT];
            const T *Cp = tc[qp % RT];
            T ou[CPL], ov[CPL], ow[CPL], oul[CPL], ovl[CPL], owl[CPL];
#pragma unroll
            for (int k = 0; k < CPL; ++k) {
                const int i = cbase + k;
                const int pc = own + k;
                const int pl = posof(i - 1), pr = posof(i + 1);
                const T Wc = W0[pc], Wn = Wp[pc];
                const T Ws = real ? Wm[pc] : T(0);
                const T WL = W0[pl], WR = W0[pr];
                const T WLn = Wp[pl], WRn = Wp[pr];
                const T WLs = real ? Wm[pl] : T(0), WRs = real ? Wm[pr] : T(0);
                const T Uc = U0[pc], Vc = V0[pc];
                const T UL = U0[pl], UR = U0[pr], VL = V0[pl], VR = V0[pr];
                const T Un = Up[pc], Vn = Vp[pc];
                const T ac = A0[pc], aL = A0[pl], aR = A0[pr];
                const T bc = B0[pc], bL = B0[pl], bR = B0[pr], bn = Bp[pc];
                const T cc = C0[pc], cn = Cp[pc];

                const T tyc = (Wn - Ws) * A.hy;
                const T tyL = (WLn - WLs) * A.hy;
                const T tyR = (WRn - WRs) * A.hy;
                const T txc = (WR - WL) * A.hx;
                const T txn = (WRn - WLn) * A.hx;
                const bool has_e = (i + 1 < nx), has_w = (i > 0);
                const T FXe = has_e ? half * (ac + aR) * ((WR - Wc) * A.idx) + half * (bc * tyc + bR * tyR) : T(0);
                const T FXw = has_w ? half * (aL + ac) * ((Wc - WL) * A.idx) + half * (bL * tyL + bc * tyc) : T(0);
                const T FYn = has_n ? half * (cc + cn) * ((Wn - Wc) * A.idy) + half * (bc * txc + bn * txn) : T(0);
                const T GXe = has_e ? (one - half * (Uc + UR)) * ((VR - Vc) * A.idx) : T(0);
                const T GXw = has_w ? (one - half * (UL + Uc)) * ((Vc - VL) * A.idx) : T(0);
                const T GYn = has_n ? (one - half * (Uc + Un)) * ((Vn - Vc) * A.idy) : T(0);
                const T divW = (FXe - FXw) * A.idx + (FYn - FYs[src][k]) * A.idy;
                const T divV = (GXe - GXw) * A.idx + (GYn - GYs[src][k]) * A.idy;
                const T fu = Uc * (one - Uc) - (A.d1 * Uc) * Wc;
                const T fv = (A.r2 * Vc) * (one - Vc) + A.D2 * divV;
                const T fw = (A.r3 * Vc - A.d3 * Wc) + divW;
                const bool inside = (i < nx);
                if constexpr (COMP) {
                    T h, l;
                    comp_add(Uc, sL[src][0][q % 3][pc], A.dt * fu, h, l);
                    ou[k] = inside ? h : T(0);
                    oul[k] = inside ? l : T(0);
                    comp_add(Vc, sL[src][1][q % 3][pc], A.dt * fv, h, l);
                    ov[k] = inside ? h : T(0);
                    ovl[k] = inside ? l : T(0);
                    comp_add(Wc, sL[src][2][q % 3][pc], A.dt * fw, h, l);
                    ow[k] = inside ? h : T(0);
                    owl[k] = inside ? l : T(0);
                } else {
                    ou[k] = inside ? Uc + A.dt * fu : T(0);
                    ov[k] = inside ? Vc + A.dt * fv : T(0);
                    ow[k] = inside ? Wc + A.dt * fw : T(0);
                }
                FYs[src][k] = FYn;
                GYs[src][k] = GYn;
            }
            if (!real) continue;
            if (s < K) {
                lds_store_vec<T, CPL>(&sW[s][q & 3][own], ow);
                lds_store_vec<T, CPL>(&sU[s][q % 3][own], ou);
                lds_store_vec<T, CPL>(&sV[s][q % 3][own], ov);
                if constexpr (COMP) {
                    lds_store_vec<T, CPL>(&sL[s][0][q % 3][own], oul);
                    lds_store_vec<T, CPL>(&sL[s][1][q % 3][own], ovl);
                    lds_store_vec<T, CPL>(&sL[s][2][q % 3][own], owl);
                }
            } else if (cbase >= o0 && cbase < o0 + OUTW && cbase < A.pitch) {
                // level K rows are exactly the output rows [j0, j1)
                const size_t o = (size_t)q * A.pitch + cbase;
                store_vec<T, CPL>(A.un + o, ou);
                store_vec<T, CPL>(A.vn + o, ov);
                store_vec<T, CPL>(A.wn + o, ow);
                if constexpr (COMP) {
                    store_vec<T, CPL>(A.unlo + o, oul);
                    store_vec<T, CPL>(A.vnlo + o, ovl);
                    store_vec<T, CPL>(A.wnlo + o, owl);
                }
            }
        }
    }
}

template <typename T, bool COMP, int CPL, int NT, int K>
hipError_t launch_fused_typed(ggfv_ctx *ctx, const void *in, void *out, double dt)
{
    constexpr int TXW = NT * CPL;
    constexpr int H = (K + CPL - 1) / CPL * CPL;
    constexpr int OUTW = TXW - 2 * H;
    const int nbx = (ctx->nx + OUTW - 1) / OUTW;
    int rows = ctx->rows_per_strip;
    if (rows <= 0) {
        // tall strips amortise the pipeline fill (3K rows); about four
        // workgroups per CU on 256 CUs
        const long target = 1024;
        long per = ((long)ctx->ny * nbx + target - 1) / target;
        const int floor_rows = 16 * K;
        rows = (int)(per < floor_rows ? floor_rows : per);
    }
    if (rows > ctx->ny) rows = ctx->ny;
    const StepArgs<T> A = make_args<T>(ctx, in, out, dt, rows);
    const int nby = (ctx->ny + rows - 1) / rows;
    hipLaunchKernelGGL((fused_kernel<T, COMP, CPL, NT, K>), dim3(nbx, nby), dim3(NT), 0, ctx->stream, A);
    return hipGetLastError();
}

template <typename T, bool COMP, int CPL>
hipError_t launch_fused_depth(ggfv_ctx *ctx, const void *in, void *out, double dt, int K)
{
    const bool narrow = ctx->threads == 64;
    switch (K) {
    case 2: return narrow ? launch_fused_typed<T, COMP, CPL, 64, 2>(ctx, in, out, dt)
                          : launch_fused_typed<T, COMP, CPL, 128, 2>(ctx, in, out, dt);
    case 3: return narrow ? launch_fused_typed<T, COMP, CPL, 64, 3>(ctx, in, out, dt)
                          : launch_fused_typed<T, COMP, CPL, 128, 3>(ctx, in, out, dt);
    case 4: return launch_fused_typed<T, COMP, CPL, 64, 4>(ctx, in, out, dt);
    default: return hipErrorInvalidValue;
    }
}

}  // namespace

hipError_t launch_step_fused(ggfv_ctx *ctx, const void *in, void *out, double dt, int K)
{
    switch (ctx->dtype) {
    case GGFV_F64: return launch_fused_depth<double, false, 1>(ctx, in, out, dt, K);
    case GGFV_F32: return launch_fused_depth<float, false, 2>(ctx, in, out, dt, K);
    case GGFV_F32C: return launch_fused_depth<float, true, 2>(ctx, in, out, dt, K);
    default: return hipErrorInvalidValue;
    }
}

}  // namespace ggfv
