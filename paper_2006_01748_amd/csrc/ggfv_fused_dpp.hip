// ggfv_fused_dpp.hip -- K steps per launch with one wave per workgroup, the
// rows of every time level held in registers and x-neighbours exchanged with
// DPP lane shifts.
//
// A wave of 64 lanes owns 64*CPL adjacent columns (lane l: columns e0 + l*CPL +
// k) and sweeps a strip upwards like the LDS-ring variant (ggfv_fused.hip), but:
//   * every lane keeps the rows it needs of each time level in its own
//     registers (rings of 4 rows for w, 3 for u, v and the low words), so no LDS
//     traffic and no barriers are needed for the state;
//   * the x-neighbour values come from the neighbouring lane through a DPP
//     wave shift (v_mov_dpp wave_shl/wave_shr), a modifier of an ordinary VALU
//     move;
//   * each x-face flux is evaluated once, by the cell on its left, and the cell
//     on its right receives it through a lane shift; both see the same bits;
//   * the tensor rows (needed by all levels, 2K+1 rows deep) sit in a per-lane
//     LDS ring, each lane reading only what it wrote.
// The lanes at the two ends of the wave receive no neighbour; they are outside
// the valid columns of every level above the old state (the valid range shrinks
// by one column per level on each side), so what they compute is discarded.
//
// Schedule.  At iteration r the old-state row r+1 is requested (it is first
// used one iteration later), and level s = 1..K computes row q = r - 2s + 1
// from rows q-1, q, q+1 of level s-1.  Level s starts one row early (a warm-up
// row) to produce its carried south-face flux, as in the other kernels.  The row
// loop is unrolled by 12 so that every register-ring slot (row mod 4, row mod 3)
// is a compile-time constant.
//
// The arithmetic per cell is the single-step kernel's, in the same order, so K
// fused steps equal K single steps bit for bit.

#include "ggfv_step_common.hpp"

namespace ggfv {
namespace {

constexpr int kWave = 64;

// DPP wave shifts.  0x138: wave_shr:1 (lane l receives lane l-1); 0x130:
// wave_shl:1 (lane l receives lane l+1).  A lane without a source keeps its own
// value (old operand); such lanes are never used.
//
// A shift must run with every lane of the wave active: a lane reading from a
// lane that is masked off does not receive that lane's value.  The compiler may
// sink a move whose result is only used under a per-lane condition into that
// condition's branch; the empty volatile asm on the result keeps the move at
// its place in the (wave-uniform) control flow.
template <int CTRL>
__device__ __forceinline__ int dpp_move_bits(int v)
{
    int r = __builtin_amdgcn_update_dpp(v, v, CTRL, 0xf, 0xf, false);
    asm volatile("" : "+v"(r));
    return r;
}

template <int CTRL>
__device__ __forceinline__ float dpp_move(float x)
{
    return __int_as_float(dpp_move_bits<CTRL>(__float_as_int(x)));
}

template <int CTRL>
__device__ __forceinline__ double dpp_move(double x)
{
    const long long v = __double_as_longlong(x);
    const int nlo = dpp_move_bits<CTRL>((int)(v & 0xffffffffLL));
    const int nhi = dpp_move_bits<CTRL>((int)(v >> 32));
    return __longlong_as_double(((long long)nhi << 32) | (long long)(unsigned)nlo);
}

template <typename T>
__device__ __forceinline__ T from_left(T x) { return dpp_move<0x138>(x); }
template <typename T>
__device__ __forceinline__ T from_right(T x) { return dpp_move<0x130>(x); }

constexpr int pmod(int x, int m) { return ((x % m) + m) % m; }

template <typename T, bool COMP, int CPL, int K>
struct DppState {
    T W[K][4][CPL];               // level s rows, slot = row mod 4
    T U[K][3][CPL];               // slot = row mod 3
    T V[K][3][CPL];
    T Wl[COMP ? K : 1][3][CPL];   // low words of the compensated state
    T Ul[COMP ? K : 1][3][CPL];
    T Vl[COMP ? K : 1][3][CPL];
    T FYs[K][CPL], GYs[K][CPL];   // carried south faces per level
    T ta[CPL], tb[CPL], tc[CPL];  // tensor row in flight (written to LDS next iteration)
};

struct DppGeom {
    int nx, ny, j0, j1, o0, e0, lane, cbase, lcol, last0;
    int lo[5], re[5], hi[5];      // per level 1..K: first swept row, first real row, end
    int outw;
};

template <typename T, bool COMP, int CPL, int K, int RT>
struct TensorLds {
    T a[RT][kWave * CPL], b[RT][kWave * CPL], c[RT][kWave * CPL];
};

template <typename T, bool COMP, int CPL, int K, int PH, int RT>
__device__ __forceinline__ void dpp_iter(const StepArgs<T> &A, const DppGeom &g, DppState<T, COMP, CPL, K> &S,
                                         TensorLds<T, COMP, CPL, K, RT> &L, const int r, const int r_start,
                                         const int r_end)
{
    if (r < r_start || r > r_end) return;
    const int own = g.lane * CPL;
    const T half = T(0.5), one = T(1);
    auto cl = [&](int j) { return j < 0 ? 0 : (j >= g.ny ? g.ny - 1 : j); };
    auto tslot = [&](int row) { return ((row % RT) + RT) % RT; };

    // The tensor row r arrived in registers during the previous iteration: store
    // it in the lane's LDS ring.  Then request old-state row r+1 (state straight
    // into the level-0 ring slots, tensor into the in-flight registers).
    if (r >= r_start + 1 && r <= g.last0) {
        const int ts = tslot(r);
#pragma unroll
        for (int k = 0; k < CPL; ++k) {
            L.a[ts][own + k] = S.ta[k];
            L.b[ts][own + k] = S.tb[k];
            L.c[ts][own + k] = S.tc[k];
        }
    }
    if (r + 1 <= g.last0) {
        const size_t base = (size_t)cl(r + 1) * A.pitch + g.lcol;
        constexpr int w1 = pmod(PH + 1, 4), u1 = pmod(PH + 1, 3);
        load_vec<T, CPL>(A.w + base, S.W[0][w1]);
        load_vec<T, CPL>(A.u + base, S.U[0][u1]);
        load_vec<T, CPL>(A.v + base, S.V[0][u1]);
        if constexpr (COMP) {
            load_vec<T, CPL>(A.wlo + base, S.Wl[0][u1]);
            load_vec<T, CPL>(A.ulo + base, S.Ul[0][u1]);
            load_vec<T, CPL>(A.vlo + base, S.Vl[0][u1]);
        }
        load_vec<T, CPL>(A.a + base, S.ta);
        load_vec<T, CPL>(A.b + base, S.tb);
        load_vec<T, CPL>(A.c + base, S.tc);
    }

#pragma unroll
    for (int s = 1; s <= K; ++s) {
        const int q = r - 2 * s + 1;
        if (q < g.lo[s] || q >= g.hi[s]) continue;              // uniform
        const bool real = q >= g.re[s];
        const bool has_n = q + 1 < g.ny;
        const bool has_s = q > 0;
        const int src = s - 1;
        // ring slots of rows q-1, q, q+1 (r = PH mod 12, q = r + 1 - 2s)
        const int sq4 = pmod(PH + 1 - 2 * s, 4), sp4 = pmod(PH + 2 - 2 * s, 4), sm4 = pmod(PH - 2 * s, 4);
        const int sq3 = pmod(PH + 1 - 2 * s, 3), sp3 = pmod(PH + 2 - 2 * s, 3);
        const int tq = tslot(q), tp = tslot(has_n ? q + 1 : q);

        T W0[CPL], Wp[CPL], Wm[CPL], U0[CPL], Up[CPL], V0[CPL], Vp[CPL], A0[CPL], B0[CPL], Bp[CPL], C0[CPL],
            Cp[CPL], TY[CPL];
#pragma unroll
        for (int k = 0; k < CPL; ++k) {
            W0[k] = S.W[src][sq4][k];
            Wp[k] = has_n ? S.W[src][sp4][k] : W0[k];
            Wm[k] = real ? (has_s ? S.W[src][sm4][k] : W0[k]) : T(0);
            U0[k] = S.U[src][sq3][k];
            V0[k] = S.V[src][sq3][k];
            Up[k] = has_n ? S.U[src][sp3][k] : U0[k];
            Vp[k] = has_n ? S.V[src][sp3][k] : V0[k];
            A0[k] = L.a[tq][own + k];
            B0[k] = L.b[tq][own + k];
            C0[k] = L.c[tq][own + k];
            Bp[k] = L.b[tp][own + k];
            Cp[k] = L.c[tp][own + k];
            TY[k] = (Wp[k] - Wm[k]) * A.hy;
        }
        // right neighbours of every column (lane shift for the last column)
        T WR[CPL], aR[CPL], bR[CPL], tyR[CPL], UR[CPL], VR[CPL], WL[CPL], WLn[CPL], WRn[CPL];
#pragma unroll
        for (int k = 0; k < CPL; ++k) {
            if (k + 1 < CPL) {
                WR[k] = W0[k + 1];
                aR[k] = A0[k + 1];
                bR[k] = B0[k + 1];
                tyR[k] = TY[k + 1];
                UR[k] = U0[k + 1];
                VR[k] = V0[k + 1];
                WRn[k] = Wp[k + 1];
            } else {
                WR[k] = from_right(W0[0]);
                aR[k] = from_right(A0[0]);
                bR[k] = from_right(B0[0]);
                tyR[k] = from_right(TY[0]);
                UR[k] = from_right(U0[0]);
                VR[k] = from_right(V0[0]);
                WRn[k] = from_right(Wp[0]);
            }
            if (k > 0) {
                WL[k] = W0[k - 1];
                WLn[k] = Wp[k - 1];
            } else {
                WL[k] = from_left(W0[CPL - 1]);
                WLn[k] = from_left(Wp[CPL - 1]);
            }
        }
        // east faces of every column
        T FXe[CPL], GXe[CPL];
#pragma unroll
        for (int k = 0; k < CPL; ++k) {
            const int i = g.cbase + k;
            const bool has_e = i + 1 < g.nx;
            FXe[k] = has_e ? half * (A0[k] + aR[k]) * ((WR[k] - W0[k]) * A.idx) + half * (B0[k] * TY[k] + bR[k] * tyR[k])
                           : T(0);
            GXe[k] = has_e ? (one - half * (U0[k] + UR[k])) * ((VR[k] - V0[k]) * A.idx) : T(0);
        }
        // west faces of the first column come from the lane on the left; the
        // shifts run outside any per-lane condition (a ?: operand is evaluated
        // conditionally)
        const T FXl = from_left(FXe[CPL - 1]), GXl = from_left(GXe[CPL - 1]);
        T ou[CPL], ov[CPL], ow[CPL], oul[CPL], ovl[CPL], owl[CPL];
#pragma unroll
        for (int k = 0; k < CPL; ++k) {
            const int i = g.cbase + k;
            const bool has_w = i > 0, has_e = i + 1 < g.nx;
            const T FXw = has_w ? (k > 0 ? FXe[k - 1] : FXl) : T(0);
            const T GXw = has_w ? (k > 0 ? GXe[k - 1] : GXl) : T(0);
            // mirrored neighbours for the tangential differences
            const T wl = has_w ? WL[k] : W0[k], wr = has_e ? WR[k] : W0[k];
            const T wln = has_w ? WLn[k] : Wp[k], wrn = has_e ? WRn[k] : Wp[k];
            const T txc = (wr - wl) * A.hx;
            const T txn = (wrn - wln) * A.hx;
            const T Wc = W0[k], Wn = Wp[k], Uc = U0[k], Vc = V0[k];
            const T FYn = has_n ? half * (C0[k] + Cp[k]) * ((Wn - Wc) * A.idy) + half * (B0[k] * txc + Bp[k] * txn)
                                : T(0);
            const T GYn = has_n ? (one - half * (Uc + Up[k])) * ((Vp[k] - Vc) * A.idy) : T(0);
            const T divW = (FXe[k] - FXw) * A.idx + (FYn - S.FYs[src][k]) * A.idy;
            const T divV = (GXe[k] - GXw) * A.idx + (GYn - S.GYs[src][k]) * A.idy;
            const T fu = Uc * (one - Uc) - (A.d1 * Uc) * Wc;
            const T fv = (A.r2 * Vc) * (one - Vc) + A.D2 * divV;
            const T fw = (A.r3 * Vc - A.d3 * Wc) + divW;
            const bool inside = i < g.nx;
            if constexpr (COMP) {
                T h, l;
                comp_add(Uc, S.Ul[src][sq3][k], A.dt * fu, h, l);
                ou[k] = inside ? h : T(0);
                oul[k] = inside ? l : T(0);
                comp_add(Vc, S.Vl[src][sq3][k], A.dt * fv, h, l);
                ov[k] = inside ? h : T(0);
                ovl[k] = inside ? l : T(0);
                comp_add(Wc, S.Wl[src][sq3][k], A.dt * fw, h, l);
                ow[k] = inside ? h : T(0);
                owl[k] = inside ? l : T(0);
            } else {
                ou[k] = inside ? Uc + A.dt * fu : T(0);
                ov[k] = inside ? Vc + A.dt * fv : T(0);
                ow[k] = inside ? Wc + A.dt * fw : T(0);
            }
            S.FYs[src][k] = FYn;
            S.GYs[src][k] = GYn;
        }
        if (!real) continue;
        if (s < K) {
#pragma unroll
            for (int k = 0; k < CPL; ++k) {
                S.W[s][sq4][k] = ow[k];
                S.U[s][sq3][k] = ou[k];
                S.V[s][sq3][k] = ov[k];
                if constexpr (COMP) {
                    S.Wl[s][sq3][k] = owl[k];
                    S.Ul[s][sq3][k] = oul[k];
                    S.Vl[s][sq3][k] = ovl[k];
                }
            }
        } else if (g.cbase >= g.o0 && g.cbase < g.o0 + g.outw && g.cbase < A.pitch) {
            const size_t o = (size_t)q * A.pitch + g.cbase;
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

template <typename T, bool COMP, int CPL, int K>
__global__ __launch_bounds__(kWave) void fused_dpp_kernel(StepArgs<T> A)
{
    constexpr int TXW = kWave * CPL;
    constexpr int H = (K + CPL - 1) / CPL * CPL;
    constexpr int OUTW = TXW - 2 * H;
    constexpr int RT = 2 * K + 1;
    static_assert(K >= 1 && K <= 4, "fused depth 1..4");
    __shared__ TensorLds<T, COMP, CPL, K, RT> L;

    const int nbx = gridDim.x;
    const int lid = xcd_local_id(blockIdx.x + nbx * blockIdx.y, gridDim.x * gridDim.y);
    const int sx = lid % nbx, sy = lid / nbx;
    DppGeom g;
    g.nx = A.nx;
    g.ny = A.ny;
    g.o0 = sx * OUTW;
    g.e0 = g.o0 - H;
    g.outw = OUTW;
    g.j0 = sy * A.rows;
    g.j1 = min(g.ny, g.j0 + A.rows);
    g.lane = threadIdx.x;
    g.cbase = g.e0 + g.lane * CPL;
    g.lcol = min(max(g.cbase, 0), A.pitch - CPL);
#pragma unroll
    for (int s = 1; s <= K; ++s) {
        g.lo[s] = max(0, g.j0 - (K - s) - 1);
        g.re[s] = max(0, g.j0 - (K - s));
        g.hi[s] = min(g.ny, g.j1 + (K - s));
    }
    g.last0 = g.hi[1];                     // last old-state row needed (clamped on load)
    const int r_begin = g.lo[1] + 1;       // level 1 computes q = r - 1
    const int r_end = g.hi[K] - 1 + 2 * K - 1;
    const int r_start = r_begin - 4;       // four load-only iterations fill the rings

    DppState<T, COMP, CPL, K> S;
#pragma unroll
    for (int s = 0; s < K; ++s)
#pragma unroll
        for (int k = 0; k < CPL; ++k) {
            S.FYs[s][k] = T(0);
            S.GYs[s][k] = T(0);
        }
    const int r0 = r_start - pmod(r_start, 12);
    for (int rb = r0; rb <= r_end; rb += 12) {
        dpp_iter<T, COMP, CPL, K, 0, RT>(A, g, S, L, rb + 0, r_start, r_end);
        dpp_iter<T, COMP, CPL, K, 1, RT>(A, g, S, L, rb + 1, r_start, r_end);
        dpp_iter<T, COMP, CPL, K, 2, RT>(A, g, S, L, rb + 2, r_start, r_end);
        dpp_iter<T, COMP, CPL, K, 3, RT>(A, g, S, L, rb + 3, r_start, r_end);
        dpp_iter<T, COMP, CPL, K, 4, RT>(A, g, S, L, rb + 4, r_start, r_end);
        dpp_iter<T, COMP, CPL, K, 5, RT>(A, g, S, L, rb + 5, r_start, r_end);
        dpp_iter<T, COMP, CPL, K, 6, RT>(A, g, S, L, rb + 6, r_start, r_end);
        dpp_iter<T, COMP, CPL, K, 7, RT>(A, g, S, L, rb + 7, r_start, r_end);
        dpp_iter<T, COMP, CPL, K, 8, RT>(A, g, S, L, rb + 8, r_start, r_end);
        dpp_iter<T, COMP, CPL, K, 9, RT>(A, g, S, L, rb + 9, r_start, r_end);
        dpp_iter<T, COMP, CPL, K, 10, RT>(A, g, S, L, rb + 10, r_start, r_end);
        dpp_iter<T, COMP, CPL, K, 11, RT>(A, g, S, L, rb + 11, r_start, r_end);
    }
}

template <typename T, bool COMP, int CPL, int K>
hipError_t launch_dpp_typed(ggfv_ctx *ctx, const void *in, void *out, double dt)
{
    constexpr int TXW = kWave * CPL;
    constexpr int H = (K + CPL - 1) / CPL * CPL;
    constexpr int OUTW = TXW - 2 * H;
    const int nbx = (ctx->nx + OUTW - 1) / OUTW;
    int rows = ctx->rows_per_strip;
    if (rows <= 0) {
        // one-wave workgroups: aim for about 16 per CU on 256 CUs, tall enough
        // to amortise the 3K-row pipeline fill
        const long target = 4096;
        long per = ((long)ctx->ny * nbx + target - 1) / target;
        const int floor_rows = 8 * K;
        rows = (int)(per < floor_rows ? floor_rows : per);
    }
    if (rows > ctx->ny) rows = ctx->ny;
    const StepArgs<T> A = make_args<T>(ctx, in, out, dt, rows);
    const int nby = (ctx->ny + rows - 1) / rows;
    hipLaunchKernelGGL((fused_dpp_kernel<T, COMP, CPL, K>), dim3(nbx, nby), dim3(kWave), 0, ctx->stream, A);
    return hipGetLastError();
}

template <typename T, bool COMP, int CPL>
hipError_t launch_dpp_depth(ggfv_ctx *ctx, const void *in, void *out, double dt, int K)
{
    switch (K) {
    case 1: return launch_dpp_typed<T, COMP, CPL, 1>(ctx, in, out, dt);
    case 2: return launch_dpp_typed<T, COMP, CPL, 2>(ctx, in, out, dt);
    case 3: return launch_dpp_typed<T, COMP, CPL, 3>(ctx, in, out, dt);
    case 4: return launch_dpp_typed<T, COMP, CPL, 4>(ctx, in, out, dt);
    default: return hipErrorInvalidValue;
    }
}

}  // namespace

hipError_t launch_step_fused_dpp(ggfv_ctx *ctx, const void *in, void *out, double dt, int K)
{
    switch (ctx->dtype) {
    case GGFV_F64: return launch_dpp_depth<double, false, 1>(ctx, in, out, dt, K);
    case GGFV_F32: return launch_dpp_depth<float, false, 2>(ctx, in, out, dt, K);
    case GGFV_F32C: return launch_dpp_depth<float, true, 2>(ctx, in, out, dt, K);
    default: return hipErrorInvalidValue;
    }
}

}  // namespace ggfv
