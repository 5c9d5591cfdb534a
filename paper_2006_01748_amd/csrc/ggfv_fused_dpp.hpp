// ggfv_fused_dpp.hpp -- K steps per launch with one wave per workgroup, the
// rows of every time level held in registers and x-neighbours exchanged with
// DPP lane shifts.
//
// A wave of 64 lanes owns 64*CPL adjacent columns (lane l: columns e0 + l*CPL +
// k) and sweeps a strip upwards.  Level s = 1..K computes row q = r - 2s + 1 at
// iteration r from rows q-1, q, q+1 of level s-1 (level 0 is the old state,
// requested one iteration ahead).
//   * every lane keeps the rows it needs of each level in registers, so the
//     state needs no LDS and no barriers;
//   * the levels of one iteration run from K down to 1, so that level s has
//     consumed a row of level s-1 before level s-1 overwrites it: w needs a ring
//     of 3 rows, u, v and the low words a ring of 2;
//   * x-neighbours come from the neighbouring lane through a DPP wave shift;
//     each x-face flux is evaluated once, by the cell on its left, and the cell
//     on its right receives it by a shift; b*dw/dy is shifted as one product;
//   * the x-difference of w of row q+1 and its right-lane neighbour are kept
//     for the next row, where they belong to the row being computed;
//   * the tensor rows (needed by all levels) sit in per-lane LDS rings, each lane
//     reading only what it wrote, stored as the half face sums (a_i + a_i+1)/2
//     and (c_j + c_j+1)/2 that the fluxes use, plus b.  A row of (a+a')/2 or b
//     is last read by level K, 2K-1 iterations after it is stored, and a row of
//     (c+c')/2 one iteration sooner; since levels K..2 read before the store of
//     an iteration, rings of 2K-1 and 2K-2 rows suffice (2 and 1 for K = 1):
//     10 KB for FP64 at K = 4, so 16 one-wave workgroups fit a CU's 160 KB;
//   * the mirrored row -1 (= row 0) of the no-flux boundary is written into
//     the rings; row ny is never computed: the only value of it that matters,
//     the y-difference of w at row ny-1, selects row ny-1 itself (the faces
//     through the top boundary are zero).
// Each level starts one row early (a warm-up row) to produce its carried south
// face, and one row before that it takes the x-difference of its first row.
// The lanes at the two ends of the wave receive no neighbour; they lie outside
// the valid columns of every level above the old state (the valid range shrinks
// by one column per level on each side), so what they compute is discarded.
//
// The arithmetic per cell is the single-step kernel's, in the same order (the
// shared sums and products are the same operations on the same operands), so K
// fused steps equal K single steps bit for bit.
//
// The FP32 instances are built in ggfv_fused_dpp.hip and the FP64 ones in
// ggfv_fused_dpp_f64.hip, each under the instruction schedule that measured
// fastest for it.

#ifndef GGFV_FUSED_DPP_HPP
#define GGFV_FUSED_DPP_HPP

#include "ggfv_dpp.hpp"
#include "ggfv_step_common.hpp"

namespace ggfv {
namespace {

constexpr int kWave = 64;
constexpr int kPeriod = 6;    // row-loop unroll: lcm of the ring lengths 3 and 2
// s_getreg operand for bit 0 of the wave's slot (HW_ID register 4, bits 3:0 hold
// the slot; size field 0 = one bit, offset 0)
constexpr int kHwIdWaveSlotBit0 = 4;

constexpr int pmod(int x, int m) { return ((x % m) + m) % m; }

template <typename T, bool COMP, int CPL, int K>
struct LaneRows {
    // input rows of level s (output rows of level s-1) at index s-1
    T W[K][3][CPL];               // slot = row mod 3
    T U[K][2][CPL], V[K][2][CPL]; // slot = row mod 2
    T Wl[COMP ? K : 1][2][CPL], Ul[COMP ? K : 1][2][CPL], Vl[COMP ? K : 1][2][CPL];
    T TX[K][CPL];                 // x-difference of w of the next row of level s
    T WR[K];                      // its w one column right of the lane's last column
    T FYs[K][CPL], GYs[K][CPL];   // carried south faces
    T ta[CPL], tb[CPL], tc[CPL];  // tensor row in flight
    T cprev[CPL];                 // c of the previous tensor row
    T KO[COMP ? 6 : 3][CPL];      // level K's output row until it is stored (late_store)
};

template <int K>
struct LaneGeom {
    int nx, ny, own, cbase, lcol, last0;
    int lo[K + 1], re[K + 1], hi[K + 1];   // per level: warm-up row, first real row, end
    int o0, span;                          // first output column of the workgroup; output columns of a row
    bool flip;                             // the strip sweeps downward (rows mirrored, see dpp_strip)
};

template <typename T, int CPL, int RTA, int RTC>
struct TensorRing {
    // a row holds column k of every lane at [k * 64 + lane]: the 64 lanes of
    // one access touch consecutive words, free of bank conflicts
    T hA[RTA][kWave * CPL];       // (a_i + a_i+1) / 2
    T B[RTA][kWave * CPL];        // b
    T hC[RTC][kWave * CPL];       // (c_j + c_j+1) / 2
};

// EDGE = false: the wave's columns and the strip's rows stay clear of the
// domain boundary, so every boundary mask is true and compiles away.
template <int CPL, bool EDGE = true>
struct ColumnMasks {
    bool ve[CPL];                 // column >= 0 and its east face inside the domain
    bool he[CPL];                 // column has an east neighbour
    bool hw0;                     // the first column has a west neighbour
    bool inside[CPL];             // column < nx
};

template <int RT>
__device__ __forceinline__ int tslot(int row) { return ((row % RT) + RT) % RT; }

// Ring slot of row rb + D, where rb is a multiple of the unroll period and
// base = tslot<RT>(rb) (0 when RT divides the period: then the slot is a
// constant).  One conditional subtract instead of a division per use.
template <int RT, int D>
__device__ __forceinline__ int ring_slot(int base)
{
    constexpr int d = pmod(D, RT);
    if constexpr (kPeriod % RT == 0) return d;
    const int x = base + d;
    return x >= RT ? x - RT : x;
}

template <int RT>
__device__ __forceinline__ int ring_base(int rb)
{
    if constexpr (kPeriod % RT == 0) return 0;
    return tslot<RT>(rb);
}

// x-difference of w along one row (mirrored at the domain edges) and the raw
// right-lane neighbour of the last column.
template <typename T, int CPL, bool EDGE>
__device__ __forceinline__ void x_difference(const T (&X)[CPL], const ColumnMasks<CPL, EDGE> &m, const T hx,
                                             T (&TXo)[CPL], T &WRo)
{
    const T WLs = from_left(X[CPL - 1]);
    const T WRs = from_right(X[0]);
#pragma unroll
    for (int k = 0; k < CPL; ++k) {
        const T wl = k > 0 ? X[k > 0 ? k - 1 : 0] : ((!EDGE || m.hw0) ? WLs : X[0]);
        const T nb = k + 1 < CPL ? X[k + 1 < CPL ? k + 1 : k] : WRs;
        const T wr = (!EDGE || m.he[k]) ? nb : X[k];
        TXo[k] = (wr - wl) * hx;
    }
    WRo = WRs;
}

// Where and how level K's output row is stored (measured on MI355X).  FP64
// with wide lanes (the headline kernel): late, after the ring update has
// waited for the loads of the iteration's old-state row, with non-temporal
// stores.  The memory counter drains in order, so a wait for a load also
// waits for every store issued before that load; stored late, a row's stores
// have the rest of the iteration before the next such wait (+1-2%, measured
// when the stores still sat behind a branch).  Every other kernel stores at level K.  The FP32
// single-context kernels write through the caches (+2-5%); FP64 and the
// ensemble kernels keep non-temporal stores (the ensemble and the narrow FP64
// kernel measured slower otherwise).
template <typename T, int CPL, int K>
constexpr bool late_store() { return sizeof(T) == 8 && CPL == 2 && K >= 2; }

// Store level K's output row q (held in R.KO): the lanes whose columns are
// outputs of this workgroup, if q is one of its rows.  Every lane issues the
// store in every iteration, as a buffer store whose range is the workgroup's
// output span of the row (empty for a row outside the strip): the hardware
// drops the lanes outside the range.  With no branch around the stores, the
// compiler's memory-counter waits can count them, so the wait for the next
// row's loads does not also wait for the stores issued before them.
template <typename T, bool COMP, int CPL, int K, bool BATCH>
__device__ __forceinline__ void store_level_k(const StepArgs<T> &A, const LaneGeom<K> &g,
                                              const LaneRows<T, COMP, CPL, K> &R, const int q)
{
    constexpr bool NT = sizeof(T) == 8 || BATCH;
    const bool row_ok = q >= g.re[K] && q < g.hi[K];                 // uniform
    const int nbytes = row_ok ? g.span * (int)sizeof(T) : 0;
    const size_t o = (size_t)(row_ok ? (g.flip ? g.ny - 1 - q : q) : 0) * A.pitch + g.o0;
    const int voff = (g.cbase - g.o0) * (int)sizeof(T);           // negative left of the span: out of range
    buffer_store_vec<T, CPL, NT>(A.un + o, nbytes, voff, R.KO[0]);
    buffer_store_vec<T, CPL, NT>(A.vn + o, nbytes, voff, R.KO[1]);
    buffer_store_vec<T, CPL, NT>(A.wn + o, nbytes, voff, R.KO[2]);
    if constexpr (COMP) {
        buffer_store_vec<T, CPL, NT>(A.unlo + o, nbytes, voff, R.KO[3]);
        buffer_store_vec<T, CPL, NT>(A.vnlo + o, nbytes, voff, R.KO[4]);
        buffer_store_vec<T, CPL, NT>(A.wnlo + o, nbytes, voff, R.KO[5]);
    }
}

template <typename T, bool COMP, int CPL, int K, int PH, int S, int RTA, int RTC, bool EDGE, bool BATCH>
__device__ __forceinline__ void level_row(const StepArgs<T> &A, const LaneGeom<K> &g, const ColumnMasks<CPL, EDGE> &m,
                                          LaneRows<T, COMP, CPL, K> &R, TensorRing<T, CPL, RTA, RTC> &L,
                                          const int r, const int ba, const int bc)
{
    const int q = r - 2 * S + 1;
    // Row hi[S] is not computed: it lies past the level's range, or it is row
    // ny, whose mirrored value only the y-difference of row ny-1 would read (the
    // faces through the top boundary are zero), and that difference takes row
    // ny-1 itself.  Leaving every register untouched on this path keeps the
    // register allocator from copying the rings on the common path.
    if (q < g.lo[S] - 1 || q >= g.hi[S]) return;                 // uniform
    constexpr int m3 = pmod(PH - 2 * S, 3), q3 = pmod(PH - 2 * S + 1, 3), p3 = pmod(PH - 2 * S + 2, 3);
    constexpr int q2 = pmod(PH + 1, 2), p2 = pmod(PH, 2);       // rows q and q +- 1
    constexpr int I = S - 1;

    // Row q = lo[S]-1 (the pre-row) runs the same code: what it carries to the
    // next row is the x-difference and right neighbour of row q+1 = lo[S], which
    // the first row needs; its other results are discarded or overwritten (its
    // south-face flux by the warm-up row; below the domain it is 0, the
    // boundary face of row 0).
    const T half = T(0.5), one = T(1);
    const bool has_n = !EDGE || (q >= 0 && q + 1 < g.ny);
    const bool top = EDGE && q + 1 >= g.ny;  // row q+1 is the mirror of row q
    // r = rb + PH with rb a multiple of the unroll period (ba, bc: its ring slots)
    const int ts = ring_slot<RTA, PH - 2 * S + 1>(ba), tp = ring_slot<RTA, PH - 2 * S + 2>(ba);
    const int tc = ring_slot<RTC, PH - 2 * S + 1>(bc);

    T W0[CPL], Wp[CPL], U0[CPL], V0[CPL], TY[CPL], BT[CPL], B0[CPL];
#pragma unroll
    for (int k = 0; k < CPL; ++k) {
        W0[k] = R.W[I][q3][k];
        Wp[k] = R.W[I][p3][k];
        U0[k] = R.U[I][q2][k];
        V0[k] = R.V[I][q2][k];
        B0[k] = L.B[ts][k * kWave + g.own];
        const T Wn = top ? W0[k] : Wp[k];
        TY[k] = (Wn - R.W[I][m3][k]) * A.hy;
        BT[k] = B0[k] * TY[k];
    }
    // shifts: b*ty, u and v from the right; x-difference of row q+1
    const T btR = from_right(BT[0]), uR = from_right(U0[0]), vR = from_right(V0[0]);
    T TXn[CPL], WRn;
    x_difference<T, CPL, EDGE>(Wp, m, A.hx, TXn, WRn);

    // east faces of every column
    T FXe[CPL], GXe[CPL];
#pragma unroll
    for (int k = 0; k < CPL; ++k) {
        const int k1 = k + 1 < CPL ? k + 1 : k;
        const T wr = k + 1 < CPL ? W0[k1] : R.WR[I];
        const T btr = k + 1 < CPL ? BT[k1] : btR;
        const T ur = k + 1 < CPL ? U0[k1] : uR;
        const T vr = k + 1 < CPL ? V0[k1] : vR;
        const T hA = L.hA[ts][k * kWave + g.own];
        const T fx = madd<T, COMP>(hA, (wr - W0[k]) * A.idx, half * (BT[k] + btr));
        const T gx = madd<T, COMP>(-half, U0[k] + ur, one) * ((vr - V0[k]) * A.idx);
        FXe[k] = (!EDGE || m.ve[k]) ? fx : T(0);
        GXe[k] = (!EDGE || m.ve[k]) ? gx : T(0);
    }
    // west face of the first column: the left lane's last east face (0 left of
    // column 0, where that face lies outside the domain)
    const T FXl = from_left(FXe[CPL - 1]), GXl = from_left(GXe[CPL - 1]);

    T ou[CPL], ov[CPL], ow[CPL], oul[CPL], ovl[CPL], owl[CPL];
#pragma unroll
    for (int k = 0; k < CPL; ++k) {
        const T Up = R.U[I][p2][k], Vp = R.V[I][p2][k];
        const T Bp = L.B[tp][k * kWave + g.own], hC = L.hC[tc][k * kWave + g.own];
        const T FXw = k > 0 ? FXe[k > 0 ? k - 1 : 0] : FXl;
        const T GXw = k > 0 ? GXe[k > 0 ? k - 1 : 0] : GXl;
        const T Wc = W0[k], Uc = U0[k], Vc = V0[k];
        const T fy = madd<T, COMP>(hC, (Wp[k] - Wc) * A.idy, half * (B0[k] * R.TX[I][k] + Bp * TXn[k]));
        const T gy = madd<T, COMP>(-half, Uc + Up, one) * ((Vp - Vc) * A.idy);
        const T FYn = has_n ? fy : T(0);
        const T GYn = has_n ? gy : T(0);
        const T divW = (FXe[k] - FXw) * A.idx + (FYn - R.FYs[I][k]) * A.idy;
        const T divV = (GXe[k] - GXw) * A.idx + (GYn - R.GYs[I][k]) * A.idy;
        const T fu = madd<T, COMP>(-(A.d1 * Uc), Wc, Uc * (one - Uc));
        const T fv = madd<T, COMP>(A.D2, divV, (A.r2 * Vc) * (one - Vc));
        const T fw = madd<T, COMP>(A.r3, Vc, -(A.d3 * Wc)) + divW;
        if constexpr (COMP) {
            comp_add(Uc, R.Ul[I][q2][k], A.dt * fu, ou[k], oul[k]);
            comp_add(Vc, R.Vl[I][q2][k], A.dt * fv, ov[k], ovl[k]);
            comp_add(Wc, R.Wl[I][q2][k], A.dt * fw, ow[k], owl[k]);
        } else {
            ou[k] = madd<T, COMP>(A.dt, fu, Uc);
            ov[k] = madd<T, COMP>(A.dt, fv, Vc);
            ow[k] = madd<T, COMP>(A.dt, fw, Wc);
        }
        R.FYs[I][k] = FYn;
        R.GYs[I][k] = GYn;
        R.TX[I][k] = TXn[k];
    }
    R.WR[I] = WRn;

    // A warm-up row's result is written into the ring like any other: the only
    // reader of that ring row is the next level's warm-up row, as the south
    // neighbour whose flux it discards.
    if constexpr (S < K) {
#pragma unroll
        for (int k = 0; k < CPL; ++k) {
            R.W[S][q3][k] = ow[k];
            R.U[S][q2][k] = ou[k];
            R.V[S][q2][k] = ov[k];
            if constexpr (COMP) {
                R.Wl[S][q2][k] = owl[k];
                R.Ul[S][q2][k] = oul[k];
                R.Vl[S][q2][k] = ovl[k];
            }
        }
        if (EDGE && q == 0) {                // mirror row -1 for level S+1
#pragma unroll
            for (int k = 0; k < CPL; ++k) R.W[S][m3][k] = ow[k];
        }
    } else {
        // columns past nx (row padding) are written as zeros
#pragma unroll
        for (int k = 0; k < CPL; ++k) {
            R.KO[0][k] = m.inside[k] ? ou[k] : T(0);
            R.KO[1][k] = m.inside[k] ? ov[k] : T(0);
            R.KO[2][k] = m.inside[k] ? ow[k] : T(0);
            if constexpr (COMP) {
                R.KO[3][k] = m.inside[k] ? oul[k] : T(0);
                R.KO[4][k] = m.inside[k] ? ovl[k] : T(0);
                R.KO[5][k] = m.inside[k] ? owl[k] : T(0);
            }
        }
        if constexpr (!late_store<T, CPL, K>()) store_level_k<T, COMP, CPL, K, BATCH>(A, g, R, q);
    }
}

template <typename T, bool COMP, int CPL, int K, int PH, int RTA, int RTC, bool EDGE, bool BATCH>
__device__ __forceinline__ void lane_iter(const StepArgs<T> &A, const LaneGeom<K> &g, const ColumnMasks<CPL, EDGE> &m,
                                          LaneRows<T, COMP, CPL, K> &R, TensorRing<T, CPL, RTA, RTC> &L,
                                          const int r, const int r_start, const int r_end, const int ba,
                                          const int bc)
{
    if (r < r_start || r > r_end) return;                        // uniform
    if constexpr (K >= 4) level_row<T, COMP, CPL, K, PH, 4, RTA, RTC, EDGE, BATCH>(A, g, m, R, L, r, ba, bc);
    if constexpr (K >= 3) level_row<T, COMP, CPL, K, PH, 3, RTA, RTC, EDGE, BATCH>(A, g, m, R, L, r, ba, bc);
    if constexpr (K >= 2) level_row<T, COMP, CPL, K, PH, 2, RTA, RTC, EDGE, BATCH>(A, g, m, R, L, r, ba, bc);

    // tensor row r (requested one iteration ago) into the ring; the c face sum
    // of row r-1 needs row r
    if (r >= r_start + 1 && r <= g.last0) {
        const T half = T(0.5);
        const T aRs = from_right(R.ta[0]);
        const int ts = ring_slot<RTA, PH>(ba), tm = ring_slot<RTC, PH - 1>(bc);
#pragma unroll
        for (int k = 0; k < CPL; ++k) {
            const T ar = k + 1 < CPL ? R.ta[k + 1 < CPL ? k + 1 : k] : aRs;
            L.hA[ts][k * kWave + g.own] = half * (R.ta[k] + ar);
            const T bneg = -R.tb[k];
            L.B[ts][k * kWave + g.own] = g.flip ? bneg : R.tb[k];
            L.hC[tm][k * kWave + g.own] = half * (R.cprev[k] + R.tc[k]);
            R.cprev[k] = R.tc[k];
        }
    }
    if constexpr (late_store<T, CPL, K>()) store_level_k<T, COMP, CPL, K, BATCH>(A, g, R, r - 2 * K + 1);
    level_row<T, COMP, CPL, K, PH, 1, RTA, RTC, EDGE, BATCH>(A, g, m, R, L, r, ba, bc);

    // request old-state row r+1 (clamped: rows -1 and ny load their mirrors).
    // The plain FP32 single-context kernel loads its rows non-temporally
    // (measured on MI355X: 441 -> 471 Gcell-updates/s at 4096^2); FP64 and the
    // compensated state measured 4.5% and 14% slower that way.
    if (r + 1 <= g.last0) {
        constexpr bool NTL = sizeof(T) == 4 && !COMP && !BATCH;
        const int row = min(max(r + 1, 0), g.ny - 1);
        const size_t base = (size_t)(g.flip ? g.ny - 1 - row : row) * A.pitch + g.lcol;
        constexpr int w1 = pmod(PH + 1, 3), u1 = pmod(PH + 1, 2);
        load_vec<T, CPL, NTL>(A.w + base, R.W[0][w1]);
        load_vec<T, CPL, NTL>(A.u + base, R.U[0][u1]);
        load_vec<T, CPL, NTL>(A.v + base, R.V[0][u1]);
        if constexpr (COMP) {
            load_vec<T, CPL>(A.wlo + base, R.Wl[0][u1]);
            load_vec<T, CPL>(A.ulo + base, R.Ul[0][u1]);
            load_vec<T, CPL>(A.vlo + base, R.Vl[0][u1]);
        }
        load_vec<T, CPL, NTL>(A.a + base, R.ta);
        load_vec<T, CPL, NTL>(A.b + base, R.tb);
        load_vec<T, CPL, NTL>(A.c + base, R.tc);
    }
}

template <int CPL, int K>
struct DppShape {
    static constexpr int TXW = kWave * CPL;               // columns a wave holds
    static constexpr int H = (K + CPL - 1) / CPL * CPL;   // halo columns on each side
    static constexpr int OUTW = TXW - 2 * H;              // output columns per workgroup
    static constexpr int RTA = K >= 2 ? 2 * K - 1 : 2;     // rows of the (a+a')/2 and b rings
    static constexpr int RTC = K >= 2 ? 2 * K - 2 : 1;     // rows of the (c+c')/2 ring
};

// Strips of odd index sweep downward: row j of the grid is row ny-1-j of the
// sweep, and b enters negated.  Mirroring the rows turns every y-face flux and
// every y-difference into its exact negative (sums commute, differences swap
// sign, and b*ty keeps its sign), so the update of every cell is the same
// bits either way.  Vertically neighbouring strips then reach the halo rows
// they share at the same time (both at the end or both at the start of their
// sweeps), so the second read finds them in L2.
__device__ __forceinline__ bool strip_flips(const int sy) { return (sy & 1) != 0; }

// Rows [j0, j1) of strip sy, in the rows of its sweep.
__device__ __forceinline__ void strip_rows(const int ny, const int rows, const int sy, int &j0, int &j1)
{
    const int p0 = sy * rows, p1 = min(ny, p0 + rows);
    j0 = strip_flips(sy) ? ny - p1 : p0;
    j1 = strip_flips(sy) ? ny - p0 : p1;
}

// One workgroup's strip: output columns [sx*OUTW, sx*OUTW + OUTW) of rows
// [sy*A.rows, sy*A.rows + A.rows), K steps from A's input to A's output planes.
template <typename T, bool COMP, int CPL, int K, bool EDGE, bool BATCH>
__device__ __forceinline__ void dpp_strip(const StepArgs<T> &A, const int sx, const int sy,
                                          TensorRing<T, CPL, DppShape<CPL, K>::RTA, DppShape<CPL, K>::RTC> &L)
{
    using Sh = DppShape<CPL, K>;
    constexpr int RTA = Sh::RTA, RTC = Sh::RTC;
    static_assert(K >= 1 && K <= 4, "fused depth 1..4");
    const int o0 = sx * Sh::OUTW, e0 = o0 - Sh::H;
    LaneGeom<K> g;
    g.nx = A.nx;
    g.ny = A.ny;
    g.own = threadIdx.x;
    g.cbase = e0 + (int)threadIdx.x * CPL;
    g.lcol = min(max(g.cbase, 0), A.pitch - CPL);
    g.o0 = o0;
    g.span = min(Sh::OUTW, A.pitch - o0);
    g.flip = strip_flips(sy);
    int j0, j1;
    strip_rows(g.ny, A.rows, sy, j0, j1);
#pragma unroll
    for (int s = 1; s <= K; ++s) {
        g.lo[s] = max(0, j0 - (K - s) - 1);
        g.re[s] = max(0, j0 - (K - s));
        g.hi[s] = min(g.ny, j1 + (K - s));
    }
    g.lo[0] = g.re[0] = g.hi[0] = 0;
    g.last0 = g.hi[1];                     // last old-state row level 1 reads
    ColumnMasks<CPL, EDGE> m;
#pragma unroll
    for (int k = 0; k < CPL; ++k) {
        const int i = g.cbase + k;
        m.ve[k] = i >= 0 && i + 1 < g.nx;
        m.he[k] = i + 1 < g.nx;
        m.inside[k] = i < g.nx;
    }
    m.hw0 = g.cbase > 0;

    LaneRows<T, COMP, CPL, K> R;
#pragma unroll
    for (int s = 0; s < K; ++s) {
#pragma unroll
        for (int k = 0; k < CPL; ++k) {
#pragma unroll
            for (int j = 0; j < 3; ++j) R.W[s][j][k] = T(0);
#pragma unroll
            for (int j = 0; j < 2; ++j) {
                R.U[s][j][k] = T(0);
                R.V[s][j][k] = T(0);
                if constexpr (COMP) {
                    R.Wl[s][j][k] = T(0);
                    R.Ul[s][j][k] = T(0);
                    R.Vl[s][j][k] = T(0);
                }
            }
            R.TX[s][k] = T(0);
            R.FYs[s][k] = T(0);
            R.GYs[s][k] = T(0);
        }
        R.WR[s] = T(0);
    }
#pragma unroll
    for (int k = 0; k < CPL; ++k) R.ta[k] = R.tb[k] = R.tc[k] = R.cprev[k] = T(0);

    // two load-only iterations: rows lo[1]-1 (row -1 mirrors row 0) and lo[1];
    // level 1 takes the x-difference of row lo[1] at r = lo[1]
    const int r_start = g.lo[1] - 2;
    const int r_end = g.hi[K] + 2 * K - 2;
    const int r0 = r_start - pmod(r_start, kPeriod);
    // Two waves share each SIMD, and among waves of equal priority the
    // instruction arbiter issues the older one first: measured on MI355X (4096²
    // FP64, one round of strips), the older wave of every SIMD pair finished
    // first, the younger one took 1.3-1.55 times as long, and for the last third
    // of the launch one wave per SIMD was left, which moves fewer bytes per
    // second.  The younger wave (odd slot in the SIMD's wave list) therefore
    // runs at raised priority for the first half of its sweep and at the common
    // one after it, so the two finish closer together.  Only the issue order
    // changes, not the arithmetic.  The compensated-FP32 ensemble kernel (many
    // rounds of short strips) measured 3.6% slower with it and runs without.
    constexpr bool raise_younger = !(BATCH && COMP);
    const unsigned int slot = __builtin_amdgcn_s_getreg(kHwIdWaveSlotBit0) & 1u;
    const int r_half = r_start + (r_end - r_start) / 2;
    for (int rb = r0; rb <= r_end; rb += kPeriod) {
        if (raise_younger && slot != 0u && rb < r_half) __builtin_amdgcn_s_setprio(1);
        else __builtin_amdgcn_s_setprio(0);
        const int ba = ring_base<RTA>(rb), bc = ring_base<RTC>(rb);
        lane_iter<T, COMP, CPL, K, 0, RTA, RTC, EDGE, BATCH>(A, g, m, R, L, rb + 0, r_start, r_end, ba, bc);
        lane_iter<T, COMP, CPL, K, 1, RTA, RTC, EDGE, BATCH>(A, g, m, R, L, rb + 1, r_start, r_end, ba, bc);
        lane_iter<T, COMP, CPL, K, 2, RTA, RTC, EDGE, BATCH>(A, g, m, R, L, rb + 2, r_start, r_end, ba, bc);
        lane_iter<T, COMP, CPL, K, 3, RTA, RTC, EDGE, BATCH>(A, g, m, R, L, rb + 3, r_start, r_end, ba, bc);
        lane_iter<T, COMP, CPL, K, 4, RTA, RTC, EDGE, BATCH>(A, g, m, R, L, rb + 4, r_start, r_end, ba, bc);
        lane_iter<T, COMP, CPL, K, 5, RTA, RTC, EDGE, BATCH>(A, g, m, R, L, rb + 5, r_start, r_end, ba, bc);
    }
}

// Whether strip (sx, sy) keeps every column of the wave and every row that any
// level touches (warm-up rows included) clear of the domain boundary.
template <int CPL, int K, typename T>
__device__ __forceinline__ bool strip_interior(const StepArgs<T> &A, const int sx, const int sy)
{
    using Sh = DppShape<CPL, K>;
    const int e0 = sx * Sh::OUTW - Sh::H;
    int j0, j1;
    strip_rows(A.ny, A.rows, sy, j0, j1);
    return e0 >= 1 && e0 + Sh::TXW < A.nx && j0 >= K + 2 && j1 + K < A.ny;
}

// Interior strips run a copy of the sweep with the boundary masks compiled
// out: for the plain state with 8-byte lanes, and for plain FP32 with wide
// lanes (measured +1.5-2% on MI355X, where the kernel is at the vector issue
// limit).  The FP64 wide-lane sweep measured 2.5% slower with two copies, and
// the compensated sweep is the largest: they keep one copy.
template <typename T, bool COMP, int CPL, int K, bool BATCH>
__device__ __forceinline__ void run_strip(const StepArgs<T> &A, const int sx, const int sy,
                                          TensorRing<T, CPL, DppShape<CPL, K>::RTA, DppShape<CPL, K>::RTC> &L)
{
    if constexpr ((sizeof(T) * CPL <= 8 || sizeof(T) == 4) && !COMP) {
        if (strip_interior<CPL, K>(A, sx, sy)) {                // uniform
            dpp_strip<T, COMP, CPL, K, false, BATCH>(A, sx, sy, L);
            return;
        }
    }
    dpp_strip<T, COMP, CPL, K, true, BATCH>(A, sx, sy, L);
}

template <typename T, bool COMP, int CPL, int K>
__global__ __launch_bounds__(kWave) __attribute__((amdgpu_waves_per_eu(2))) void fused_dpp_kernel(StepArgs<T> A)
{
    __shared__ TensorRing<T, CPL, DppShape<CPL, K>::RTA, DppShape<CPL, K>::RTC> L;
    const int nbx = gridDim.x;
    const int lid = xcd_local_id(blockIdx.x + nbx * blockIdx.y, gridDim.x * gridDim.y);
    run_strip<T, COMP, CPL, K, false>(A, lid % nbx, lid / nbx, L);
}

// Ensemble form: the workgroups of all instances in one launch.  Instance i owns
// the work items [prefix[i], prefix[i+1]) and its own step description D[i]
// (sizes, planes, parameters, dt and strip height).
template <typename T, bool COMP, int CPL, int K>
__global__ __launch_bounds__(kWave) __attribute__((amdgpu_waves_per_eu(2))) void fused_dpp_batch_kernel(const StepArgs<T> *__restrict__ D,
                                                                const int *__restrict__ prefix, int n)
{
    __shared__ TensorRing<T, CPL, DppShape<CPL, K>::RTA, DppShape<CPL, K>::RTC> L;
    const int lid = xcd_local_id(blockIdx.x, gridDim.x);
    int lo = 0, hi = n;                    // prefix[lo] <= lid < prefix[hi]
    while (hi - lo > 1) {
        const int mid = (lo + hi) >> 1;
        if (prefix[mid] <= lid) lo = mid;
        else hi = mid;
    }
    const StepArgs<T> A = D[lo];
    const int nbx = (A.nx + DppShape<CPL, K>::OUTW - 1) / DppShape<CPL, K>::OUTW;
    const int local = lid - prefix[lo];
    run_strip<T, COMP, CPL, K, true>(A, local % nbx, local / nbx, L);
}

// Resident one-wave workgroups of a lane-shift kernel per CU (its registers and
// LDS ring decide), queried once per kernel.
template <typename T, bool COMP, int CPL, int K>
int lane_shift_blocks_per_cu()
{
    static const int n = [] {
        int b = 0;
        if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&b, fused_dpp_kernel<T, COMP, CPL, K>, kWave, 0) !=
                hipSuccess ||
            b < 1)
            b = 1;
        return b;
    }();
    return n;
}

// The tallest strips whose waves still fill the resident slots rounds2/2 times
// over, so that the last round is not a partial one: every strip repeats the
// 2K+2-row pipeline fill, and a partial last round leaves CUs idle.  Never
// below 8K rows nor above ny.
template <typename T, bool COMP, int CPL, int K>
int fit_rows_typed(const ggfv_ctx *ctx, int rounds2)
{
    constexpr int OUTW = DppShape<CPL, K>::OUTW;
    const long nbx = (ctx->nx + OUTW - 1) / OUTW;
    const long slots = (long)lane_shift_blocks_per_cu<T, COMP, CPL, K>() * (ctx->cus > 0 ? ctx->cus : 1);
    long strips = slots * rounds2 / 2 / nbx;
    if (strips < 1) strips = 1;
    long rows = (ctx->ny + strips - 1) / strips;
    if (rows < 8 * K) rows = 8 * K;
    if (rows > ctx->ny) rows = ctx->ny;
    return (int)rows;
}

template <typename T, bool COMP, int CPL, int K>
hipError_t launch_dpp_typed(ggfv_ctx *ctx, const void *in, void *out, double dt)
{
    constexpr int OUTW = DppShape<CPL, K>::OUTW;
    const int nbx = (ctx->nx + OUTW - 1) / OUTW;
    int rows = ctx->rows_per_strip;
    if (rows <= 0) rows = fit_rows_typed<T, COMP, CPL, K>(ctx, 2);
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

template <typename T, bool COMP, int CPL, int K>
hipError_t launch_dpp_batch_typed(const BatchLaunch &b, hipStream_t stream)
{
    hipLaunchKernelGGL((fused_dpp_batch_kernel<T, COMP, CPL, K>), dim3(b.items), dim3(kWave), 0, stream,
                       static_cast<const StepArgs<T> *>(b.desc), b.prefix, b.n);
    return hipGetLastError();
}

template <typename T, bool COMP, int CPL>
hipError_t launch_dpp_batch_depth(const BatchLaunch &b, hipStream_t stream)
{
    switch (b.fused) {
    case 1: return launch_dpp_batch_typed<T, COMP, CPL, 1>(b, stream);
    case 2: return launch_dpp_batch_typed<T, COMP, CPL, 2>(b, stream);
    case 3: return launch_dpp_batch_typed<T, COMP, CPL, 3>(b, stream);
    case 4: return launch_dpp_batch_typed<T, COMP, CPL, 4>(b, stream);
    default: return hipErrorInvalidValue;
    }
}

template <typename T, bool COMP, int CPL>
int fit_rows_depth(const ggfv_ctx *ctx, int K, int rounds2)
{
    switch (K) {
    case 1: return fit_rows_typed<T, COMP, CPL, 1>(ctx, rounds2);
    case 2: return fit_rows_typed<T, COMP, CPL, 2>(ctx, rounds2);
    case 3: return fit_rows_typed<T, COMP, CPL, 3>(ctx, rounds2);
    default: return fit_rows_typed<T, COMP, CPL, 4>(ctx, rounds2);
    }
}

}  // namespace
}  // namespace ggfv

#endif  // GGFV_FUSED_DPP_HPP
