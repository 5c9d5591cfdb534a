// ggfv3.hip -- the three-dimensional form of the explicit finite-volume step.
//
// The scheme of Section 2 (eq. (3)) with the same flux form in three
// directions: acid faces with the full symmetric tensor (19-point stencil),
// tumour-cell faces with the mobility 1 - (U_l + U_r)/2 (7 points), the
// reactions and the forward-Euler update of the 2D scheme, zero flux through
// boundary faces and the boundary cell as its own missing neighbour in the
// tangential differences.
//
// Layout: a plane of a field is ny rows of `pitch` values (nx rounded up to
// 64), x fastest.  The fields of one plane lie next to each other: the state
// buffer holds plane k of u, v, w at planes 3k, 3k+1, 3k+2, the tensor buffer
// plane k of axx, ayy, azz, axy, axz, ayz at planes 6k .. 6k+5.  Two state
// buffers alternate.  A kernel then reaches every field of a plane through one
// buffer resource (a scalar base) and a scalar field offset.
//
// Step kernel (one wave per workgroup, a pencil of cells):
//   * the 64 lanes of a wave hold 64 adjacent columns x0-1 .. x0+62; lanes 1..62
//     produce output, lanes 0 and 63 only supply neighbour values, so strips of
//     62 columns tile x;
//   * each lane holds R adjacent rows j0..j0+R-1 plus the rows j0-1 and j0+R
//     that the y-faces and tangential differences need, and the wave marches
//     up a strip of planes k0..k1-1, starting one plane early (at k0-1, no
//     output) to produce the flux through the strip's bottom face;
//   * x-neighbours come from the neighbouring lane through DPP wave shifts;
//     every x-face flux is evaluated once, by the cell on its left, and passed
//     to the cell on its right; every z-face flux once, by the cell below, and
//     carried in registers to the next plane; the two y-faces at the ends of a
//     row group are also evaluated by the neighbouring groups, from the same
//     operands in the same order;
//   * the state of plane k+1, the tz-difference of plane k and the tensor
//     entries of plane k+1 that the z-face needs are carried in registers, and
//     in FP64 so are u, v and ayz of the halo rows, read one plane ahead
//     together with the neighbouring groups that own them;
//     every input value enters the wave once per plane (halo rows and halo
//     lanes aside), and the neighbouring row groups of a plane run on the same
//     XCD so that halo rows come from its L2.
// Rows and columns outside the grid are read clamped to the last row or column
// (the mirrored ghost value of the tangential differences); their results are
// not stored.  The arithmetic order is
//   FX(i+1/2) = 0.5*(axx_l + axx_r)*((W_r - W_l)*idx)
//             + 0.5*(axy_l*ty_l + axy_r*ty_r) + 0.5*(axz_l*tz_l + axz_r*tz_r)
//   (FY, FZ alike), GX = (1 - 0.5*(U_l + U_r))*((V_r - V_l)*idx),
//   divW = ((FX_e - FX_w)*idx + (FY_n - FY_s)*idy) + (FZ_t - FZ_b)*idz,
// with no contraction into FMA, so FP64 results equal a plain CPU loop's.

#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <new>
#include <string>

#include "ggfv3.h"
#include "ggfv_dpp.hpp"
#include "ggfv_internal.hpp"

struct ggfv3_ctx {
    int nx = 0, ny = 0, nz = 0, pitch = 0;
    double lx = 1.0, ly = 1.0, lz = 1.0;
    int dtype = 0, device = 0;
    hipStream_t stream = nullptr;
    size_t plane = 0;              // values per plane of one field (ny * pitch)
    size_t elem = 0;               // bytes per value
    void *state[2] = {nullptr, nullptr};
    int cur = 0;
    void *tensor = nullptr;        // 6 fields, plane-interleaved
    void *staging = nullptr;       // dense io arrays (FP64-sized)
    size_t staging_bytes = 0;
    double *scratch = nullptr;     // reduction partials and results
    ggfv_params prm{};
    bool has_params = false, has_tensor = false, has_state = false;
    double t = 0.0;
    long long steps = 0;
    int zs = 0;                    // planes per strip (0: default)
    int rows = 0;                  // rows per wave (0: default)
    int wx = 0, wy = 0;            // waves per workgroup along x, y (0: default)
    std::string err;
};

namespace {

thread_local std::string g3_create_error;
constexpr int kRed3 = 256;         // reduction workgroup
constexpr int kRed3Blocks = 512;   // reduction partial blocks
constexpr int kRed3Slots = 5;      // three state sums, the Gershgorin max, non-definite cells

int fail3(ggfv3_ctx *ctx, int code, const char *fmt, ...) __attribute__((format(printf, 3, 4)));

int fail3(ggfv3_ctx *ctx, int code, const char *fmt, ...)
{
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    if (ctx)
        ctx->err = buf;
    else
        g3_create_error = buf;
    return code;
}

#define GGFV3_HIP(ctx, call)                                                                 \
    do {                                                                                     \
        hipError_t e_ = (call);                                                              \
        if (e_ != hipSuccess)                                                                \
            return fail3((ctx), GGFV_EHIP, "%s failed: %s", #call, hipGetErrorString(e_));   \
    } while (0)

struct Guard3 {
    int prev = -1;
    explicit Guard3(int dev)
    {
        (void)hipGetDevice(&prev);
        (void)hipSetDevice(dev);
    }
    ~Guard3()
    {
        if (prev >= 0) (void)hipSetDevice(prev);
    }
};

template <typename T>
struct Step3Args {
    const T *s;                    // state in (u, v, w interleaved by plane)
    T *o;                          // state out
    const T *t;                    // tensor (axx, ayy, azz, axy, axz, ayz interleaved by plane)
    int nx, ny, nz, pitch, zs;
    unsigned pb;                   // bytes per plane of one field
    T idx, idy, idz, hx, hy, hz, dt;
    T d1, r2, D2, r3, d3;
};

constexpr int kStrip = 62;     // output columns per wave

__device__ __forceinline__ int xcd_local_id3(int bid, int nb)
{
    // workgroups are dealt round-robin to the eight XCDs: give each XCD one
    // contiguous range of pencils
    const int xcd = bid & 7, q = nb >> 3, rem = nb & 7;
    return xcd * q + min(xcd, rem) + (bid >> 3);
}

// Loads and stores through a buffer resource per plane group (wave-uniform base
// and size in scalar registers), a scalar field offset and a 32-bit per-lane
// byte offset, so no lane keeps a 64-bit address.  A plane group holds fewer
// than 2^32 bytes.
typedef unsigned int u32x2_t __attribute__((ext_vector_type(2)));
constexpr int kRsrcWord3 = 0x00020000;          // raw buffer, 32-bit data format

__device__ __forceinline__ __amdgpu_buffer_rsrc_t group_rsrc(const void *base, unsigned bytes)
{
    return __builtin_amdgcn_make_buffer_rsrc(const_cast<void *>(base), (short)0, (int)bytes, kRsrcWord3);
}

template <typename T>
__device__ __forceinline__ T gld(__amdgpu_buffer_rsrc_t r, unsigned voff, unsigned soff);

template <>
__device__ __forceinline__ double gld<double>(__amdgpu_buffer_rsrc_t r, unsigned voff, unsigned soff)
{
    return __builtin_bit_cast(double, __builtin_amdgcn_raw_buffer_load_b64(r, voff, soff, 0));
}

template <>
__device__ __forceinline__ float gld<float>(__amdgpu_buffer_rsrc_t r, unsigned voff, unsigned soff)
{
    return __builtin_bit_cast(float, __builtin_amdgcn_raw_buffer_load_b32(r, voff, soff, 0));
}

__device__ __forceinline__ void gst(__amdgpu_buffer_rsrc_t r, unsigned voff, unsigned soff, double v)
{
    __builtin_amdgcn_raw_buffer_store_b64(__builtin_bit_cast(u32x2_t, v), r, voff, soff, 0);
}

__device__ __forceinline__ void gst(__amdgpu_buffer_rsrc_t r, unsigned voff, unsigned soff, float v)
{
    __builtin_amdgcn_raw_buffer_store_b32(__builtin_bit_cast(unsigned, v), r, voff, soff, 0);
}

// Pencils of one workgroup: wx x-strips by wy row groups, marching in step (one
// barrier per plane) so that the columns and rows they share are read from
// the caches at about the same time.
struct PencilGrid {
    int nbx, nby, nzb;             // workgroups along x, y, z
    int wx, wy;                    // waves per workgroup along x, y
};

constexpr int kMaxWaves3 = 8;

template <typename T, int R>
__global__ __launch_bounds__(64 * kMaxWaves3) void step3_pencil_kernel(Step3Args<T> A, PencilGrid G)
{
    using ggfv::from_left;
    using ggfv::from_right;
    constexpr int NR = R + 2;                      // rows held: j0-1 .. j0+R
    // FP64: read u, v, ayz of the halo rows one plane ahead (see below); FP32's
    // working set stays in L2 either way, and the later read is faster there
    constexpr bool AHEAD = sizeof(T) == 8;
    // FP32 with four rows per wave issues all of a plane's loads in one round
    // trip (11% faster than reading the face tensors in the output branch).
    // FP64 keeps them there: with two rows the early loads raise the registers
    // from 168 to 170, one wave per SIMD fewer, and the step is slower; with
    // four they spill.  FP32 with one or two rows measured no gain.
    // FP64 recomputes the x-difference of w of its own rows every plane instead
    // of carrying it (fewer live registers: two-row waves keep three waves per
    // SIMD while loading axx before the first store of a plane); FP32 carries it.
    constexpr bool RTX = sizeof(T) == 8;
    constexpr bool EARLY = sizeof(T) == 4 && R == 4;
    const int lid = xcd_local_id3(blockIdx.x, G.nbx * G.nby * G.nzb);
    const int bx = lid % G.nbx, rest = lid / G.nbx;
    const int by = rest % G.nby, zb = rest / G.nby;
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int sx = bx * G.wx + wave % G.wx;        // strips and row groups past the grid
    const int gy = by * G.wy + wave / G.wx;        // read clamped and store nothing
    const bool sync = G.wx * G.wy > 1;
    const int x = sx * kStrip - 1 + lane;
    const int xl = min(max(x, 0), A.nx - 1);
    const bool east_edge = x >= A.nx - 1, west_edge = x <= 0;
    const bool out_lane = lane >= 1 && lane <= kStrip && x < A.nx;
    const int j0 = gy * R;
    const int k0 = zb * A.zs, k1 = min(A.nz, k0 + A.zs);
    const size_t P = (size_t)A.ny * A.pitch;
    const unsigned PB = A.pb;
    // field offsets within a plane group
    const unsigned fU = 0, fV = PB, fW = 2 * PB;
    const unsigned fXX = 0, fYY = PB, fZZ = 2 * PB, fXY = 3 * PB, fXZ = 4 * PB, fYZ = 5 * PB;
    const T half = T(0.5), one = T(1);
    auto state_at = [&](int k) { return group_rsrc(A.s + (size_t)k * 3 * P, 3 * PB); };
    auto tensor_at = [&](int k) { return group_rsrc(A.t + (size_t)k * 6 * P, 6 * PB); };

    unsigned off[NR];                              // clamped byte offsets within a plane
    bool face_ok[R + 1];                           // y-face between rows f and f+1 inside the grid
    bool row_ok[NR];
#pragma unroll
    for (int r = 0; r < NR; ++r) {
        const int j = j0 - 1 + r;
        off[r] = (unsigned)(min(max(j, 0), A.ny - 1) * A.pitch + xl) * (unsigned)sizeof(T);
        row_ok[r] = j < A.ny;
    }
#pragma unroll
    for (int f = 0; f <= R; ++f) face_ok[f] = (j0 - 1 + f) >= 0 && (j0 + f) <= A.ny - 1;

    const int kstart = k0 > 0 ? k0 - 1 : 0;
    // registers carried from plane to plane
    T Wc[NR], Wn[NR], TZc[NR];                     // w of planes k and k+1, tz of plane k
    T Uc[NR], Vc[NR];                              // u, v of plane k (own rows carried)
    T zz[NR], xz[NR], yz[NR];                      // azz, axz, ayz of plane k (own rows carried)
    T TXc[NR];                                     // tx of plane k, own rows (carried when !RTX)
    T FZb[NR], GZb[NR];                            // fluxes through the bottom faces
    {
        const auto Sm = state_at(max(kstart - 1, 0)), Sc = state_at(kstart);
        const auto Sn = state_at(min(kstart + 1, A.nz - 1));
        const auto Tc = tensor_at(kstart);
#pragma unroll
        for (int r = 0; r < NR; ++r) {
            Wc[r] = gld<T>(Sc, off[r], fW);
            Wn[r] = gld<T>(Sn, off[r], fW);
            const T m = gld<T>(Sm, off[r], fW);
            TZc[r] = (Wn[r] - m) * A.hz;
        }
#pragma unroll
        for (int r = 1; r <= R; ++r) {
            if constexpr (!RTX) {
                const T e = from_right(Wc[r]), w = from_left(Wc[r]);
                const T er = east_edge ? Wc[r] : e;
                const T wl = west_edge ? Wc[r] : w;
                TXc[r] = (er - wl) * A.hx;
            }
            Uc[r] = gld<T>(Sc, off[r], fU);
            Vc[r] = gld<T>(Sc, off[r], fV);
            zz[r] = gld<T>(Tc, off[r], fZZ);
            xz[r] = gld<T>(Tc, off[r], fXZ);
            yz[r] = gld<T>(Tc, off[r], fYZ);
            FZb[r] = T(0);
            GZb[r] = T(0);
        }
        if constexpr (AHEAD) {
#pragma unroll
            for (int r = 0; r < NR; r += R + 1) {
                Uc[r] = gld<T>(Sc, off[r], fU);
                Vc[r] = gld<T>(Sc, off[r], fV);
                yz[r] = gld<T>(Tc, off[r], fYZ);
            }
        }
    }

    for (int k = kstart; k < k1; ++k) {
        const bool top = k + 1 < A.nz;
        const auto Sn = state_at(min(k + 1, A.nz - 1)), S2 = state_at(min(k + 2, A.nz - 1));
        const auto Tn = tensor_at(min(k + 1, A.nz - 1));
        // w of plane k+2 -> tz of plane k+1
        T W2[NR], TZn[NR];
#pragma unroll
        for (int r = 0; r < NR; ++r) {
            W2[r] = gld<T>(S2, off[r], fW);
            TZn[r] = (W2[r] - Wc[r]) * A.hz;
        }
        // values of plane k+1: the top faces' (own rows), and (AHEAD) u, v, ayz
        // of the halo rows, which the y-faces of plane k+1 need one iteration
        // later.  Reading those together with the neighbouring groups, which
        // read the same rows as their own now, keeps the re-read within the
        // L2's reach: a plane-iteration later, an FP64 XCD has streamed about
        // its L2's size and they would have been evicted.
        T Un[NR], Vn[NR], zzn[NR], xzn[NR], yzn[NR];
        constexpr int r0 = AHEAD ? 0 : 1, r1 = AHEAD ? NR : R + 1;
#pragma unroll
        for (int r = r0; r < r1; ++r) {
            Un[r] = gld<T>(Sn, off[r], fU);
            Vn[r] = gld<T>(Sn, off[r], fV);
            yzn[r] = gld<T>(Tn, off[r], fYZ);
        }
#pragma unroll
        for (int r = 1; r <= R; ++r) {
            zzn[r] = gld<T>(Tn, off[r], fZZ);
            xzn[r] = gld<T>(Tn, off[r], fXZ);
        }
        // the x- and y-face tensor entries of plane k and (not AHEAD) u, v, ayz
        // of its halo rows
        const auto Tk = tensor_at(k);
        T yy[NR], xy[NR], xx[NR];
        auto load_plane_k = [&]() {
#pragma unroll
            for (int r = 0; r < NR; ++r) {
                yy[r] = gld<T>(Tk, off[r], fYY);
                xy[r] = gld<T>(Tk, off[r], fXY);
            }
            // axx of every own row before the plane's first store: a load issued
            // after a store waits for that store too (the memory counter drains
            // in order).  Four FP64 rows load it at its use instead, for the
            // registers.
            if constexpr (EARLY || R <= 2) {
#pragma unroll
                for (int r = 1; r <= R; ++r) xx[r] = gld<T>(Tk, off[r], fXX);
            }
            if constexpr (!AHEAD) {
                const auto Sk = state_at(k);
#pragma unroll
                for (int r = 0; r < NR; r += R + 1) {
                    Uc[r] = gld<T>(Sk, off[r], fU);
                    Vc[r] = gld<T>(Sk, off[r], fV);
                    yz[r] = gld<T>(Tk, off[r], fYZ);
                }
            }
        };
        if constexpr (EARLY) {
            // issued with the loads above, so that one memory round trip
            // serves the whole plane.  The empty statement that may write
            // memory keeps them here: the optimizer would otherwise move each
            // load next to its only use in the output branch below, where it
            // waits for a second (and third) round trip.  It emits no
            // instruction and no wait.
            load_plane_k();
            asm volatile("" ::: "memory");
        }
        // tx of plane k, own rows
        T TX[NR];
#pragma unroll
        for (int r = 1; r <= R; ++r) {
            if constexpr (RTX) {
                const T e = from_right(Wc[r]), w = from_left(Wc[r]);
                const T er = east_edge ? Wc[r] : e;
                const T wl = west_edge ? Wc[r] : w;
                TX[r] = (er - wl) * A.hx;
            } else {
                TX[r] = TXc[r];
            }
        }
        // top faces (also in the warm-up plane)
        T FZt[NR], GZt[NR], TXn[NR];
#pragma unroll
        for (int r = 1; r <= R; ++r) {
            const T ty = (Wc[r + 1] - Wc[r - 1]) * A.hy;
            const T tyn = (Wn[r + 1] - Wn[r - 1]) * A.hy;
            const T e = from_right(Wn[r]), w = from_left(Wn[r]);
            const T er = east_edge ? Wn[r] : e;
            const T wl = west_edge ? Wn[r] : w;
            TXn[r] = (er - wl) * A.hx;
            const T fz = half * (zz[r] + zzn[r]) * ((Wn[r] - Wc[r]) * A.idz) + half * (xz[r] * TX[r] + xzn[r] * TXn[r]) +
                         half * (yz[r] * ty + yzn[r] * tyn);
            const T gz = (one - half * (Uc[r] + Un[r])) * ((Vn[r] - Vc[r]) * A.idz);
            FZt[r] = top ? fz : T(0);
            GZt[r] = top ? gz : T(0);
        }
        if (k >= k0) {                             // wave-uniform
            if constexpr (!EARLY) load_plane_k();
            // plane k: tx of the halo rows
#pragma unroll
            for (int r = 0; r < NR; r += R + 1) {
                const T e = from_right(Wc[r]), w = from_left(Wc[r]);
                const T er = east_edge ? Wc[r] : e;
                const T wl = west_edge ? Wc[r] : w;
                TX[r] = (er - wl) * A.hx;
            }
            // y-faces f between rows f and f+1
            T FY[R + 1], GY[R + 1];
#pragma unroll
            for (int f = 0; f <= R; ++f) {
                const T fy = half * (yy[f] + yy[f + 1]) * ((Wc[f + 1] - Wc[f]) * A.idy) +
                             half * (xy[f] * TX[f] + xy[f + 1] * TX[f + 1]) + half * (yz[f] * TZc[f] + yz[f + 1] * TZc[f + 1]);
                const T gy = (one - half * (Uc[f] + Uc[f + 1])) * ((Vc[f + 1] - Vc[f]) * A.idy);
                FY[f] = face_ok[f] ? fy : T(0);
                GY[f] = face_ok[f] ? gy : T(0);
            }
            const auto Ok = group_rsrc(A.o + (size_t)k * 3 * P, 3 * PB);
#pragma unroll
            for (int r = 1; r <= R; ++r) {
                if constexpr (!EARLY && R > 2) xx[r] = gld<T>(Tk, off[r], fXX);   // at its use: fewer live registers
                const T ty = (Wc[r + 1] - Wc[r - 1]) * A.hy;
                const T xxE = from_right(xx[r]), xyE = from_right(xy[r]), xzE = from_right(xz[r]);
                const T wE = from_right(Wc[r]), tyE = from_right(ty), tzE = from_right(TZc[r]);
                const T uE = from_right(Uc[r]), vE = from_right(Vc[r]);
                const T fx = half * (xx[r] + xxE) * ((wE - Wc[r]) * A.idx) + half * (xy[r] * ty + xyE * tyE) +
                             half * (xz[r] * TZc[r] + xzE * tzE);
                const T gx = (one - half * (Uc[r] + uE)) * ((vE - Vc[r]) * A.idx);
                const T FXe = east_edge ? T(0) : fx;
                const T GXe = east_edge ? T(0) : gx;
                const T fw = from_left(FXe), gw = from_left(GXe);
                const T FXw = west_edge ? T(0) : fw;
                const T GXw = west_edge ? T(0) : gw;
                const T divW = ((FXe - FXw) * A.idx + (FY[r] - FY[r - 1]) * A.idy) + (FZt[r] - FZb[r]) * A.idz;
                const T divV = ((GXe - GXw) * A.idx + (GY[r] - GY[r - 1]) * A.idy) + (GZt[r] - GZb[r]) * A.idz;
                const T U = Uc[r], V = Vc[r], W = Wc[r];
                const T un = U + A.dt * (U * (one - U) - (A.d1 * U) * W);
                const T vn = V + A.dt * ((A.r2 * V) * (one - V) + A.D2 * divV);
                const T wn = W + A.dt * ((A.r3 * V - A.d3 * W) + divW);
                if (out_lane && row_ok[r]) {
                    gst(Ok, off[r], fU, un);
                    gst(Ok, off[r], fV, vn);
                    gst(Ok, off[r], fW, wn);
                }
            }
        }
        // advance one plane
#pragma unroll
        for (int r = 0; r < NR; ++r) {
            Wc[r] = Wn[r];
            Wn[r] = W2[r];
            TZc[r] = TZn[r];
            if (AHEAD || (r >= 1 && r <= R)) {
                Uc[r] = Un[r];
                Vc[r] = Vn[r];
                yz[r] = yzn[r];
            }
        }
#pragma unroll
        for (int r = 1; r <= R; ++r) {
            if constexpr (!RTX) TXc[r] = TXn[r];
            zz[r] = zzn[r];
            xz[r] = xzn[r];
            FZb[r] = FZt[r];
            GZb[r] = GZt[r];
        }
        if (sync) __syncthreads();                 // workgroup-uniform
    }
}

// dense (nz, ny, nx) io array -> field f of NF plane-interleaved fields
template <typename S, typename T>
__global__ void pack3_kernel(const S *__restrict__ src, T *__restrict__ dst, int nx, int ny, int nz, int pitch,
                             int nf, int f)
{
    const long n = (long)nx * ny * nz;
    for (long q = blockIdx.x * (long)blockDim.x + threadIdx.x; q < n; q += (long)gridDim.x * blockDim.x) {
        const long row = q / nx;
        const int i = (int)(q - row * nx);
        const long k = row / ny;
        const int j = (int)(row - k * ny);
        dst[((size_t)(k * nf + f) * ny + j) * pitch + i] = T(src[q]);
    }
}

template <typename T, typename D>
__global__ void unpack3_kernel(const T *__restrict__ src, D *__restrict__ dst, int nx, int ny, int nz, int pitch,
                               int nf, int f)
{
    const long n = (long)nx * ny * nz;
    for (long q = blockIdx.x * (long)blockDim.x + threadIdx.x; q < n; q += (long)gridDim.x * blockDim.x) {
        const long row = q / nx;
        const int i = (int)(q - row * nx);
        const long k = row / ny;
        const int j = (int)(row - k * ny);
        dst[q] = D(src[((size_t)(k * nf + f) * ny + j) * pitch + i]);
    }
}

__device__ __forceinline__ double wave_sum(double x)
{
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) x += __shfl_xor(x, off, 64);
    return x;
}

__device__ __forceinline__ double wave_max(double x)
{
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) x = fmax(x, __shfl_xor(x, off, 64));
    return x;
}

// Per-block partial sums of the three state fields (fixed partition and order),
// the Gershgorin bound of the tensor (max) and the number of cells whose tensor
// is not positive definite, written to parts[block*kRed3Slots + q].  A cell is
// positive definite when all three leading principal minors are positive
// (Sylvester's criterion), evaluated in FP64 on the stored entries.
template <typename T>
__global__ __launch_bounds__(kRed3) void reduce3_kernel(const T *__restrict__ st, const T *__restrict__ ten, int nx,
                                                       int ny, int nz, int pitch, double *__restrict__ parts)
{
    __shared__ double sm[kRed3 / 64][kRed3Slots];
    double x[kRed3Slots] = {0.0, 0.0, 0.0, 0.0, 0.0};
    const long n = (long)nx * ny * nz;
    const size_t P = (size_t)ny * pitch;
    for (long q = blockIdx.x * (long)kRed3 + threadIdx.x; q < n; q += (long)gridDim.x * kRed3) {
        const long row = q / nx;
        const int i = (int)(q - row * nx);
        const long k = row / ny;
        const size_t o = (size_t)(row - k * ny) * pitch + i;
        if (st) {
            const T *sk = st + (size_t)k * 3 * P + o;
#pragma unroll
            for (int f = 0; f < 3; ++f) x[f] += double(sk[f * P]);
        }
        if (ten) {
            const T *tk = ten + (size_t)k * 6 * P + o;
            const double axx = tk[0], ayy = tk[P], azz = tk[2 * P];
            const double axy = tk[3 * P], axz = tk[4 * P], ayz = tk[5 * P];
            const double r0 = fabs(axx) + fabs(axy) + fabs(axz);
            const double r1 = fabs(axy) + fabs(ayy) + fabs(ayz);
            const double r2 = fabs(axz) + fabs(ayz) + fabs(azz);
            x[3] = fmax(x[3], fmax(r0, fmax(r1, r2)));
            const double m2 = axx * ayy - axy * axy;
            const double m3 = axx * (ayy * azz - ayz * ayz) - axy * (axy * azz - ayz * axz) +
                              axz * (axy * ayz - ayy * axz);
            const bool finite = isfinite(axx) && isfinite(ayy) && isfinite(azz) && isfinite(axy) &&
                                isfinite(axz) && isfinite(ayz);
            if (!(finite && axx > 0.0 && m2 > 0.0 && m3 > 0.0)) x[4] += 1.0;
        }
    }
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
#pragma unroll
    for (int f = 0; f < 3; ++f) x[f] = wave_sum(x[f]);
    x[3] = wave_max(x[3]);
    x[4] = wave_sum(x[4]);
    if (lane == 0) {
#pragma unroll
        for (int f = 0; f < kRed3Slots; ++f) sm[wv][f] = x[f];
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        double s[kRed3Slots];
        for (int f = 0; f < kRed3Slots; ++f) s[f] = sm[0][f];
        for (int w = 1; w < kRed3 / 64; ++w) {
            for (int f = 0; f < 3; ++f) s[f] += sm[w][f];
            s[3] = fmax(s[3], sm[w][3]);
            s[4] += sm[w][4];
        }
        for (int f = 0; f < kRed3Slots; ++f) parts[(size_t)blockIdx.x * kRed3Slots + f] = s[f];
    }
}

// Fold the partials in block order (one thread: a fixed order).
__global__ void reduce3_final_kernel(const double *__restrict__ parts, int nb, double *__restrict__ out)
{
    if (threadIdx.x != 0 || blockIdx.x != 0) return;
    double s[kRed3Slots] = {0.0, 0.0, 0.0, 0.0, 0.0};
    for (int b = 0; b < nb; ++b) {
        const double *p = parts + (size_t)b * kRed3Slots;
        for (int f = 0; f < 3; ++f) s[f] += p[f];
        s[3] = fmax(s[3], p[3]);
        s[4] += p[4];
    }
    for (int f = 0; f < kRed3Slots; ++f) out[f] = s[f];
}

size_t io_bytes(int io) { return io == GGFV_F64 ? 8 : 4; }

int check_io(ggfv3_ctx *ctx, int where, int io)
{
    if (where != GGFV_HOST && where != GGFV_DEVICE) return fail3(ctx, GGFV_EINVAL, "where must be HOST or DEVICE");
    if (io != GGFV_F64 && io != GGFV_F32) return fail3(ctx, GGFV_EINVAL, "io dtype must be F64 or F32");
    return GGFV_OK;
}

long rows_of(const ggfv3_ctx *ctx) { return (long)ctx->ny * ctx->nz; }

int ensure_staging3(ggfv3_ctx *ctx, int narrays)
{
    const size_t need = (size_t)narrays * ctx->nx * rows_of(ctx) * sizeof(double);
    if (ctx->staging && ctx->staging_bytes >= need) return GGFV_OK;
    if (ctx->staging) {
        (void)hipStreamSynchronize(ctx->stream);
        (void)hipFree(ctx->staging);
        ctx->staging = nullptr;
    }
    if (hipMalloc(&ctx->staging, need) != hipSuccess) {
        ctx->staging = nullptr;
        return fail3(ctx, GGFV_ENOMEM, "cannot allocate %zu bytes of staging memory", need);
    }
    ctx->staging_bytes = need;
    return GGFV_OK;
}

// Pack n dense io arrays (host or device) into consecutive fields at dst.
int pack_fields(ggfv3_ctx *ctx, const void *const *src, int n, int where, int io, void *dst)
{
    const size_t count = (size_t)ctx->nx * rows_of(ctx);
    const void *d[6];
    if (where == GGFV_HOST) {
        int rc = ensure_staging3(ctx, n);
        if (rc) return rc;
        for (int p = 0; p < n; ++p) {
            char *s = static_cast<char *>(ctx->staging) + p * count * io_bytes(io);
            GGFV3_HIP(ctx, hipMemcpyAsync(s, src[p], count * io_bytes(io), hipMemcpyHostToDevice, ctx->stream));
            d[p] = s;
        }
    } else {
        for (int p = 0; p < n; ++p) d[p] = src[p];
    }
    const int blocks = 1024;
    const int gd[4] = {ctx->nx, ctx->ny, ctx->nz, ctx->pitch};
    for (int p = 0; p < n; ++p) {
        if (ctx->dtype == GGFV_F64 && io == GGFV_F64)
            hipLaunchKernelGGL((pack3_kernel<double, double>), dim3(blocks), dim3(256), 0, ctx->stream,
                               (const double *)d[p], (double *)dst, gd[0], gd[1], gd[2], gd[3], n, p);
        else if (ctx->dtype == GGFV_F64)
            hipLaunchKernelGGL((pack3_kernel<float, double>), dim3(blocks), dim3(256), 0, ctx->stream,
                               (const float *)d[p], (double *)dst, gd[0], gd[1], gd[2], gd[3], n, p);
        else if (io == GGFV_F64)
            hipLaunchKernelGGL((pack3_kernel<double, float>), dim3(blocks), dim3(256), 0, ctx->stream,
                               (const double *)d[p], (float *)dst, gd[0], gd[1], gd[2], gd[3], n, p);
        else
            hipLaunchKernelGGL((pack3_kernel<float, float>), dim3(blocks), dim3(256), 0, ctx->stream,
                               (const float *)d[p], (float *)dst, gd[0], gd[1], gd[2], gd[3], n, p);
        GGFV3_HIP(ctx, hipGetLastError());
    }
    // the host staging area is reused by the next call
    if (where == GGFV_HOST) GGFV3_HIP(ctx, hipStreamSynchronize(ctx->stream));
    return GGFV_OK;
}

// Reduction over the state and/or tensor: host[0..2] masses' sums, host[3]
// the Gershgorin max, host[4] the count of non-definite cells (synchronizes).
int reduce3(ggfv3_ctx *ctx, bool state, bool tensor, double *host)
{
    double *parts = ctx->scratch, *res = ctx->scratch + (size_t)kRed3Blocks * kRed3Slots;
    const void *st = state ? ctx->state[ctx->cur] : nullptr;
    const void *tn = tensor ? ctx->tensor : nullptr;
    if (ctx->dtype == GGFV_F64)
        hipLaunchKernelGGL((reduce3_kernel<double>), dim3(kRed3Blocks), dim3(kRed3), 0, ctx->stream,
                           (const double *)st, (const double *)tn, ctx->nx, ctx->ny, ctx->nz, ctx->pitch, parts);
    else
        hipLaunchKernelGGL((reduce3_kernel<float>), dim3(kRed3Blocks), dim3(kRed3), 0, ctx->stream,
                           (const float *)st, (const float *)tn, ctx->nx, ctx->ny, ctx->nz, ctx->pitch, parts);
    GGFV3_HIP(ctx, hipGetLastError());
    hipLaunchKernelGGL(reduce3_final_kernel, dim3(1), dim3(64), 0, ctx->stream, parts, kRed3Blocks, res);
    GGFV3_HIP(ctx, hipGetLastError());
    GGFV3_HIP(ctx, hipMemcpyAsync(host, res, kRed3Slots * sizeof(double), hipMemcpyDeviceToHost, ctx->stream));
    GGFV3_HIP(ctx, hipStreamSynchronize(ctx->stream));
    return GGFV_OK;
}

template <typename T>
Step3Args<T> args3(const ggfv3_ctx *ctx, double dt)
{
    Step3Args<T> A{};
    A.s = static_cast<const T *>(ctx->state[ctx->cur]);
    A.o = static_cast<T *>(ctx->state[1 - ctx->cur]);
    A.t = static_cast<const T *>(ctx->tensor);
    A.nx = ctx->nx;
    A.ny = ctx->ny;
    A.nz = ctx->nz;
    A.pitch = ctx->pitch;
    A.pb = (unsigned)(ctx->plane * sizeof(T));
    const double idx = ctx->nx / ctx->lx, idy = ctx->ny / ctx->ly, idz = ctx->nz / ctx->lz;
    A.idx = T(idx);
    A.idy = T(idy);
    A.idz = T(idz);
    A.hx = T(0.5 * idx);
    A.hy = T(0.5 * idy);
    A.hz = T(0.5 * idz);
    A.dt = T(dt);
    A.d1 = T(ctx->prm.delta1);
    A.r2 = T(ctx->prm.rho2);
    A.D2 = T(ctx->prm.Delta2);
    A.r3 = T(ctx->prm.rho3);
    A.d3 = T(ctx->prm.delta3);
    A.zs = 1;
    return A;
}

struct Shape3 {
    int rows, nsx, ngy, zs;
    PencilGrid G;
};

// Pencil shape: rows per wave (1, 2 or 4), planes per strip and waves per
// workgroup.  Defaults (measured on the 256^3 workload): about 2560 waves in
// the grid; FP64 with two rows per wave and two row groups per workgroup,
// FP32 with four rows per wave and every x-strip of a row group in one
// workgroup (up to 8).
Shape3 shape3(const ggfv3_ctx *ctx)
{
    Shape3 S{};
    const bool f64 = ctx->dtype == GGFV_F64;
    S.rows = ctx->rows > 0 ? ctx->rows : (f64 ? 2 : 4);
    S.nsx = (ctx->nx + kStrip - 1) / kStrip;
    S.ngy = (ctx->ny + S.rows - 1) / S.rows;
    if (ctx->wx > 0 || ctx->wy > 0) {
        S.G.wx = ctx->wx > 0 ? ctx->wx : 1;
        S.G.wy = ctx->wy > 0 ? ctx->wy : 1;
    } else if (f64) {
        S.G.wx = 1;
        S.G.wy = 2;
    } else {
        S.G.wx = S.nsx <= kMaxWaves3 ? S.nsx : 1;
        S.G.wy = 1;
    }
    int zs = ctx->zs;
    if (zs <= 0) {
        const long pencils = (long)S.nsx * S.ngy;
        const long target = 2560;
        long nzb = (target + pencils - 1) / pencils;
        if (nzb < 1) nzb = 1;
        zs = (int)((ctx->nz + nzb - 1) / nzb);
        if (zs < 8) zs = 8;
    }
    S.zs = zs > ctx->nz ? ctx->nz : zs;
    S.G.nbx = (S.nsx + S.G.wx - 1) / S.G.wx;
    S.G.nby = (S.ngy + S.G.wy - 1) / S.G.wy;
    S.G.nzb = (ctx->nz + S.zs - 1) / S.zs;
    return S;
}

long long workgroups3(const Shape3 &S) { return (long long)S.G.nbx * S.G.nby * S.G.nzb; }

template <typename T>
hipError_t launch3(ggfv3_ctx *ctx, double dt)
{
    Step3Args<T> A = args3<T>(ctx, dt);
    const Shape3 S = shape3(ctx);
    A.zs = S.zs;
    const long long nb = workgroups3(S);
    if (nb > 0x7fffffffLL) return hipErrorInvalidConfiguration;
    const dim3 grid((unsigned)nb), block(64 * S.G.wx * S.G.wy);
    switch (S.rows) {
    case 1:
        hipLaunchKernelGGL((step3_pencil_kernel<T, 1>), grid, block, 0, ctx->stream, A, S.G);
        break;
    case 2:
        hipLaunchKernelGGL((step3_pencil_kernel<T, 2>), grid, block, 0, ctx->stream, A, S.G);
        break;
    default:
        hipLaunchKernelGGL((step3_pencil_kernel<T, 4>), grid, block, 0, ctx->stream, A, S.G);
        break;
    }
    return hipGetLastError();
}

}  // namespace

extern "C" {

int ggfv3_create(ggfv3_ctx **out, int nx, int ny, int nz, double lx, double ly, double lz, int dtype,
                 int device, void *hip_stream)
{
    if (!out) return fail3(nullptr, GGFV_EINVAL, "null output pointer");
    *out = nullptr;
    if (nx < 1 || ny < 1 || nz < 1) return fail3(nullptr, GGFV_EINVAL, "sizes must be >= 1");
    if ((long long)nx * ny * nz > (1LL << 31))
        return fail3(nullptr, GGFV_EINVAL, "grid of %lld cells is too large", (long long)nx * ny * nz);
    // the six tensor planes of one z-level are addressed with 32-bit offsets
    if (6LL * ggfv::round_up(nx, ggfv::kRowAlign) * ny * (dtype == GGFV_F64 ? 8 : 4) >= (1LL << 32))
        return fail3(nullptr, GGFV_EINVAL, "a %dx%d plane is too large for 32-bit plane offsets", nx, ny);
    if (!(lx > 0.0) || !(ly > 0.0) || !(lz > 0.0) || !std::isfinite(lx) || !std::isfinite(ly) || !std::isfinite(lz))
        return fail3(nullptr, GGFV_EINVAL, "domain lengths must be finite and > 0");
    if (dtype != GGFV_F64 && dtype != GGFV_F32) return fail3(nullptr, GGFV_EINVAL, "dtype must be F64 or F32");
    int ndev = 0;
    hipError_t he = hipGetDeviceCount(&ndev);
    if (he != hipSuccess) return fail3(nullptr, GGFV_EHIP, "hipGetDeviceCount failed: %s", hipGetErrorString(he));
    if (device < 0 || device >= ndev) return fail3(nullptr, GGFV_EINVAL, "device %d out of range [0, %d)", device, ndev);
    ggfv3_ctx *c = new (std::nothrow) ggfv3_ctx;
    if (!c) return fail3(nullptr, GGFV_ENOMEM, "out of host memory");
    c->nx = nx;
    c->ny = ny;
    c->nz = nz;
    c->lx = lx;
    c->ly = ly;
    c->lz = lz;
    c->dtype = dtype;
    c->device = device;
    c->stream = static_cast<hipStream_t>(hip_stream);
    c->pitch = ggfv::round_up(nx, ggfv::kRowAlign);
    c->plane = (size_t)ny * c->pitch;
    const size_t field = c->plane * nz;
    c->elem = dtype == GGFV_F64 ? 8 : 4;
    Guard3 g(device);
    bool ok = hipMalloc(&c->state[0], 3 * field * c->elem) == hipSuccess &&
              hipMalloc(&c->state[1], 3 * field * c->elem) == hipSuccess &&
              hipMalloc(&c->tensor, 6 * field * c->elem) == hipSuccess &&
              hipMalloc(reinterpret_cast<void **>(&c->scratch),
                        ((size_t)kRed3Blocks * kRed3Slots + 8) * sizeof(double)) ==
                  hipSuccess;
    if (ok) ok = hipMemset(c->state[0], 0, 3 * field * c->elem) == hipSuccess &&
                 hipMemset(c->state[1], 0, 3 * field * c->elem) == hipSuccess &&
                 hipMemset(c->tensor, 0, 6 * field * c->elem) == hipSuccess;
    if (!ok) {
        ggfv3_destroy(c);
        return fail3(nullptr, GGFV_ENOMEM, "cannot allocate device memory for a %dx%dx%d grid", nx, ny, nz);
    }
    *out = c;
    return GGFV_OK;
}

void ggfv3_destroy(ggfv3_ctx *ctx)
{
    if (!ctx) return;
    {
        Guard3 g(ctx->device);
        (void)hipStreamSynchronize(ctx->stream);
        for (void *p : {ctx->state[0], ctx->state[1], ctx->tensor, ctx->staging, static_cast<void *>(ctx->scratch)})
            if (p) (void)hipFree(p);
    }
    delete ctx;
}

int ggfv3_set_params(ggfv3_ctx *ctx, const ggfv_params *p)
{
    if (!ctx) return GGFV_EINVAL;
    if (!p) return fail3(ctx, GGFV_EINVAL, "null params");
    const double v[5] = {p->delta1, p->rho2, p->Delta2, p->rho3, p->delta3};
    for (double x : v)
        if (!std::isfinite(x)) return fail3(ctx, GGFV_EINVAL, "parameters must be finite");
    ctx->prm = *p;
    ctx->has_params = true;
    return GGFV_OK;
}

int ggfv3_set_tensor(ggfv3_ctx *ctx, const void *axx, const void *ayy, const void *azz, const void *axy,
                     const void *axz, const void *ayz, int where, int io)
{
    if (!ctx) return GGFV_EINVAL;
    int rc = check_io(ctx, where, io);
    if (rc) return rc;
    const void *src[6] = {axx, ayy, azz, axy, axz, ayz};
    for (const void *p : src)
        if (!p) return fail3(ctx, GGFV_EINVAL, "null tensor field");
    Guard3 g(ctx->device);
    ctx->has_tensor = false;
    if ((rc = pack_fields(ctx, src, 6, where, io, ctx->tensor))) return rc;
    double r[kRed3Slots];
    if ((rc = reduce3(ctx, false, true, r))) return rc;
    if (r[4] > 0.0)
        return fail3(ctx, GGFV_EINVAL,
                     "tensor is not positive definite in %.0f cells (need axx > 0, axx*ayy - axy^2 > 0, det > 0)",
                     r[4]);
    ctx->has_tensor = true;
    return GGFV_OK;
}

int ggfv3_set_state(ggfv3_ctx *ctx, const void *u, const void *v, const void *w, int where, int io)
{
    if (!ctx) return GGFV_EINVAL;
    int rc = check_io(ctx, where, io);
    if (rc) return rc;
    if (!u || !v || !w) return fail3(ctx, GGFV_EINVAL, "null state field");
    Guard3 g(ctx->device);
    const void *src[3] = {u, v, w};
    if ((rc = pack_fields(ctx, src, 3, where, io, ctx->state[ctx->cur]))) return rc;
    ctx->has_state = true;
    ctx->t = 0.0;
    ctx->steps = 0;
    return GGFV_OK;
}

int ggfv3_get_state(ggfv3_ctx *ctx, void *u, void *v, void *w, int where, int io)
{
    if (!ctx) return GGFV_EINVAL;
    int rc = check_io(ctx, where, io);
    if (rc) return rc;
    if (!u || !v || !w) return fail3(ctx, GGFV_EINVAL, "null output field");
    if (!ctx->has_state) return fail3(ctx, GGFV_ESTATE, "state not set");
    Guard3 g(ctx->device);
    const size_t count = (size_t)ctx->nx * rows_of(ctx);
    void *dst[3] = {u, v, w};
    if (where == GGFV_HOST && (rc = ensure_staging3(ctx, 3))) return rc;
    const int gd[4] = {ctx->nx, ctx->ny, ctx->nz, ctx->pitch};
    for (int p = 0; p < 3; ++p) {
        const void *src = ctx->state[ctx->cur];
        void *d = where == GGFV_HOST ? static_cast<char *>(ctx->staging) + p * count * io_bytes(io) : dst[p];
        if (ctx->dtype == GGFV_F64 && io == GGFV_F64)
            hipLaunchKernelGGL((unpack3_kernel<double, double>), dim3(1024), dim3(256), 0, ctx->stream,
                               (const double *)src, (double *)d, gd[0], gd[1], gd[2], gd[3], 3, p);
        else if (ctx->dtype == GGFV_F64)
            hipLaunchKernelGGL((unpack3_kernel<double, float>), dim3(1024), dim3(256), 0, ctx->stream,
                               (const double *)src, (float *)d, gd[0], gd[1], gd[2], gd[3], 3, p);
        else if (io == GGFV_F64)
            hipLaunchKernelGGL((unpack3_kernel<float, double>), dim3(1024), dim3(256), 0, ctx->stream,
                               (const float *)src, (double *)d, gd[0], gd[1], gd[2], gd[3], 3, p);
        else
            hipLaunchKernelGGL((unpack3_kernel<float, float>), dim3(1024), dim3(256), 0, ctx->stream,
                               (const float *)src, (float *)d, gd[0], gd[1], gd[2], gd[3], 3, p);
        GGFV3_HIP(ctx, hipGetLastError());
        if (where == GGFV_HOST)
            GGFV3_HIP(ctx, hipMemcpyAsync(dst[p], d, count * io_bytes(io), hipMemcpyDeviceToHost, ctx->stream));
    }
    if (where == GGFV_HOST) GGFV3_HIP(ctx, hipStreamSynchronize(ctx->stream));
    return GGFV_OK;
}

int ggfv3_stable_dt(ggfv3_ctx *ctx, double safety, double *dt)
{
    if (!ctx) return GGFV_EINVAL;
    if (!dt) return fail3(ctx, GGFV_EINVAL, "null dt");
    if (!(safety > 0.0) || !std::isfinite(safety)) return fail3(ctx, GGFV_EINVAL, "safety must be > 0");
    if (!ctx->has_tensor || !ctx->has_params) return fail3(ctx, GGFV_ESTATE, "tensor and parameters must be set");
    Guard3 g(ctx->device);
    double r[kRed3Slots];
    int rc = reduce3(ctx, false, true, r);
    if (rc) return rc;
    double gmax = ctx->prm.Delta2;
    if (r[3] > gmax) gmax = r[3];
    if (!(gmax > 0.0)) return fail3(ctx, GGFV_EINVAL, "no positive diffusion: step bound undefined");
    const double idx = ctx->nx / ctx->lx, idy = ctx->ny / ctx->ly, idz = ctx->nz / ctx->lz;
    *dt = safety / (2.0 * gmax * (idx * idx + idy * idy + idz * idz));
    return GGFV_OK;
}

int ggfv3_step(ggfv3_ctx *ctx, double dt, long long nsteps)
{
    if (!ctx) return GGFV_EINVAL;
    if (!(dt > 0.0) || !std::isfinite(dt)) return fail3(ctx, GGFV_EINVAL, "dt must be finite and > 0");
    if (nsteps < 0) return fail3(ctx, GGFV_EINVAL, "nsteps must be >= 0");
    if (!ctx->has_state || !ctx->has_tensor || !ctx->has_params)
        return fail3(ctx, GGFV_ESTATE, "state, tensor and parameters must be set before stepping");
    Guard3 g(ctx->device);
    for (long long s = 0; s < nsteps; ++s) {
        GGFV3_HIP(ctx, ctx->dtype == GGFV_F64 ? launch3<double>(ctx, dt) : launch3<float>(ctx, dt));
        ctx->cur ^= 1;
    }
    const double dt_used = ctx->dtype == GGFV_F64 ? dt : (double)(float)dt;
    ctx->t += dt_used * (double)nsteps;
    ctx->steps += nsteps;
    return GGFV_OK;
}

int ggfv3_mass(ggfv3_ctx *ctx, double *mass3)
{
    if (!ctx) return GGFV_EINVAL;
    if (!mass3) return fail3(ctx, GGFV_EINVAL, "null output");
    if (!ctx->has_state) return fail3(ctx, GGFV_ESTATE, "state not set");
    Guard3 g(ctx->device);
    double r[kRed3Slots];
    int rc = reduce3(ctx, true, false, r);
    if (rc) return rc;
    const double vol = (ctx->lx / ctx->nx) * (ctx->ly / ctx->ny) * (ctx->lz / ctx->nz);
    for (int f = 0; f < 3; ++f) mass3[f] = vol * r[f];
    return GGFV_OK;
}

int ggfv3_time(const ggfv3_ctx *ctx, double *t, long long *steps)
{
    if (!ctx) return GGFV_EINVAL;
    if (t) *t = ctx->t;
    if (steps) *steps = ctx->steps;
    return GGFV_OK;
}

int ggfv3_set_tuning(ggfv3_ctx *ctx, int z_per_strip, int rows_per_wave, int waves_x, int waves_y)
{
    if (!ctx) return GGFV_EINVAL;
    if (z_per_strip < 0) return fail3(ctx, GGFV_EINVAL, "z_per_strip must be >= 0");
    if (rows_per_wave != 0 && rows_per_wave != 1 && rows_per_wave != 2 && rows_per_wave != 4)
        return fail3(ctx, GGFV_EINVAL, "rows_per_wave must be 0, 1, 2 or 4");
    if (waves_x < 0 || waves_y < 0 || (waves_x > 0 ? waves_x : 1) * (waves_y > 0 ? waves_y : 1) > kMaxWaves3)
        return fail3(ctx, GGFV_EINVAL, "waves_x and waves_y must be >= 0 with at most %d waves per workgroup",
                     kMaxWaves3);
    ctx->zs = z_per_strip;
    ctx->rows = rows_per_wave;
    ctx->wx = waves_x;
    ctx->wy = waves_y;
    return GGFV_OK;
}

int ggfv3_get_tuning(const ggfv3_ctx *ctx, int *z_per_strip, int *rows_per_wave, int *waves_x, int *waves_y,
                     long long *workgroups)
{
    if (!ctx) return GGFV_EINVAL;
    const Shape3 S = shape3(ctx);
    if (z_per_strip) *z_per_strip = S.zs;
    if (rows_per_wave) *rows_per_wave = S.rows;
    if (waves_x) *waves_x = S.G.wx;
    if (waves_y) *waves_y = S.G.wy;
    if (workgroups) *workgroups = workgroups3(S);
    return GGFV_OK;
}

const char *ggfv3_last_error(const ggfv3_ctx *ctx) { return ctx ? ctx->err.c_str() : g3_create_error.c_str(); }

}  // extern "C"
