// ggfv_step_common.hpp -- device helpers shared by the single-step and the
// fused multi-step kernels: the step description, vector row access, the
// compensated update and the XCD-aware work order.
#pragma once

#include "ggfv_internal.hpp"

namespace ggfv {
namespace {

template <typename T, int N>
struct alignas(sizeof(T) * N) VecN {
    T v[N];
};

template <typename T>
struct StepArgs {
    const T *u, *v, *w, *ulo, *vlo, *wlo;   // old level (lo only if compensated)
    T *un, *vn, *wn, *unlo, *vnlo, *wnlo;   // new level
    const T *a, *b, *c;
    int nx, ny, pitch, rows;
    T idx, idy, hx, hy, dt;
    T d1, r2, D2, r3, d3;
};

// NT = true loads non-temporally (the row is not kept in the caches for a
// later reader).
template <typename T, int CPL, bool NT = false>
__device__ __forceinline__ void load_vec(const T *__restrict__ p, T (&out)[CPL])
{
    if constexpr (NT) {
        typedef T vec_t __attribute__((ext_vector_type(CPL)));
        const vec_t x = __builtin_nontemporal_load(reinterpret_cast<const vec_t *>(p));
#pragma unroll
        for (int k = 0; k < CPL; ++k) out[k] = x[k];
    } else {
        VecN<T, CPL> x = *reinterpret_cast<const VecN<T, CPL> *>(p);
#pragma unroll
        for (int k = 0; k < CPL; ++k) out[k] = x.v[k];
    }
}

// Output rows are written with non-temporal stores by default: the next step
// reads them again, but the state of a large grid does not fit in any cache
// level, and streaming stores keep the caches for the input rows' halos.
// NT = false writes through the caches (faster for the FP32 lane-shift
// kernels, measured).
template <typename T, int CPL, bool NT = true>
__device__ __forceinline__ void store_vec(T *__restrict__ p, const T (&in)[CPL])
{
    if constexpr (CPL == 1) {
        if constexpr (NT) __builtin_nontemporal_store(in[0], p);
        else *p = in[0];
    } else {
        typedef T vec_t __attribute__((ext_vector_type(CPL)));
        vec_t x;
#pragma unroll
        for (int k = 0; k < CPL; ++k) x[k] = in[k];
        if constexpr (NT) __builtin_nontemporal_store(x, reinterpret_cast<vec_t *>(p));
        else *reinterpret_cast<vec_t *>(p) = x;
    }
}

// Store CPL values at byte offset voff of a buffer of nbytes bytes starting at
// base (base and nbytes uniform across the wave).  A lane whose offset lies
// outside [0, nbytes) (a negative offset reads as a large unsigned one) stores
// nothing: the hardware's range check of buffer accesses drops it.  Offsets
// and nbytes are multiples of the store's width, so a store is never partly
// in range.
template <typename T, int CPL, bool NT>
__device__ __forceinline__ void buffer_store_vec(T *base, int nbytes, int voff, const T (&in)[CPL])
{
    constexpr int kBytes = (int)sizeof(T) * CPL;
    static_assert(kBytes == 4 || kBytes == 8 || kBytes == 16, "4, 8 or 16 bytes per lane");
    // word 3 of a gfx9 buffer resource: 32-bit data format, no swizzle, no index
    const __amdgpu_buffer_rsrc_t rsrc = __builtin_amdgcn_make_buffer_rsrc(base, (short)0, nbytes, 0x00020000);
    constexpr int aux = NT ? 2 : 0;                      // 2: the non-temporal bit
    unsigned int w[kBytes / 4];
    __builtin_memcpy(w, in, kBytes);
    if constexpr (kBytes == 16) {
        typedef unsigned int u4 __attribute__((ext_vector_type(4)));
        const u4 x = {w[0], w[1], w[2], w[3]};
        __builtin_amdgcn_raw_buffer_store_b128(x, rsrc, voff, 0, aux);
    } else if constexpr (kBytes == 8) {
        typedef unsigned int u2 __attribute__((ext_vector_type(2)));
        const u2 x = {w[0], w[1]};
        __builtin_amdgcn_raw_buffer_store_b64(x, rsrc, voff, 0, aux);
    } else {
        __builtin_amdgcn_raw_buffer_store_b32(w[0], rsrc, voff, 0, aux);
    }
}

template <typename T, int CPL>
__device__ __forceinline__ void lds_store_vec(T *p, const T (&in)[CPL])
{
    VecN<T, CPL> x;
#pragma unroll
    for (int k = 0; k < CPL; ++k) x.v[k] = in[k];
    *reinterpret_cast<VecN<T, CPL> *>(p) = x;
}

// a * b + c.  The plain FP32 state evaluates it as one fused multiply-add (one
// rounding); FP64 and the compensated FP32 state keep the multiply and the add,
// so that FP64 follows the oracle's operations one for one.  The single-step
// and the fused kernels call it at the same places with the same operands, so
// they keep giving the same bits in every precision.  The places are the face
// fluxes of w, the mobilities 1 - (U + U')/2, the reactions and the Euler
// updates: each is its own expression, so transposing the grid, mirroring it
// or sweeping a strip downward maps it to itself or to its exact negative
// (fma(a, -b, -c) = -fma(a, b, c)), and those symmetries stay bit for bit.
// The divergences keep their separate products: fusing one of their two
// terms would make the transposed grid round differently.
template <typename T, bool COMP>
__device__ __forceinline__ T madd(T a, T b, T c)
{
    if constexpr (sizeof(T) == 4 && !COMP) return __builtin_fmaf(a, b, c);
    else return a * b + c;
}

// x + inc with the compensated pair (hi, lo): returns new (hi, lo).
template <typename T>
__device__ __forceinline__ void comp_add(T hi, T lo, T inc_dt, T &nhi, T &nlo)
{
    const T d = inc_dt + lo;
    const T s = hi + d;
    const T bb = s - hi;
    const T e = (hi - (s - bb)) + (d - bb);
    nhi = s;
    nlo = e;
}

// Workgroups are dealt round-robin to the eight XCDs; map the linear id so that
// each XCD receives one contiguous range of work items.
__device__ __forceinline__ int xcd_local_id(int bid, int nb)
{
    const int xcd = bid & 7, q = nb >> 3, rem = nb & 7;
    return xcd * q + min(xcd, rem) + (bid >> 3);
}

template <typename T>
StepArgs<T> make_args(const ggfv_ctx *ctx, const void *in_base, void *out_base, double dt, int rows)
{
    StepArgs<T> A{};
    const T *in = static_cast<const T *>(in_base);
    T *out = static_cast<T *>(out_base);
    const size_t P = ctx->plane;
    A.u = in;
    A.v = in + P;
    A.w = in + 2 * P;
    A.un = out;
    A.vn = out + P;
    A.wn = out + 2 * P;
    if (ctx->dtype == GGFV_F32C) {
        A.ulo = in + 3 * P;
        A.vlo = in + 4 * P;
        A.wlo = in + 5 * P;
        A.unlo = out + 3 * P;
        A.vnlo = out + 4 * P;
        A.wnlo = out + 5 * P;
    }
    const T *tn = static_cast<const T *>(ctx->tensor);
    A.a = tn;
    A.b = tn + P;
    A.c = tn + 2 * P;
    A.nx = ctx->nx;
    A.ny = ctx->ny;
    A.pitch = ctx->pitch;
    A.rows = rows;
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
    return A;
}

}  // namespace
}  // namespace ggfv
