// ggfv_dpp.hpp -- cross-lane moves of one wave by DPP wave shifts (gfx9).
#pragma once

#include <hip/hip_runtime.h>

namespace ggfv {

// DPP wave shifts.  0x138: wave_shr:1 (lane l receives lane l-1); 0x130:
// wave_shl:1 (lane l receives lane l+1).  A lane without a source receives 0
// (bound_ctrl); such lanes are never used.
//
// A shift must run with every lane of the wave active: a lane reading from a
// lane that is masked off does not receive that lane's value.  All shifts here
// sit in wave-uniform control flow and outside every ?: operand (which C
// evaluates conditionally); the DPP builtin is convergent, so the compiler does
// not move it under a per-lane condition either.  Every value a select chooses
// between is computed in a statement of its own, so the select stays a select
// rather than a branch around the computation.
template <int CTRL>
__device__ __forceinline__ int dpp_bits(int v)
{
    return __builtin_amdgcn_mov_dpp(v, CTRL, 0xf, 0xf, true);
}

template <int CTRL>
__device__ __forceinline__ float dpp_move(float x)
{
    return __int_as_float(dpp_bits<CTRL>(__float_as_int(x)));
}

template <int CTRL>
__device__ __forceinline__ double dpp_move(double x)
{
    const long long v = __double_as_longlong(x);
    const int nlo = dpp_bits<CTRL>((int)(v & 0xffffffffLL));
    const int nhi = dpp_bits<CTRL>((int)(v >> 32));
    return __longlong_as_double(((long long)nhi << 32) | (long long)(unsigned)nlo);
}

template <typename T>
__device__ __forceinline__ T from_left(T x) { return dpp_move<0x138>(x); }
template <typename T>
__device__ __forceinline__ T from_right(T x) { return dpp_move<0x130>(x); }

}  // namespace ggfv
