// Device helpers shared by the kernels of libjacobi.so (gfx950, wave64).
#pragma once

#include <hip/hip_runtime.h>

namespace jac {

// ---------------------------------------------------------------- division --
// Correctly rounded s/6 in three operations (Markstein's correction step):
// q0 = s * fl(1/6) is within one ulp of s/6, the residual s - 6 q0 is exact in
// an FMA, and q0 + r * fl(1/6) rounds to the correctly rounded quotient
// (P. Markstein, IBM J. Res. Dev. 34(1), 1990; Muller et al., Handbook of
// Floating-Point Arithmetic, division by a correctly rounded reciprocal).
// Valid away from overflow and underflow, i.e. for |s| in [2^-1020, 2^1020]
// and s = 0; the tests compare it bitwise with IEEE division.
__device__ __forceinline__ double div6(double s)
{
    const double c = 0x1.5555555555555p-3;  // the double nearest 1/6
    const double q = s * c;
    const double r = __fma_rn(-6.0, q, s);
    return __fma_rn(r, c, q);
}

__device__ __forceinline__ float div6(float s)
{
    return s * (1.0f / 6.0f);
}

// ------------------------------------------------------- cross-lane moves --
// DPP wave shifts (GFX9 wave_shr:1 / wave_shl:1): lane l receives the value
// of lane l-1 (shr) or l+1 (shl); bound_ctrl makes the lane with no source
// read 0, so no old value has to be materialised.
template <int CTRL>
__device__ __forceinline__ double dpp_move(double v)
{
    const int lo = __double2loint(v), hi = __double2hiint(v);
    const int l2 = __builtin_amdgcn_mov_dpp(lo, CTRL, 0xf, 0xf, true);
    const int h2 = __builtin_amdgcn_mov_dpp(hi, CTRL, 0xf, 0xf, true);
    return __hiloint2double(h2, l2);
}

template <int CTRL>
__device__ __forceinline__ float dpp_move(float v)
{
    return __int_as_float(__builtin_amdgcn_mov_dpp(__float_as_int(v), CTRL, 0xf, 0xf, true));
}

constexpr int DPP_WAVE_SHL1 = 0x130;
constexpr int DPP_WAVE_SHR1 = 0x138;

template <typename real>
__device__ __forceinline__ real from_left(real v) { return dpp_move<DPP_WAVE_SHR1>(v); }
template <typename real>
__device__ __forceinline__ real from_right(real v) { return dpp_move<DPP_WAVE_SHL1>(v); }

}  // namespace jac
