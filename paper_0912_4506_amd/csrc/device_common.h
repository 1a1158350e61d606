// Device helpers shared by the kernels of libjacobi.so (gfx950, wave64).
#pragma once

#include <hip/hip_runtime.h>

namespace jac {

// ---------------------------------------------------------------- division --
// s/6 in three operations (Markstein's correction step): q0 = s * fl(1/6) is
// within one ulp of s/6, the residual 6 q0 - s is exact in an FMA, and
// q0 - r * fl(1/6) rounds to the correctly rounded quotient (P. Markstein,
// IBM J. Res. Dev. 34(1), 1990; Muller et al., Handbook of Floating-Point
// Arithmetic, division by a correctly rounded reciprocal).  Taking the
// residual with the opposite sign keeps the sign of a zero quotient: for
// s = -0 the last FMA adds -0 to -0.
//
// Where the three operations can differ from IEEE s/6:
//  * s = +-Inf: 6 q0 - s is Inf - Inf, so the result is NaN (IEEE: +-Inf);
//  * a quotient in the subnormal range: there s/6 can fall exactly half way
//    between two subnormals (s = 9 * 2^-1074 gives 1.5 * 2^-1074), and
//    q0 - r * fl(1/6), a hair below that, rounds the other way.
// A quotient that comes out as a normal number or zero is the IEEE one: in
// the normal range s/6 is never a tie (a tie would make s an odd multiple of
// three half-ulps of the quotient, which needs more than 53 bits), and the
// FMA's error is far below the distance to the nearest midpoint.  So
// div6_suspect flags exactly the results worth recomputing (NaN, Inf,
// subnormal) and callers redo those with div6_ieee; for finite data away from
// the subnormal range the check never fires.
__device__ __forceinline__ double div6(double s)
{
    const double c = 0x1.5555555555555p-3;  // the double nearest 1/6
    const double q = s * c;
    const double r = __fma_rn(6.0, q, -s);
    return __fma_rn(-r, c, q);
}

__device__ __forceinline__ float div6(float s)
{
    return s * (1.0f / 6.0f);
}

// v_cmp_class mask: signalling and quiet NaN, -Inf, -subnormal, +subnormal,
// +Inf (the zero and normal classes are exact results of div6)
constexpr int kDiv6SuspectClass = 0x001 | 0x002 | 0x004 | 0x010 | 0x080 | 0x200;

__device__ __forceinline__ bool div6_suspect(double q)
{
    return __builtin_amdgcn_class(q, kDiv6SuspectClass);
}

// FP32 sweeps multiply by the float nearest 1/6; nothing to recompute
__device__ __forceinline__ bool div6_suspect(float) { return false; }

// IEEE division (the compiler's correctly rounded sequence, valid for every
// input, including subnormals and infinities)
__device__ __forceinline__ double div6_ieee(double s) { return s / 6.0; }
__device__ __forceinline__ float div6_ieee(float s) { return s * (1.0f / 6.0f); }

// s/6 with the IEEE result everywhere: the fast quotient, recomputed where it
// may differ (one class test per value; used outside the blocked pass)
template <typename real>
__device__ __forceinline__ real div6_exact(real s)
{
    const real q = div6(s);
    return div6_suspect(q) ? div6_ieee(s) : q;
}

// An opaque copy of v: the compiler cannot prove it equal to v, so an
// expression recomputed from it is not merged with the original (which
// would keep the original result live in registers until the recompute).
template <typename real>
__device__ __forceinline__ real opaque(real v)
{
    asm volatile("" : "+v"(v));
    return v;
}

// s_waitcnt immediate (gfx9 encoding) that waits until at most n vector
// memory operations are outstanding, leaving the LDS and export counters free.
constexpr int vmcnt_imm(int n) { return (n & 15) | ((n >> 4) << 14) | (7 << 4) | (15 << 8); }

// ------------------------------------------------------------ plane stores --
// Stores into one plane through a buffer resource (gfx9 raw buffer: base,
// stride 0, record count in bytes).  An offset at or past the record count
// is dropped by the hardware, so a caller can issue the same number of
// stores on every path and mask cells by offset instead of by branch
// (kDropOffset, kernels.h).  (The non-temporal hint measured 2% slower on
// the blocked pass, with 5% more bytes written to HBM.)

__device__ __forceinline__ __amdgpu_buffer_rsrc_t plane_rsrc(const void *base, int bytes)
{
    return __builtin_amdgcn_make_buffer_rsrc(const_cast<void *>(base), 0, bytes, 0x00020000);
}

__device__ __forceinline__ void plane_store(double v, __amdgpu_buffer_rsrc_t r, int off)
{
    typedef unsigned int u2 __attribute__((ext_vector_type(2)));
    __builtin_amdgcn_raw_buffer_store_b64(__builtin_bit_cast(u2, v), r, off, 0, 0);
}

__device__ __forceinline__ void plane_store(float v, __amdgpu_buffer_rsrc_t r, int off)
{
    __builtin_amdgcn_raw_buffer_store_b32(__builtin_bit_cast(unsigned int, v), r, off, 0, 0);
}

// Workgroup ids reach the eight XCDs round robin (id mod 8), and each XCD has
// its own L2.  Remap so that XCD x works through a contiguous range of
// logical blocks: blocks that share halo cells then run on the same L2 at the
// same time.
__device__ __forceinline__ int xcd_remap(int b, int n)
{
    const int q = n >> 3, rem = n & 7, x = b & 7, idx = b >> 3;
    return x * q + min(x, rem) + idx;
}

// The 3-D block index of a launch after xcd_remap (x fastest).
__device__ __forceinline__ void remapped_block(int &bx, int &by, int &bz)
{
    const int gx = gridDim.x, gy = gridDim.y;
    const int total = gx * gy * gridDim.z;
    const int l = xcd_remap(blockIdx.x + gx * (blockIdx.y + gy * blockIdx.z), total);
    bx = l % gx;
    by = (l / gx) % gy;
    bz = l / (gx * gy);
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
