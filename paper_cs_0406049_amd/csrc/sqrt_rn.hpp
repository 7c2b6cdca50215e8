// sqrt_rn.hpp -- a correctly rounded binary32 square root for the arguments
// the Huygens term produces (x = rho^2 + L^2 >= 2^-96), without the scaling
// of tiny arguments and the special-value selects that a general correctly
// rounded square root needs.
//
// Method: the hardware estimate s = v_sqrt_f32(x) is within one ulp of
// sqrt(x); the correctly rounded result is s or one of its neighbours
// s- = pred(s), s+ = succ(s).  The residuals r- = x - s- * s and
// r+ = x - s+ * s, each formed with one rounding by a fused multiply-add,
// decide: r- <= 0 means sqrt(x) lies at or below the midpoint of s- and s,
// so s- is the rounded root; r+ > 0 means it lies above the midpoint of s and
// s+, so s+ is.  (The residual test for correctly rounded square roots; the
// product s- * s stands for the squared midpoint, from which it differs by
// ulp^2 / 4, too little to move the sign of a residual of x.)  For
// 2^-96 <= x <= FLT_MAX this equals IEEE sqrt(x); +inf and NaN pass through
// the neighbours' NaN residuals unchanged, and +0 gives +0.  The library's
// GPU tests check it against the IEEE square root on every binary32 in
// [2^-96, +inf] and on NaN.
#pragma once

#include <hip/hip_runtime.h>

namespace mi355 {

// Smallest argument for which sqrt_rn equals IEEE sqrt (2^-96).
constexpr float kSqrtRnMin = 0x1p-96f;

__device__ __forceinline__ float sqrt_rn(float x)
{
    const float s = __builtin_amdgcn_sqrtf(x);
    const float below = __builtin_bit_cast(float, __builtin_bit_cast(int, s) - 1);
    const float above = __builtin_bit_cast(float, __builtin_bit_cast(int, s) + 1);
    const float r_below = __builtin_fmaf(-below, s, x);
    const float r_above = __builtin_fmaf(-above, s, x);
    const float t = r_below <= 0.0f ? below : s;
    return r_above > 0.0f ? above : t;
}

// Five instructions for finite arguments: the hardware reciprocal square
// root estimate y, the root estimate s = x y, and one Newton correction
// with a fused multiply-add, s + (x - s^2) (y / 2).  On the GPU this equals
// IEEE sqrt(x) for every binary32 2^-96 <= x <= FLT_MAX (an exhaustive GPU
// test checks it); at +inf it gives NaN, so callers use it only where the
// argument is known to be finite.
__device__ __forceinline__ float sqrt_rn_finite(float x)
{
    const float y = __builtin_amdgcn_rsqf(x);
    const float s = x * y;
    const float h = 0.5f * y;
    const float r = __builtin_fmaf(-s, s, x);
    return __builtin_fmaf(r, h, s);
}

}  // namespace mi355
