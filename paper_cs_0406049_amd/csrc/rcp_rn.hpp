// rcp_rn.hpp -- correctly rounded binary32 reciprocal on a bounded range.
//
// The hardware reciprocal estimate is within one ulp of 1/x; one Newton step
// with fused multiply-adds, y + y (1 - x y), then lands on the correctly
// rounded reciprocal for every binary32 x with 2^-126 <= |x| < 2^126 (a GPU
// test compares it with IEEE 1/x on every such bit pattern of either sign).
// Outside that range -- subnormal x, or 1/x subnormal or zero -- it is not
// the IEEE result, and callers must not use it there.  Three instructions
// against about ten for the general IEEE division sequence, which also
// handles scaling and special cases.
#pragma once

namespace mi355 {

constexpr float kRcpRnMin = 0x1p-126f;
constexpr float kRcpRnMax = 0x1p126f;  // exclusive

__device__ __forceinline__ float rcp_rn(float x)
{
    const float y = __builtin_amdgcn_rcpf(x);
    const float e = __builtin_fmaf(-x, y, 1.0f);
    return __builtin_fmaf(e, y, y);
}

}  // namespace mi355
