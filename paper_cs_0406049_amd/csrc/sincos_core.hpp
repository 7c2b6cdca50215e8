// sincos_core.hpp -- device arithmetic of the branch-free single-precision
// sine-cosine pair (Mendenhall 2004), for gfx950.
//
// One lane computes one pair with binary32 VALU operations only: no branch,
// no table, no FP64, no packed FP32 (the library is built with packed FP32
// disabled), IEEE subnormals kept (no flush).  Steps, as Sec. II of the paper
// orders them:
//   1. x1 = x * fl(1/(2 pi)); q1 = x1 - rint(x1)         (reduction mod 1)
//   2. q2 = q1^2; s1 = q1 * P_s(q2); c1 = P_c(q2)        (quarter-angle series)
//   3. (s2, c2) = (2 s1 c1, c1^2 - s1^2)                  (eq. (1) doubling)
//   4. m = 2 - c2^2 - s2^2  (method 1)  or  1 / (s2^2 + c2^2)  (method 2)
//   5. (s3, c3) = (2 s2 c2, c2^2 - s2^2)                  (second doubling)
//   6. (s, c) = (s3 m, c3 m)                               (magnitude fix)
// The magnitude factor is formed after the first doubling and applied to the
// final pair, where the paper's sample implementation (Fig. 1) takes it.
//
// rint() is v_rndne_f32: round to nearest, ties to even, so q1 lies in
// [-1/2, 1/2] and the subtraction is exact.  The paper writes every plain
// product as a multiply-add with a +0 addend (AltiVec has no plain multiply);
// here a product is a product, which changes no output (the reduced angle is
// never -0).  2 * (s * c) keeps the product rounded first: the doubling of a
// rounded product is exact, the rounding of 2s * c differs for subnormals.
#pragma once

#include <hip/hip_runtime.h>

namespace mi355 {

enum class Arith : int { Fused = 0, Split = 1, Contract = 2 };
enum class Method : int { Normalized = 0, Arctan = 1 };

// 1/(2 pi) with pi written to ten decimals, rounded to binary32 (Fig. 1).
constexpr float kInvTwoPi = 0x1.45f306p-3f;
static_assert(kInvTwoPi == (float)(1.0 / (2.0 * 3.1415926536)), "reduction constant");

// Series coefficients: sin(pi q/2) ~ q (ss1 + ss2 q^2 + ss3 q^4 + ss4 q^6),
// cos(pi q/2) ~ 1 + cc1 q^2 + cc2 q^4 + cc3 q^6.  Hex literals are the
// binary32 roundings of the decimals printed in Sec. II (checked below).
template <Method M> struct Series;

template <> struct Series<Method::Normalized> {  // first method (Sec. II)
    static constexpr float ss1 = 0x1.921fb6p+0f;
    static constexpr float ss2 = -0x1.4abbbep-1f;
    static constexpr float ss3 = 0x1.46609cp-4f;
    static constexpr float ss4 = -0x1.2df648p-8f;
    static constexpr float cc1 = -0x1.3bd39ep+0f;
    static constexpr float cc2 = 0x1.03b1fap-2f;
    static constexpr float cc3 = -0x1.4ee010p-6f;
};
static_assert(Series<Method::Normalized>::ss1 == 1.5707963235f, "ss1");
static_assert(Series<Method::Normalized>::ss2 == -0.645963615f, "ss2");
static_assert(Series<Method::Normalized>::ss3 == 0.0796819754f, "ss3");
static_assert(Series<Method::Normalized>::ss4 == -0.0046075748f, "ss4");
static_assert(Series<Method::Normalized>::cc1 == -1.2336977925f, "cc1");
static_assert(Series<Method::Normalized>::cc2 == 0.2536086171f, "cc2");
static_assert(Series<Method::Normalized>::cc3 == -0.0204391631f, "cc3");

template <> struct Series<Method::Arctan> {  // second method (Sec. II)
    static constexpr float ss1 = 0x1.921fb6p+0f;
    static constexpr float ss2 = -0x1.4b143ap-1f;  // text value -0.6466386936
    static constexpr float ss3 = 0x1.16296cp-4f;
    static constexpr float ss4 = -0x1.2f6682p-10f;
    static constexpr float cc1 = -0x1.3beff2p+0f;
    static constexpr float cc2 = 0x1.f8e08ap-3f;
    static constexpr float cc3 = -0x1.9614d0p-7f;
};
static_assert(Series<Method::Arctan>::ss1 == 1.5707963268f, "ss1");
static_assert(Series<Method::Arctan>::ss2 == -0.6466386936f, "ss2");
static_assert(Series<Method::Arctan>::ss3 == 0.0679105987f, "ss3");
static_assert(Series<Method::Arctan>::ss4 == -0.0011573807f, "ss4");
static_assert(Series<Method::Arctan>::cc1 == -1.2341299769f, "cc1");
static_assert(Series<Method::Arctan>::cc2 == 0.2465220241f, "cc2");
static_assert(Series<Method::Arctan>::cc3 == -0.0123926179f, "cc3");

// a*b + c and c - a*b.  Fused: one rounding (v_fma_f32).  Split: product and
// sum rounded separately; the translation unit is compiled with
// -ffp-contract=off, so the compiler cannot fuse them.
template <Arith A> __device__ __forceinline__ float mul_add(float a, float b, float c)
{
    if constexpr (A == Arith::Fused) {
        return __builtin_fmaf(a, b, c);
    } else {
        const float p = a * b;
        return p + c;
    }
}

template <Arith A> __device__ __forceinline__ float mul_sub_from(float a, float b, float c)
{
    if constexpr (A == Arith::Fused) {
        return __builtin_fmaf(-a, b, c);
    } else {
        const float p = a * b;
        return c - p;
    }
}

// Steps 1-6 with Fused or Split arithmetic.
template <Arith A, Method M>
__device__ __forceinline__ void pair_exact(float x, float &s, float &c)
{
    using S = Series<M>;
    const float x1 = x * kInvTwoPi;
    const float q1 = x1 - __builtin_rintf(x1);
    const float q2 = q1 * q1;

    float t = mul_add<A>(q2, S::ss4, S::ss3);
    t = mul_add<A>(q2, t, S::ss2);
    t = mul_add<A>(q2, t, S::ss1);
    const float s1 = q1 * t;
    float u = mul_add<A>(q2, S::cc3, S::cc2);
    u = mul_add<A>(q2, u, S::cc1);
    const float c1 = mul_add<A>(q2, u, 1.0f);

    const float c2 = mul_sub_from<A>(s1, s1, c1 * c1);
    const float s2 = 2.0f * (s1 * c1);

    float m;
    if constexpr (M == Method::Normalized) {
        m = mul_sub_from<A>(s2, s2, mul_sub_from<A>(c2, c2, 2.0f));
    } else {
        m = 1.0f / mul_add<A>(s2, s2, c2 * c2);  // IEEE division (correctly rounded)
    }

    const float c3 = mul_sub_from<A>(s2, s2, c2 * c2);
    const float s3 = 2.0f * (s2 * c2);
    s = s3 * m;
    c = c3 * m;
}

// The Split expression tree with contraction allowed: the compiler may fuse
// any product into the sum that consumes it.
template <Method M>
__device__ __forceinline__ void pair_contract(float x, float &s, float &c)
{
#pragma clang fp contract(fast)
    using S = Series<M>;
    const float x1 = x * kInvTwoPi;
    const float q1 = x1 - __builtin_rintf(x1);
    const float q2 = q1 * q1;
    const float s1 = q1 * (((q2 * S::ss4 + S::ss3) * q2 + S::ss2) * q2 + S::ss1);
    const float c1 = ((q2 * S::cc3 + S::cc2) * q2 + S::cc1) * q2 + 1.0f;
    const float c2 = c1 * c1 - s1 * s1;
    const float s2 = 2.0f * (s1 * c1);
    float m;
    if constexpr (M == Method::Normalized) {
        m = (2.0f - c2 * c2) - s2 * s2;
    } else {
        m = 1.0f / (s2 * s2 + c2 * c2);
    }
    const float c3 = c2 * c2 - s2 * s2;
    const float s3 = 2.0f * (s2 * c2);
    s = s3 * m;
    c = c3 * m;
}

template <Arith A, Method M>
__device__ __forceinline__ void sincos_pair(float x, float &s, float &c)
{
    if constexpr (A == Arith::Contract) {
        pair_contract<M>(x, s, c);
    } else {
        pair_exact<A, M>(x, s, c);
    }
}

}  // namespace mi355
