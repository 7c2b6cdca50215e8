// sincos_core.hpp -- device arithmetic of the branch-free single-precision
// sine-cosine pair (Mendenhall 2004), for gfx950.
//
// One lane computes one pair (or N pairs in lockstep, on fvec<N> values)
// with binary32 VALU operations only: no branch,
// no table, no FP64, no packed FP32 (the library is built with packed FP32
// disabled), IEEE subnormals kept (no flush).  The method of Sec. II:
//   reduce   the angle times 1/(2 pi), less its nearest integer: the fraction
//            of a turn x in [-1/2, 1/2] (round to nearest even, v_rndne_f32;
//            the subtraction is exact);
//   series   sine and cosine of the quarter angle pi x / 2: an odd and an
//            even polynomial in x, Horner's rule in x^2;
//   double   eq. (1) twice.  By the stability analysis of Sec. II a doubling
//            squares the pair's magnitude and keeps its relative angle error;
//   correct  after two doublings the magnitude is a^4, which is also the
//            squared magnitude of the pair after the first doubling.  From
//            that pair, |p|^2 = 1 + e, comes the factor 1/(1 + e): to first
//            order 2 - |p|^2 (first method) or exactly 1 / |p|^2 (second).
//            Formed there, it is computed beside the last doubling, whose
//            result it rescales.
// In FUSED arithmetic every product that feeds a sum is fused into it; in the
// sums of two squares the cosine's square is the inner term and the sine's is
// fused last, as in the paper's own implementation (Fig. 1), whose rounding
// its printed accuracy figures reflect.  A plain product stays a product (the
// vector unit the paper used has none and adds +0; the reduced angle is never
// -0, so no output changes).  The sine of a doubling rounds s * c before
// doubling it: doubling a rounded product is exact, rounding 2s * c is not
// the same among subnormals.
#pragma once

#include <hip/hip_runtime.h>

#include <type_traits>

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

// The arithmetic below is written for a value type V: float (one pair per
// lane), or fvec<N>, N pairs per lane in lockstep.  On a vector every
// operation is the scalar one applied to each element (the library is built
// without packed FP32, so each becomes N scalar instructions, the N chains
// interleaved), hence each element's bits are the scalar path's.
template <int N> using fvec = float __attribute__((ext_vector_type(N)));

// a*b + c and c - a*b.  Fused: one rounding (v_fma_f32).  Split: product and
// sum rounded separately; the translation unit is compiled with
// -ffp-contract=off, so the compiler cannot fuse them.
template <typename V> __device__ __forceinline__ V fma_v(V a, V b, V c)
{
    if constexpr (std::is_same_v<V, float>)
        return __builtin_fmaf(a, b, c);
    else
        return __builtin_elementwise_fma(a, b, c);
}

template <Arith A, typename V> __device__ __forceinline__ V mul_add(V a, V b, V c)
{
    if constexpr (A == Arith::Fused) {
        return fma_v(a, b, c);
    } else {
        const V p = a * b;
        return p + c;
    }
}

template <Arith A, typename V> __device__ __forceinline__ V mul_sub_from(V a, V b, V c)
{
    if constexpr (A == Arith::Fused) {
        return fma_v(-a, b, c);
    } else {
        const V p = a * b;
        return c - p;
    }
}

// A sine-cosine pair (or N of them).
template <typename V> struct PairT {
    V s, c;
};
using Pair = PairT<float>;

// Reduction: theta / (2 pi) less its nearest integer (round to nearest even).
template <typename V> __device__ __forceinline__ V reduce_turns(V theta)
{
    const V turns = theta * kInvTwoPi;
    if constexpr (std::is_same_v<V, float>)
        return turns - __builtin_rintf(turns);
    else
        return turns - __builtin_elementwise_rint(turns);
}

// Horner's rule in x2: k0 + x2 (k1 + x2 (k2 + ...)).
template <Arith A, typename V> __device__ __forceinline__ V horner(V, float top)
{
    return (V)top;
}
template <Arith A, typename V, typename... R>
__device__ __forceinline__ V horner(V x2, float k0, R... rest)
{
    return mul_add<A>(x2, horner<A>(x2, rest...), (V)k0);
}

// Series: (sin, cos) of the quarter angle pi x / 2.  On vectors both
// polynomials are written before the product x * (sine polynomial): the same
// operations, in an order from which the compiler schedules N interleaved
// chains better (measured on the Huygens kernel).
template <Arith A, Method M, typename V> __device__ __forceinline__ PairT<V> quarter_pair(V x)
{
    using S = Series<M>;
    const V x2 = x * x;
    if constexpr (std::is_same_v<V, float>) {
        return {x * horner<A>(x2, S::ss1, S::ss2, S::ss3, S::ss4),
                horner<A>(x2, 1.0f, S::cc1, S::cc2, S::cc3)};
    } else {
        const V ps = horner<A>(x2, S::ss1, S::ss2, S::ss3, S::ss4);
        const V pc = horner<A>(x2, 1.0f, S::cc1, S::cc2, S::cc3);
        return {x * ps, pc};
    }
}

// eq. (1): (sin 2u, cos 2u) = (2 s c, c^2 - s^2).
template <Arith A, typename V = float> __device__ __forceinline__ PairT<V> double_angle(PairT<V> p)
{
    return {2.0f * (p.s * p.c), mul_sub_from<A>(p.s, p.s, p.c * p.c)};
}

// Magnitude factor 1/(1 + e) from a pair with |p|^2 = 1 + e.
template <Arith A, Method M, typename V = float>
__device__ __forceinline__ V norm_factor(PairT<V> p)
{
    if constexpr (M == Method::Normalized)
        return mul_sub_from<A>(p.s, p.s, mul_sub_from<A>(p.c, p.c, (V)2.0f));  // 1 - e
    else
        return (V)1.0f / mul_add<A>(p.s, p.s, p.c * p.c);  // IEEE division, correctly rounded
}

// The method with FUSED or SPLIT arithmetic.
template <Arith A, Method M, typename V>
__device__ __forceinline__ void pair_exact(V theta, V &s, V &c)
{
    const PairT<V> half = double_angle<A, V>(quarter_pair<A, M>(reduce_turns(theta)));
    const V m = norm_factor<A, M, V>(half);  // |half|^2 is the final magnitude
    const PairT<V> whole = double_angle<A, V>(half);
    s = whole.s * m;
    c = whole.c * m;
}

// The Split expression tree with contraction allowed: the compiler may fuse
// any product into the sum that consumes it.
template <Method M>
__device__ __forceinline__ void pair_contract(float theta, float &s, float &c)
{
#pragma clang fp contract(fast)
    using S = Series<M>;
    const float turns = theta * kInvTwoPi;
    const float x = turns - __builtin_rintf(turns);
    const float x2 = x * x;
    const float qs = x * (((x2 * S::ss4 + S::ss3) * x2 + S::ss2) * x2 + S::ss1);
    const float qc = ((x2 * S::cc3 + S::cc2) * x2 + S::cc1) * x2 + 1.0f;
    const float hc = qc * qc - qs * qs;
    const float hs = 2.0f * (qs * qc);
    float m;
    if constexpr (M == Method::Normalized) {
        m = (2.0f - hc * hc) - hs * hs;
    } else {
        m = 1.0f / (hs * hs + hc * hc);
    }
    const float wc = hc * hc - hs * hs;
    const float ws = 2.0f * (hs * hc);
    s = ws * m;
    c = wc * m;
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
