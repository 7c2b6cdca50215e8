// ablation.hip -- the ablations of Sec. II on the GPU, for analysis and
// measurement (the product's pair is pair_exact in sincos_core.hpp, whose
// steps these kernels reuse):
//   * the method's alternatives: no magnitude fix; the text's fix
//     (3 - s^2 - c^2)/2 applied to the final pair; both doublings with the
//     rejected eq. (2), cos 2a = 1 - 2 sin^2 a;
//   * the general form: a series for sin and cos of 2 pi q / 2^n followed by
//     n eq. (1) doublings, with the factor 2 - s^2 - c^2 taken from the pair
//     before the last doubling (for n = 0, the text's factor on the series
//     pair).  n = 2 with the printed series and the fix is the method.
// Each element is reduced as in step 1 first.  The arrays stream as in the
// plain kernel (one 64-thread wave per tile of 64 float4, buffer loads and
// stores with the same cache policies), so a timing difference is the
// arithmetic's.  x, s, c are 16-byte aligned.
#include "../../include/sincos.h"
#include "internal.hpp"
#include "sincos_core.hpp"
#include "stream.hpp"

#include <algorithm>

namespace mi355 {

namespace {

// eq. (2): (s, c) <- (2 s c, 1 - 2 s^2)
template <Arith A> __device__ __forceinline__ void double_eq2(float &s, float &c)
{
    const float c2 = mul_sub_from<A>(2.0f * s, s, 1.0f);
    const float s2 = 2.0f * (s * c);
    s = s2;
    c = c2;
}

// The text's factor (3 - c^2 - s^2) / 2.
template <Arith A> __device__ __forceinline__ float text_factor(float s, float c)
{
    return 0.5f * mul_sub_from<A>(s, s, mul_sub_from<A>(c, c, 3.0f));
}

template <Arith A, Method M, int V>
__device__ __forceinline__ void pair_variant(float x, float &s, float &c)
{
    const Pair quarter = quarter_pair<A, M>(reduce_turns(x));
    if constexpr (V == SINCOS_VARIANT_EQ2) {
        float sv = quarter.s, cv = quarter.c;
        double_eq2<A>(sv, cv);
        const float m = norm_factor<A, M>({sv, cv});
        double_eq2<A>(sv, cv);
        s = sv * m;
        c = cv * m;
    } else {
        const Pair half = double_angle<A>(quarter);
        const float m = norm_factor<A, M>(half);  // used by the method's variant only
        const Pair whole = double_angle<A>(half);
        if constexpr (V == SINCOS_VARIANT_NO_FIX) {
            s = whole.s;
            c = whole.c;
        } else if constexpr (V == SINCOS_VARIANT_TEXT_FIX) {
            const float mt = text_factor<A>(whole.s, whole.c);
            s = whole.s * mt;
            c = whole.c * mt;
        } else {
            s = whole.s * m;
            c = whole.c * m;
        }
    }
}

struct DoublingArgs {
    float ss[kMaxSeriesTerms];
    float cc[kMaxSeriesTerms];
    int32_t ns, nc, ndoub, fix;
};

// Four elements at a time, so that each trip of the runtime-length loops
// carries four independent chains (each element's operations and their order
// are those of one element alone).
template <Arith A>
__device__ __forceinline__ void pair_doublings4(const float (&x)[4], const DoublingArgs &g,
                                                float (&s)[4], float (&c)[4])
{
    float xr[4], x2[4], t[4], u[4], m[4];
#pragma unroll
    for (int r = 0; r < 4; ++r) {
        xr[r] = reduce_turns(x[r]);
        x2[r] = xr[r] * xr[r];
        t[r] = g.ss[g.ns - 1];
        u[r] = g.cc[g.nc - 1];
        m[r] = 1.0f;
    }
    for (int k = g.ns - 2; k >= 0; --k) {
        const float a = g.ss[k];
#pragma unroll
        for (int r = 0; r < 4; ++r)
            t[r] = mul_add<A>(x2[r], t[r], a);
    }
    for (int k = g.nc - 2; k >= 0; --k) {
        const float a = g.cc[k];
#pragma unroll
        for (int r = 0; r < 4; ++r)
            u[r] = mul_add<A>(x2[r], u[r], a);
    }
    float sv[4], cv[4];
#pragma unroll
    for (int r = 0; r < 4; ++r) {
        sv[r] = xr[r] * t[r];
        cv[r] = mul_add<A>(x2[r], u[r], 1.0f);
    }
    if (g.ndoub == 0 && g.fix) {
#pragma unroll
        for (int r = 0; r < 4; ++r)
            m[r] = text_factor<A>(sv[r], cv[r]);
    }
    for (int d = 0; d < g.ndoub; ++d) {
        if (g.fix && d == g.ndoub - 1) {
#pragma unroll
            for (int r = 0; r < 4; ++r)
                m[r] = norm_factor<A, Method::Normalized>({sv[r], cv[r]});
        }
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            const Pair d2 = double_angle<A>({sv[r], cv[r]});
            sv[r] = d2.s;
            cv[r] = d2.c;
        }
    }
#pragma unroll
    for (int r = 0; r < 4; ++r) {
        s[r] = g.fix ? sv[r] * m[r] : sv[r];
        c[r] = g.fix ? cv[r] * m[r] : cv[r];
    }
}

// x, s, c 16-byte aligned: tiles of 64 float4 (one per workgroup, grid-
// stride past max_grid workgroups); the last n % 4 elements by the first lanes of
// workgroup 0.  Each element is read before its outputs are written by the
// same lane, so x may be s or c.
template <class Pair4>
__device__ __forceinline__ void stream_pairs(const float *x, float *s, float *c, int64_t n,
                                             const Pair4 &pair4)
{
    const int64_t n4 = n >> 2;
    const f4 *xv = reinterpret_cast<const f4 *>(x);
    f4 *sv = reinterpret_cast<f4 *>(s);
    f4 *cv = reinterpret_cast<f4 *>(c);
    const int bd = blockDim.x;
    const int off = (int)threadIdx.x * 16;
    for (int64_t t0 = (int64_t)blockIdx.x * bd; t0 < n4; t0 += (int64_t)gridDim.x * bd) {
        const int64_t bytes = min<int64_t>(bd, n4 - t0) * 16;
        const f4 v = __builtin_bit_cast(
            f4, __builtin_amdgcn_raw_buffer_load_b128(tile_rsrc(xv + t0, bytes), off, 0, kLoadPolicy));
        const float xa[4] = {v.x, v.y, v.z, v.w};
        float sa[4], ca[4];
        pair4(xa, sa, ca);
        const f4 so = {sa[0], sa[1], sa[2], sa[3]};
        const f4 co = {ca[0], ca[1], ca[2], ca[3]};
        __builtin_amdgcn_raw_buffer_store_b128(__builtin_bit_cast(u4, so), tile_rsrc(sv + t0, bytes),
                                               off, 0, kStorePolicy);
        __builtin_amdgcn_raw_buffer_store_b128(__builtin_bit_cast(u4, co), tile_rsrc(cv + t0, bytes),
                                               off, 0, kStorePolicy);
    }
    if (blockIdx.x == 0 && (int64_t)threadIdx.x < n - 4 * n4) {
        const int64_t i = 4 * n4 + threadIdx.x;
        const float xi = x[i];
        const float xa[4] = {xi, xi, xi, xi};
        float sa[4], ca[4];
        pair4(xa, sa, ca);
        s[i] = sa[0];
        c[i] = ca[0];
    }
}

template <Arith A, Method M, int V>
__global__ void __launch_bounds__(64) k_variant(const float *x, float *s, float *c, int64_t n)
{
    stream_pairs(x, s, c, n, [](const float (&a)[4], float (&sv)[4], float (&cv)[4]) {
#pragma unroll
        for (int r = 0; r < 4; ++r)
            pair_variant<A, M, V>(a[r], sv[r], cv[r]);
    });
}

template <Arith A>
__global__ void __launch_bounds__(64) k_doublings(const float *x, float *s, float *c, int64_t n,
                                                   const DoublingArgs g)
{
    stream_pairs(x, s, c, n, [&g](const float (&a)[4], float (&sv)[4], float (&cv)[4]) {
        pair_doublings4<A>(a, g, sv, cv);
    });
}

constexpr int kAblBlock = 64;  // the plain kernel's shape

dim3 abl_grid(int64_t n)
{
    const int64_t tiles = ((n >> 2) + kAblBlock - 1) / kAblBlock;
    return dim3((unsigned)std::min<int64_t>(std::max<int64_t>(tiles, 1), max_grid(kAblBlock)));
}

template <Arith A, Method M>
hipError_t launch_variant_am(const float *x, float *s, float *c, int64_t n, int variant,
                             hipStream_t st)
{
    const dim3 g = abl_grid(n), b(kAblBlock);
    switch (variant) {
    case SINCOS_VARIANT_NO_FIX:
        hipLaunchKernelGGL((k_variant<A, M, SINCOS_VARIANT_NO_FIX>), g, b, 0, st, x, s, c, n);
        break;
    case SINCOS_VARIANT_TEXT_FIX:
        hipLaunchKernelGGL((k_variant<A, M, SINCOS_VARIANT_TEXT_FIX>), g, b, 0, st, x, s, c, n);
        break;
    case SINCOS_VARIANT_EQ2:
        hipLaunchKernelGGL((k_variant<A, M, SINCOS_VARIANT_EQ2>), g, b, 0, st, x, s, c, n);
        break;
    default:
        hipLaunchKernelGGL((k_variant<A, M, SINCOS_VARIANT_LISTING>), g, b, 0, st, x, s, c, n);
        break;
    }
    return hipGetLastError();
}

}  // namespace

hipError_t launch_variant(const float *x, float *s, float *c, int64_t n, int arith, int method,
                          int variant, hipStream_t st)
{
    const bool m2 = method == (int)Method::Arctan;
    if (arith == (int)Arith::Split)
        return m2 ? launch_variant_am<Arith::Split, Method::Arctan>(x, s, c, n, variant, st)
                  : launch_variant_am<Arith::Split, Method::Normalized>(x, s, c, n, variant, st);
    return m2 ? launch_variant_am<Arith::Fused, Method::Arctan>(x, s, c, n, variant, st)
              : launch_variant_am<Arith::Fused, Method::Normalized>(x, s, c, n, variant, st);
}

hipError_t launch_doublings(const float *x, float *s, float *c, int64_t n, int arith, int ndoub,
                            const float *ss, int ns, const float *cc, int nc, int fix,
                            hipStream_t st)
{
    DoublingArgs g{};
    std::copy(ss, ss + ns, g.ss);
    std::copy(cc, cc + nc, g.cc);
    g.ns = ns;
    g.nc = nc;
    g.ndoub = ndoub;
    g.fix = fix ? 1 : 0;
    const dim3 gr = abl_grid(n), b(kAblBlock);
    if (arith == (int)Arith::Split)
        hipLaunchKernelGGL((k_doublings<Arith::Split>), gr, b, 0, st, x, s, c, n, g);
    else
        hipLaunchKernelGGL((k_doublings<Arith::Fused>), gr, b, 0, st, x, s, c, n, g);
    return hipGetLastError();
}

}  // namespace mi355
