// stream.hpp -- device helpers shared by the streaming kernels: one lane's
// float4 of pairs, and one block's share of a float4 or scalar stream.
#pragma once

#include "sincos_core.hpp"

namespace mi355 {

typedef float f4 __attribute__((ext_vector_type(4)));

// ---------------------------------------------------------------------------
// Small device helpers.

template <Arith A, Method M>
__device__ __forceinline__ void pair4(const f4 v, f4 &so, f4 &co)
{
    float s0, s1, s2, s3, c0, c1, c2, c3;
    sincos_pair<A, M>(v.x, s0, c0);
    sincos_pair<A, M>(v.y, s1, c1);
    sincos_pair<A, M>(v.z, s2, c2);
    sincos_pair<A, M>(v.w, s3, c3);
    so = f4{s0, s1, s2, s3};
    co = f4{c0, c1, c2, c3};
}

template <Arith A, Method M>
__device__ __forceinline__ void pair1_store(const float *x, float *s, float *c, int64_t i)
{
    float so, co;
    sincos_pair<A, M>(x[i], so, co);
    s[i] = so;
    c[i] = co;
}

// One block's share of a float4 stream: U float4 per lane, lanes strided by
// the block size so that each of the U loads is one coalesced row.
template <Arith A, Method M, int U>
__device__ __forceinline__ void stream_vec_tile(const f4 *xv, f4 *sv, f4 *cv, int64_t base,
                                                int64_t n4, int64_t bd)
{
    f4 v[U];
#pragma unroll
    for (int u = 0; u < U; ++u) {
        const int64_t j = base + u * bd;
        v[u] = j < n4 ? __builtin_nontemporal_load(xv + j) : f4{0.f, 0.f, 0.f, 0.f};
    }
#pragma unroll
    for (int u = 0; u < U; ++u) {
        const int64_t j = base + u * bd;
        if (j < n4) {
            f4 so, co;
            pair4<A, M>(v[u], so, co);
            __builtin_nontemporal_store(so, sv + j);
            __builtin_nontemporal_store(co, cv + j);
        }
    }
}

// Scalar version: U*4 elements per lane per trip.
template <Arith A, Method M, int U>
__device__ __forceinline__ void stream_scalar_tile(const float *x, float *s, float *c,
                                                   int64_t base, int64_t n, int64_t bd)
{
    constexpr int R = 4 * U;
    float v[R];
#pragma unroll
    for (int r = 0; r < R; ++r) {
        const int64_t j = base + r * bd;
        v[r] = j < n ? __builtin_nontemporal_load(x + j) : 0.f;
    }
#pragma unroll
    for (int r = 0; r < R; ++r) {
        const int64_t j = base + r * bd;
        if (j < n) {
            float so, co;
            sincos_pair<A, M>(v[r], so, co);
            __builtin_nontemporal_store(so, s + j);
            __builtin_nontemporal_store(co, c + j);
        }
    }
}

}  // namespace mi355
