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

// Buffer-instruction version of a tile, used by the plain kernel.  Each
// tile gets its own buffer resource (64-bit base at the tile's start, a
// byte range of at most the tile), so 32-bit offsets suffice for any array
// size and the hardware range check drops the lanes past the end (loads
// return 0, stores are discarded): no per-lane bounds test.  Cache policy:
// loads non-temporal (nt), stores with sc1 (measured fastest for this
// 1-read / 2-write stream on gfx950).
constexpr int kLoadPolicy = 2;    // nt
constexpr int kStorePolicy = 16;  // sc1

typedef unsigned u4 __attribute__((ext_vector_type(4)));

__device__ __forceinline__ __amdgpu_buffer_rsrc_t tile_rsrc(const void *base, int64_t bytes)
{
    // dword3 = 0x00020000: raw (untyped) 32-bit data format for gfx9-family parts
    return __builtin_amdgcn_make_buffer_rsrc(const_cast<void *>(base), (short)0, (int)bytes,
                                             0x00020000);
}

template <Arith A, Method M, int U>
__device__ __forceinline__ void buffer_vec_tile(const f4 *xv, f4 *sv, f4 *cv, int64_t tile_f4,
                                                int64_t n4, int bd)
{
    const int64_t bytes = min<int64_t>((int64_t)bd * U, n4 - tile_f4) * 16;
    const __amdgpu_buffer_rsrc_t rx = tile_rsrc(xv + tile_f4, bytes);
    const __amdgpu_buffer_rsrc_t rs = tile_rsrc(sv + tile_f4, bytes);
    const __amdgpu_buffer_rsrc_t rc = tile_rsrc(cv + tile_f4, bytes);
    f4 v[U];
#pragma unroll
    for (int u = 0; u < U; ++u) {
        const int off = (int)(threadIdx.x + u * bd) * 16;
        v[u] = __builtin_bit_cast(f4, __builtin_amdgcn_raw_buffer_load_b128(rx, off, 0, kLoadPolicy));
    }
#pragma unroll
    for (int u = 0; u < U; ++u) {
        const int off = (int)(threadIdx.x + u * bd) * 16;
        f4 so, co;
        pair4<A, M>(v[u], so, co);
        __builtin_amdgcn_raw_buffer_store_b128(__builtin_bit_cast(u4, so), rs, off, 0, kStorePolicy);
        __builtin_amdgcn_raw_buffer_store_b128(__builtin_bit_cast(u4, co), rc, off, 0, kStorePolicy);
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
