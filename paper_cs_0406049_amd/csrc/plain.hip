// plain.hip -- the plain form's kernel (and its scalar fallback and the
// bandwidth-ceiling copy), their launchers and the default launch shape.
//
// The plain form is bound by HBM traffic (4 bytes read, 8 bytes written per
// element), so the kernel streams: one float4 load and two float4 stores per
// lane as buffer instructions with explicit cache policy (non-temporal loads,
// sc1 stores), one tile per workgroup, a buffer resource per tile.
#include "internal.hpp"
#include "stream.hpp"

#include <algorithm>

namespace mi355 {

// ---------------------------------------------------------------------------
// K1: plain form.  x, s, c share their offset modulo 16 bytes; `head` scalar
// elements precede the 16-byte aligned float4 body of n4 vectors and `tail`
// scalar elements follow it.  Block 0 also does the <= 6 scalar elements.

template <Arith A, Method M, int U>
__global__ void __launch_bounds__(1024) k_sincos_vec(const float *x, float *s, float *c,
                                                     int64_t n4, int head, int tail)
{
    if (blockIdx.x == 0) {
        const int t = threadIdx.x;
        if (t < head) {
            pair1_store<A, M>(x, s, c, t);
        } else if (t >= 4 && t < 4 + tail) {
            pair1_store<A, M>(x, s, c, head + 4 * n4 + (t - 4));
        }
    }
    const f4 *xv = reinterpret_cast<const f4 *>(x + head);
    f4 *sv = reinterpret_cast<f4 *>(s + head);
    f4 *cv = reinterpret_cast<f4 *>(c + head);
    const int bd = blockDim.x;
    const int64_t tile = (int64_t)bd * U;
    for (int64_t t0 = (int64_t)blockIdx.x * tile; t0 < n4; t0 += (int64_t)gridDim.x * tile)
        buffer_vec_tile<A, M, U>(xv, sv, cv, t0, n4, bd);
}

// x, s, c with different offsets modulo 16 bytes: scalar stream.
template <Arith A, Method M, int U>
__global__ void __launch_bounds__(1024) k_sincos_scalar(const float *x, float *s, float *c,
                                                        int64_t n)
{
    const int64_t bd = blockDim.x;
    const int64_t stride = (int64_t)gridDim.x * bd * U * 4;
    for (int64_t base = (int64_t)blockIdx.x * bd * U * 4 + threadIdx.x; base < n; base += stride)
        stream_scalar_tile<A, M, U>(x, s, c, base, n, bd);
}

// Bandwidth ceiling: the plain kernel's traffic, instructions and cache
// policy with no arithmetic (s = c = x).
template <int U>
__global__ void __launch_bounds__(1024) k_copy_1r2w(const f4 *x, f4 *s, f4 *c, int64_t n4)
{
    const int bd = blockDim.x;
    const int64_t tile = (int64_t)bd * U;
    for (int64_t t0 = (int64_t)blockIdx.x * tile; t0 < n4; t0 += (int64_t)gridDim.x * tile) {
        const int64_t bytes = min<int64_t>(tile, n4 - t0) * 16;
        const __amdgpu_buffer_rsrc_t rx = tile_rsrc(x + t0, bytes);
        const __amdgpu_buffer_rsrc_t rs = tile_rsrc(s + t0, bytes);
        const __amdgpu_buffer_rsrc_t rc = tile_rsrc(c + t0, bytes);
        u4 v[U];
#pragma unroll
        for (int u = 0; u < U; ++u)
            v[u] = __builtin_amdgcn_raw_buffer_load_b128(rx, (int)(threadIdx.x + u * bd) * 16, 0,
                                                         kLoadPolicy);
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const int off = (int)(threadIdx.x + u * bd) * 16;
            __builtin_amdgcn_raw_buffer_store_b128(v[u], rs, off, 0, kStorePolicy);
            __builtin_amdgcn_raw_buffer_store_b128(v[u], rc, off, 0, kStorePolicy);
        }
    }
}

// ---------------------------------------------------------------------------
// Launchers.

LaunchShape resolve_plain_shape(const LaunchShape &req, int64_t, const DeviceInfo &)
{
    // default: one workgroup per tile, up to max_grid; the kernels
    // grid-stride past that.  A grid-stride loop over two or more
    // tiles per workgroup runs slower per byte than one tile each (0.95x at
    // 2^29 elements with two tiles per workgroup).
    LaunchShape sh = req;
    const int64_t cap = max_grid(sh.block);
    if (sh.grid <= 0 || sh.grid > cap)
        sh.grid = (int)cap;
    return sh;
}

namespace {

template <Arith A, Method M>
hipError_t launch_plain_am(const float *x, float *s, float *c, int64_t n,
                           const LaunchShape &sh, hipStream_t st)
{
    const uintptr_t ax = reinterpret_cast<uintptr_t>(x), as = reinterpret_cast<uintptr_t>(s),
                    ac = reinterpret_cast<uintptr_t>(c);
    const bool same_phase = (ax & 15) == (as & 15) && (ax & 15) == (ac & 15);
    const int64_t head = same_phase ? (int64_t)(((16 - (ax & 15)) & 15) >> 2) : 0;
    if (!same_phase || n < head + 4) {
        const int64_t per_block = (int64_t)sh.block * sh.unroll * 4;
        int64_t grid = (n + per_block - 1) / per_block;
        if (sh.grid > 0)
            grid = std::min<int64_t>(grid, sh.grid);
        grid = std::max<int64_t>(grid, 1);
#define MI355_SCALAR(UU)                                                                  \
    hipLaunchKernelGGL((k_sincos_scalar<A, M, UU>), dim3((unsigned)grid), dim3(sh.block),   \
                       (unsigned)sh.lds, st, x, s, c, n)
        switch (sh.unroll) {
        case 1: MI355_SCALAR(1); break;
        case 2: MI355_SCALAR(2); break;
        case 8: MI355_SCALAR(8); break;
        default: MI355_SCALAR(4); break;
        }
#undef MI355_SCALAR
        return hipGetLastError();
    }
    const int64_t n4 = (n - head) / 4;
    const int tail = (int)(n - head - 4 * n4);
    const int64_t per_block = (int64_t)sh.block * sh.unroll;
    int64_t grid = (n4 + per_block - 1) / per_block;
    if (sh.grid > 0)
        grid = std::min<int64_t>(grid, sh.grid);
    grid = std::max<int64_t>(grid, 1);
#define MI355_VEC(UU)                                                                   \
    hipLaunchKernelGGL((k_sincos_vec<A, M, UU>), dim3((unsigned)grid), dim3(sh.block),   \
                       (unsigned)sh.lds, st, x, s, c, n4, (int)head, tail)
    switch (sh.unroll) {
    case 1: MI355_VEC(1); break;
    case 2: MI355_VEC(2); break;
    case 8: MI355_VEC(8); break;
    default: MI355_VEC(4); break;
    }
#undef MI355_VEC
    return hipGetLastError();
}

}  // namespace

hipError_t launch_sincos(const float *x, float *s, float *c, int64_t n, int arith, int method,
                         const LaunchShape &sh, hipStream_t st)
{
    const bool m2 = method == (int)Method::Arctan;
    switch (arith) {
    case (int)Arith::Split:
        return m2 ? launch_plain_am<Arith::Split, Method::Arctan>(x, s, c, n, sh, st)
                  : launch_plain_am<Arith::Split, Method::Normalized>(x, s, c, n, sh, st);
    case (int)Arith::Contract:
        return m2 ? launch_plain_am<Arith::Contract, Method::Arctan>(x, s, c, n, sh, st)
                  : launch_plain_am<Arith::Contract, Method::Normalized>(x, s, c, n, sh, st);
    default:
        return m2 ? launch_plain_am<Arith::Fused, Method::Arctan>(x, s, c, n, sh, st)
                  : launch_plain_am<Arith::Fused, Method::Normalized>(x, s, c, n, sh, st);
    }
}

hipError_t launch_copy_ceiling(const float *x, float *s, float *c, int64_t n,
                               const LaunchShape &sh, hipStream_t st)
{
    const int64_t n4 = n / 4;  // caller guarantees 16-byte alignment and n % 4 == 0
    const int64_t per_block = (int64_t)sh.block * sh.unroll;
    int64_t grid = (n4 + per_block - 1) / per_block;
    if (sh.grid > 0)
        grid = std::min<int64_t>(grid, sh.grid);
    grid = std::max<int64_t>(grid, 1);
    const f4 *xv = reinterpret_cast<const f4 *>(x);
    f4 *sv = reinterpret_cast<f4 *>(s);
    f4 *cv = reinterpret_cast<f4 *>(c);
#define MI355_COPY(UU)                                                                   \
    hipLaunchKernelGGL((k_copy_1r2w<UU>), dim3((unsigned)grid), dim3(sh.block),           \
                       (unsigned)sh.lds, st, xv, sv, cv, n4)
    switch (sh.unroll) {
    case 1: MI355_COPY(1); break;
    case 2: MI355_COPY(2); break;
    case 8: MI355_COPY(8); break;
    default: MI355_COPY(4); break;
    }
#undef MI355_COPY
    return hipGetLastError();
}

}  // namespace mi355
