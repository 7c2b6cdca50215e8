// probes.hip -- memory-traffic probes for the plain form's roofline: the same
// buffer instructions and cache policy as the plain kernel, with no
// arithmetic, in several access schedules.  They answer what the HBM allows
// for one read stream, for two write streams, and for the plain kernel's
// 1-read / 2-write mix when its reads and writes are arranged differently.
#include "internal.hpp"
#include "stream.hpp"

#include <algorithm>

namespace mi355 {

namespace {

// Loads are kept live by folding their bits into one word per lane, which is
// stored (to out[0]) only if it equals a constant no ordinary input hits.
constexpr unsigned kKeepAlive = 0x7fbadc0du;

template <int U, int LP>
__global__ void __launch_bounds__(1024) k_probe_read(const f4 *x, int64_t n4, float *out)
{
    const int bd = blockDim.x;
    const int64_t tile = (int64_t)bd * U;
    unsigned acc = 0;
    for (int64_t t0 = (int64_t)blockIdx.x * tile; t0 < n4; t0 += (int64_t)gridDim.x * tile) {
        const __amdgpu_buffer_rsrc_t rx = tile_rsrc(x + t0, min<int64_t>(tile, n4 - t0) * 16);
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const u4 v = __builtin_amdgcn_raw_buffer_load_b128(rx, (int)(threadIdx.x + u * bd) * 16,
                                                               0, LP);
            acc ^= v.x ^ v.y ^ v.z ^ v.w;
        }
    }
    if (acc == kKeepAlive)
        out[0] = __builtin_bit_cast(float, acc);
}

// Two write streams (s and c), the plain kernel's stores with no loads (c
// null: one stream).
template <int U, int SP>
__global__ void __launch_bounds__(1024) k_probe_write(f4 *s, f4 *c, int64_t n4)
{
    const int bd = blockDim.x;
    const int64_t tile = (int64_t)bd * U;
    for (int64_t t0 = (int64_t)blockIdx.x * tile; t0 < n4; t0 += (int64_t)gridDim.x * tile) {
        const int64_t bytes = min<int64_t>(tile, n4 - t0) * 16;
        const __amdgpu_buffer_rsrc_t rs = tile_rsrc(s + t0, bytes);
        const __amdgpu_buffer_rsrc_t rc = tile_rsrc(c ? c + t0 : s, c ? bytes : 0);
        const unsigned tag = (unsigned)t0;
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const int off = (int)(threadIdx.x + u * bd) * 16;
            const u4 v = u4{tag, (unsigned)off, tag ^ 1u, (unsigned)off ^ 1u};
            __builtin_amdgcn_raw_buffer_store_b128(v, rs, off, 0, SP);
            if (c)
                __builtin_amdgcn_raw_buffer_store_b128(v, rc, off, 0, SP);
        }
    }
}

// 1-read / 2-write in the plain kernel's schedule: a tile of block * U
// float4 per workgroup, each row loaded, then stored to s and to c.
template <int U, int SP>
__global__ void __launch_bounds__(1024) k_probe_copy(const f4 *x, f4 *s, f4 *c, int64_t n4)
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
            __builtin_amdgcn_raw_buffer_store_b128(v[u], rs, off, 0, SP);
            __builtin_amdgcn_raw_buffer_store_b128(v[u], rc, off, 0, SP);
        }
    }
}

// 1-read / 2-write, batched: a workgroup loads U rows of its tile before it
// stores anything, then stores all U rows of s, then all U rows of c (the
// plain kernel with unroll U alternates s and c row by row).
template <int U>
__global__ void __launch_bounds__(1024) k_probe_copy_batch(const f4 *x, f4 *s, f4 *c, int64_t n4)
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
        for (int u = 0; u < U; ++u)
            __builtin_amdgcn_raw_buffer_store_b128(v[u], rs, (int)(threadIdx.x + u * bd) * 16, 0,
                                                   kStorePolicy);
#pragma unroll
        for (int u = 0; u < U; ++u)
            __builtin_amdgcn_raw_buffer_store_b128(v[u], rc, (int)(threadIdx.x + u * bd) * 16, 0,
                                                   kStorePolicy);
    }
}

// 1-read / 2-write, one write stream per wave: a workgroup of two waves
// takes a tile of 64 float4; both waves load it (the second load is served
// by the cache), wave 0 stores it to s and wave 1 to c.
__global__ void __launch_bounds__(128) k_probe_copy_split(const f4 *x, f4 *s, f4 *c, int64_t n4)
{
    const int lane = threadIdx.x & 63;
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    for (int64_t t0 = (int64_t)blockIdx.x * 64; t0 < n4; t0 += (int64_t)gridDim.x * 64) {
        const int64_t bytes = min<int64_t>(64, n4 - t0) * 16;
        const __amdgpu_buffer_rsrc_t rx = tile_rsrc(x + t0, bytes);
        const __amdgpu_buffer_rsrc_t rd = tile_rsrc((wave == 0 ? s : c) + t0, bytes);
        const u4 v = __builtin_amdgcn_raw_buffer_load_b128(rx, lane * 16, 0, kLoadPolicy);
        __builtin_amdgcn_raw_buffer_store_b128(v, rd, lane * 16, 0, kStorePolicy);
    }
}

// 1-read / 2-write, one write stream per wave through LDS: a workgroup of two
// waves reads a tile of 128 float4 once (one float4 per thread) into LDS;
// wave 0 then stores the whole tile to s and wave 1 to c, each as two
// contiguous 1 KiB rows.
__global__ void __launch_bounds__(128) k_probe_copy_lds(const f4 *x, f4 *s, f4 *c, int64_t n4)
{
    __shared__ u4 buf[128];
    const int lane = threadIdx.x & 63;
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    for (int64_t t0 = (int64_t)blockIdx.x * 128; t0 < n4; t0 += (int64_t)gridDim.x * 128) {
        const int64_t bytes = min<int64_t>(128, n4 - t0) * 16;
        const __amdgpu_buffer_rsrc_t rx = tile_rsrc(x + t0, bytes);
        const __amdgpu_buffer_rsrc_t rd = tile_rsrc((wave == 0 ? s : c) + t0, bytes);
        buf[threadIdx.x] =
            __builtin_amdgcn_raw_buffer_load_b128(rx, (int)threadIdx.x * 16, 0, kLoadPolicy);
        __syncthreads();
        __builtin_amdgcn_raw_buffer_store_b128(buf[lane], rd, lane * 16, 0, kStorePolicy);
        __builtin_amdgcn_raw_buffer_store_b128(buf[64 + lane], rd, (64 + lane) * 16, 0,
                                               kStorePolicy);
        __syncthreads();  // both waves have read buf before the next tile overwrites it
    }
}

// 1-read / 2-write, the plain kernel's tile, with workgroups mapped to tiles
// so that each of the 8 XCDs (which take workgroups round-robin) takes runs
// of `run` consecutive tiles: XCD x gets tiles x*run .. x*run + run - 1 of
// every 8*run.  run = 1 is the plain order; run = ceil(tiles / 8) gives each
// XCD a contiguous eighth of the array.  One tile per workgroup; workgroups
// past the last tile do nothing.
__global__ void __launch_bounds__(1024) k_probe_copy_xcd(const f4 *x, f4 *s, f4 *c, int64_t n4,
                                                         int64_t run)
{
    const int bd = blockDim.x;
    const int64_t k = blockIdx.x / 8;  // this workgroup's index on its XCD
    const int64_t tile_idx = (k / run) * 8 * run + (int64_t)(blockIdx.x % 8) * run + k % run;
    const int64_t t0 = tile_idx * bd;
    if (t0 >= n4)
        return;
    const int64_t bytes = min<int64_t>(bd, n4 - t0) * 16;
    const __amdgpu_buffer_rsrc_t rx = tile_rsrc(x + t0, bytes);
    const __amdgpu_buffer_rsrc_t rs = tile_rsrc(s + t0, bytes);
    const __amdgpu_buffer_rsrc_t rc = tile_rsrc(c + t0, bytes);
    const int off = (int)threadIdx.x * 16;
    const u4 v = __builtin_amdgcn_raw_buffer_load_b128(rx, off, 0, kLoadPolicy);
    __builtin_amdgcn_raw_buffer_store_b128(v, rs, off, 0, kStorePolicy);
    __builtin_amdgcn_raw_buffer_store_b128(v, rc, off, 0, kStorePolicy);
}

int64_t grid_for(int64_t n4, int64_t per_block, int requested)
{
    int64_t grid = (n4 + per_block - 1) / per_block;
    if (requested > 0)
        grid = std::min<int64_t>(grid, requested);
    return std::max<int64_t>(std::min<int64_t>(grid, int64_t(1) << 20), 1);
}

// A kernel template over (unroll, cache policy) launched for run-time values.
template <template <int, int> class Launch, int P, typename... Args>
hipError_t by_unroll(int unroll, Args... args)
{
    switch (unroll) {
    case 1: Launch<1, P>::run(args...); break;
    case 2: Launch<2, P>::run(args...); break;
    case 8: Launch<8, P>::run(args...); break;
    default: Launch<4, P>::run(args...); break;
    }
    return hipGetLastError();
}

template <template <int, int> class Launch, int Default, typename... Args>
hipError_t by_policy(int policy, int unroll, Args... args)
{
    switch (policy) {
    case -1: return by_unroll<Launch, Default>(unroll, args...);
    case 0: return by_unroll<Launch, 0>(unroll, args...);
    case 1: return by_unroll<Launch, 1>(unroll, args...);
    case 2: return by_unroll<Launch, 2>(unroll, args...);
    case 16: return by_unroll<Launch, 16>(unroll, args...);
    case 17: return by_unroll<Launch, 17>(unroll, args...);
    case 18: return by_unroll<Launch, 18>(unroll, args...);
    default: return hipErrorInvalidValue;
    }
}

template <int U, int P> struct ReadLaunch {
    static void run(dim3 g, dim3 b, unsigned lds, hipStream_t st, const f4 *x, int64_t n4, float *out)
    {
        hipLaunchKernelGGL((k_probe_read<U, P>), g, b, lds, st, x, n4, out);
    }
};
template <int U, int P> struct WriteLaunch {
    static void run(dim3 g, dim3 b, unsigned lds, hipStream_t st, f4 *s, f4 *c, int64_t n4)
    {
        hipLaunchKernelGGL((k_probe_write<U, P>), g, b, lds, st, s, c, n4);
    }
};
template <int U, int P> struct CopyLaunch {
    static void run(dim3 g, dim3 b, unsigned lds, hipStream_t st, const f4 *x, f4 *s, f4 *c, int64_t n4)
    {
        hipLaunchKernelGGL((k_probe_copy<U, P>), g, b, lds, st, x, s, c, n4);
    }
};
template <int U, int P> struct BatchLaunch {
    static void run(dim3 g, dim3 b, unsigned lds, hipStream_t st, const f4 *x, f4 *s, f4 *c, int64_t n4)
    {
        hipLaunchKernelGGL((k_probe_copy_batch<U>), g, b, lds, st, x, s, c, n4);
    }
};

}  // namespace

bool probe_takes_policy(int probe)
{
    return probe == kProbeRead || probe == kProbeWrite || probe == kProbeWrite1 ||
           probe == kProbeCopy;
}

bool probe_policy_ok(int policy)
{
    return policy == -1 || policy == 0 || policy == 1 || policy == 2 || policy == 16 ||
           policy == 17 || policy == 18;
}

int probe_block(int probe, const LaunchShape &sh)
{
    return (probe == kProbeCopySplit || probe == kProbeCopyLds) ? 128 : sh.block;
}

hipError_t launch_stream_probe(int probe, int policy, const float *x, float *s, float *c,
                               int64_t n, const LaunchShape &sh, hipStream_t st)
{
    const unsigned lds = (unsigned)sh.lds;
    const int64_t n4 = n / 4;  // caller guarantees 16-byte alignment and n % 4 == 0
    const f4 *xv = reinterpret_cast<const f4 *>(x);
    f4 *sv = reinterpret_cast<f4 *>(s);
    f4 *cv = reinterpret_cast<f4 *>(c);
    const int bd = probe_block(probe, sh);
    const dim3 grid((unsigned)grid_for(n4, (int64_t)bd * sh.unroll, sh.grid));
    switch (probe) {
    case kProbeRead:
        return by_policy<ReadLaunch, kLoadPolicy>(policy, sh.unroll, grid, dim3(bd), lds, st, xv, n4, s);
    case kProbeWrite:
        return by_policy<WriteLaunch, kStorePolicy>(policy, sh.unroll, grid, dim3(bd), lds, st, sv, cv,
                                                    n4);
    case kProbeWrite1:
        return by_policy<WriteLaunch, kStorePolicy>(policy, sh.unroll, grid, dim3(bd), lds, st, sv,
                                                    (f4 *)nullptr, n4);
    case kProbeCopy:
        return by_policy<CopyLaunch, kStorePolicy>(policy, sh.unroll, grid, dim3(bd), lds, st, xv, sv,
                                                   cv, n4);
    case kProbeCopyBatch:
        return by_unroll<BatchLaunch, kStorePolicy>(sh.unroll, grid, dim3(bd), lds, st, xv, sv, cv, n4);
    case kProbeCopySplit: {
        const unsigned g = (unsigned)grid_for(n4, 64, sh.grid);
        hipLaunchKernelGGL(k_probe_copy_split, dim3(g), dim3(128), lds, st, xv, sv, cv, n4);
        break;
    }
    case kProbeCopyLds: {
        const unsigned g = (unsigned)grid_for(n4, 128, sh.grid);
        hipLaunchKernelGGL(k_probe_copy_lds, dim3(g), dim3(128), lds, st, xv, sv, cv, n4);
        break;
    }
    case kProbeCopyXcd: {
        const int64_t tiles = (n4 + bd - 1) / bd;
        const int64_t run = std::max<int64_t>(1, std::min<int64_t>(sh.grid, (tiles + 7) / 8));
        const int64_t grid = (tiles + 8 * run - 1) / (8 * run) * 8 * run;
        hipLaunchKernelGGL(k_probe_copy_xcd, dim3((unsigned)grid), dim3(bd), lds, st, xv, sv, cv,
                           n4, run);
        break;
    }
    default:
        return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

}  // namespace mi355
