// forms.hip -- the kernels built around the plain form's arithmetic: the
// interleaved-output, ragged, adjoint, sinusoid-model and Huygens kernels and
// their launchers.  All arithmetic is binary32 VALU (sincos_core.hpp).
#include "internal.hpp"
#include "rcp_rn.hpp"
#include "sqrt_rn.hpp"
#include "stream.hpp"

#include <algorithm>
#include <cfloat>
#include <mutex>
#include <type_traits>

namespace mi355 {

// ---------------------------------------------------------------------------
// K1b: interleaved outputs.  Each lane computes 4 consecutive pairs; their 8
// output floats go to LDS at the lane's own 32-byte slot, in the chosen
// order, and the wave then stores its 2 KB as two fully contiguous float4
// rows (lane l writes float4 l and 64 + l of the wave's region) instead of
// two half-filled rows.
//   LAYOUT 0: complex64 e^{ix}: out[2i] = cos x_i, out[2i + 1] = sin x_i
//   LAYOUT 1: the paper's phase blocks: per 4 elements, 4 sines then 4 cosines
// x and out 16-byte aligned; n4 = n / 4 whole blocks (the caller does the
// tail).  Two waves per workgroup: measured on MI355X at 6.6 TB/s, against
// 6.4 with one or four.

constexpr int kIntWaves = 2;

template <int LAYOUT>
__global__ void __launch_bounds__(64 * kIntWaves) k_sincos_interleaved(const f4 *x, f4 *out,
                                                                      int64_t n4)
{
    __shared__ f4 stage[kIntWaves][128];
    const int lane = threadIdx.x & 63;
    const int wave = threadIdx.x >> 6;
    // grid-stride over tiles of 64 * kIntWaves float4 of x
    for (int64_t tile = blockIdx.x; tile * (64 * kIntWaves) < n4; tile += gridDim.x) {
        const int64_t i = tile * (64 * kIntWaves) + threadIdx.x;
        // first float4 of x for this wave
        const int64_t wbase = tile * (64 * kIntWaves) + wave * 64;
        if (wbase >= n4)
            return;  // whole wave past the end (wave-uniform); later tiles are too
        f4 so = f4{0.f, 0.f, 0.f, 0.f}, co = so;
        if (i < n4)
            pair4<Arith::Fused, Method::Normalized>(__builtin_nontemporal_load(x + i), so, co);
        if (LAYOUT == 0) {
            stage[wave][2 * lane] = f4{co.x, so.x, co.y, so.y};
            stage[wave][2 * lane + 1] = f4{co.z, so.z, co.w, so.w};
        } else {
            stage[wave][2 * lane] = so;
            stage[wave][2 * lane + 1] = co;
        }
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
        const int64_t valid = min<int64_t>(64, n4 - wbase);  // float4 of x this wave covers
        f4 *dst = out + 2 * wbase;
        if (lane < 2 * valid)
            __builtin_nontemporal_store(stage[wave][lane], dst + lane);
        if (64 + lane < 2 * valid)
            __builtin_nontemporal_store(stage[wave][64 + lane], dst + 64 + lane);
        // the wave's reads of its stage rows finish before the next tile writes them
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    }
}

// The last n % 4 elements of an interleaved output (complex layout: pair i at
// out[2i], out[2i+1]; block layout: a final partial block of 4 sines then 4
// cosines, its unused slots untouched).
__global__ void __launch_bounds__(64) k_interleaved_tail(const float *x, float *out, int64_t lo,
                                                         int64_t n, int layout)
{
    const int64_t i = lo + threadIdx.x;
    if (i >= n)
        return;
    float sv, cv;
    sincos_pair<Arith::Fused, Method::Normalized>(x[i], sv, cv);
    if (layout == 0) {
        out[2 * i] = cv;
        out[2 * i + 1] = sv;
    } else {
        out[2 * lo + (i - lo)] = sv;
        out[2 * lo + 4 + (i - lo)] = cv;
    }
}

// ---------------------------------------------------------------------------
// K2: ragged form, one persistent launch over many segments.
// Work is cut into units: a vector segment's unit is block*U float4 of its
// body (unit 0 also does its <= 6 head/tail scalars), a scalar segment's unit
// is block*U*4 elements.  ubeg[j] is the first unit of segment j (ubeg[count]
// = total).  Block b owns the contiguous units [b*per, (b+1)*per): it finds
// its first segment by binary search and then walks forward, so segment
// lookups cost O(1) per unit.  Segment fields are wave-uniform (scalar loads).

// The per-workgroup body over a table of descriptors and unit offsets.  Tab
// is either a pair of device pointers (staged or planned tables) or the
// table itself passed as a kernel argument (small batches): both index as
// tab.desc[j] and tab.ubeg[j].
template <Arith A, Method M, int U, class Tab>
__device__ __forceinline__ void ragged_block(const Tab &tab, int32_t count, int64_t total_units,
                                             int64_t per_block)
{
    const int64_t u0 = (int64_t)blockIdx.x * per_block;
    const int64_t u1 = min(u0 + per_block, total_units);
    if (u0 >= u1)
        return;
    int lo = 0, hi = count - 1;
    while (lo < hi) {  // largest j with ubeg[j] <= u0
        const int mid = (lo + hi + 1) >> 1;
        if (tab.ubeg[mid] <= u0)
            lo = mid;
        else
            hi = mid - 1;
    }
    int seg = lo;
    const int64_t bd = blockDim.x;
    for (int64_t unit = u0; unit < u1; ++unit) {
        while (tab.ubeg[seg + 1] <= unit)
            ++seg;
        const RaggedDesc d = tab.desc[seg];
        const int64_t local = unit - tab.ubeg[seg];
        if (d.vec) {
            if (local == 0) {
                const int t = threadIdx.x;
                const int tail = (int)(d.n - d.head - 4 * d.n4);
                if (t < d.head)
                    pair1_store<A, M>(d.x, d.s, d.c, t);
                else if (t >= 4 && t < 4 + tail)
                    pair1_store<A, M>(d.x, d.s, d.c, d.head + 4 * d.n4 + (t - 4));
            }
            const f4 *xv = reinterpret_cast<const f4 *>(d.x + d.head);
            f4 *sv = reinterpret_cast<f4 *>(d.s + d.head);
            f4 *cv = reinterpret_cast<f4 *>(d.c + d.head);
            // global non-temporal loads and stores: over thousands of separate
            // arrays the plain kernel's sc1 store policy measured 12 % slower
            // (buffer or global loads, nt stores: the same rate)
            stream_vec_tile<A, M, U>(xv, sv, cv, local * bd * U + threadIdx.x, d.n4, bd);
        } else {
            stream_scalar_tile<A, M, U>(d.x, d.s, d.c, local * bd * U * 4 + threadIdx.x, d.n, bd);
        }
    }
}

struct RaggedPtrs {
    const RaggedDesc *__restrict__ desc;
    const int64_t *__restrict__ ubeg;
};

template <Arith A, Method M, int U>
__global__ void __launch_bounds__(1024) k_ragged(const RaggedDesc *__restrict__ desc,
                                                 const int64_t *__restrict__ ubeg, int32_t count,
                                                 int64_t total_units, int64_t per_block)
{
    ragged_block<A, M, U>(RaggedPtrs{desc, ubeg}, count, total_units, per_block);
}

// Small tables travel in the kernel arguments: no staging copy before the
// launch (the runtime copies the arguments when it enqueues the kernel).
template <Arith A, Method M, int U>
__global__ void __launch_bounds__(1024) k_ragged_inline(const RaggedInline tab, int32_t count,
                                                        int64_t total_units, int64_t per_block)
{
    ragged_block<A, M, U>(tab, count, total_units, per_block);
}

// ---------------------------------------------------------------------------
// K3: adjoint of the pair, gx = gs*c - gc*s (absent gradient = 0).

template <bool GS, bool GC>
__device__ __forceinline__ float adjoint1(float s, float c, float gs, float gc)
{
    const float a = GS ? gs * c : 0.0f;
    const float b = GC ? gc * s : 0.0f;
    return a - b;
}

// Float4 body: one float4 per lane, one 64-thread wave per workgroup and
// tile (grid-stride past max_grid tiles), buffer loads and stores with the
// non-temporal policy -- measured on MI355X at 6.5 TB/s against 6.1 for
// 512-thread workgroups of global loads and stores.  Each workgroup reserves
// 8 KiB of LDS it does not use, so that at most 20 are resident per CU: with
// fewer tiles in flight the stream runs 1.3 % faster (6.53 against 6.45
// TB/s; 7-8 KiB reserved measured alike, less or none slower).
constexpr int kBwdBlock = 64;
constexpr int kBwdStorePolicy = 2;  // nt
constexpr unsigned kBwdLdsReserve = 8192;

template <bool GS, bool GC>
__global__ void __launch_bounds__(kBwdBlock) k_backward_vec(const f4 *s, const f4 *c,
                                                            const f4 *gs, const f4 *gc, f4 *gx,
                                                            int64_t n4)
{
    const int bd = blockDim.x;
    const int off = (int)threadIdx.x * 16;
    for (int64_t t0 = (int64_t)blockIdx.x * bd; t0 < n4; t0 += (int64_t)gridDim.x * bd) {
        // the tile's byte range: lanes past the end load 0 and store nothing
        const int64_t bytes = min<int64_t>(bd, n4 - t0) * 16;
        auto load = [&](const f4 *p) {
            return __builtin_bit_cast(
                f4, __builtin_amdgcn_raw_buffer_load_b128(tile_rsrc(p + t0, bytes), off, 0,
                                                          kLoadPolicy));
        };
        const f4 sv = load(s);
        const f4 cv = load(c);
        f4 a = f4{0.f, 0.f, 0.f, 0.f}, b = f4{0.f, 0.f, 0.f, 0.f};
        if (GS)
            a = load(gs);
        if (GC)
            b = load(gc);
        f4 r;
        r.x = adjoint1<GS, GC>(sv.x, cv.x, a.x, b.x);
        r.y = adjoint1<GS, GC>(sv.y, cv.y, a.y, b.y);
        r.z = adjoint1<GS, GC>(sv.z, cv.z, a.z, b.z);
        r.w = adjoint1<GS, GC>(sv.w, cv.w, a.w, b.w);
        __builtin_amdgcn_raw_buffer_store_b128(__builtin_bit_cast(u4, r), tile_rsrc(gx + t0, bytes),
                                               off, 0, kBwdStorePolicy);
    }
}

template <bool GS, bool GC>
__global__ void __launch_bounds__(256) k_backward_scalar(const float *s, const float *c,
                                                         const float *gs, const float *gc,
                                                         float *gx, int64_t lo, int64_t hi)
{
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t i = lo + (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < hi; i += stride)
        gx[i] = adjoint1<GS, GC>(s[i], c[i], GS ? gs[i] : 0.f, GC ? gc[i] : 0.f);
}

// ---------------------------------------------------------------------------
// K4: sinusoid model forward, y_i = sum_k A_k sin(w_k t_i + phi_k).
// Lane <-> sample: each lane keeps IPT samples and walks k in order, so the
// sum order is k = 0..K-1 exactly; A_k, w_k, phi_k are wave-uniform (scalar
// loads).  Only the sine of each pair is used; the cosine-only operations
// are dropped by the compiler.
// RESID: write the residual r_i = y_i - y_obs_i instead of y_i, and the
// workgroup's sum of r_i^2 to loss_part[blockIdx.x]: each lane adds its r^2
// with fma in sample order, then a fixed 256-way tree in LDS.

constexpr int kFwdIPT = 8;
constexpr int kFwdBlock = 256;

template <bool RESID>
__global__ void __launch_bounds__(kFwdBlock) k_sinusoid_fwd(const float *t, int64_t N,
                                                            const float *__restrict__ A,
                                                            const float *__restrict__ w,
                                                            const float *__restrict__ phi,
                                                            int32_t K, float *y,
                                                            const float *y_obs, float *loss_part)
{
    const int64_t bd = blockDim.x;
    const int64_t stride = (int64_t)gridDim.x * bd * kFwdIPT;
    float sq = 0.0f;
    for (int64_t base = (int64_t)blockIdx.x * bd * kFwdIPT + threadIdx.x; base < N;
         base += stride) {
        float ti[kFwdIPT], acc[kFwdIPT];
#pragma unroll
        for (int r = 0; r < kFwdIPT; ++r) {
            const int64_t i = base + r * bd;
            ti[r] = i < N ? t[i] : 0.f;
            acc[r] = 0.0f;
        }
#pragma unroll 4
        for (int32_t k = 0; k < K; ++k) {
            const float wk = w[k], pk = phi[k], ak = A[k];
#pragma unroll
            for (int r = 0; r < kFwdIPT; ++r) {
                float sv, cv;
                sincos_pair<Arith::Fused, Method::Normalized>(__builtin_fmaf(wk, ti[r], pk), sv, cv);
                acc[r] = __builtin_fmaf(ak, sv, acc[r]);
            }
        }
#pragma unroll
        for (int r = 0; r < kFwdIPT; ++r) {
            const int64_t i = base + r * bd;
            if (i < N) {
                float v = acc[r];
                if (RESID) {
                    v = v - y_obs[i];
                    sq = __builtin_fmaf(v, v, sq);
                }
                y[i] = v;
            }
        }
    }
    if (RESID) {
        __shared__ float red[kFwdBlock];
        red[threadIdx.x] = sq;
        __syncthreads();
        for (int h = kFwdBlock / 2; h > 0; h >>= 1) {
            if ((int)threadIdx.x < h)
                red[threadIdx.x] += red[threadIdx.x + h];
            __syncthreads();
        }
        if (threadIdx.x == 0)
            loss_part[blockIdx.x] = red[0];
    }
}

// Sum of p[start], p[start + step], ... below n, added in that order.  The
// loads go out eight at a time so their latencies overlap; the additions
// keep the order, so the result does not depend on the grouping.
__device__ __forceinline__ float strided_sum(const float *p, int64_t n, int64_t start,
                                             int64_t step)
{
    float acc = 0.0f;
    int64_t j = start;
    for (; j + 7 * step < n; j += 8 * step) {
        float v[8];
#pragma unroll
        for (int u = 0; u < 8; ++u)
            v[u] = p[j + u * step];
#pragma unroll
        for (int u = 0; u < 8; ++u)
            acc += v[u];
    }
    for (; j < n; j += step)
        acc += p[j];
    return acc;
}

// Sum of row[0..n) by one 256-thread workgroup: strided per-thread sums,
// then a fixed 256-way tree (the result is in red[0] for every thread after
// the last barrier).
__device__ __forceinline__ float block_sum_256(const float *row, int64_t n, float *red)
{
    red[threadIdx.x] = strided_sum(row, n, threadIdx.x, 256);
    __syncthreads();
    for (int h = 128; h > 0; h >>= 1) {
        if ((int)threadIdx.x < h)
            red[threadIdx.x] += red[threadIdx.x + h];
        __syncthreads();
    }
    return red[0];
}

// loss = 1/2 * (sum of the workgroup partials): one workgroup.
__global__ void __launch_bounds__(256) k_loss_reduce(const float *part, int64_t nparts, float *loss)
{
    __shared__ float red[256];
    const float v = block_sum_256(part, nparts, red);
    if (threadIdx.x == 0)
        loss[0] = 0.5f * v;
}

// K5: sinusoid adjoint.  Lane <-> frequency k (a wave covers 64 of them),
// wave <-> chunk of consecutive samples: t_i and g_i are wave-uniform (scalar
// loads), so each lane accumulates its own three sums with no cross-lane
// traffic.  The block's waves then add their sums in LDS in a fixed pairwise
// tree, and the block writes one partial per (j, k) to
// partial[(j * Kpad + k) * nparts + block] (j = 0: A, 1: phi, 2: w);
// k_sinusoid_reduce adds each row in a fixed tree order (deterministic) and
// applies A_k.

constexpr int64_t kAdjChunk = 128;  // samples per wave (measured 6 % faster than 512)
constexpr int kAdjWaves = 16;       // waves per block (one chunk each)
static_assert((kAdjWaves & (kAdjWaves - 1)) == 0 && kAdjWaves >= 3, "pairwise tree over the waves");

__global__ void __launch_bounds__(64 * kAdjWaves) k_sinusoid_adj(const float *__restrict__ t,
                                                      const float *__restrict__ g, int64_t N,
                                                      const float *__restrict__ w,
                                                      const float *__restrict__ phi, int32_t K,
                                                      int64_t nchunks, float *partial)
{
    __shared__ float sums[3][kAdjWaves][64];
    const int lane = threadIdx.x & 63;
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int64_t chunk = (int64_t)blockIdx.x * kAdjWaves + wave;
    const int64_t nparts = gridDim.x;
    const int32_t Kpad = (int32_t)gridDim.y * 64;
    const int32_t k = (int32_t)blockIdx.y * 64 + lane;
    const bool active = k < K;
    const float wk = active ? w[k] : 0.f;
    const float pk = active ? phi[k] : 0.f;
    float sa = 0.f, sp = 0.f, sw = 0.f;
    if (chunk < nchunks) {  // waves past the last chunk add zeros
        const int64_t i0 = chunk * kAdjChunk;
        const int64_t i1 = min(i0 + kAdjChunk, N);
#pragma unroll 8
        for (int64_t i = i0; i < i1; ++i) {
            const float ti = t[i], gi = g[i];
            float sv, cv;
            sincos_pair<Arith::Fused, Method::Normalized>(__builtin_fmaf(wk, ti, pk), sv, cv);
            sa = __builtin_fmaf(gi, sv, sa);
            sp = __builtin_fmaf(gi, cv, sp);
            sw = __builtin_fmaf(gi * ti, cv, sw);
        }
    }
    sums[0][wave][lane] = sa;
    sums[1][wave][lane] = sp;
    sums[2][wave][lane] = sw;
    __syncthreads();
    if (wave < 3) {  // wave j adds sum j over the block's waves
        float v[kAdjWaves];
#pragma unroll
        for (int q = 0; q < kAdjWaves; ++q)
            v[q] = sums[wave][q][lane];
#pragma unroll
        for (int h = kAdjWaves / 2; h > 0; h >>= 1)
#pragma unroll
            for (int q = 0; q < h; ++q)
                v[q] = v[q] + v[q + h];
        partial[((int64_t)wave * Kpad + k) * nparts + blockIdx.x] = v[0];
    }
}

// One block per output (j, k): each thread sums a strided share of the row
// of block partials, then a fixed-shape tree in LDS.
__global__ void __launch_bounds__(256) k_sinusoid_reduce(const float *partial, int64_t nparts,
                                                         int32_t Kpad, int32_t K, const float *A,
                                                         float *gA, float *gw, float *gphi)
{
    const int32_t k = blockIdx.x;
    const int j = blockIdx.y;  // 0: A, 1: phi, 2: w
    __shared__ float red[256];
    const float v = block_sum_256(partial + ((int64_t)j * Kpad + k) * nparts, nparts, red);
    if (threadIdx.x == 0 && k < K) {
        if (j == 0)
            gA[k] = v;
        else if (j == 1)
            gphi[k] = A[k] * v;
        else
            gw[k] = A[k] * v;
    }
}

// K5b: one step of the least-squares fit in one pass over the samples.  A
// workgroup of kAdjWaves waves owns kAdjWaves * kAdjChunk consecutive
// samples.  Phase 1, lane <-> sample: y_i as the forward model computes it,
// r_i = y_i - y_obs_i, kept in LDS as (t_i, r_i, r_i t_i) (the residual
// never goes to HBM), and the workgroup's partial of sum r_i^2.  Phase 2,
// lane <-> frequency: exactly the adjoint kernel's sums over the same chunks
// in the same order, each sample one LDS read, its product r_i t_i rounded
// once per sample instead of once per frequency (the same value the adjoint
// kernel rounds per pair), and the same tree over the waves.  The gradients
// are therefore the same bits as the forward kernel's residual followed by
// the adjoint kernel.
constexpr int kFitSamples = kAdjWaves * (int)kAdjChunk;  // 2048

__global__ void __launch_bounds__(64 * kAdjWaves) k_sinusoid_fit(
    const float *__restrict__ t, const float *__restrict__ y_obs, int64_t N,
    const float *__restrict__ A, const float *__restrict__ w, const float *__restrict__ phi,
    int32_t K, int32_t kgroups, float *partial, float *loss_part)
{
    __shared__ f4 samp[kFitSamples];  // (t, r, r t, unused) per sample
    __shared__ float sums[3][kAdjWaves][64];
    __shared__ float red[64 * kAdjWaves];
    const int64_t base = (int64_t)blockIdx.x * kFitSamples;
    const int64_t nparts = gridDim.x;
    const int32_t Kpad = kgroups * 64;

    // phase 1: two samples per thread, each the forward model in k order from
    // +0; both samples in one pass over k, so that each frequency's
    // parameters serve two terms (and the two chains overlap)
    float sq = 0.0f;
    float ti[2], acc[2];
#pragma unroll
    for (int h = 0; h < 2; ++h) {
        const int64_t i = base + (int)threadIdx.x + h * 64 * kAdjWaves;
        ti[h] = i < N ? t[i] : 0.0f;
        acc[h] = 0.0f;
    }
#pragma unroll 4
    for (int32_t k = 0; k < K; ++k) {
        const float wk = w[k], pk = phi[k], ak = A[k];
#pragma unroll
        for (int h = 0; h < 2; ++h) {
            float sv, cv;
            sincos_pair<Arith::Fused, Method::Normalized>(__builtin_fmaf(wk, ti[h], pk), sv, cv);
            acc[h] = __builtin_fmaf(ak, sv, acc[h]);
        }
    }
#pragma unroll
    for (int h = 0; h < 2; ++h) {
        const int li = (int)threadIdx.x + h * 64 * kAdjWaves;
        const int64_t i = base + li;
        float r = 0.0f;
        if (i < N) {
            r = acc[h] - y_obs[i];
            sq = __builtin_fmaf(r, r, sq);
        }
        samp[li] = f4{ti[h], r, r * ti[h], 0.0f};
    }
    red[threadIdx.x] = sq;
    __syncthreads();
    for (int h = 64 * kAdjWaves / 2; h > 0; h >>= 1) {
        if ((int)threadIdx.x < h)
            red[threadIdx.x] += red[threadIdx.x + h];
        __syncthreads();
    }
    if (threadIdx.x == 0)
        loss_part[blockIdx.x] = red[0];

    // phase 2: the adjoint sums, one k group of 64 frequencies at a time
    const int lane = threadIdx.x & 63;
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int32_t j0 = wave * (int32_t)kAdjChunk;  // this wave's samples, block-local
    const int32_t j1 = (int32_t)min<int64_t>(j0 + kAdjChunk, N - base);
    for (int32_t kg = 0; kg < kgroups; ++kg) {
        const int32_t k = kg * 64 + lane;
        const bool active = k < K;
        const float wk = active ? w[k] : 0.f;
        const float pk = active ? phi[k] : 0.f;
        float sa = 0.f, sp = 0.f, sw = 0.f;
#pragma unroll 8
        for (int32_t j = j0; j < j1; ++j) {
            const f4 q = samp[j];  // one LDS read: t, r and the product r t
            float sv, cv;
            sincos_pair<Arith::Fused, Method::Normalized>(__builtin_fmaf(wk, q.x, pk), sv, cv);
            sa = __builtin_fmaf(q.y, sv, sa);
            sp = __builtin_fmaf(q.y, cv, sp);
            sw = __builtin_fmaf(q.z, cv, sw);
        }
        if (kg > 0)
            __syncthreads();  // the previous group's tree has read sums
        sums[0][wave][lane] = sa;
        sums[1][wave][lane] = sp;
        sums[2][wave][lane] = sw;
        __syncthreads();
        if (wave < 3) {
            float v[kAdjWaves];
#pragma unroll
            for (int q = 0; q < kAdjWaves; ++q)
                v[q] = sums[wave][q][lane];
#pragma unroll
            for (int h = kAdjWaves / 2; h > 0; h >>= 1)
#pragma unroll
                for (int q = 0; q < h; ++q)
                    v[q] = v[q] + v[q + h];
            partial[((int64_t)wave * Kpad + k) * nparts + blockIdx.x] = v[0];
        }
    }
}

// The fit step's reduction in one launch: blocks (k, j < 3) as
// k_sinusoid_reduce, block (0, 3) the loss.
__global__ void __launch_bounds__(256) k_fit_reduce(const float *partial, const float *loss_part,
                                                    int64_t nparts, int32_t Kpad, int32_t K,
                                                    const float *A, float *gA, float *gw,
                                                    float *gphi, float *loss)
{
    const int32_t k = blockIdx.x;
    const int j = blockIdx.y;
    __shared__ float red[256];
    if (j == 3) {
        if (k != 0)
            return;
        const float v = block_sum_256(loss_part, nparts, red);
        if (threadIdx.x == 0)
            loss[0] = 0.5f * v;
        return;
    }
    const float v = block_sum_256(partial + ((int64_t)j * Kpad + k) * nparts, nparts, red);
    if (threadIdx.x == 0 && k < K) {
        if (j == 0)
            gA[k] = v;
        else if (j == 1)
            gphi[k] = A[k] * v;
        else
            gw[k] = A[k] * v;
    }
}

// ---------------------------------------------------------------------------
// K6: Huygens point-source sum, U_i = sum_j (a_j / r_ij) exp(i (k (r_ij - L) +
// phi_j)), the path difference as rho^2 / (r + L), both quotients from one
// reciprocal: e = r + L, g = 1 / (r e), d = rho^2 (r g), w = a (e g), each
// operation rounded (two divisions, d = rho^2 / e and w = a / r, where r e
// is not a normal binary32).  The sources are summed in kHuyBlocks
// contiguous blocks of ceil(S / kHuyBlocks), each in source order with fma
// from +0, and the block sums are added in block order.  One wave per block: a 256-thread
// workgroup takes 64 screen points, wave b sums block b for all 64 and the
// four partial fields meet in LDS.  Four waves per point give the
// diffraction workload (262,144 points) 16,384 waves instead of 4096, enough
// to keep 8 resident on every SIMD: the term's long dependency chains need
// them.  The source table (x, y, a, phi) is read with wave-uniform float4
// scalar loads, and the loads of the next kHuyGroup sources are issued
// before the current group is evaluated, so their latency hides behind
// that arithmetic; the group's sine-cosine pairs are evaluated in lockstep.
// The square root and the reciprocal are correctly rounded.

constexpr int kHuyGroup = 2;
constexpr int kHuyBlocks = 4;
constexpr int kHuyPoints = 256 / kHuyBlocks;  // screen points per workgroup (one wave)
// The short square root and rcp_rn serve a group when every coordinate of
// the wave's points and of the group's sources is below 2^60 in magnitude
// and 2^-48 <= L < 2^60 (checked by the launcher): then 2^-96 <= rho^2 + L^2
// < 2^124, r < 2^62, r + L < 2^63 and 2^-96 <= r (r + L) < 2^125, inside
// both helpers' ranges.  Otherwise (huge, infinite or NaN coordinates) the
// group takes sqrt_rn and the IEEE reciprocal, or the two divisions.
constexpr uint32_t kHuyCoordMaxBits = 0x5D800000u;  // 2^60

__device__ __forceinline__ bool huy_coord_ok(float v)
{
    return (__builtin_bit_cast(uint32_t, v) & 0x7FFFFFFFu) < kHuyCoordMaxBits;
}

// The terms of G sources for one screen point, added to (re, im) in source
// order.  SQRT_RN: L^2 >= 2^-96, so rho^2 + L^2 is in the range where
// sqrt_rn is the IEEE square root (7 fewer instructions than the general
// sequence).  fast (wave-uniform): every coordinate is in range (see
// kHuyCoordMaxBits), so rho^2 + L^2 is finite and sqrt_rn_finite is the IEEE
// square root, and r (r + L) is in rcp_rn's range, so rcp_rn is the IEEE
// reciprocal and the one-reciprocal form applies; otherwise, lane by lane,
// sqrt_rn, then the IEEE reciprocal while r (r + L) is a normal binary32 and
// two IEEE divisions where it is not.  One branch per group around the root
// and the quotients: the rest of the arithmetic is shared.
template <int G, bool SQRT_RN>
__device__ __forceinline__ void huygens_terms(float px, float py, const f4 *sq, bool fast,
                                              float k, float L, float L2, float &re, float &im)
{
    float rho2[G], r2[G], d[G], w[G];
#pragma unroll
    for (int u = 0; u < G; ++u) {
        const float dx = px - sq[u].x;
        const float dy = py - sq[u].y;
        const float dy2 = dy * dy;
        rho2[u] = __builtin_fmaf(dx, dx, dy2);
        r2[u] = rho2[u] + L2;
    }
    if (fast) {
        // 2^-96 <= r2 < 2^124: sqrt_rn_finite is the IEEE square root there
#pragma unroll
        for (int u = 0; u < G; ++u) {
            const float rr = sqrt_rn_finite(r2[u]);
            const float e = rr + L;
            const float g = rcp_rn(rr * e);
            d[u] = rho2[u] * (rr * g);
            w[u] = sq[u].z * (e * g);
        }
    } else {
#pragma unroll
        for (int u = 0; u < G; ++u) {
            const float rr = SQRT_RN ? sqrt_rn(r2[u]) : __builtin_sqrtf(r2[u]);
            const float e = rr + L;
            const float x = rr * e;
            const bool normal = x >= FLT_MIN && x <= FLT_MAX;
            const float g = 1.0f / x;
            d[u] = normal ? rho2[u] * (rr * g) : rho2[u] / e;
            w[u] = normal ? sq[u].z * (e * g) : sq[u].z / rr;
        }
    }
    if constexpr (G > 1) {
        fvec<G> th, sv, cv;  // the group's pairs in lockstep
#pragma unroll
        for (int u = 0; u < G; ++u)
            th[u] = __builtin_fmaf(k, d[u], sq[u].w);
        pair_exact<Arith::Fused, Method::Normalized>(th, sv, cv);
#pragma unroll
        for (int u = 0; u < G; ++u) {
            re = __builtin_fmaf(w[u], cv[u], re);
            im = __builtin_fmaf(w[u], sv[u], im);
        }
    } else {
        float sv, cv;
        sincos_pair<Arith::Fused, Method::Normalized>(__builtin_fmaf(k, d[0], sq[0].w), sv, cv);
        re = __builtin_fmaf(w[0], cv, re);
        im = __builtin_fmaf(w[0], sv, im);
    }
}

// Whether every source coordinate of a group is below 2^60 in magnitude: the
// running maximum of the magnitude bit patterns against 2^60, no branches.
// The values are wave-uniform; the empty asm statements pin each maximum to a
// scalar register, which keeps the compiler from merging them into a vector
// three-input maximum (a vector result the branch would then wait for), so
// the check stays on the scalar unit.  The elements are copied to scalars
// first: __builtin_bit_cast applied to a vector element reads the vector's
// first element with this compiler.
template <int G>
__device__ __forceinline__ bool huy_sources_ok(const f4 *sq)
{
    uint32_t acc = 0;
#pragma unroll
    for (int u = 0; u < G; ++u) {
        const float x = sq[u].x, y = sq[u].y;
        uint32_t m = max(__builtin_bit_cast(uint32_t, x) & 0x7FFFFFFFu,
                         __builtin_bit_cast(uint32_t, y) & 0x7FFFFFFFu);
        asm("" : "+s"(m));
        acc = max(acc, m);
        asm("" : "+s"(acc));
    }
    return acc < kHuyCoordMaxBits;
}

// WRAP = 0: source j is src[j] (the sum).  WRAP = 8: source j is src[j % 8],
// the term's own ceiling: the same code with the sources served from an
// 8-entry table that stays in the scalar cache, i.e. the arithmetic with
// (almost) no source traffic.  rcp_ok: the launcher's part of the rcp_rn
// condition (2^-48 <= L < 2^60, with SQRT_RN).
template <int WRAP, bool SQRT_RN>
__global__ void __launch_bounds__(256) k_huygens(const float *xo, const float *yo, int64_t P,
                                                 const f4 *__restrict__ src, int32_t S, float k,
                                                 float L, float L2, int rcp_ok, float *re,
                                                 float *im)
{
    static_assert(WRAP == 0 || WRAP % kHuyGroup == 0, "groups stay within the table");
    static_assert(kHuyPoints == 64, "one wave per source block");
    auto at = [](int32_t j) { return WRAP ? (j & (WRAP - 1)) : j; };
    __shared__ float part_re[kHuyBlocks][kHuyPoints], part_im[kHuyBlocks][kHuyPoints];
    const int lane = threadIdx.x % kHuyPoints;
    const int blk = __builtin_amdgcn_readfirstlane(threadIdx.x / kHuyPoints);  // the wave
    // this wave's block of sources: [lo, lo + cnt)
    const int32_t per = (int32_t)(((int64_t)S + kHuyBlocks - 1) / kHuyBlocks);
    const int32_t lo = (int32_t)min<int64_t>(S, (int64_t)blk * per);
    const int32_t cnt = (int32_t)min<int64_t>(S - lo, per);
    const int32_t full = cnt / kHuyGroup * kHuyGroup;  // sources in whole groups
    // k in a vector register: theta = fma(k, d, phi) then reads one scalar
    // operand (phi), which a vector instruction can take without a copy
    float kv;
    asm volatile("v_mov_b32 %0, %1" : "=v"(kv) : "s"(k));
    for (int64_t base = (int64_t)blockIdx.x * kHuyPoints; base < P;
         base += (int64_t)gridDim.x * kHuyPoints) {  // workgroup-uniform loop
        const int64_t i = base + lane;
        const float px = i < P ? xo[i] : 0.f;
        const float py = i < P ? yo[i] : 0.f;
        // wave-uniform: rcp_rn is allowed for this wave's points
        const bool pts_ok =
            SQRT_RN && rcp_ok &&
            __builtin_amdgcn_ballot_w64(!(huy_coord_ok(px) && huy_coord_ok(py))) == 0;
        float ar = 0.0f, ai = 0.0f;
        f4 cur[kHuyGroup];
        bool fast = false;
        if (full > 0) {
#pragma unroll
            for (int u = 0; u < kHuyGroup; ++u)
                cur[u] = src[at(lo + u)];
            fast = pts_ok & huy_sources_ok<kHuyGroup>(cur);
        }
        for (int32_t q = 0; q < full; q += kHuyGroup) {
            // the next group; the last group reloads itself, so every index is < lo + cnt
            const int32_t nq = min(q + kHuyGroup, full - kHuyGroup);
            f4 nxt[kHuyGroup];
#pragma unroll
            for (int u = 0; u < kHuyGroup; ++u)
                nxt[u] = src[at(lo + nq + u)];
            huygens_terms<kHuyGroup, SQRT_RN>(px, py, cur, fast, kv, L, L2, ar, ai);
            // the next group's path, decided once its sources have arrived
            fast = pts_ok & huy_sources_ok<kHuyGroup>(nxt);
#pragma unroll
            for (int u = 0; u < kHuyGroup; ++u)
                cur[u] = nxt[u];
        }
        for (int32_t q = full; q < cnt; ++q) {
            const f4 sq = src[at(lo + q)];
            huygens_terms<1, SQRT_RN>(px, py, &sq, pts_ok & huy_sources_ok<1>(&sq), kv, L, L2,
                                      ar, ai);
        }
        part_re[blk][lane] = ar;
        part_im[blk][lane] = ai;
        __syncthreads();
        if (blk == 0 && i < P) {
            float fr = part_re[0][lane], fi = part_im[0][lane];
#pragma unroll
            for (int b = 1; b < kHuyBlocks; ++b) {
                fr = fr + part_re[b][lane];
                fi = fi + part_im[b][lane];
            }
            re[i] = fr;
            im[i] = fi;
        }
        __syncthreads();  // the partials are read before the next tile writes them
    }
}

// ---------------------------------------------------------------------------
// K7: VALU ceiling for the pair's instruction mix: lane i runs kCeilChains
// independent angle chains theta_r = x_i + r, each step adding 1, for `reps`
// steps, and sums the sines and the cosines of each chain in binary32 in step
// order; out[i] = sum over r, in order, of (sines_r + cosines_r).  Nothing but
// registers between the one load and the one store, so its rate is the VALU's.
constexpr int kCeilChains = 8;

__global__ void __launch_bounds__(256) k_pair_ceiling(const float *x, float *out, int64_t n,
                                                      int32_t reps)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const float x0 = i < n ? x[i] : 0.0f;
    float th[kCeilChains], sums[kCeilChains], sumc[kCeilChains];
#pragma unroll
    for (int r = 0; r < kCeilChains; ++r) {
        th[r] = x0 + (float)r;
        sums[r] = 0.0f;
        sumc[r] = 0.0f;
    }
    for (int32_t j = 0; j < reps; ++j) {
#pragma unroll
        for (int r = 0; r < kCeilChains; ++r) {
            float sv, cv;
            sincos_pair<Arith::Fused, Method::Normalized>(th[r], sv, cv);
            sums[r] = sums[r] + sv;
            sumc[r] = sumc[r] + cv;
            th[r] = th[r] + 1.0f;
        }
    }
    float o = 0.0f;
#pragma unroll
    for (int r = 0; r < kCeilChains; ++r)
        o = o + (sums[r] + sumc[r]);
    if (i < n)
        out[i] = o;
}

// ---------------------------------------------------------------------------
// Launchers.

namespace {

// Tab: RaggedPtrs (device table) or RaggedInline (table in the arguments).
template <Arith A, Method M, class Tab>
hipError_t launch_ragged_am(const Tab &tab, int32_t count, int64_t total_units,
                            const LaunchShape &sh, hipStream_t st)
{
    const int64_t grid = std::max(1, sh.grid);
    const int64_t per = (total_units + grid - 1) / grid;
#define MI355_RAGGED(UU)                                                                          \
    do {                                                                                          \
        if constexpr (std::is_same<Tab, RaggedInline>::value)                                     \
            hipLaunchKernelGGL((k_ragged_inline<A, M, UU>), dim3((unsigned)grid), dim3(sh.block),  \
                               (unsigned)sh.lds, st, tab, count, total_units, per);               \
        else                                                                                      \
            hipLaunchKernelGGL((k_ragged<A, M, UU>), dim3((unsigned)grid), dim3(sh.block),         \
                               (unsigned)sh.lds, st, tab.desc, tab.ubeg, count, total_units, per); \
    } while (0)
    switch (sh.unroll) {
    case 1: MI355_RAGGED(1); break;
    case 2: MI355_RAGGED(2); break;
    case 8: MI355_RAGGED(8); break;
    default: MI355_RAGGED(4); break;
    }
#undef MI355_RAGGED
    return hipGetLastError();
}

template <class Tab>
hipError_t launch_ragged_tab(const Tab &tab, int32_t count, int64_t total_units, int arith,
                             int method, const LaunchShape &sh, hipStream_t st)
{
    const bool m2 = method == (int)Method::Arctan;
    switch (arith) {
    case (int)Arith::Split:
        return m2 ? launch_ragged_am<Arith::Split, Method::Arctan>(tab, count, total_units, sh, st)
                  : launch_ragged_am<Arith::Split, Method::Normalized>(tab, count, total_units, sh, st);
    case (int)Arith::Contract:
        return m2 ? launch_ragged_am<Arith::Contract, Method::Arctan>(tab, count, total_units, sh, st)
                  : launch_ragged_am<Arith::Contract, Method::Normalized>(tab, count, total_units, sh, st);
    default:
        return m2 ? launch_ragged_am<Arith::Fused, Method::Arctan>(tab, count, total_units, sh, st)
                  : launch_ragged_am<Arith::Fused, Method::Normalized>(tab, count, total_units, sh, st);
    }
}

}  // namespace

hipError_t launch_sincos_interleaved(const float *x, float *out, int64_t n, int layout,
                                     hipStream_t st)
{
    const int64_t n4 = n / 4;
    if (n4 > 0) {
        const int per_block = 64 * kIntWaves;
        // one tile per workgroup up to max_grid, grid-stride past it
        const int64_t grid = std::min<int64_t>((n4 + per_block - 1) / per_block, max_grid(per_block));
        if (layout == 0)
            hipLaunchKernelGGL(k_sincos_interleaved<0>, dim3((unsigned)grid), dim3(per_block), 0,
                               st, reinterpret_cast<const f4 *>(x), reinterpret_cast<f4 *>(out), n4);
        else
            hipLaunchKernelGGL(k_sincos_interleaved<1>, dim3((unsigned)grid), dim3(per_block), 0,
                               st, reinterpret_cast<const f4 *>(x), reinterpret_cast<f4 *>(out), n4);
        hipError_t e = hipGetLastError();
        if (e != hipSuccess)
            return e;
    }
    const int64_t rem = n - 4 * n4;
    if (rem > 0) {
        hipLaunchKernelGGL(k_interleaved_tail, dim3(1), dim3(64), 0, st, x, out, n4 * 4, n, layout);
        return hipGetLastError();
    }
    return hipSuccess;
}

hipError_t launch_ragged(const RaggedDesc *desc, const int64_t *ubeg, int32_t count,
                         int64_t total_units, int arith, int method, const LaunchShape &sh,
                         hipStream_t st)
{
    return launch_ragged_tab(RaggedPtrs{desc, ubeg}, count, total_units, arith, method, sh, st);
}

hipError_t launch_ragged_inline(const RaggedInline &tab, int32_t count, int64_t total_units,
                                int arith, int method, const LaunchShape &sh, hipStream_t st)
{
    if (count < 1 || count > kInlineSegs)
        return hipErrorInvalidValue;
    return launch_ragged_tab(tab, count, total_units, arith, method, sh, st);
}

int64_t ragged_units(const RaggedDesc &d, const LaunchShape &sh)
{
    if (d.vec) {
        const int64_t per = (int64_t)sh.block * sh.unroll;
        return std::max<int64_t>(1, (d.n4 + per - 1) / per);
    }
    const int64_t per = (int64_t)sh.block * sh.unroll * 4;
    return (d.n + per - 1) / per;
}

RaggedDesc make_desc(const float *x, float *s, float *c, int64_t n)
{
    RaggedDesc d{x, s, c, n, 0, 0, 0};
    const uintptr_t ax = reinterpret_cast<uintptr_t>(x), as = reinterpret_cast<uintptr_t>(s),
                    ac = reinterpret_cast<uintptr_t>(c);
    const bool same_phase = (ax & 15) == (as & 15) && (ax & 15) == (ac & 15);
    const int64_t head = same_phase ? (int64_t)(((16 - (ax & 15)) & 15) >> 2) : 0;
    if (same_phase && n >= head + 16) {
        d.vec = 1;
        d.head = (int32_t)head;
        d.n4 = (n - head) / 4;
    }
    return d;
}

hipError_t launch_backward(const float *s, const float *c, const float *gs, const float *gc,
                           float *gx, int64_t n, hipStream_t st)
{
    const uintptr_t phase = reinterpret_cast<uintptr_t>(s) & 15;
    bool vec = (reinterpret_cast<uintptr_t>(c) & 15) == phase &&
               (reinterpret_cast<uintptr_t>(gx) & 15) == phase &&
               (!gs || (reinterpret_cast<uintptr_t>(gs) & 15) == phase) &&
               (!gc || (reinterpret_cast<uintptr_t>(gc) & 15) == phase);
    const int64_t head = vec ? (int64_t)(((16 - phase) & 15) >> 2) : 0;
    if (n < head + 4)
        vec = false;
    const int64_t n4 = vec ? (n - head) / 4 : 0;
    const int64_t body_end = vec ? head + 4 * n4 : 0;
    auto scalar = [&](int64_t lo, int64_t hi) {
        if (hi <= lo)
            return;
        const int64_t grid = std::min<int64_t>((hi - lo + 255) / 256, 8192);
#define MI355_BWD_S(GS, GC)                                                                       \
    hipLaunchKernelGGL((k_backward_scalar<GS, GC>), dim3((unsigned)grid), dim3(256), 0, st, s, c, \
                       gs, gc, gx, lo, hi)
        if (gs && gc) MI355_BWD_S(true, true);
        else if (gs) MI355_BWD_S(true, false);
        else if (gc) MI355_BWD_S(false, true);
        else MI355_BWD_S(false, false);
#undef MI355_BWD_S
    };
    if (!vec) {
        scalar(0, n);
        return hipGetLastError();
    }
    scalar(0, head);
    // one float4 per thread, one tile per workgroup (grid-stride past max_grid)
    const int64_t grid = std::max<int64_t>(
        1, std::min<int64_t>((n4 + kBwdBlock - 1) / kBwdBlock, max_grid(kBwdBlock)));
    const f4 *sv = reinterpret_cast<const f4 *>(s + head);
    const f4 *cv = reinterpret_cast<const f4 *>(c + head);
    const f4 *gsv = gs ? reinterpret_cast<const f4 *>(gs + head) : nullptr;
    const f4 *gcv = gc ? reinterpret_cast<const f4 *>(gc + head) : nullptr;
    f4 *gxv = reinterpret_cast<f4 *>(gx + head);
#define MI355_BWD_V(GS, GC)                                                                       \
    hipLaunchKernelGGL((k_backward_vec<GS, GC>), dim3((unsigned)grid), dim3(kBwdBlock),      \
                       kBwdLdsReserve, st, sv, cv, gsv, gcv, gxv, n4)
    if (gs && gc) MI355_BWD_V(true, true);
    else if (gs) MI355_BWD_V(true, false);
    else if (gc) MI355_BWD_V(false, true);
    else MI355_BWD_V(false, false);
#undef MI355_BWD_V
    scalar(body_end, n);
    return hipGetLastError();
}

int64_t sinusoid_fwd_blocks(int64_t N)
{
    // one tile of samples per workgroup; the kernel's grid-stride loop covers
    // any N beyond 2^20 workgroups
    const int64_t per_block = (int64_t)kFwdBlock * kFwdIPT;
    return std::max<int64_t>(1, std::min<int64_t>((N + per_block - 1) / per_block, int64_t(1) << 20));
}

hipError_t launch_sinusoid_forward(const float *t, int64_t N, const float *A, const float *w,
                                   const float *phi, int32_t K, float *y, hipStream_t st)
{
    const int64_t grid = sinusoid_fwd_blocks(N);
    hipLaunchKernelGGL(k_sinusoid_fwd<false>, dim3((unsigned)grid), dim3(kFwdBlock), 0, st, t, N,
                       A, w, phi, K, y, nullptr, nullptr);
    return hipGetLastError();
}

hipError_t launch_sinusoid_residual(const float *t, const float *y_obs, int64_t N, const float *A,
                                    const float *w, const float *phi, int32_t K, float *r,
                                    float *loss, float *part, hipStream_t st)
{
    const int64_t grid = sinusoid_fwd_blocks(N);
    if (N > 0) {
        hipLaunchKernelGGL(k_sinusoid_fwd<true>, dim3((unsigned)grid), dim3(kFwdBlock), 0, st, t,
                           N, A, w, phi, K, r, y_obs, part);
        hipError_t e = hipGetLastError();
        if (e != hipSuccess)
            return e;
    }
    hipLaunchKernelGGL(k_loss_reduce, dim3(1), dim3(256), 0, st, part, N > 0 ? grid : 0, loss);
    return hipGetLastError();
}

hipError_t launch_huygens(const float *xo, const float *yo, int64_t P, const float *src,
                          int32_t S, float k, float L, float *re, float *im, hipStream_t st)
{
    // 64 points per workgroup; grid-stride past 2^20 workgroups
    const int64_t grid = std::min<int64_t>(
        std::max<int64_t>(1, (P + kHuyPoints - 1) / kHuyPoints), int64_t(1) << 20);
    const float L2 = L * L;
    const int rcp_ok = L2 >= kSqrtRnMin && L < 0x1p60f;
    if (L2 >= kSqrtRnMin)
        hipLaunchKernelGGL((k_huygens<0, true>), dim3((unsigned)grid), dim3(256), 0, st, xo, yo,
                           P, reinterpret_cast<const f4 *>(src), S, k, L, L2, rcp_ok, re, im);
    else
        hipLaunchKernelGGL((k_huygens<0, false>), dim3((unsigned)grid), dim3(256), 0, st, xo, yo,
                           P, reinterpret_cast<const f4 *>(src), S, k, L, L2, 0, re, im);
    return hipGetLastError();
}

hipError_t launch_huygens_ceiling(const float *xo, const float *yo, int64_t P, const float *src,
                                  int32_t reps, float k, float L, float *re, float *im,
                                  hipStream_t st)
{
    const int64_t grid = std::min<int64_t>(
        std::max<int64_t>(1, (P + kHuyPoints - 1) / kHuyPoints), int64_t(1) << 20);
    const int64_t S = (int64_t)kHuygensCeilingSources * reps;  // below 2^31: reps < 2^28
    const float L2 = L * L;
    const int rcp_ok = L2 >= kSqrtRnMin && L < 0x1p60f;
    if (L2 >= kSqrtRnMin)
        hipLaunchKernelGGL((k_huygens<kHuygensCeilingSources, true>), dim3((unsigned)grid),
                           dim3(256), 0, st, xo, yo, P, reinterpret_cast<const f4 *>(src),
                           (int32_t)S, k, L, L2, rcp_ok, re, im);
    else
        hipLaunchKernelGGL((k_huygens<kHuygensCeilingSources, false>), dim3((unsigned)grid),
                           dim3(256), 0, st, xo, yo, P, reinterpret_cast<const f4 *>(src),
                           (int32_t)S, k, L, L2, 0, re, im);
    return hipGetLastError();
}

int64_t sinusoid_chunks(int64_t N) { return (N + kAdjChunk - 1) / kAdjChunk; }
int64_t sinusoid_parts(int64_t N) { return (sinusoid_chunks(N) + kAdjWaves - 1) / kAdjWaves; }
int64_t sinusoid_kgroups(int32_t K) { return std::max<int64_t>(1, ((int64_t)K + 63) / 64); }

hipError_t launch_sinusoid_backward(const float *t, const float *g, int64_t N, const float *A,
                                    const float *w, const float *phi, int32_t K, float *gA,
                                    float *gw, float *gphi, float *partial, hipStream_t st)
{
    const int64_t nchunks = sinusoid_chunks(N);
    const int64_t nparts = sinusoid_parts(N);  // one workgroup per kAdjWaves chunks
    const int64_t kg = sinusoid_kgroups(K);
    const int32_t Kpad = (int32_t)(kg * 64);
    if (nchunks > 0) {
        hipLaunchKernelGGL(k_sinusoid_adj, dim3((unsigned)nparts, (unsigned)kg), dim3(64 * kAdjWaves),
                           0, st, t, g, N, w, phi, K, nchunks, partial);
        hipError_t e = hipGetLastError();
        if (e != hipSuccess)
            return e;
    }
    hipLaunchKernelGGL(k_sinusoid_reduce, dim3((unsigned)Kpad, 3), dim3(256), 0, st, partial,
                       nparts, Kpad, K, A, gA, gw, gphi);
    return hipGetLastError();
}

int64_t sinusoid_fit_parts(int64_t N) { return (N + kFitSamples - 1) / kFitSamples; }

hipError_t launch_sinusoid_fit(const float *t, const float *y_obs, int64_t N, const float *A,
                               const float *w, const float *phi, int32_t K, float *loss,
                               float *gA, float *gw, float *gphi, float *partial,
                               float *loss_part, hipStream_t st)
{
    const int64_t nparts = sinusoid_fit_parts(N);
    const int64_t kg = sinusoid_kgroups(K);
    const int32_t Kpad = (int32_t)(kg * 64);
    if (nparts > 0) {
        hipLaunchKernelGGL(k_sinusoid_fit, dim3((unsigned)nparts), dim3(64 * kAdjWaves), 0, st, t,
                           y_obs, N, A, w, phi, K, (int32_t)kg, partial, loss_part);
        hipError_t e = hipGetLastError();
        if (e != hipSuccess)
            return e;
    }
    hipLaunchKernelGGL(k_fit_reduce, dim3((unsigned)Kpad, 4), dim3(256), 0, st, partial, loss_part,
                       nparts, Kpad, K, A, gA, gw, gphi, loss);
    return hipGetLastError();
}

// Library-owned partials of the allocation-free fit step: one copy per GPU,
// held until the process ends.  Host code never passes the array's name to a
// kernel (on the host it is only a stand-in for the symbol); it uses the
// device address that fit_scratch() looks up once per device.
static __device__ __align__(256) float scratch[kFitScratchBytes / sizeof(float)];

hipError_t fit_scratch(int device, float **out)
{
    static std::mutex mu;
    static float *addr[kMaxScratchDevices] = {};
    if (device < 0 || device >= kMaxScratchDevices)
        return hipErrorInvalidDevice;
    std::lock_guard<std::mutex> lk(mu);
    if (!addr[device]) {
        void *p = nullptr;
        const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess)
            return e;
        addr[device] = static_cast<float *>(p);
    }
    *out = addr[device];
    return hipSuccess;
}

hipError_t launch_pair_ceiling(const float *x, float *out, int64_t n, int32_t reps,
                               hipStream_t st)
{
    const int64_t grid = (n + 255) / 256;
    hipLaunchKernelGGL(k_pair_ceiling, dim3((unsigned)grid), dim3(256), 0, st, x, out, n, reps);
    return hipGetLastError();
}

}  // namespace mi355
