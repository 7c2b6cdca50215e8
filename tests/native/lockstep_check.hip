// lockstep_check.hip -- test helper: compares the library's pair arithmetic on
// N-element vectors (N pairs per lane in lockstep, as the Huygens kernel
// evaluates a group of sources) with the same arithmetic on one float, on
// every binary32 bit pattern in [lo, hi], on the GPU.  Lane element u takes
// the pattern b + u * 0x9E3779B9 (mod 2^32), so the N elements of a vector
// hold unrelated arguments and the range covers every pattern in each
// element.  With `planted` set the scalar side takes the next bit pattern
// instead, a difference the check must report.  Built by
// __graft_entry__.build() into tests/native/liblockstep_check.so; used by
// tests/test_gpu_lockstep.py.
#include <hip/hip_runtime.h>

#include <cstdint>

#include "../../paper_cs_0406049_amd/csrc/sincos_core.hpp"

using namespace mi355;

__device__ __forceinline__ bool same_bits(float a, float b)
{
    return __builtin_bit_cast(uint32_t, a) == __builtin_bit_cast(uint32_t, b) ||
           (a != a && b != b);
}

template <int N, Arith A, Method M>
__global__ void k_lockstep_check(uint32_t lo, uint32_t hi, int planted,
                                 unsigned long long *mismatches, uint32_t *first_bad)
{
    const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
    for (uint64_t b = (uint64_t)lo + (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; b <= hi;
         b += stride) {
        uint32_t bits[N];
        fvec<N> th, s, c;
#pragma unroll
        for (int u = 0; u < N; ++u) {
            bits[u] = (uint32_t)b + (uint32_t)u * 0x9E3779B9u;
            th[u] = __builtin_bit_cast(float, bits[u]);
        }
        pair_exact<A, M>(th, s, c);
        bool ok = true;
#pragma unroll
        for (int u = 0; u < N; ++u) {
            float s1, c1;
            pair_exact<A, M>(__builtin_bit_cast(float, bits[u] + (planted ? 1u : 0u)), s1, c1);
            const float su = s[u], cu = c[u];  // scalar copies before the comparison
            ok = ok && same_bits(su, s1) && same_bits(cu, c1);
        }
        if (!ok) {
            atomicAdd(mismatches, 1ull);
            atomicMin(first_bad, (uint32_t)b);
        }
    }
}

template <int N, Arith A, Method M>
static hipError_t launch(uint32_t lo, uint32_t hi, int planted, unsigned long long *d_count,
                         uint32_t *d_first)
{
    hipLaunchKernelGGL((k_lockstep_check<N, A, M>), dim3(4096), dim3(256), 0, 0, lo, hi, planted,
                       d_count, d_first);
    return hipGetLastError();
}

template <int N>
static hipError_t dispatch(int arith, int method, uint32_t lo, uint32_t hi, int planted,
                           unsigned long long *d_count, uint32_t *d_first)
{
    if (arith == 0 && method == 0)
        return launch<N, Arith::Fused, Method::Normalized>(lo, hi, planted, d_count, d_first);
    if (arith == 0 && method == 1)
        return launch<N, Arith::Fused, Method::Arctan>(lo, hi, planted, d_count, d_first);
    if (arith == 1 && method == 0)
        return launch<N, Arith::Split, Method::Normalized>(lo, hi, planted, d_count, d_first);
    return launch<N, Arith::Split, Method::Arctan>(lo, hi, planted, d_count, d_first);
}

// width: 2 or 4 pairs per lane; arith: 0 fused, 1 split; method: 0 first,
// 1 second.  Returns 0 on success (the number of mismatching patterns b in
// *mismatches and the smallest in *first_bad, 0xffffffff if none), else a
// hipError_t.
extern "C" __attribute__((visibility("default"))) int lockstep_check(
    int width, int arith, int method, uint32_t lo, uint32_t hi, int planted,
    unsigned long long *mismatches, uint32_t *first_bad)
{
    if (lo > hi || !mismatches || !first_bad || (width != 2 && width != 4) || arith < 0 ||
        arith > 1 || method < 0 || method > 1)
        return (int)hipErrorInvalidValue;
    unsigned long long *d_count = nullptr;
    uint32_t *d_first = nullptr;
    hipError_t e = hipMalloc((void **)&d_count, sizeof *d_count);
    if (e == hipSuccess)
        e = hipMalloc((void **)&d_first, sizeof *d_first);
    const unsigned long long zero = 0;
    const uint32_t none = 0xffffffffu;
    if (e == hipSuccess)
        e = hipMemcpy(d_count, &zero, sizeof zero, hipMemcpyHostToDevice);
    if (e == hipSuccess)
        e = hipMemcpy(d_first, &none, sizeof none, hipMemcpyHostToDevice);
    if (e == hipSuccess)
        e = width == 2 ? dispatch<2>(arith, method, lo, hi, planted, d_count, d_first)
                       : dispatch<4>(arith, method, lo, hi, planted, d_count, d_first);
    if (e == hipSuccess)
        e = hipMemcpy(mismatches, d_count, sizeof *mismatches, hipMemcpyDeviceToHost);
    if (e == hipSuccess)
        e = hipMemcpy(first_bad, d_first, sizeof *first_bad, hipMemcpyDeviceToHost);
    if (d_count)
        (void)hipFree(d_count);
    if (d_first)
        (void)hipFree(d_first);
    return (int)e;
}
