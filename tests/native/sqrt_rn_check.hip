// sqrt_rn_check.hip -- test helper: compares the library's sqrt_rn (and
// sqrt_rn_finite) with the compiler's IEEE (correctly rounded) binary32
// square root on every bit pattern in [lo, hi], on the GPU.  With `planted` set it compares against
// the IEEE root of the next binary32 instead, a difference the check must
// report (so that a check that sees nothing cannot pass).  Built by __graft_entry__.build() into
// tests/native/libsqrt_rn_check.so; used by tests/test_gpu_sqrt_rn.py.
#include <hip/hip_runtime.h>

#include <cstdint>

#include "../../paper_cs_0406049_amd/csrc/sqrt_rn.hpp"

template <int FINITE>
__global__ void k_sqrt_rn_check(uint32_t lo, uint32_t hi, int planted,
                                unsigned long long *mismatches, uint32_t *first_bad)
{
    const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
    for (uint64_t b = (uint64_t)lo + (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; b <= hi;
         b += stride) {
        const float x = __builtin_bit_cast(float, (uint32_t)b);
        const float got = FINITE ? mi355::sqrt_rn_finite(x) : mi355::sqrt_rn(x);
        const float want = __builtin_sqrtf(
            planted ? __builtin_bit_cast(float, (uint32_t)b + 1u) : x);
        const bool same = __builtin_bit_cast(uint32_t, got) == __builtin_bit_cast(uint32_t, want) ||
                          (got != got && want != want);
        if (!same) {
            atomicAdd(mismatches, 1ull);
            atomicMin(first_bad, (uint32_t)b);
        }
    }
}

// Returns 0 on success (counts in *mismatches and the smallest mismatching
// bit pattern in *first_bad, 0xffffffff if none), else a hipError_t.
template <int FINITE>
static int run_check(uint32_t lo, uint32_t hi, int planted, unsigned long long *mismatches,
                     uint32_t *first_bad)
{
    if (lo > hi || !mismatches || !first_bad)
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
    if (e == hipSuccess) {
        hipLaunchKernelGGL(k_sqrt_rn_check<FINITE>, dim3(4096), dim3(256), 0, 0, lo, hi, planted,
                           d_count, d_first);
        e = hipGetLastError();
    }
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

// sqrt_rn, and sqrt_rn_finite (the five-instruction root for finite
// arguments), against the IEEE square root.
extern "C" __attribute__((visibility("default"))) int sqrt_rn_check(
    uint32_t lo, uint32_t hi, int planted, unsigned long long *mismatches, uint32_t *first_bad)
{
    return run_check<0>(lo, hi, planted, mismatches, first_bad);
}

extern "C" __attribute__((visibility("default"))) int sqrt_rn_finite_check(
    uint32_t lo, uint32_t hi, int planted, unsigned long long *mismatches, uint32_t *first_bad)
{
    return run_check<1>(lo, hi, planted, mismatches, first_bad);
}
