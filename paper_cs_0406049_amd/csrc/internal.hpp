// internal.hpp -- declarations shared by the library's translation units
// (kernel launchers, the C ABI and the request server).  Not installed.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <string>
#include <vector>

namespace mi355 {

// One ragged segment as the kernel reads it (device memory, 48 bytes).
struct RaggedDesc {
    const float *x;
    float *s;
    float *c;
    int64_t n;     // elements in the segment
    int64_t n4;    // float4 in the body (vector segments); 0 for scalar ones
    int32_t head;  // scalar elements before the float4 body (vector segments)
    int32_t vec;   // 1: float4 body + head/tail scalars; 0: all scalar
};
static_assert(sizeof(RaggedDesc) == 48, "descriptor layout");

// A launch shape: threads per workgroup, float4 per thread per loop trip,
// workgroups (0 = one per tile / unit of work), bytes of LDS each workgroup
// reserves (0 = none; a reservation caps the workgroups resident per CU).
struct LaunchShape {
    int block = 256;
    int unroll = 1;
    int grid = 0;
    int lds = 0;
};

// Process-wide defaults per form, installed by sincos_set_tuning.
enum { kFormPlain = 0, kFormRagged = 1 };

// Built-in defaults (what sincos_set_tuning(NULL) restores).  Plain form: one
// 64-thread wave per workgroup, one float4 per thread, one tile per
// workgroup -- the fastest measured shape for its 1-read / 2-write stream on
// MI355X (3 % ahead of 256 threads) -- and 7 KiB of LDS reserved per
// workgroup, so that at most 22 are resident per CU: fewer tiles in flight
// keep fewer DRAM rows open at once (1-2 % faster than no cap; a cap below
// about 20 workgroups starves the reads).  Ragged form: 256 threads, where
// the per-unit segment lookup is amortized over more work.
constexpr LaunchShape kBuiltinShape[2] = {{64, 1, 0, 7168}, {256, 1, 0, 0}};
LaunchShape default_shape(int form);
int validate_shape(const LaunchShape &sh, const char *who);

// Device facts the launchers need (cached per device).
struct DeviceInfo {
    int device = -1;
    int cus = 0;
    int arch_ok = 0;
    std::string arch;
};
const DeviceInfo &device_info(int device);

// ---- launchers (plain.hip, forms.hip); each returns the hipError_t of the launch ----
hipError_t launch_sincos(const float *x, float *s, float *c, int64_t n, int arith, int method,
                         const LaunchShape &shape, hipStream_t stream);
hipError_t launch_sincos_interleaved(const float *x, float *out, int64_t n, int layout,
                                     hipStream_t stream);
hipError_t launch_copy_ceiling(const float *x, float *s, float *c, int64_t n,
                               const LaunchShape &shape, hipStream_t stream);
// Memory-traffic probes (probes.hip): the kinds of sincos_stream_probe_f32;
// policy -1 is the plain kernel's cache policy, else the aux bits of the
// probe's stores (of its loads for the read probe).
enum {
    kProbeRead = 0,
    kProbeWrite = 1,
    kProbeWrite1 = 2,
    kProbeCopy = 3,
    kProbeCopyBatch = 4,
    kProbeCopySplit = 5,
    kProbeCopyLds = 6,
    kProbeCopyXcd = 7,
    kProbeCount = 8
};
bool probe_takes_policy(int probe);
bool probe_policy_ok(int policy);
int probe_block(int probe, const LaunchShape &shape);
hipError_t launch_stream_probe(int probe, int policy, const float *x, float *s, float *c,
                               int64_t n, const LaunchShape &shape, hipStream_t stream);
hipError_t launch_pair_ceiling(const float *x, float *out, int64_t n, int32_t reps,
                               hipStream_t stream);
hipError_t launch_ragged(const RaggedDesc *desc, const int64_t *ubeg, int32_t count,
                         int64_t total_units, int arith, int method, const LaunchShape &shape,
                         hipStream_t stream);

// Ablations of Sec. II (ablation.hip): variant in SINCOS_VARIANT_*; the
// general form with ndoub doublings after series of ns and nc terms.
constexpr int kMaxSeriesTerms = 16;
constexpr int kMaxDoublings = 8;
hipError_t launch_variant(const float *x, float *s, float *c, int64_t n, int arith, int method,
                          int variant, hipStream_t stream);
hipError_t launch_doublings(const float *x, float *s, float *c, int64_t n, int arith, int ndoub,
                            const float *ss, int ns, const float *cc, int nc, int fix,
                            hipStream_t stream);

// A small ragged table passed whole as a kernel argument (3.6 KB), so the
// launch needs no staging copy: up to kInlineSegs non-empty segments.
constexpr int kInlineSegs = 64;
struct RaggedInline {
    RaggedDesc desc[kInlineSegs];
    int64_t ubeg[kInlineSegs + 1];
};
static_assert(sizeof(RaggedInline) <= 3600, "kernel arguments stay well under 4 KB");
hipError_t launch_ragged_inline(const RaggedInline &tab, int32_t count, int64_t total_units,
                                int arith, int method, const LaunchShape &shape,
                                hipStream_t stream);
hipError_t launch_backward(const float *s, const float *c, const float *gs, const float *gc,
                           float *gx, int64_t n, hipStream_t stream);
hipError_t launch_sinusoid_forward(const float *t, int64_t N, const float *A, const float *w,
                                   const float *phi, int32_t K, float *y, hipStream_t stream);
int64_t sinusoid_fwd_blocks(int64_t N);
hipError_t launch_sinusoid_residual(const float *t, const float *y_obs, int64_t N, const float *A,
                                    const float *w, const float *phi, int32_t K, float *r,
                                    float *loss, float *part, hipStream_t stream);
hipError_t launch_huygens(const float *xo, const float *yo, int64_t P, const float *src,
                          int32_t S, float k, float L, float *re, float *im, hipStream_t stream);
// The Huygens term over 8 register-resident sources, `reps` passes.
constexpr int kHuygensCeilingSources = 8;
hipError_t launch_huygens_ceiling(const float *xo, const float *yo, int64_t P, const float *src,
                                  int32_t reps, float k, float L, float *re, float *im,
                                  hipStream_t stream);
int64_t sinusoid_chunks(int64_t N);
int64_t sinusoid_parts(int64_t N);
int64_t sinusoid_kgroups(int32_t K);
// One fit step (forward, residual, loss and gradients): workgroup partials of
// the gradients in partial[3][Kpad][parts], of the loss in loss_part[parts].
int64_t sinusoid_fit_parts(int64_t N);
hipError_t launch_sinusoid_fit(const float *t, const float *y_obs, int64_t N, const float *A,
                               const float *w, const float *phi, int32_t K, float *loss,
                               float *gA, float *gw, float *gphi, float *partial,
                               float *loss_part, hipStream_t stream);
// The allocation-free fit step's partials live in a static device array of
// kFitScratchBytes per GPU; fit_scratch() returns its device address on
// `device` (which must be current), looked up on the first call per device.
constexpr int64_t kFitScratchBytes = int64_t(8) << 20;
constexpr int kMaxScratchDevices = 64;
hipError_t fit_scratch(int device, float **out);
hipError_t launch_sinusoid_backward(const float *t, const float *g, int64_t N, const float *A,
                                    const float *w, const float *phi, int32_t K, float *gA,
                                    float *gw, float *gphi, float *partial, hipStream_t stream);

// Units of work of one ragged segment for a launch shape (host and plan use).
int64_t ragged_units(const RaggedDesc &d, const LaunchShape &shape);
// Build a descriptor for (x, s, c, n); n > 0.
RaggedDesc make_desc(const float *x, float *s, float *c, int64_t n);

// Default launch shapes (resolved against the device).
// Most workgroups one launch of `block`-thread workgroups may have: 2^30,
// and grid * block below 2^32 (the dispatch packet counts work-items in 32
// bits).  The streaming kernels take one tile per workgroup up to this and
// grid-stride past it.
inline int64_t max_grid(int block)
{
    const int64_t by_items = int64_t(UINT32_MAX) / (block > 0 ? block : 1);
    return by_items < (int64_t(1) << 30) ? by_items : (int64_t(1) << 30);
}
LaunchShape resolve_plain_shape(const LaunchShape &req, int64_t n, const DeviceInfo &dev);
LaunchShape resolve_ragged_shape(const LaunchShape &req, int64_t total_units,
                                 const DeviceInfo &dev);

// Host table of a ragged batch: descriptors of the non-empty segments, then
// their first-unit offsets (count + 1 entries).
struct RaggedTable {
    std::vector<RaggedDesc> desc;
    std::vector<int64_t> ubeg;
    int64_t elements = 0;
};
// Append one segment (n > 0) to a table under construction.
void table_add(RaggedTable &t, const float *x, float *s, float *c, int64_t n,
               const LaunchShape &shape);
// Pinned host + device buffers for one staged descriptor table.
struct StagingBuffers {
    char *host = nullptr;
    char *dev = nullptr;
    size_t cap = 0;
};
size_t staged_bytes(const RaggedTable &t);
// Make b hold at least `bytes` (reallocates; the caller knows b is idle).
int grow_staging(StagingBuffers &b, size_t bytes);
void free_staging(StagingBuffers &b);
// Copy the table into `host`, enqueue its copy to `dev_buf` and the ragged
// kernel on `stream`.  The buffers must stay untouched until the stream has
// passed the launch.
int stage_and_launch(const RaggedTable &t, char *host, char *dev_buf, int arith, int method,
                     const LaunchShape &shape, const DeviceInfo &dev, hipStream_t stream);
// Launch a table of at most kInlineSegs segments with the table in the
// kernel arguments (nothing to stage or keep alive).
int launch_table_inline(const RaggedTable &t, int arith, int method, const LaunchShape &shape,
                        const DeviceInfo &dev, hipStream_t stream);
// Launch the ragged kernel on `stream`: small tables inline, larger ones
// staged through the library's pinned/device ring.  Returns a sincos status.
int ragged_enqueue(const RaggedTable &t, int arith, int method, const LaunchShape &shape,
                   const DeviceInfo &dev, hipStream_t stream);

// Thread-local error reporting used by every C entry point.
int set_error(int status, const std::string &msg);
void clear_error();

}  // namespace mi355
