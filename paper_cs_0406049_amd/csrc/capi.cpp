// capi.cpp -- the C ABI of libmi355_sincos.so (declared in include/sincos.h):
// argument checks, launch-shape resolution, descriptor staging for the ragged
// form, ragged plans with graph replay, and error reporting.
#include "../../include/sincos.h"
#include "internal.hpp"

#include <algorithm>
#include <climits>
#include <cstdio>
#include <cstring>
#include <initializer_list>
#include <map>
#include <memory>
#include <mutex>
#include <string>
#include <vector>

namespace mi355 {

// ---------------------------------------------------------------------------
// Errors

static thread_local std::string g_last_error;

int set_error(int status, const std::string &msg)
{
    g_last_error = msg;
    return status;
}

void clear_error() { g_last_error.clear(); }

static int hip_error(hipError_t e, const char *what)
{
    return set_error(SINCOS_EHIP, std::string(what) + ": " + hipGetErrorString(e));
}

// ---------------------------------------------------------------------------
// Device facts

static std::mutex g_dev_mu;
static std::map<int, std::unique_ptr<DeviceInfo>> g_devs;

const DeviceInfo &device_info(int device)
{
    std::lock_guard<std::mutex> lk(g_dev_mu);
    auto it = g_devs.find(device);
    if (it != g_devs.end())
        return *it->second;
    auto info = std::make_unique<DeviceInfo>();
    info->device = device;
    hipDeviceProp_t prop;
    if (hipGetDeviceProperties(&prop, device) == hipSuccess) {
        info->cus = prop.multiProcessorCount;
        info->arch = prop.gcnArchName;
        info->arch_ok = std::strncmp(prop.gcnArchName, "gfx950", 6) == 0;
    }
    const DeviceInfo &ref = *info;
    g_devs[device] = std::move(info);
    return ref;
}

// The current device, checked to be a gfx950.
static int current_device(const DeviceInfo **out)
{
    int dev = -1;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess)
        return set_error(SINCOS_ENODEV, std::string("no HIP device: ") + hipGetErrorString(e));
    const DeviceInfo &info = device_info(dev);
    if (!info.arch_ok)
        return set_error(SINCOS_ENODEV, "device " + std::to_string(dev) + " is " +
                                             (info.arch.empty() ? "unknown" : info.arch) +
                                             ", this library is built for gfx950 only");
    *out = &info;
    return SINCOS_OK;
}

// ---------------------------------------------------------------------------
// Launch shapes

// A caller's shape over the form's current default (0 in a field = default).
static int check_shape(const sincos_launch_t *req, int form, LaunchShape *out)
{
    LaunchShape sh = default_shape(form);
    if (req) {
        if (req->block != 0)
            sh.block = req->block;
        if (req->unroll != 0)
            sh.unroll = req->unroll;
        if (req->grid != 0)
            sh.grid = req->grid;
        if (req->lds != 0)
            sh.lds = req->lds < 0 ? 0 : req->lds;
    }
    const int rc = validate_shape(sh, "launch");
    if (rc == SINCOS_OK)
        *out = sh;
    return rc;
}

LaunchShape resolve_ragged_shape(const LaunchShape &req, int64_t total_units,
                                 const DeviceInfo &dev)
{
    (void)dev;
    LaunchShape sh = req;
    // default: one workgroup per unit of work (measured faster than a
    // persistent grid); a requested grid is capped to the number of units
    // and to max_grid; each workgroup then takes a contiguous run of units
    const int64_t cap = std::min<int64_t>(std::max<int64_t>(total_units, 1), max_grid(sh.block));
    sh.grid = (int)(sh.grid <= 0 ? cap : std::min<int64_t>(sh.grid, cap));
    return sh;
}

// ---------------------------------------------------------------------------
// Argument checks

static bool ranges_overlap(const void *a, int64_t na, const void *b, int64_t nb)
{
    const uintptr_t pa = reinterpret_cast<uintptr_t>(a), pb = reinterpret_cast<uintptr_t>(b);
    return pa < pb + (uintptr_t)nb * 4 && pb < pa + (uintptr_t)na * 4;
}

static bool aligned4(const void *p) { return (reinterpret_cast<uintptr_t>(p) & 3) == 0; }

// A device array of n floats, named for error messages (n <= 0 or a null
// pointer: nothing to check).
struct Span {
    const void *p;
    int64_t n;
    const char *name;
};

// Every output span disjoint from every input span and from the other
// outputs; `same_ok` lets an output equal one input exactly (in place).
static int check_disjoint(std::initializer_list<Span> outs, std::initializer_list<Span> ins,
                          const char *who, const void *same_ok_out = nullptr,
                          const void *same_ok_in_a = nullptr, const void *same_ok_in_b = nullptr)
{
    auto live = [](const Span &a) { return a.p && a.n > 0; };
    for (auto o = outs.begin(); o != outs.end(); ++o) {
        if (!live(*o))
            continue;
        for (auto q = o + 1; q != outs.end(); ++q)
            if (live(*q) && ranges_overlap(o->p, o->n, q->p, q->n))
                return set_error(SINCOS_EOVERLAP, std::string(who) + ": " + o->name + " overlaps " +
                                                      q->name);
        for (const Span &in : ins) {
            if (!live(in) || !ranges_overlap(o->p, o->n, in.p, in.n))
                continue;
            const bool in_place = o->p == same_ok_out && in.p == o->p && in.n == o->n &&
                                  (in.p == same_ok_in_a || in.p == same_ok_in_b);
            if (!in_place)
                return set_error(SINCOS_EOVERLAP, std::string(who) + ": " + o->name + " overlaps " +
                                                      in.name);
        }
    }
    return SINCOS_OK;
}

static bool all_aligned4(std::initializer_list<const void *> ps)
{
    for (const void *p : ps)
        if (p && !aligned4(p))
            return false;
    return true;
}

static int check_triplet(const float *x, const float *s, const float *c, int64_t n,
                         const char *who)
{
    if (n < 0)
        return set_error(SINCOS_EINVAL, std::string(who) + ": n < 0");
    if (n == 0)
        return SINCOS_OK;
    if (!x || !s || !c)
        return set_error(SINCOS_EINVAL, std::string(who) + ": null pointer with n > 0");
    if (!aligned4(x) || !aligned4(s) || !aligned4(c))
        return set_error(SINCOS_EINVAL, std::string(who) + ": pointers must be 4-byte aligned");
    if (n > (int64_t(1) << 60))
        return set_error(SINCOS_EINVAL, std::string(who) + ": n too large");
    if (ranges_overlap(s, n, c, n))
        return set_error(SINCOS_EOVERLAP, std::string(who) + ": s and c overlap");
    if (x != s && ranges_overlap(x, n, s, n))
        return set_error(SINCOS_EOVERLAP, std::string(who) + ": x partially overlaps s");
    if (x != c && ranges_overlap(x, n, c, n))
        return set_error(SINCOS_EOVERLAP, std::string(who) + ": x partially overlaps c");
    return SINCOS_OK;
}

static int check_modes(int32_t arith, int32_t method)
{
    if (arith < 0 || arith > 2)
        return set_error(SINCOS_EINVAL, "arith must be FUSED, SPLIT or CONTRACT");
    if (method < 0 || method > 1)
        return set_error(SINCOS_EINVAL, "method must be NORMALIZED or ARCTAN");
    return SINCOS_OK;
}

// Cross-segment aliasing: outputs pairwise disjoint; an input may overlap an
// output only as the exact in-place case of its own segment.
struct Interval {
    uintptr_t lo, hi;
    int32_t seg;
};

static int check_ragged_aliasing(const sincos_seg_t *segs, const int64_t *lens, int32_t count)
{
    std::vector<Interval> outs;
    outs.reserve((size_t)count * 2);
    for (int32_t j = 0; j < count; ++j) {
        if (lens[j] == 0)
            continue;
        const uintptr_t b = (uintptr_t)lens[j] * 4;
        outs.push_back({reinterpret_cast<uintptr_t>(segs[j].s), reinterpret_cast<uintptr_t>(segs[j].s) + b, j});
        outs.push_back({reinterpret_cast<uintptr_t>(segs[j].c), reinterpret_cast<uintptr_t>(segs[j].c) + b, j});
    }
    std::sort(outs.begin(), outs.end(), [](const Interval &a, const Interval &b) { return a.lo < b.lo; });
    for (size_t i = 1; i < outs.size(); ++i)
        if (outs[i].lo < outs[i - 1].hi)
            return set_error(SINCOS_EOVERLAP, "ragged: outputs of segments " +
                                                  std::to_string(outs[i - 1].seg) + " and " +
                                                  std::to_string(outs[i].seg) + " overlap");
    for (int32_t j = 0; j < count; ++j) {
        if (lens[j] == 0)
            continue;
        const uintptr_t lo = reinterpret_cast<uintptr_t>(segs[j].x), hi = lo + (uintptr_t)lens[j] * 4;
        auto it = std::lower_bound(outs.begin(), outs.end(), hi,
                                   [](const Interval &a, uintptr_t v) { return a.lo < v; });
        if (it == outs.begin())
            continue;
        --it;  // the output with the largest start below hi
        if (it->hi <= lo)
            continue;
        if (!(it->seg == j && it->lo == lo))
            return set_error(SINCOS_EOVERLAP, "ragged: input of segment " + std::to_string(j) +
                                                  " overlaps an output of segment " +
                                                  std::to_string(it->seg));
    }
    return SINCOS_OK;
}

static int check_ragged(const sincos_seg_t *segs, const int64_t *lens, int32_t count)
{
    if (count < 0)
        return set_error(SINCOS_EINVAL, "ragged: count < 0");
    if (count == 0)
        return SINCOS_OK;
    if (!segs || !lens)
        return set_error(SINCOS_EINVAL, "ragged: null segment or length table");
    for (int32_t j = 0; j < count; ++j) {
        int rc = check_triplet(segs[j].x, segs[j].s, segs[j].c, lens[j], "ragged segment");
        if (rc != SINCOS_OK)
            return set_error(rc, g_last_error + " (segment " + std::to_string(j) + ")");
    }
    return check_ragged_aliasing(segs, lens, count);
}

void table_add(RaggedTable &t, const float *x, float *s, float *c, int64_t n,
               const LaunchShape &sh)
{
    if (t.ubeg.empty())
        t.ubeg.push_back(0);
    RaggedDesc d = make_desc(x, s, c, n);
    t.desc.push_back(d);
    t.ubeg.push_back(t.ubeg.back() + ragged_units(d, sh));
    t.elements += n;
}

static void build_table(const sincos_seg_t *segs, const int64_t *lens, int32_t count,
                        const LaunchShape &sh, RaggedTable &t)
{
    t.desc.clear();
    t.ubeg.assign(1, 0);
    t.elements = 0;
    for (int32_t j = 0; j < count; ++j)
        if (lens[j] > 0)
            table_add(t, segs[j].x, segs[j].s, segs[j].c, lens[j], sh);
}

// ---------------------------------------------------------------------------
// Staging ring for one-shot ragged calls: pinned host + device buffer per
// slot, reused once the event recorded after its last use has completed.

struct StageSlot {
    StagingBuffers buf;
    hipEvent_t done = nullptr;
    bool pending = false;
};

struct StageRing {
    std::mutex mu;
    std::vector<StageSlot> slots;
    size_t next = 0;
};

static std::mutex g_ring_mu;
static std::map<int, std::unique_ptr<StageRing>> g_rings;
constexpr int kStageSlots = 8;

static StageRing &ring_for(int device)
{
    std::lock_guard<std::mutex> lk(g_ring_mu);
    auto &r = g_rings[device];
    if (!r) {
        r = std::make_unique<StageRing>();
        r->slots.resize(kStageSlots);
    }
    return *r;
}

size_t staged_bytes(const RaggedTable &t)
{
    return sizeof(RaggedDesc) * t.desc.size() + sizeof(int64_t) * t.ubeg.size();
}

int stage_and_launch(const RaggedTable &t, char *host, char *dev_buf, int arith, int method,
                     const LaunchShape &shape, const DeviceInfo &dev, hipStream_t stream)
{
    const int32_t count = (int32_t)t.desc.size();
    if (count == 0)
        return SINCOS_OK;
    const int64_t total = t.ubeg.back();
    const LaunchShape sh = resolve_ragged_shape(shape, total, dev);
    const size_t desc_bytes = sizeof(RaggedDesc) * (size_t)count;
    const size_t bytes = staged_bytes(t);
    std::memcpy(host, t.desc.data(), desc_bytes);
    std::memcpy(host + desc_bytes, t.ubeg.data(), sizeof(int64_t) * (size_t)(count + 1));
    hipError_t e = hipMemcpyAsync(dev_buf, host, bytes, hipMemcpyHostToDevice, stream);
    if (e != hipSuccess)
        return hip_error(e, "ragged: staging copy");
    e = launch_ragged(reinterpret_cast<const RaggedDesc *>(dev_buf),
                      reinterpret_cast<const int64_t *>(dev_buf + desc_bytes), count, total, arith,
                      method, sh, stream);
    if (e != hipSuccess)
        return hip_error(e, "ragged: kernel launch");
    return SINCOS_OK;
}

int launch_table_inline(const RaggedTable &t, int arith, int method, const LaunchShape &shape,
                        const DeviceInfo &dev, hipStream_t stream)
{
    const int32_t count = (int32_t)t.desc.size();
    if (count == 0)
        return SINCOS_OK;
    if (count > kInlineSegs)
        return set_error(SINCOS_EINVAL, "ragged: table too large to pass inline");
    const int64_t total = t.ubeg.back();
    RaggedInline tab{};
    std::memcpy(tab.desc, t.desc.data(), sizeof(RaggedDesc) * (size_t)count);
    std::memcpy(tab.ubeg, t.ubeg.data(), sizeof(int64_t) * (size_t)(count + 1));
    const hipError_t e = launch_ragged_inline(tab, count, total, arith, method,
                                              resolve_ragged_shape(shape, total, dev), stream);
    return e == hipSuccess ? SINCOS_OK : hip_error(e, "ragged: kernel launch");
}

int grow_staging(StagingBuffers &b, size_t bytes)
{
    if (b.cap >= bytes)
        return SINCOS_OK;
    if (b.host)
        (void)hipHostFree(b.host);
    if (b.dev)
        (void)hipFree(b.dev);
    b.host = nullptr;
    b.dev = nullptr;
    b.cap = 0;
    const size_t cap = std::max<size_t>(bytes, 64 * 1024);
    if (hipHostMalloc((void **)&b.host, cap, hipHostMallocDefault) != hipSuccess ||
        hipMalloc((void **)&b.dev, cap) != hipSuccess) {
        if (b.host)
            (void)hipHostFree(b.host);
        b.host = nullptr;
        b.dev = nullptr;
        return set_error(SINCOS_ENOMEM, "ragged: cannot allocate the staging buffers");
    }
    b.cap = cap;
    return SINCOS_OK;
}

void free_staging(StagingBuffers &b)
{
    if (b.host)
        (void)hipHostFree(b.host);
    if (b.dev)
        (void)hipFree(b.dev);
    b = StagingBuffers{};
}

int ragged_enqueue(const RaggedTable &t, int arith, int method, const LaunchShape &shape,
                   const DeviceInfo &dev, hipStream_t stream)
{
    if (t.desc.empty())
        return SINCOS_OK;
    if (t.desc.size() <= (size_t)kInlineSegs)  // small tables need no staging
        return launch_table_inline(t, arith, method, shape, dev, stream);
    StageRing &ring = ring_for(dev.device);
    std::lock_guard<std::mutex> lk(ring.mu);
    StageSlot &slot = ring.slots[ring.next];
    ring.next = (ring.next + 1) % ring.slots.size();
    hipError_t e;
    if (slot.pending) {
        e = hipEventSynchronize(slot.done);
        if (e != hipSuccess)
            return hip_error(e, "ragged: waiting for a staging slot");
        slot.pending = false;
    }
    int rc = grow_staging(slot.buf, staged_bytes(t));
    if (rc != SINCOS_OK)
        return rc;
    if (!slot.done && hipEventCreateWithFlags(&slot.done, hipEventDisableTiming) != hipSuccess)
        return set_error(SINCOS_EHIP, "ragged: cannot create an event");
    rc = stage_and_launch(t, slot.buf.host, slot.buf.dev, arith, method, shape, dev, stream);
    // Guard the slot even when the launch failed: the staging copy may already
    // be enqueued and still read the pinned buffer.
    e = hipEventRecord(slot.done, stream);
    if (e == hipSuccess)
        slot.pending = true;
    else
        (void)hipStreamSynchronize(stream);  // the slot cannot be proven idle: drain instead
    if (rc != SINCOS_OK)
        return rc;
    return e == hipSuccess ? SINCOS_OK : hip_error(e, "ragged: event record");
}

}  // namespace mi355

using namespace mi355;

// ---------------------------------------------------------------------------
// Plain form

extern "C" int sincos_f32_ex(const float *x, float *s, float *c, int64_t n, int32_t arith,
                             int32_t method, const sincos_launch_t *launch, void *stream)
{
    clear_error();
    int rc = check_triplet(x, s, c, n, "sincos_f32");
    if (rc != SINCOS_OK)
        return rc;
    if ((rc = check_modes(arith, method)) != SINCOS_OK)
        return rc;
    LaunchShape sh;
    if ((rc = check_shape(launch, kFormPlain, &sh)) != SINCOS_OK)
        return rc;
    if (n == 0)
        return SINCOS_OK;
    const DeviceInfo *dev;
    if ((rc = current_device(&dev)) != SINCOS_OK)
        return rc;
    hipError_t e = launch_sincos(x, s, c, n, arith, method, resolve_plain_shape(sh, n, *dev),
                                 (hipStream_t)stream);
    return e == hipSuccess ? SINCOS_OK : hip_error(e, "sincos_f32: kernel launch");
}

extern "C" int sincos_f32(const float *x, float *s, float *c, int64_t n, void *stream)
{
    return sincos_f32_ex(x, s, c, n, SINCOS_ARITH_FUSED, SINCOS_METHOD_NORMALIZED, nullptr,
                         stream);
}

extern "C" int sincos_f32_interleaved(const float *x, float *out, int64_t n, int32_t layout,
                                      void *stream)
{
    clear_error();
    if (n < 0)
        return set_error(SINCOS_EINVAL, "sincos_f32_interleaved: n < 0");
    if (layout != 0 && layout != 1)
        return set_error(SINCOS_EINVAL, "sincos_f32_interleaved: layout must be 0 or 1");
    if (n == 0)
        return SINCOS_OK;
    if (!x || !out)
        return set_error(SINCOS_EINVAL, "sincos_f32_interleaved: null pointer with n > 0");
    if ((reinterpret_cast<uintptr_t>(x) | reinterpret_cast<uintptr_t>(out)) & 15)
        return set_error(SINCOS_EINVAL, "sincos_f32_interleaved: x and out must be 16-byte aligned");
    if (n > (int64_t(1) << 36))  // 256 GiB of angles: beyond any device memory
        return set_error(SINCOS_EINVAL, "sincos_f32_interleaved: n too large");
    // out holds 2n floats (layout 1 rounds the last block up to 8 floats)
    const int64_t out_floats = layout == 0 ? 2 * n : 8 * ((n + 3) / 4);
    if (ranges_overlap(x, n, out, out_floats))
        return set_error(SINCOS_EOVERLAP, "sincos_f32_interleaved: x overlaps out");
    const DeviceInfo *dev;
    int rc;
    if ((rc = current_device(&dev)) != SINCOS_OK)
        return rc;
    hipError_t e = launch_sincos_interleaved(x, out, n, layout, (hipStream_t)stream);
    return e == hipSuccess ? SINCOS_OK : hip_error(e, "sincos_f32_interleaved: kernel launch");
}

extern "C" int sincos_copy_ceiling_f32(const float *x, float *s, float *c, int64_t n,
                                       const sincos_launch_t *launch, void *stream)
{
    clear_error();
    int rc = check_triplet(x, s, c, n, "sincos_copy_ceiling_f32");
    if (rc != SINCOS_OK)
        return rc;
    if (x == s || x == c)
        return set_error(SINCOS_EOVERLAP, "sincos_copy_ceiling_f32: no in-place use");
    const uintptr_t bits = reinterpret_cast<uintptr_t>(x) | reinterpret_cast<uintptr_t>(s) |
                           reinterpret_cast<uintptr_t>(c);
    if ((bits & 15) != 0 || n % 4 != 0)
        return set_error(SINCOS_EINVAL,
                         "sincos_copy_ceiling_f32: needs 16-byte aligned arrays and n % 4 == 0");
    LaunchShape sh;
    if ((rc = check_shape(launch, kFormPlain, &sh)) != SINCOS_OK)
        return rc;
    if (n == 0)
        return SINCOS_OK;
    const DeviceInfo *dev;
    if ((rc = current_device(&dev)) != SINCOS_OK)
        return rc;
    hipError_t e = launch_copy_ceiling(x, s, c, n, resolve_plain_shape(sh, n, *dev),
                                       (hipStream_t)stream);
    return e == hipSuccess ? SINCOS_OK : hip_error(e, "sincos_copy_ceiling_f32: kernel launch");
}

extern "C" int sincos_stream_probe_f32(int32_t probe, int32_t policy, const float *x, float *s,
                                       float *c, int64_t n, const sincos_launch_t *launch,
                                       void *stream)
{
    clear_error();
    const char *who = "sincos_stream_probe_f32";
    if (probe < 0 || probe >= kProbeCount)
        return set_error(SINCOS_EINVAL, std::string(who) + ": unknown probe " +
                                            std::to_string(probe));
    if (!probe_policy_ok(policy) || (policy != -1 && !probe_takes_policy(probe)))
        return set_error(SINCOS_EINVAL, std::string(who) + ": policy " + std::to_string(policy) +
                                            " not available for this probe");
    if (n < 0 || n % 4 != 0)
        return set_error(SINCOS_EINVAL, std::string(who) + ": n must be >= 0 and a multiple of 4");
    const bool reads = probe != kProbeWrite && probe != kProbeWrite1;
    const bool writes_c = probe != kProbeRead && probe != kProbeWrite1;
    if ((reads && !x) || !s || (writes_c && !c))
        return set_error(SINCOS_EINVAL, std::string(who) + ": null array");
    const uintptr_t bits = reinterpret_cast<uintptr_t>(reads ? x : nullptr) |
                           reinterpret_cast<uintptr_t>(s) |
                           reinterpret_cast<uintptr_t>(writes_c ? c : nullptr);
    if ((bits & 15) != 0)
        return set_error(SINCOS_EINVAL, std::string(who) + ": arrays must be 16-byte aligned");
    // outputs: s (one float for the read probe) and c; input: x
    const int64_t ns = probe == kProbeRead ? 1 : n;
    int rc = check_disjoint({{s, ns, "s"}, {writes_c ? c : nullptr, n, "c"}},
                            {{reads ? x : nullptr, n, "x"}}, who);
    if (rc != SINCOS_OK)
        return rc;
    LaunchShape sh;
    if ((rc = check_shape(launch, kFormPlain, &sh)) != SINCOS_OK)
        return rc;
    // the XCD schedule launches up to twice the tiles: keep grid * block below 2^32
    if (probe == kProbeCopyXcd && n / 4 > (int64_t(1) << 30))
        return set_error(SINCOS_EINVAL, std::string(who) + ": n too large for the XCD schedule");
    if (n == 0)
        return SINCOS_OK;
    const DeviceInfo *dev;
    if ((rc = current_device(&dev)) != SINCOS_OK)
        return rc;
    hipError_t e = launch_stream_probe(probe, policy, x, s, c, n,
                                       resolve_plain_shape(sh, n, *dev), (hipStream_t)stream);
    return e == hipSuccess ? SINCOS_OK : hip_error(e, "sincos_stream_probe_f32: kernel launch");
}

extern "C" int sincos_pair_ceiling_f32(const float *x, float *out, int64_t n, int32_t reps,
                                       void *stream)
{
    clear_error();
    if (n < 0 || reps < 0)
        return set_error(SINCOS_EINVAL, "sincos_pair_ceiling_f32: n < 0 or reps < 0");
    if (n == 0)
        return SINCOS_OK;
    if (n > (int64_t)(UINT32_MAX / 256) * 256)  // one 256-thread workgroup per 256 lanes
        return set_error(SINCOS_EINVAL, "sincos_pair_ceiling_f32: n too large");
    if (!x || !out || !aligned4(x) || !aligned4(out))
        return set_error(SINCOS_EINVAL, "sincos_pair_ceiling_f32: null or misaligned pointer");
    if (ranges_overlap(x, n, out, n) && x != out)
        return set_error(SINCOS_EOVERLAP, "sincos_pair_ceiling_f32: x partly overlaps out");
    const DeviceInfo *dev;
    int rc;
    if ((rc = current_device(&dev)) != SINCOS_OK)
        return rc;
    hipError_t e = launch_pair_ceiling(x, out, n, reps, (hipStream_t)stream);
    return e == hipSuccess ? SINCOS_OK : hip_error(e, "sincos_pair_ceiling_f32: kernel launch");
}

// ---------------------------------------------------------------------------
// Ablations

static int check_ablation_arrays(const float *x, float *s, float *c, int64_t n, int32_t arith,
                                 const char *who)
{
    int rc = check_triplet(x, s, c, n, who);
    if (rc != SINCOS_OK)
        return rc;
    if (arith != SINCOS_ARITH_FUSED && arith != SINCOS_ARITH_SPLIT)
        return set_error(SINCOS_EINVAL, std::string(who) + ": arith must be FUSED or SPLIT");
    const uintptr_t bits = reinterpret_cast<uintptr_t>(x) | reinterpret_cast<uintptr_t>(s) |
                           reinterpret_cast<uintptr_t>(c);
    if (n > 0 && (bits & 15) != 0)
        return set_error(SINCOS_EINVAL, std::string(who) + ": x, s and c must be 16-byte aligned");
    return SINCOS_OK;
}

extern "C" int sincos_f32_variant(const float *x, float *s, float *c, int64_t n, int32_t arith,
                                  int32_t method, int32_t variant, void *stream)
{
    clear_error();
    int rc = check_ablation_arrays(x, s, c, n, arith, "sincos_f32_variant");
    if (rc != SINCOS_OK)
        return rc;
    if (method != SINCOS_METHOD_NORMALIZED && method != SINCOS_METHOD_ARCTAN)
        return set_error(SINCOS_EINVAL, "sincos_f32_variant: method must be NORMALIZED or ARCTAN");
    if (variant < SINCOS_VARIANT_LISTING || variant > SINCOS_VARIANT_EQ2)
        return set_error(SINCOS_EINVAL, "sincos_f32_variant: unknown variant");
    if (n == 0)
        return SINCOS_OK;
    const DeviceInfo *dev;
    if ((rc = current_device(&dev)) != SINCOS_OK)
        return rc;
    hipError_t e = launch_variant(x, s, c, n, arith, method, variant, (hipStream_t)stream);
    return e == hipSuccess ? SINCOS_OK : hip_error(e, "sincos_f32_variant: kernel launch");
}

extern "C" int sincos_f32_doublings(const float *x, float *s, float *c, int64_t n, int32_t arith,
                                    int32_t ndoub, const float *ss, int32_t ns, const float *cc,
                                    int32_t nc, int32_t fix, void *stream)
{
    clear_error();
    int rc = check_ablation_arrays(x, s, c, n, arith, "sincos_f32_doublings");
    if (rc != SINCOS_OK)
        return rc;
    if (ndoub < 0 || ndoub > kMaxDoublings)
        return set_error(SINCOS_EINVAL, "sincos_f32_doublings: ndoub must be in [0, " +
                                            std::to_string(kMaxDoublings) + "]");
    if (!ss || !cc || ns < 1 || ns > kMaxSeriesTerms || nc < 1 || nc > kMaxSeriesTerms)
        return set_error(SINCOS_EINVAL, "sincos_f32_doublings: need 1 to " +
                                            std::to_string(kMaxSeriesTerms) +
                                            " host coefficients in ss and in cc");
    if (n == 0)
        return SINCOS_OK;
    const DeviceInfo *dev;
    if ((rc = current_device(&dev)) != SINCOS_OK)
        return rc;
    hipError_t e = launch_doublings(x, s, c, n, arith, ndoub, ss, ns, cc, nc, fix,
                                    (hipStream_t)stream);
    return e == hipSuccess ? SINCOS_OK : hip_error(e, "sincos_f32_doublings: kernel launch");
}

// ---------------------------------------------------------------------------
// Ragged form

extern "C" int sincos_f32_ragged_ex(const sincos_seg_t *segs, const int64_t *lens, int32_t count,
                                    int32_t arith, int32_t method, const sincos_launch_t *launch,
                                    void *stream)
{
    clear_error();
    int rc = check_ragged(segs, lens, count);
    if (rc != SINCOS_OK)
        return rc;
    if ((rc = check_modes(arith, method)) != SINCOS_OK)
        return rc;
    LaunchShape sh;
    if ((rc = check_shape(launch, kFormRagged, &sh)) != SINCOS_OK)
        return rc;
    if (count == 0)
        return SINCOS_OK;
    const DeviceInfo *dev;
    if ((rc = current_device(&dev)) != SINCOS_OK)
        return rc;
    hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
    if (hipStreamIsCapturing((hipStream_t)stream, &cs) == hipSuccess &&
        cs != hipStreamCaptureStatusNone)
        return set_error(SINCOS_EINVAL,
                         "sincos_f32_ragged: stream is being captured; use a ragged plan");
    RaggedTable t;
    build_table(segs, lens, count, sh, t);
    return ragged_enqueue(t, arith, method, sh, *dev, (hipStream_t)stream);
}

extern "C" int sincos_f32_ragged(const sincos_seg_t *segs, const int64_t *lens, int32_t count,
                                 void *stream)
{
    return sincos_f32_ragged_ex(segs, lens, count, SINCOS_ARITH_FUSED, SINCOS_METHOD_NORMALIZED,
                                nullptr, stream);
}

struct sincos_ragged_plan {
    int device = -1;
    int arith = 0, method = 0;
    LaunchShape shape;
    int32_t count = 0;
    int64_t total_units = 0;
    int64_t elements = 0;
    char *dev_buf = nullptr;
    RaggedDesc *d_desc = nullptr;
    int64_t *d_ubeg = nullptr;
    hipStream_t capture_stream = nullptr;
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
};

extern "C" int sincos_ragged_plan_create(const sincos_seg_t *segs, const int64_t *lens,
                                         int32_t count, int32_t arith, int32_t method,
                                         const sincos_launch_t *launch,
                                         sincos_ragged_plan_t **out_plan)
{
    clear_error();
    if (!out_plan)
        return set_error(SINCOS_EINVAL, "plan_create: null out_plan");
    *out_plan = nullptr;
    int rc = check_ragged(segs, lens, count);
    if (rc != SINCOS_OK)
        return rc;
    if ((rc = check_modes(arith, method)) != SINCOS_OK)
        return rc;
    LaunchShape sh;
    if ((rc = check_shape(launch, kFormRagged, &sh)) != SINCOS_OK)
        return rc;
    const DeviceInfo *dev;
    if ((rc = current_device(&dev)) != SINCOS_OK)
        return rc;
    RaggedTable t;
    build_table(segs, lens, count, sh, t);
    auto plan = std::make_unique<sincos_ragged_plan>();
    plan->device = dev->device;
    plan->arith = arith;
    plan->method = method;
    plan->count = (int32_t)t.desc.size();
    plan->total_units = t.ubeg.back();
    plan->elements = t.elements;
    plan->shape = resolve_ragged_shape(sh, plan->total_units, *dev);
    if (plan->count > 0) {
        const size_t desc_bytes = sizeof(RaggedDesc) * t.desc.size();
        const size_t bytes = desc_bytes + sizeof(int64_t) * t.ubeg.size();
        if (hipMalloc((void **)&plan->dev_buf, bytes) != hipSuccess)
            return set_error(SINCOS_ENOMEM, "plan_create: cannot allocate the device table");
        std::vector<char> host(bytes);
        std::memcpy(host.data(), t.desc.data(), desc_bytes);
        std::memcpy(host.data() + desc_bytes, t.ubeg.data(), sizeof(int64_t) * t.ubeg.size());
        hipError_t e = hipMemcpy(plan->dev_buf, host.data(), bytes, hipMemcpyHostToDevice);
        if (e != hipSuccess) {
            (void)hipFree(plan->dev_buf);
            return hip_error(e, "plan_create: table copy");
        }
        plan->d_desc = reinterpret_cast<RaggedDesc *>(plan->dev_buf);
        plan->d_ubeg = reinterpret_cast<int64_t *>(plan->dev_buf + desc_bytes);
    }
    *out_plan = plan.release();
    return SINCOS_OK;
}

// Plans hold device addresses of the device they were made on.
static int check_plan_device(const sincos_ragged_plan *plan, const char *who)
{
    int dev = -1;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess)
        return hip_error(e, who);
    if (dev != plan->device)
        return set_error(SINCOS_EINVAL, std::string(who) + ": plan made on device " +
                                            std::to_string(plan->device) + ", current device is " +
                                            std::to_string(dev));
    return SINCOS_OK;
}

extern "C" int sincos_ragged_plan_launch(const sincos_ragged_plan_t *plan, void *stream)
{
    clear_error();
    if (!plan)
        return set_error(SINCOS_EINVAL, "plan_launch: null plan");
    if (plan->count == 0)
        return SINCOS_OK;
    int rc = check_plan_device(plan, "plan_launch");
    if (rc != SINCOS_OK)
        return rc;
    hipError_t e = launch_ragged(plan->d_desc, plan->d_ubeg, plan->count, plan->total_units,
                                 plan->arith, plan->method, plan->shape, (hipStream_t)stream);
    return e == hipSuccess ? SINCOS_OK : hip_error(e, "plan_launch: kernel launch");
}

extern "C" int sincos_ragged_plan_graph_launch(sincos_ragged_plan_t *plan, void *stream)
{
    clear_error();
    if (!plan)
        return set_error(SINCOS_EINVAL, "plan_graph_launch: null plan");
    if (plan->count == 0)
        return SINCOS_OK;
    int rc = check_plan_device(plan, "plan_graph_launch");
    if (rc != SINCOS_OK)
        return rc;
    hipError_t e;
    if (!plan->exec) {
        if (!plan->capture_stream &&
            (e = hipStreamCreateWithFlags(&plan->capture_stream, hipStreamNonBlocking)) != hipSuccess)
            return hip_error(e, "plan_graph_launch: capture stream");
        if ((e = hipStreamBeginCapture(plan->capture_stream, hipStreamCaptureModeThreadLocal)) != hipSuccess)
            return hip_error(e, "plan_graph_launch: begin capture");
        hipError_t le = launch_ragged(plan->d_desc, plan->d_ubeg, plan->count, plan->total_units,
                                      plan->arith, plan->method, plan->shape, plan->capture_stream);
        hipGraph_t g = nullptr;
        e = hipStreamEndCapture(plan->capture_stream, &g);
        if (le != hipSuccess || e != hipSuccess) {
            if (g)
                (void)hipGraphDestroy(g);
            return hip_error(le != hipSuccess ? le : e, "plan_graph_launch: capture");
        }
        plan->graph = g;
        if ((e = hipGraphInstantiate(&plan->exec, g, nullptr, nullptr, 0)) != hipSuccess) {
            plan->exec = nullptr;
            return hip_error(e, "plan_graph_launch: instantiate");
        }
    }
    e = hipGraphLaunch(plan->exec, (hipStream_t)stream);
    return e == hipSuccess ? SINCOS_OK : hip_error(e, "plan_graph_launch: graph launch");
}

extern "C" int sincos_ragged_plan_info(const sincos_ragged_plan_t *plan, int32_t *block,
                                       int32_t *unroll, int32_t *grid, int64_t *units,
                                       int64_t *elements)
{
    clear_error();
    if (!plan)
        return set_error(SINCOS_EINVAL, "plan_info: null plan");
    if (block)
        *block = plan->shape.block;
    if (unroll)
        *unroll = plan->shape.unroll;
    if (grid)
        *grid = plan->shape.grid;
    if (units)
        *units = plan->total_units;
    if (elements)
        *elements = plan->elements;
    return SINCOS_OK;
}

extern "C" int sincos_ragged_plan_destroy(sincos_ragged_plan_t *plan)
{
    clear_error();
    if (!plan)
        return SINCOS_OK;
    if (plan->exec)
        (void)hipGraphExecDestroy(plan->exec);
    if (plan->graph)
        (void)hipGraphDestroy(plan->graph);
    if (plan->capture_stream)
        (void)hipStreamDestroy(plan->capture_stream);
    if (plan->dev_buf)
        (void)hipFree(plan->dev_buf);
    delete plan;
    return SINCOS_OK;
}

// ---------------------------------------------------------------------------
// Adjoints

extern "C" int sincos_f32_backward(const float *s, const float *c, const float *gs,
                                   const float *gc, float *gx, int64_t n, void *stream)
{
    clear_error();
    if (n < 0)
        return set_error(SINCOS_EINVAL, "sincos_f32_backward: n < 0");
    if (n == 0)
        return SINCOS_OK;
    if (!s || !c || !gx)
        return set_error(SINCOS_EINVAL, "sincos_f32_backward: null s, c or gx with n > 0");
    if (!aligned4(s) || !aligned4(c) || !aligned4(gx) || (gs && !aligned4(gs)) ||
        (gc && !aligned4(gc)))
        return set_error(SINCOS_EINVAL, "sincos_f32_backward: pointers must be 4-byte aligned");
    if (ranges_overlap(gx, n, s, n) || ranges_overlap(gx, n, c, n))
        return set_error(SINCOS_EOVERLAP, "sincos_f32_backward: gx overlaps s or c");
    if (gs && gs != gx && ranges_overlap(gx, n, gs, n))
        return set_error(SINCOS_EOVERLAP, "sincos_f32_backward: gx partially overlaps gs");
    if (gc && gc != gx && ranges_overlap(gx, n, gc, n))
        return set_error(SINCOS_EOVERLAP, "sincos_f32_backward: gx partially overlaps gc");
    const DeviceInfo *dev;
    int rc;
    if ((rc = current_device(&dev)) != SINCOS_OK)
        return rc;
    hipError_t e = launch_backward(s, c, gs, gc, gx, n, (hipStream_t)stream);
    return e == hipSuccess ? SINCOS_OK : hip_error(e, "sincos_f32_backward: kernel launch");
}

static int check_params(const float *A, const float *w, const float *phi, int32_t K,
                        const char *who)
{
    if (K < 0)
        return set_error(SINCOS_EINVAL, std::string(who) + ": K < 0");
    if (K > 0 && (!A || !w || !phi))
        return set_error(SINCOS_EINVAL, std::string(who) + ": null parameter array with K > 0");
    if (K > (1 << 20))
        return set_error(SINCOS_EINVAL, std::string(who) + ": K too large");
    return SINCOS_OK;
}

extern "C" int sinusoid_f32_forward(const float *t, int64_t N, const float *A, const float *w,
                                    const float *phi, int32_t K, float *y, void *stream)
{
    clear_error();
    if (N < 0)
        return set_error(SINCOS_EINVAL, "sinusoid_f32_forward: N < 0");
    int rc = check_params(A, w, phi, K, "sinusoid_f32_forward");
    if (rc != SINCOS_OK)
        return rc;
    if (N == 0)
        return SINCOS_OK;
    if (!t || !y)
        return set_error(SINCOS_EINVAL, "sinusoid_f32_forward: null t or y with N > 0");
    if (!all_aligned4({t, y, A, w, phi}))
        return set_error(SINCOS_EINVAL, "sinusoid_f32_forward: pointers must be 4-byte aligned");
    if ((rc = check_disjoint({{y, N, "y"}},
                             {{t, N, "t"}, {A, K, "A"}, {w, K, "w"}, {phi, K, "phi"}},
                             "sinusoid_f32_forward", y, t)) != SINCOS_OK)
        return rc;
    const DeviceInfo *dev;
    if ((rc = current_device(&dev)) != SINCOS_OK)
        return rc;
    hipError_t e = launch_sinusoid_forward(t, N, A, w, phi, K, y, (hipStream_t)stream);
    return e == hipSuccess ? SINCOS_OK : hip_error(e, "sinusoid_f32_forward: kernel launch");
}

extern "C" int64_t sinusoid_f32_residual_workspace_bytes(int64_t N)
{
    if (N < 0)
        return -1;
    return sinusoid_fwd_blocks(N) * (int64_t)sizeof(float);
}

extern "C" int sinusoid_f32_residual(const float *t, const float *y_obs, int64_t N, const float *A,
                                     const float *w, const float *phi, int32_t K, float *r,
                                     float *loss, void *workspace, int64_t workspace_bytes,
                                     void *stream)
{
    clear_error();
    if (N < 0)
        return set_error(SINCOS_EINVAL, "sinusoid_f32_residual: N < 0");
    int rc = check_params(A, w, phi, K, "sinusoid_f32_residual");
    if (rc != SINCOS_OK)
        return rc;
    if (!loss)
        return set_error(SINCOS_EINVAL, "sinusoid_f32_residual: null loss");
    if (N > 0) {
        if (!t || !y_obs || !r)
            return set_error(SINCOS_EINVAL, "sinusoid_f32_residual: null t, y_obs or r with N > 0");
        if (!all_aligned4({t, y_obs, r, loss, A, w, phi, workspace}))
            return set_error(SINCOS_EINVAL, "sinusoid_f32_residual: pointers must be 4-byte aligned");
        const int64_t need = sinusoid_f32_residual_workspace_bytes(N);
        if (!workspace || workspace_bytes < need)
            return set_error(SINCOS_EINVAL, "sinusoid_f32_residual: workspace needs " +
                                                std::to_string(need) + " bytes");
        if ((rc = check_disjoint({{r, N, "r"}, {loss, 1, "loss"}, {workspace, need / 4, "workspace"}},
                                 {{t, N, "t"}, {y_obs, N, "y_obs"}, {A, K, "A"}, {w, K, "w"},
                                  {phi, K, "phi"}},
                                 "sinusoid_f32_residual", r, t, y_obs)) != SINCOS_OK)
            return rc;
    } else if (!aligned4(loss)) {
        return set_error(SINCOS_EINVAL, "sinusoid_f32_residual: loss must be 4-byte aligned");
    }
    const DeviceInfo *dev;
    if ((rc = current_device(&dev)) != SINCOS_OK)
        return rc;
    hipError_t e = launch_sinusoid_residual(t, y_obs, N, A, w, phi, K, r, loss,
                                            static_cast<float *>(workspace), (hipStream_t)stream);
    return e == hipSuccess ? SINCOS_OK : hip_error(e, "sinusoid_f32_residual: kernel launch");
}

extern "C" int64_t sinusoid_f32_backward_workspace_bytes(int64_t N, int32_t K)
{
    if (N < 0 || K < 0)
        return -1;
    return sinusoid_parts(N) * 3 * sinusoid_kgroups(K) * 64 * (int64_t)sizeof(float);
}

extern "C" int sinusoid_f32_backward(const float *t, const float *g, int64_t N, const float *A,
                                     const float *w, const float *phi, int32_t K, float *gA,
                                     float *gw, float *gphi, void *workspace,
                                     int64_t workspace_bytes, void *stream)
{
    clear_error();
    if (N < 0)
        return set_error(SINCOS_EINVAL, "sinusoid_f32_backward: N < 0");
    if (sinusoid_parts(N) > (int64_t)(UINT32_MAX / 1024))  // 1024-thread workgroups
        return set_error(SINCOS_EINVAL, "sinusoid_f32_backward: N too large");
    int rc = check_params(A, w, phi, K, "sinusoid_f32_backward");
    if (rc != SINCOS_OK)
        return rc;
    if (K == 0)
        return SINCOS_OK;
    if (!gA || !gw || !gphi)
        return set_error(SINCOS_EINVAL, "sinusoid_f32_backward: null gradient output");
    if (N > 0 && (!t || !g))
        return set_error(SINCOS_EINVAL, "sinusoid_f32_backward: null t or g with N > 0");
    if (!all_aligned4({t, g, A, w, phi, gA, gw, gphi, workspace}))
        return set_error(SINCOS_EINVAL, "sinusoid_f32_backward: pointers must be 4-byte aligned");
    const int64_t need = sinusoid_f32_backward_workspace_bytes(N, K);
    if (N > 0 && (!workspace || workspace_bytes < need))
        return set_error(SINCOS_EINVAL, "sinusoid_f32_backward: workspace needs " +
                                            std::to_string(need) + " bytes");
    if ((rc = check_disjoint({{gA, K, "gA"}, {gw, K, "gw"}, {gphi, K, "gphi"},
                              {N > 0 ? workspace : nullptr, need / 4, "workspace"}},
                             {{t, N, "t"}, {g, N, "g"}, {A, K, "A"}, {w, K, "w"}, {phi, K, "phi"}},
                             "sinusoid_f32_backward")) != SINCOS_OK)
        return rc;
    const DeviceInfo *dev;
    if ((rc = current_device(&dev)) != SINCOS_OK)
        return rc;
    hipError_t e = launch_sinusoid_backward(t, g, N, A, w, phi, K, gA, gw, gphi,
                                            static_cast<float *>(workspace), (hipStream_t)stream);
    return e == hipSuccess ? SINCOS_OK : hip_error(e, "sinusoid_f32_backward: kernel launch");
}

extern "C" int64_t sinusoid_f32_fit_step_workspace_bytes(int64_t N, int32_t K)
{
    if (N < 0 || K < 0)
        return -1;
    return sinusoid_fit_parts(N) * (3 * sinusoid_kgroups(K) * 64 + 1) * (int64_t)sizeof(float);
}

// Checks shared by the two fit-step entry points (everything but the
// partials' buffer).
static int check_fit_step(const float *t, const float *y_obs, int64_t N, const float *A,
                          const float *w, const float *phi, int32_t K, const float *loss,
                          const float *gA, const float *gw, const float *gphi, const char *who)
{
    if (N < 0)
        return set_error(SINCOS_EINVAL, std::string(who) + ": N < 0");
    if (sinusoid_fit_parts(N) > (int64_t)(UINT32_MAX / 1024))  // 1024-thread workgroups
        return set_error(SINCOS_EINVAL, std::string(who) + ": N too large");
    int rc = check_params(A, w, phi, K, who);
    if (rc != SINCOS_OK)
        return rc;
    if (!loss || (K > 0 && (!gA || !gw || !gphi)))
        return set_error(SINCOS_EINVAL, std::string(who) + ": null loss or gradient output");
    if (N > 0 && (!t || !y_obs))
        return set_error(SINCOS_EINVAL, std::string(who) + ": null t or y_obs with N > 0");
    if (!all_aligned4({t, y_obs, A, w, phi, loss, gA, gw, gphi}))
        return set_error(SINCOS_EINVAL, std::string(who) + ": pointers must be 4-byte aligned");
    return SINCOS_OK;
}

extern "C" int sinusoid_f32_fit_step(const float *t, const float *y_obs, int64_t N, const float *A,
                                     const float *w, const float *phi, int32_t K, float *loss,
                                     float *gA, float *gw, float *gphi, void *workspace,
                                     int64_t workspace_bytes, void *stream)
{
    clear_error();
    const char *who = "sinusoid_f32_fit_step";
    int rc = check_fit_step(t, y_obs, N, A, w, phi, K, loss, gA, gw, gphi, who);
    if (rc != SINCOS_OK)
        return rc;
    if (!aligned4(workspace))
        return set_error(SINCOS_EINVAL, std::string(who) + ": pointers must be 4-byte aligned");
    const int64_t need = sinusoid_f32_fit_step_workspace_bytes(N, K);
    if (N > 0 && (!workspace || workspace_bytes < need))
        return set_error(SINCOS_EINVAL, std::string(who) + ": workspace needs " +
                                            std::to_string(need) + " bytes");
    if ((rc = check_disjoint({{loss, 1, "loss"}, {gA, K, "gA"}, {gw, K, "gw"}, {gphi, K, "gphi"},
                              {N > 0 ? workspace : nullptr, need / 4, "workspace"}},
                             {{t, N, "t"}, {y_obs, N, "y_obs"}, {A, K, "A"}, {w, K, "w"},
                              {phi, K, "phi"}},
                             who)) != SINCOS_OK)
        return rc;
    const DeviceInfo *dev;
    if ((rc = current_device(&dev)) != SINCOS_OK)
        return rc;
    float *part = static_cast<float *>(workspace);
    const int64_t parts = sinusoid_fit_parts(N);
    float *loss_part = part ? part + 3 * sinusoid_kgroups(K) * 64 * parts : nullptr;
    hipError_t e = launch_sinusoid_fit(t, y_obs, N, A, w, phi, K, loss, gA, gw, gphi, part,
                                       loss_part, (hipStream_t)stream);
    return e == hipSuccess ? SINCOS_OK : hip_error(e, "sinusoid_f32_fit_step: kernel launch");
}

extern "C" int sinusoid_f32_fit_step_noalloc(const float *t, const float *y_obs, int64_t N,
                                             const float *A, const float *w, const float *phi,
                                             int32_t K, float *loss, float *gA, float *gw,
                                             float *gphi, void *stream)
{
    clear_error();
    const char *who = "sinusoid_f32_fit_step_noalloc";
    int rc = check_fit_step(t, y_obs, N, A, w, phi, K, loss, gA, gw, gphi, who);
    if (rc != SINCOS_OK)
        return rc;
    const int64_t need = sinusoid_f32_fit_step_workspace_bytes(N, K);
    if (need > kFitScratchBytes)
        return set_error(SINCOS_EINVAL, std::string(who) + ": needs " + std::to_string(need) +
                                            " bytes of partials, more than its " +
                                            std::to_string(kFitScratchBytes) +
                                            "-byte scratch; use sinusoid_f32_fit_step");
    if ((rc = check_disjoint({{loss, 1, "loss"}, {gA, K, "gA"}, {gw, K, "gw"}, {gphi, K, "gphi"}},
                             {{t, N, "t"}, {y_obs, N, "y_obs"}, {A, K, "A"}, {w, K, "w"},
                              {phi, K, "phi"}},
                             who)) != SINCOS_OK)
        return rc;
    const DeviceInfo *dev;
    if ((rc = current_device(&dev)) != SINCOS_OK)
        return rc;
    float *part = nullptr;
    hipError_t e = fit_scratch(dev->device, &part);
    if (e != hipSuccess)
        return hip_error(e, "sinusoid_f32_fit_step_noalloc: scratch address");
    const int64_t parts = sinusoid_fit_parts(N);
    float *loss_part = part + 3 * sinusoid_kgroups(K) * 64 * parts;
    e = launch_sinusoid_fit(t, y_obs, N, A, w, phi, K, loss, gA, gw, gphi, part, loss_part,
                            (hipStream_t)stream);
    return e == hipSuccess ? SINCOS_OK
                           : hip_error(e, "sinusoid_f32_fit_step_noalloc: kernel launch");
}

// Checks shared by the Huygens sum and its term ceiling (S sources in src).
static int check_huygens(const float *xo, const float *yo, int64_t P, const float *src, int64_t S,
                         float L, const float *re, const float *im, const std::string &who)
{
    if (P < 0 || S < 0)
        return set_error(SINCOS_EINVAL, who + ": P < 0 or S < 0");
    if (P > (int64_t(1) << 36))  // beyond any device memory
        return set_error(SINCOS_EINVAL, who + ": P too large");
    if (P == 0)
        return SINCOS_OK;
    if (!xo || !yo || !re || !im || (S > 0 && !src))
        return set_error(SINCOS_EINVAL, who + ": null pointer");
    if (!aligned4(xo) || !aligned4(yo) || !aligned4(re) || !aligned4(im) ||
        (S > 0 && (reinterpret_cast<uintptr_t>(src) & 15)))
        return set_error(SINCOS_EINVAL, who + ": arrays must be 4-byte aligned, src 16-byte aligned");
    if (!(L > 0.0f) || !(L < 1e18f))
        return set_error(SINCOS_EINVAL, who + ": L must be in (0, 1e18)");
    if (ranges_overlap(re, P, im, P) || ranges_overlap(re, P, xo, P) ||
        ranges_overlap(re, P, yo, P) || ranges_overlap(im, P, xo, P) ||
        ranges_overlap(im, P, yo, P) ||
        (S > 0 && (ranges_overlap(re, P, src, 4 * S) || ranges_overlap(im, P, src, 4 * S))))
        return set_error(SINCOS_EOVERLAP, who + ": outputs overlap inputs or each other");
    return SINCOS_OK;
}

extern "C" int huygens_f32(const float *xo, const float *yo, int64_t P, const float *src,
                           int32_t S, float k, float L, float *re, float *im, void *stream)
{
    clear_error();
    int rc = check_huygens(xo, yo, P, src, S, L, re, im, "huygens_f32");
    if (rc != SINCOS_OK || P == 0)
        return rc;
    const DeviceInfo *dev;
    if ((rc = current_device(&dev)) != SINCOS_OK)
        return rc;
    hipError_t e = launch_huygens(xo, yo, P, src, S, k, L, re, im, (hipStream_t)stream);
    return e == hipSuccess ? SINCOS_OK : hip_error(e, "huygens_f32: kernel launch");
}

extern "C" int huygens_term_ceiling_f32(const float *xo, const float *yo, int64_t P,
                                        const float *src8, int32_t reps, float k, float L,
                                        float *re, float *im, void *stream)
{
    clear_error();
    if (reps < 0 || reps >= (1 << 28))
        return set_error(SINCOS_EINVAL, "huygens_term_ceiling_f32: reps must be in [0, 2^28)");
    int rc = check_huygens(xo, yo, P, src8, kHuygensCeilingSources, L, re, im,
                           "huygens_term_ceiling_f32");
    if (rc != SINCOS_OK || P == 0)
        return rc;
    const DeviceInfo *dev;
    if ((rc = current_device(&dev)) != SINCOS_OK)
        return rc;
    hipError_t e = launch_huygens_ceiling(xo, yo, P, src8, reps, k, L, re, im, (hipStream_t)stream);
    return e == hipSuccess ? SINCOS_OK : hip_error(e, "huygens_term_ceiling_f32: kernel launch");
}

// ---------------------------------------------------------------------------

extern "C" const char *sincos_last_error(void) { return g_last_error.c_str(); }

extern "C" const char *sincos_version(void) { return "mi355-sincos 0.1 (gfx950)"; }
