// serve.cpp -- request server: continuous batching of sine-cosine requests
// (declared in include/sincos.h, sincos_server_*).
//
// One scheduler thread per server.  Each loop trip it
//   1. moves newly submitted requests to the FIFO of pending requests;
//   2. checks the batches on the device (event queries) and completes the
//      requests of every finished batch;
//   3. admits pending requests in arrival order while the head request's
//      12 n bytes fit in the budget and an arena block for its outputs is
//      free (no overtaking, so no request starves);
//   4. if a slot is free, sends every admitted, unlaunched request of the
//      oldest one's size class (up to the batch caps) to the device as one
//      ragged launch (mode 0), or one request as one plain launch (mode 1).
// Requests that arrive while batches run are admitted as budget frees up and
// ride in the next batch: up to max_inflight batches are on the device.  By
// default a batch runs on its size class's stream, behind the earlier
// batches of that class, so each batch has the device to itself but for the
// other class's work; with stream_per_slot every slot has its own stream and
// all batches in flight share the device.
#include "../../include/sincos.h"
#include "internal.hpp"
#include "serve.hpp"

#include <algorithm>
#include <atomic>
#include <chrono>
#include <condition_variable>
#include <deque>
#include <memory>
#include <mutex>
#include <string>
#include <thread>
#include <unordered_map>
#include <vector>

namespace mi355 {

static int64_t now_ns()
{
    return std::chrono::duration_cast<std::chrono::nanoseconds>(
               std::chrono::steady_clock::now().time_since_epoch())
        .count();
}

struct Request {
    int64_t id = 0;
    uint64_t tag = 0;
    const float *x = nullptr;
    int64_t n = 0;
    int64_t arena_off = -1;
    uint64_t arena_bytes = 0;
    float *s = nullptr;
    float *c = nullptr;
    int32_t status = SINCOS_OK;
    int32_t batch_requests = 0;
    int64_t t_submit = 0, t_admit = 0, t_launch = 0, t_complete = 0;
    bool released = false;
    hipEvent_t ready = nullptr;  // recorded on the submitter's stream: x is ready after it
};

// Where batches run.  launch() starts a batch on a slot; query() reports
// 1 (finished), 0 (running) or a negative status.
class Executor {
public:
    virtual ~Executor() = default;
    virtual int init(int slots) = 0;
    virtual int launch(int slot, const std::vector<Request *> &batch) = 0;
    virtual int query(int slot) = 0;
    virtual void wait(int slot) = 0;
    // After a failed launch: wait for whatever part of it was enqueued, so
    // that its memory can be reused.
    virtual void drain(int slot) = 0;
    virtual char *arena_base() = 0;
};

class GpuExecutor : public Executor {
public:
    // class_split > 0: one stream per size class (requests of more than
    // class_split elements form class 1; 0 when there is one class), and a
    // batch runs on its class's stream; class_split < 0: each slot's stream.
    GpuExecutor(int device, uint64_t arena_bytes, int arith, int method, int mode,
                int64_t class_split)
        : device_(device), arena_bytes_(arena_bytes), arith_(arith), method_(method), mode_(mode),
          class_split_(class_split)
    {
    }
    ~GpuExecutor() override
    {
        int prev = -1;
        const bool restore = hipGetDevice(&prev) == hipSuccess && prev != device_;
        (void)hipSetDevice(device_);
        for (hipStream_t &s : class_streams_)
            if (s) {
                (void)hipStreamSynchronize(s);
                (void)hipStreamDestroy(s);
            }
        for (auto &sl : slots_) {
            if (sl.stream)
                (void)hipStreamSynchronize(sl.stream);
            if (sl.done)
                (void)hipEventDestroy(sl.done);
            if (sl.stream)
                (void)hipStreamDestroy(sl.stream);
            free_staging(sl.staging);
        }
        if (arena_)
            (void)hipFree(arena_);
        if (restore)
            (void)hipSetDevice(prev);  // the destroying thread keeps its device
    }
    int init(int slots) override
    {
        if (hipSetDevice(device_) != hipSuccess)
            return set_error(SINCOS_ENODEV, "server: cannot select the device");
        const DeviceInfo &info = device_info(device_);
        if (!info.arch_ok)
            return set_error(SINCOS_ENODEV, "server: device is not gfx950");
        dev_ = &info;
        if (hipMalloc((void **)&arena_, arena_bytes_) != hipSuccess) {
            arena_ = nullptr;
            return set_error(SINCOS_ENOMEM, "server: cannot allocate the output arena");
        }
        slots_.resize(slots);
        for (auto &sl : slots_) {  // a stream per slot only where batches run on it
            if ((class_split_ < 0 &&
                 hipStreamCreateWithFlags(&sl.stream, hipStreamNonBlocking) != hipSuccess) ||
                hipEventCreateWithFlags(&sl.done, hipEventDisableTiming) != hipSuccess)
                return set_error(SINCOS_EHIP, "server: cannot create streams and events");
        }
        if (class_split_ >= 0)
            for (hipStream_t &s : class_streams_)
                if (hipStreamCreateWithFlags(&s, hipStreamNonBlocking) != hipSuccess)
                    return set_error(SINCOS_EHIP, "server: cannot create the class streams");
        return SINCOS_OK;
    }
    int launch(int slot, const std::vector<Request *> &batch) override
    {
        Slot &sl = slots_[slot];
        // the batch's stream: its class's (batches of a class run in order), or the slot's
        const hipStream_t st =
            class_split_ < 0 ? sl.stream
                             : class_streams_[class_split_ > 0 && batch.front()->n > class_split_];
        sl.used = st;
        const LaunchShape shape = default_shape(mode_ == 1 ? kFormPlain : kFormRagged);
        int rc = SINCOS_OK;
        for (Request *r : batch)  // inputs produced on the submitters' streams
            if (r->ready && hipStreamWaitEvent(st, r->ready, 0) != hipSuccess)
                return set_error(SINCOS_EHIP, "server: cannot wait for a request's input");
        if (mode_ == 1) {
            for (Request *r : batch) {
                hipError_t e = launch_sincos(r->x, r->s, r->c, r->n, arith_, method_,
                                             resolve_plain_shape(shape, r->n, *dev_), st);
                if (e != hipSuccess)
                    return set_error(SINCOS_EHIP, std::string("server: ") + hipGetErrorString(e));
            }
        } else {
            table_.desc.clear();
            table_.ubeg.assign(1, 0);
            table_.elements = 0;
            for (Request *r : batch)
                table_add(table_, r->x, r->s, r->c, r->n, shape);
            if (table_.desc.size() <= (size_t)kInlineSegs) {
                // small batch: the table travels in the kernel arguments
                rc = launch_table_inline(table_, arith_, method_, shape, *dev_, st);
            } else {
                rc = grow_staging(sl.staging, staged_bytes(table_));
                if (rc == SINCOS_OK)
                    rc = stage_and_launch(table_, sl.staging.host, sl.staging.dev, arith_,
                                          method_, shape, *dev_, st);
            }
            if (rc != SINCOS_OK)
                return rc;
        }
        if (hipEventRecord(sl.done, st) != hipSuccess)
            return set_error(SINCOS_EHIP, "server: event record failed");
        return SINCOS_OK;
    }
    int query(int slot) override
    {
        hipError_t e = hipEventQuery(slots_[slot].done);
        if (e == hipSuccess)
            return 1;
        if (e == hipErrorNotReady)
            return 0;
        return SINCOS_EHIP;
    }
    void wait(int slot) override { (void)hipEventSynchronize(slots_[slot].done); }
    void drain(int slot) override
    {
        const Slot &sl = slots_[slot];
        if (sl.used)  // set by the slot's last launch
            (void)hipStreamSynchronize(sl.used);
    }
    char *arena_base() override { return arena_; }

private:
    struct Slot {
        hipStream_t stream = nullptr;
        hipStream_t used = nullptr;  // the stream of the slot's last batch
        hipEvent_t done = nullptr;
        StagingBuffers staging;  // reused only after the slot's batch finished
    };
    int device_;
    uint64_t arena_bytes_;
    int arith_, method_, mode_;
    int64_t class_split_;
    hipStream_t class_streams_[2] = {nullptr, nullptr};
    const DeviceInfo *dev_ = nullptr;
    char *arena_ = nullptr;
    std::vector<Slot> slots_;
    RaggedTable table_;
};

// No device work: a batch "runs" for a computed time; every k-th fails.
// Output addresses are fake (never dereferenced by the server).
class SimExecutor : public Executor {
public:
    SimExecutor(int64_t batch_ns, int64_t elem_ps, int fail_every)
        : batch_ns_(batch_ns), elem_ps_(elem_ps), fail_every_(fail_every)
    {
    }
    int init(int slots) override
    {
        deadline_.assign(slots, 0);
        fails_.assign(slots, false);
        return SINCOS_OK;
    }
    int launch(int slot, const std::vector<Request *> &batch) override
    {
        int64_t elems = 0;
        for (Request *r : batch)
            elems += r->n;
        deadline_[slot] = now_ns() + batch_ns_ + elems * elem_ps_ / 1000;
        ++count_;
        fails_[slot] = fail_every_ > 0 && count_ % fail_every_ == 0;
        return SINCOS_OK;
    }
    int query(int slot) override
    {
        if (now_ns() < deadline_[slot])
            return 0;
        return fails_[slot] ? SINCOS_EHIP : 1;
    }
    void wait(int slot) override
    {
        while (now_ns() < deadline_[slot])
            std::this_thread::yield();
    }
    void drain(int) override {}
    char *arena_base() override { return reinterpret_cast<char *>(uintptr_t(1) << 40); }

private:
    int64_t batch_ns_, elem_ps_;
    int fail_every_;
    int64_t count_ = 0;
    std::vector<int64_t> deadline_;
    std::vector<bool> fails_;
};

}  // namespace mi355

using namespace mi355;

struct sincos_server {
    sincos_server_config_t cfg{};
    uint64_t budget = 0;
    std::unique_ptr<Executor> exec;

    // Shared state, guarded by mu (held only for short bookkeeping).
    std::mutex mu;
    std::condition_variable cv_sched, cv_done;
    bool stop = false;
    int64_t next_id = 1;
    std::deque<Request *> incoming;
    std::unordered_map<int64_t, std::unique_ptr<Request>> all;
    std::deque<Request *> done;
    Arena arena;
    uint64_t budget_used = 0;
    sincos_server_stats_t stats{};
    std::vector<hipEvent_t> event_pool;  // ready events not attached to a request

    // Owned by the scheduler thread alone.
    std::deque<Request *> pending;
    std::vector<Request *> admitted;
    struct Slot {
        bool busy = false;
        std::vector<Request *> batch;
    };
    std::vector<Slot> slots;
    std::thread thread;
    int device = 0;

    uint64_t charge(const Request *r) const { return (uint64_t)r->n * 12; }

    // caller holds mu
    void free_request_memory(Request *r)
    {
        if (r->arena_off >= 0) {
            arena.release((uint64_t)r->arena_off, r->arena_bytes);
            r->arena_off = -1;
            budget_used -= charge(r);
            stats.budget_in_use = (int64_t)budget_used;
        }
    }

    // caller holds mu
    void complete(Request *r, int status, int64_t t)
    {
        if (r->ready) {  // the batch that waited on it has finished (or never ran)
            event_pool.push_back(r->ready);
            r->ready = nullptr;
        }
        r->status = status;
        r->t_complete = t;
        if (status == SINCOS_OK) {
            stats.completed++;
            stats.elements_completed += r->n;
        } else {
            stats.failed++;
        }
        if (cfg.auto_release || status != SINCOS_OK)
            free_request_memory(r);
        done.push_back(r);
    }

    // caller holds mu: admit in arrival order while the head fits
    void admit()
    {
        while (!pending.empty()) {
            Request *r = pending.front();
            if (budget_used + charge(r) > budget)
                break;
            // outputs s then c; each placed at the input's offset modulo 16
            // bytes so the kernel keeps its float4 body
            const uint64_t phase = reinterpret_cast<uintptr_t>(r->x) & 15;
            const uint64_t span = ((uint64_t)r->n * 4 + phase + 255) / 256 * 256;
            const int64_t off = arena.alloc(2 * span);
            if (off < 0)
                break;
            r->arena_off = off;
            r->arena_bytes = 2 * span;
            char *base = exec->arena_base() + off;
            r->s = reinterpret_cast<float *>(base + phase);
            r->c = reinterpret_cast<float *>(base + span + phase);
            r->t_admit = now_ns();
            budget_used += charge(r);
            stats.budget_in_use = (int64_t)budget_used;
            stats.budget_peak = std::max(stats.budget_peak, (int64_t)budget_used);
            stats.admitted++;
            pending.pop_front();
            admitted.push_back(r);
        }
    }

    // Move the next batch out of `admitted` (scheduler thread): in arrival
    // order up to the caps, and with a size split only requests of the
    // oldest one's class (the others keep their places).
    void form_batch(std::vector<Request *> &batch)
    {
        batch.clear();
        const size_t cap = cfg.mode == 1 ? 1 : (size_t)cfg.max_batch_requests;
        const bool split = cfg.split_elems > 0;
        const bool large = split && admitted.front()->n > cfg.split_elems;
        int64_t elems = 0;
        size_t keep = 0, j = 0;
        for (; j < admitted.size() && batch.size() < cap; ++j) {
            Request *r = admitted[j];
            const bool fits = !split || (r->n > cfg.split_elems) == large;
            if (fits && !batch.empty() && cfg.max_batch_elems > 0 &&
                elems + r->n > cfg.max_batch_elems)
                break;
            if (fits) {
                elems += r->n;
                batch.push_back(r);
            } else {
                admitted[keep++] = r;
            }
        }
        for (; j < admitted.size(); ++j)
            admitted[keep++] = admitted[j];
        admitted.resize(keep);
    }

    // Check the device; complete the requests of finished batches.
    // Returns the number of batches still running.
    int reap(bool *progressed)
    {
        int inflight = 0;
        std::vector<std::pair<Request *, int>> fin;
        for (size_t k = 0; k < slots.size(); ++k) {
            Slot &sl = slots[k];
            if (!sl.busy)
                continue;
            const int q = exec->query((int)k);
            if (q == 0) {
                ++inflight;
                continue;
            }
            for (Request *r : sl.batch)
                fin.emplace_back(r, q == 1 ? SINCOS_OK : SINCOS_EHIP);
            sl.batch.clear();
            sl.busy = false;
        }
        if (!fin.empty()) {
            const int64_t t = now_ns();
            {
                std::lock_guard<std::mutex> lk(mu);
                for (auto &f : fin)
                    complete(f.first, f.second, t);
            }
            cv_done.notify_all();
            *progressed = true;
        }
        return inflight;
    }

    void drain_and_cancel()
    {
        {
            std::lock_guard<std::mutex> lk(mu);
            const int64_t t = now_ns();
            for (Request *r : pending)
                complete(r, SINCOS_ECANCELED, t);
            for (Request *r : admitted)
                complete(r, SINCOS_ECANCELED, t);
        }
        pending.clear();
        admitted.clear();
        for (size_t k = 0; k < slots.size(); ++k) {
            if (!slots[k].busy)
                continue;
            exec->wait((int)k);
            const int q = exec->query((int)k);
            std::lock_guard<std::mutex> lk(mu);
            const int64_t t = now_ns();
            for (Request *r : slots[k].batch)
                complete(r, q == 1 ? SINCOS_OK : SINCOS_EHIP, t);
            slots[k].batch.clear();
            slots[k].busy = false;
        }
        cv_done.notify_all();
    }

    void run()
    {
        if (cfg.executor == 0)
            (void)hipSetDevice(device);
        int idle = 0;
        for (;;) {
            bool stopping;
            {
                std::lock_guard<std::mutex> lk(mu);
                while (!incoming.empty()) {
                    pending.push_back(incoming.front());
                    incoming.pop_front();
                }
                stopping = stop;
            }
            bool progressed = false;
            int inflight = reap(&progressed);
            if (stopping) {
                drain_and_cancel();
                return;
            }
            if (!pending.empty()) {
                std::lock_guard<std::mutex> lk(mu);
                admit();
            }
            for (size_t k = 0; k < slots.size() && !admitted.empty(); ++k) {
                Slot &sl = slots[k];
                if (sl.busy)
                    continue;
                form_batch(sl.batch);
                const size_t take = sl.batch.size();
                const int64_t t = now_ns();
                for (Request *r : sl.batch) {
                    r->t_launch = t;
                    r->batch_requests = (int32_t)take;
                }
                const int rc = exec->launch((int)k, sl.batch);
                if (rc != SINCOS_OK)
                    exec->drain((int)k);  // before the batch's outputs return to the arena
                std::lock_guard<std::mutex> lk(mu);
                if (rc != SINCOS_OK) {
                    for (Request *r : sl.batch)
                        complete(r, SINCOS_EHIP, now_ns());
                    sl.batch.clear();
                    cv_done.notify_all();
                    continue;
                }
                sl.busy = true;
                stats.batches++;
                ++inflight;
                stats.inflight_peak = std::max(stats.inflight_peak, inflight);
                progressed = true;
            }
            if (progressed) {
                idle = 0;
                continue;
            }
            // Nothing moved.  With work on the device (or waiting for budget)
            // poll again soon: arrivals and completions are microseconds
            // apart.  Otherwise sleep until a submission arrives.
            std::unique_lock<std::mutex> lk(mu);
            if (!incoming.empty() || stop)
                continue;
            if (inflight > 0 || !pending.empty() || !admitted.empty()) {
                if (++idle < 4096) {
                    lk.unlock();
                    std::this_thread::yield();
                } else {
                    cv_sched.wait_for(lk, std::chrono::microseconds(20));
                    idle = 0;
                }
            } else {
                cv_sched.wait_for(lk, std::chrono::milliseconds(5));
                idle = 0;
            }
        }
    }
};

extern "C" int sincos_server_create(const sincos_server_config_t *cfg, sincos_server_t **out)
{
    clear_error();
    if (!cfg || !out)
        return set_error(SINCOS_EINVAL, "server_create: null argument");
    *out = nullptr;
    sincos_server_config_t c = *cfg;
    if (c.budget_bytes < 0 || c.max_inflight < 0 || c.max_batch_requests < 0 ||
        c.max_batch_elems < 0 || c.sim_batch_ns < 0 || c.sim_elem_ps < 0 || c.sim_fail_every < 0 ||
        c.split_elems < -1)
        return set_error(SINCOS_EINVAL, "server_create: negative setting");
    if (c.split_elems == 0)
        c.split_elems = int64_t(1) << 22;
    if (c.budget_bytes == 0)
        c.budget_bytes = int64_t(8) << 30;
    if (c.max_inflight == 0)
        c.max_inflight = 4;
    if (c.max_inflight > 16)
        return set_error(SINCOS_EINVAL, "server_create: max_inflight must be <= 16");
    if (c.max_batch_requests == 0)
        c.max_batch_requests = 4096;
    if (c.arith < 0 || c.arith > 2 || c.method < 0 || c.method > 1)
        return set_error(SINCOS_EINVAL, "server_create: bad arith or method");
    if (c.mode != 0 && c.mode != 1)
        return set_error(SINCOS_EINVAL, "server_create: mode must be 0 or 1");
    if (c.executor != 0 && c.executor != 1)
        return set_error(SINCOS_EINVAL, "server_create: executor must be 0 or 1");
    if (c.stream_per_slot != 0 && c.stream_per_slot != 1)
        return set_error(SINCOS_EINVAL, "server_create: stream_per_slot must be 0 or 1");
    auto srv = std::make_unique<sincos_server>();
    srv->cfg = c;
    srv->budget = (uint64_t)c.budget_bytes;
    // outputs take 8 of every 12 charged bytes; blocks are rounded up to
    // 256-byte granules (at most 542 bytes per request, under 7 % of the 8000
    // output bytes of the smallest useful request), so the arena is 3/4 of
    // the budget: admission is limited by the budget, not the arena
    const uint64_t arena_bytes = srv->budget / 4 * 3 + (uint64_t(1) << 20);
    srv->arena.reset(arena_bytes, 256);
    if (c.executor == 0) {
        if (hipGetDevice(&srv->device) != hipSuccess)
            return set_error(SINCOS_ENODEV, "server_create: no HIP device");
        const int64_t class_split =
            c.mode == 1 || c.stream_per_slot ? -1 : std::max<int64_t>(c.split_elems, 0);
        srv->exec = std::make_unique<GpuExecutor>(srv->device, srv->arena.capacity(), c.arith,
                                                  c.method, c.mode, class_split);
    } else {
        srv->exec = std::make_unique<SimExecutor>(c.sim_batch_ns, c.sim_elem_ps, c.sim_fail_every);
    }
    int rc = srv->exec->init(c.max_inflight);
    if (rc != SINCOS_OK)
        return rc;
    srv->slots.resize(c.max_inflight);
    sincos_server *raw = srv.get();
    srv->thread = std::thread([raw] { raw->run(); });
    *out = srv.release();
    return SINCOS_OK;
}

static int submit_request(sincos_server_t *srv, const float *x, int64_t n, uint64_t tag,
                          hipEvent_t ready, int64_t *out_id)
{
    auto r = std::make_unique<Request>();
    r->x = x;
    r->n = n;
    r->tag = tag;
    r->ready = ready;
    r->t_submit = now_ns();
    {
        std::lock_guard<std::mutex> lk(srv->mu);
        if (srv->stop) {
            if (ready)
                srv->event_pool.push_back(ready);
            return set_error(SINCOS_ECANCELED, "server_submit: server is stopping");
        }
        r->id = srv->next_id++;
        if (out_id)
            *out_id = r->id;
        srv->incoming.push_back(r.get());
        srv->all[r->id] = std::move(r);
        srv->stats.submitted++;
    }
    srv->cv_sched.notify_one();
    return SINCOS_OK;
}

static int check_submit(sincos_server_t *srv, const float *x, int64_t n, const char *who)
{
    if (!srv)
        return set_error(SINCOS_EINVAL, std::string(who) + ": null server");
    if (n <= 0 || !x || (reinterpret_cast<uintptr_t>(x) & 3))
        return set_error(SINCOS_EINVAL,
                         std::string(who) + ": need n >= 1 and a 4-byte aligned input");
    if ((uint64_t)n * 12 > srv->budget)
        return set_error(SINCOS_EBUDGET, std::string(who) + ": request exceeds the whole budget");
    return SINCOS_OK;
}

extern "C" int sincos_server_submit(sincos_server_t *srv, const float *x, int64_t n, uint64_t tag,
                                    int64_t *out_id)
{
    clear_error();
    const int rc = check_submit(srv, x, n, "server_submit");
    return rc != SINCOS_OK ? rc : submit_request(srv, x, n, tag, nullptr, out_id);
}

extern "C" int sincos_server_submit_on(sincos_server_t *srv, const float *x, int64_t n,
                                       uint64_t tag, void *stream, int64_t *out_id)
{
    clear_error();
    int rc = check_submit(srv, x, n, "server_submit_on");
    if (rc != SINCOS_OK)
        return rc;
    if (srv->cfg.executor != 0)  // simulated: no device work to wait for
        return submit_request(srv, x, n, tag, nullptr, out_id);
    int dev = -1;
    if (hipGetDevice(&dev) != hipSuccess || dev != srv->device)
        return set_error(SINCOS_EINVAL, "server_submit_on: the calling thread's current device "
                                        "is not the server's");
    hipEvent_t ev = nullptr;
    {
        std::lock_guard<std::mutex> lk(srv->mu);
        if (!srv->event_pool.empty()) {
            ev = srv->event_pool.back();
            srv->event_pool.pop_back();
        }
    }
    if (!ev && hipEventCreateWithFlags(&ev, hipEventDisableTiming) != hipSuccess)
        return set_error(SINCOS_EHIP, "server_submit_on: cannot create an event");
    if (hipEventRecord(ev, (hipStream_t)stream) != hipSuccess) {
        std::lock_guard<std::mutex> lk(srv->mu);
        srv->event_pool.push_back(ev);
        return set_error(SINCOS_EHIP, "server_submit_on: cannot record on the stream");
    }
    return submit_request(srv, x, n, tag, ev, out_id);
}

static void fill_completion(const Request *r, bool auto_release, sincos_completion_t *o)
{
    o->id = r->id;
    o->tag = r->tag;
    o->status = r->status;
    o->batch_requests = r->batch_requests;
    const bool have = !auto_release && r->status == SINCOS_OK;
    o->s = have ? r->s : nullptr;
    o->c = have ? r->c : nullptr;
    o->n = r->n;
    o->t_submit_ns = r->t_submit;
    o->t_admit_ns = r->t_admit;
    o->t_launch_ns = r->t_launch;
    o->t_complete_ns = r->t_complete;
}

extern "C" int sincos_server_poll(sincos_server_t *srv, sincos_completion_t *out, int32_t max,
                                  int32_t *count, int64_t timeout_ns)
{
    clear_error();
    if (!srv || !out || !count || max < 0)
        return set_error(SINCOS_EINVAL, "server_poll: bad argument");
    *count = 0;
    std::unique_lock<std::mutex> lk(srv->mu);
    if (srv->done.empty() && timeout_ns > 0)
        srv->cv_done.wait_for(lk, std::chrono::nanoseconds(timeout_ns),
                              [srv] { return !srv->done.empty(); });
    int32_t k = 0;
    while (k < max && !srv->done.empty()) {
        Request *r = srv->done.front();
        srv->done.pop_front();
        fill_completion(r, srv->cfg.auto_release != 0, &out[k++]);
        if (srv->cfg.auto_release || r->status != SINCOS_OK)
            srv->all.erase(r->id);  // nothing left to release
    }
    *count = k;
    return SINCOS_OK;
}

extern "C" int sincos_server_release(sincos_server_t *srv, int64_t id)
{
    clear_error();
    if (!srv)
        return set_error(SINCOS_EINVAL, "server_release: null server");
    {
        std::lock_guard<std::mutex> lk(srv->mu);
        auto it = srv->all.find(id);
        if (it == srv->all.end() || it->second->t_complete == 0)
            return set_error(SINCOS_EINVAL, "server_release: unknown or unfinished request");
        srv->free_request_memory(it->second.get());
        srv->all.erase(it);
    }
    srv->cv_sched.notify_one();
    return SINCOS_OK;
}

extern "C" int sincos_server_stats(const sincos_server_t *srv, sincos_server_stats_t *out)
{
    clear_error();
    if (!srv || !out)
        return set_error(SINCOS_EINVAL, "server_stats: null argument");
    auto *s = const_cast<sincos_server_t *>(srv);
    std::lock_guard<std::mutex> lk(s->mu);
    *out = s->stats;
    return SINCOS_OK;
}

extern "C" int sincos_server_replay(sincos_server_t *srv, const float *const *xs,
                                    const int64_t *ns, const int64_t *arrival_ns, int32_t count,
                                    sincos_completion_t *out)
{
    clear_error();
    if (!srv || count < 0 || (count > 0 && (!xs || !ns || !arrival_ns || !out)))
        return set_error(SINCOS_EINVAL, "server_replay: bad argument");
    for (int32_t j = 0; j < count; ++j)
        if (ns[j] <= 0 || (uint64_t)ns[j] * 12 > srv->budget || !xs[j] || arrival_ns[j] < 0)
            return set_error(SINCOS_EINVAL, "server_replay: request " + std::to_string(j) +
                                                " has a bad size, input or arrival time");
    std::vector<int64_t> ids(count, -1);
    std::unordered_map<int64_t, int32_t> index;
    std::mutex idx_mu;
    std::atomic<int> submit_rc{SINCOS_OK};
    const int64_t t0 = now_ns();
    std::thread gen([&] {
        for (int32_t j = 0; j < count; ++j) {
            const int64_t due = t0 + arrival_ns[j];
            while (now_ns() < due)
                if (due - now_ns() > 200000)
                    std::this_thread::sleep_for(std::chrono::microseconds(50));
            int64_t id = -1;
            std::lock_guard<std::mutex> lk(idx_mu);
            int rc = sincos_server_submit(srv, xs[j], ns[j], (uint64_t)j, &id);
            if (rc != SINCOS_OK) {
                submit_rc = rc;
                return;
            }
            ids[j] = id;
            index[id] = j;
        }
    });
    int32_t got = 0;
    std::vector<sincos_completion_t> buf(256);
    int rc = SINCOS_OK;
    while (got < count) {
        int32_t k = 0;
        sincos_server_poll(srv, buf.data(), (int32_t)buf.size(), &k, 2000000);
        for (int32_t i = 0; i < k; ++i) {
            const int32_t j = (int32_t)buf[i].tag;
            if (j < 0 || j >= count)
                continue;
            out[j] = buf[i];
            if (buf[i].status != SINCOS_OK && rc == SINCOS_OK)
                rc = buf[i].status;
            if (!srv->cfg.auto_release && buf[i].status == SINCOS_OK)
                sincos_server_release(srv, buf[i].id);
            ++got;
        }
        if (submit_rc != SINCOS_OK && got >= count)
            break;
        if (submit_rc != SINCOS_OK) {
            // the generator stopped early: wait only for what was submitted
            std::lock_guard<std::mutex> lk(idx_mu);
            int32_t submitted = (int32_t)index.size();
            if (got >= submitted)
                break;
        }
    }
    gen.join();
    if (submit_rc != SINCOS_OK)
        return set_error(submit_rc, "server_replay: a submission failed");
    if (rc != SINCOS_OK)
        return set_error(rc, "server_replay: some requests failed");
    return SINCOS_OK;
}

extern "C" int sincos_server_destroy(sincos_server_t *srv)
{
    clear_error();
    if (!srv)
        return SINCOS_OK;
    {
        std::lock_guard<std::mutex> lk(srv->mu);
        srv->stop = true;
    }
    srv->cv_sched.notify_all();
    if (srv->thread.joinable())
        srv->thread.join();
    srv->exec.reset();
    if (srv->cfg.executor == 0) {
        int prev = -1;
        const bool restore = hipGetDevice(&prev) == hipSuccess && prev != srv->device;
        (void)hipSetDevice(srv->device);
        for (hipEvent_t ev : srv->event_pool)
            (void)hipEventDestroy(ev);
        for (auto &kv : srv->all)  // requests never completed keep theirs
            if (kv.second->ready)
                (void)hipEventDestroy(kv.second->ready);
        if (restore)
            (void)hipSetDevice(prev);
    }
    delete srv;
    return SINCOS_OK;
}
