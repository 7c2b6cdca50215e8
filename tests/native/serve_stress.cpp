// Multi-threaded stress of the request server with the simulated executor:
// several submitting threads, a polling/releasing thread, stats readers and a
// shutdown while requests are pending.  Built with ThreadSanitizer on the host
// code by tests/test_native_tsan.py; exits non-zero on a logic failure.
#include "../../include/sincos.h"

#include <atomic>
#include <cstdio>
#include <cstdlib>
#include <thread>
#include <vector>

#define CHECK(cond)                                                        \
    do {                                                                   \
        if (!(cond)) {                                                     \
            std::fprintf(stderr, "check failed: %s (line %d)\n", #cond, __LINE__); \
            std::exit(1);                                                  \
        }                                                                  \
    } while (0)

static const float *fake_input(int j) { return reinterpret_cast<const float *>(uintptr_t(1) << 33) + 64 * j; }

static void scenario(int auto_release, int fail_every, int mode)
{
    sincos_server_config_t cfg{};
    cfg.budget_bytes = 12 * 40000;
    cfg.max_inflight = 3;
    cfg.executor = 1;
    cfg.sim_batch_ns = 20000;
    cfg.sim_elem_ps = 100;
    cfg.sim_fail_every = fail_every;
    cfg.auto_release = auto_release;
    cfg.mode = mode;
    sincos_server_t *srv = nullptr;
    CHECK(sincos_server_create(&cfg, &srv) == SINCOS_OK);
    const int producers = 4, per = 300;
    std::atomic<int> submitted{0};
    std::vector<std::thread> ths;
    for (int p = 0; p < producers; ++p)
        ths.emplace_back([&, p] {
            for (int j = 0; j < per; ++j) {
                int64_t id;
                CHECK(sincos_server_submit(srv, fake_input(j), 100 + (j * 37 + p) % 3000,
                                           (uint64_t)(p * per + j), &id) == SINCOS_OK);
                submitted++;
                if (j % 50 == 0)
                    std::this_thread::yield();
            }
        });
    std::atomic<int> completed{0}, failed{0};
    std::thread consumer([&] {
        std::vector<sincos_completion_t> buf(64);
        while (completed + failed < producers * per) {
            int32_t k = 0;
            CHECK(sincos_server_poll(srv, buf.data(), 64, &k, 1000000) == SINCOS_OK);
            for (int i = 0; i < k; ++i) {
                if (buf[i].status == SINCOS_OK) {
                    completed++;
                    if (!auto_release)
                        CHECK(sincos_server_release(srv, buf[i].id) == SINCOS_OK);
                } else {
                    failed++;
                }
            }
        }
    });
    std::thread watcher([&] {
        sincos_server_stats_t st;
        for (int i = 0; i < 200; ++i) {
            CHECK(sincos_server_stats(srv, &st) == SINCOS_OK);
            CHECK(st.budget_in_use <= cfg.budget_bytes);
            std::this_thread::yield();
        }
    });
    for (auto &t : ths)
        t.join();
    consumer.join();
    watcher.join();
    sincos_server_stats_t st;
    CHECK(sincos_server_stats(srv, &st) == SINCOS_OK);
    CHECK(st.submitted == producers * per);
    CHECK(st.completed + st.failed == producers * per);
    CHECK(st.budget_in_use == 0);
    CHECK(st.inflight_peak <= 3);
    if (fail_every == 0)
        CHECK(st.failed == 0);
    // shutdown with work pending
    for (int j = 0; j < 50; ++j) {
        int64_t id;
        CHECK(sincos_server_submit(srv, fake_input(j), 30000, 7, &id) == SINCOS_OK);
    }
    CHECK(sincos_server_destroy(srv) == SINCOS_OK);
}

int main()
{
    scenario(1, 0, 0);
    scenario(0, 0, 0);
    scenario(1, 5, 0);
    scenario(0, 0, 1);
    std::printf("serve_stress: ok\n");
    return 0;
}
