// Randomized check of the request server's output arena (serve.hpp) against
// a plain model: the set of allocated blocks, with first fit computed by
// scanning the gaps between them in address order.  After every operation
// the arena's offset, used bytes, number of free fragments (coalesced) and
// largest free block must equal the model's.  Exits non-zero on a mismatch.
#include "../../paper_cs_0406049_amd/csrc/serve.hpp"

#include <cstdint>
#include <cstdio>
#include <cstdlib>
#include <map>
#include <random>
#include <vector>

#define CHECK(cond)                                                                \
    do {                                                                           \
        if (!(cond)) {                                                             \
            std::fprintf(stderr, "check failed: %s (line %d)\n", #cond, __LINE__); \
            std::exit(1);                                                          \
        }                                                                          \
    } while (0)

struct Model {
    uint64_t cap, align;
    std::map<uint64_t, uint64_t> blocks;  // offset -> rounded length

    uint64_t round(uint64_t b) const { return (b + align - 1) / align * align; }
    // gaps between blocks, in address order
    std::vector<std::pair<uint64_t, uint64_t>> gaps() const
    {
        std::vector<std::pair<uint64_t, uint64_t>> g;
        uint64_t at = 0;
        for (auto &kv : blocks) {
            if (kv.first > at)
                g.push_back({at, kv.first - at});
            at = kv.first + kv.second;
        }
        if (cap > at)
            g.push_back({at, cap - at});
        return g;
    }
    int64_t alloc(uint64_t bytes)
    {
        const uint64_t need = round(bytes);
        if (need == 0)
            return -1;
        for (auto &gp : gaps())
            if (gp.second >= need) {
                blocks[gp.first] = need;
                return (int64_t)gp.first;
            }
        return -1;
    }
    uint64_t used() const
    {
        uint64_t u = 0;
        for (auto &kv : blocks)
            u += kv.second;
        return u;
    }
};

static void agree(const mi355::Arena &a, const Model &m)
{
    const auto g = m.gaps();
    uint64_t largest = 0;
    for (auto &gp : g)
        largest = gp.second > largest ? gp.second : largest;
    CHECK(a.used() == m.used());
    CHECK(a.fragments() == g.size());
    CHECK(a.largest_free() == largest);
}

static void run(uint64_t capacity, uint64_t align, int ops, uint32_t seed)
{
    mi355::Arena a(capacity, align);
    Model m{capacity / align * align, align, {}};
    CHECK(a.capacity() == m.cap);
    std::mt19937_64 rng(seed);
    std::vector<std::pair<uint64_t, uint64_t>> live;  // (offset, bytes asked)
    for (int op = 0; op < ops; ++op) {
        const bool do_alloc = live.empty() || (rng() % 100) < 55;
        if (do_alloc) {
            // sizes from 0 to a quarter of the capacity, small ones more often
            const uint64_t span = 1 + rng() % 4;
            const uint64_t bytes = rng() % (m.cap / (span * span * 4) + 2);
            const int64_t want = m.alloc(bytes);
            const int64_t got = a.alloc(bytes);
            CHECK(got == want);
            if (got >= 0) {
                CHECK(got % (int64_t)align == 0);
                live.push_back({(uint64_t)got, bytes});
            }
        } else {
            const size_t k = rng() % live.size();
            a.release(live[k].first, live[k].second);
            m.blocks.erase(live[k].first);
            live[k] = live.back();
            live.pop_back();
        }
        agree(a, m);
    }
    for (auto &b : live)
        a.release(b.first, b.second);
    CHECK(a.used() == 0);
    CHECK(a.fragments() == (m.cap > 0 ? 1u : 0u));
    CHECK(a.largest_free() == m.cap);
    // whole-capacity requests on the empty arena
    if (m.cap > 0) {
        CHECK(a.alloc(m.cap) == 0);
        CHECK(a.alloc(1) == -1);
        a.release(0, m.cap);
        CHECK(a.alloc(m.cap + 1) == -1);
    }
    CHECK(a.alloc(0) == -1);
}

int main()
{
    run(64 * 1024, 256, 200000, 1);
    run(64 * 1024 + 100, 256, 50000, 2);  // capacity rounds down to whole granules
    run(1 << 20, 4096, 50000, 3);
    run(4096, 256, 50000, 4);             // 16 granules: full and nearly full often
    run(255, 256, 100, 5);                // no granule at all
    std::printf("arena_model: ok\n");
    return 0;
}
