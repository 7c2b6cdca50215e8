// Host-side paths of the C ABI that need no GPU, for a sanitizer build:
// the tuning parser on every prefix of valid documents and on random bytes
// (each string in a heap block of exactly its size, so a read past the
// terminator is caught), sincos_get_tuning with every buffer size, and the
// argument checks of the entry points.  Exits non-zero on a logic failure.
#include "../../include/sincos.h"

#include <cstdint>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <random>
#include <string>

#define CHECK(cond)                                                                \
    do {                                                                           \
        if (!(cond)) {                                                             \
            std::fprintf(stderr, "check failed: %s (line %d)\n", #cond, __LINE__); \
            std::exit(1);                                                          \
        }                                                                          \
    } while (0)

static int set_exact(const std::string &text)
{
    char *buf = static_cast<char *>(std::malloc(text.size() + 1));
    std::memcpy(buf, text.c_str(), text.size() + 1);
    const int rc = sincos_set_tuning(buf);
    std::free(buf);
    return rc;
}

static std::string current()
{
    const int64_t n = sincos_get_tuning(nullptr, 0);
    CHECK(n > 0 && n < 4096);
    std::string s(static_cast<size_t>(n) + 1, '\0');
    CHECK(sincos_get_tuning(&s[0], n + 1) == n);
    s.resize(static_cast<size_t>(n));
    return s;
}

int main()
{
    const char *docs[] = {
        "{\"plain\": {\"block\": 512, \"unroll\": 2, \"grid\": 7}, \"ragged\": {\"grid\": 9}}",
        " { \"ragged\" : { \"unroll\" : 8 , \"block\" : 1024 } } ",
        "{}",
    };
    for (const char *d : docs) {
        const std::string doc(d);
        CHECK(set_exact(doc) == SINCOS_OK);
        const std::string good = current();
        // every proper prefix is invalid and leaves the shapes unchanged
        for (size_t len = 0; len < doc.size(); ++len) {
            const std::string cut = doc.substr(0, len);
            bool blank = true;
            for (char ch : cut)
                blank = blank && (ch == ' ');
            if (set_exact(cut) == SINCOS_OK) {
                // only a prefix that is a complete document may parse
                CHECK(!blank);
                CHECK(cut.find('{') != std::string::npos);
            }
            CHECK(std::strlen(sincos_last_error()) < 4096);
            CHECK(set_exact(doc) == SINCOS_OK);
        }
        CHECK(current() == good);
    }
    // random bytes, and random edits of a valid document
    std::mt19937 rng(12345);
    const std::string alphabet = "{}[]\":,-0123456789 abcdeghiklnoprstuxyz.\\\t\n";
    for (int it = 0; it < 20000; ++it) {
        std::string s;
        const int len = static_cast<int>(rng() % 64);
        for (int k = 0; k < len; ++k)
            s.push_back(alphabet[rng() % alphabet.size()]);
        const int rc = set_exact(s);
        CHECK(rc == SINCOS_OK || rc == SINCOS_EINVAL);
    }
    const std::string base(docs[0]);
    for (int it = 0; it < 20000; ++it) {
        std::string s = base;
        const int edits = 1 + static_cast<int>(rng() % 3);
        for (int e = 0; e < edits; ++e) {
            const size_t pos = rng() % s.size();
            switch (rng() % 3) {
            case 0: s[pos] = alphabet[rng() % alphabet.size()]; break;
            case 1: s.erase(pos, 1); break;
            default: s.insert(pos, 1, alphabet[rng() % alphabet.size()]); break;
            }
            if (s.empty())
                s = "{";
        }
        const int rc = set_exact(s);
        CHECK(rc == SINCOS_OK || rc == SINCOS_EINVAL);
    }
    CHECK(sincos_set_tuning(nullptr) == SINCOS_OK);

    // get_tuning into buffers of every size up to the full length
    const std::string full = current();
    for (int64_t cap = 0; cap <= (int64_t)full.size() + 2; ++cap) {
        char *buf = cap ? static_cast<char *>(std::malloc(static_cast<size_t>(cap))) : nullptr;
        CHECK(sincos_get_tuning(buf, cap) == (int64_t)full.size());
        if (cap) {
            CHECK(std::strlen(buf) == static_cast<size_t>(std::min<int64_t>(cap - 1, full.size())));
            CHECK(full.compare(0, std::strlen(buf), buf) == 0);
        }
        std::free(buf);
    }

    // argument checks (rejected before any device work)
    float *const fake = reinterpret_cast<float *>(uintptr_t(1) << 33);
    CHECK(sincos_f32(fake, fake + 1024, fake + 2048, -1, nullptr) == SINCOS_EINVAL);
    CHECK(sincos_f32(fake, fake + 1024, fake + 1024, 16, nullptr) == SINCOS_EOVERLAP);
    sincos_launch_t bad = {100, 1, 0, 0};
    CHECK(sincos_f32_ex(fake, fake + 1024, fake + 2048, 16, 0, 0, &bad, nullptr) == SINCOS_EINVAL);
    sincos_seg_t segs[2] = {{fake, fake + 1024, fake + 2048}, {fake, fake + 1024, fake + 4096}};
    int64_t lens[2] = {16, 16};
    CHECK(sincos_f32_ragged(segs, lens, 2, nullptr) == SINCOS_EOVERLAP);
    CHECK(sincos_f32_ragged(segs, lens, -1, nullptr) == SINCOS_EINVAL);
    CHECK(sincos_f32_interleaved(fake, fake + 4, 8, 0, nullptr) == SINCOS_EOVERLAP);
    CHECK(huygens_f32(fake, fake, 4, fake, 4, 1.0f, -1.0f, fake + 4096, fake + 8192, nullptr) ==
          SINCOS_EINVAL);
    CHECK(sincos_pair_ceiling_f32(fake, fake + 2, 16, 1, nullptr) == SINCOS_EOVERLAP);
    CHECK(sinusoid_f32_backward_workspace_bytes(-1, 1) == -1);
    sincos_server_config_t cfg{};
    cfg.executor = 7;
    sincos_server_t *srv = nullptr;
    CHECK(sincos_server_create(&cfg, &srv) == SINCOS_EINVAL && srv == nullptr);
    std::printf("host_paths: ok\n");
    return 0;
}
