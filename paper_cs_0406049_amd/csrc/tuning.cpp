// tuning.cpp -- process-wide default launch shapes (sincos_set_tuning /
// sincos_get_tuning).  An autotuner measures shapes and installs its choice
// here; every call that passes no launch shape (or 0 in a field) then uses it.
//
// The accepted text is a small JSON subset:
//   {"plain": {"block": 256, "unroll": 1, "grid": 0, "lds": 8192},
//    "ragged": {"block": 512, "unroll": 2, "grid": 0}}
// Both forms and all four fields are optional; a missing field takes the
// built-in default (kBuiltinShape).  Anything else (unknown keys,
// non-integers, numbers JSON does not allow, escapes in keys, a repeated key,
// trailing text) is rejected, leaving the current shapes unchanged.
#include "../../include/sincos.h"
#include "internal.hpp"

#include <cctype>
#include <climits>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <string>

namespace mi355 {

static std::mutex g_tune_mu;
static LaunchShape g_tuned[2] = {kBuiltinShape[kFormPlain], kBuiltinShape[kFormRagged]};

LaunchShape default_shape(int form)
{
    std::lock_guard<std::mutex> lk(g_tune_mu);
    return g_tuned[form == kFormRagged ? kFormRagged : kFormPlain];
}

int validate_shape(const LaunchShape &sh, const char *who)
{
    if (sh.block < 64 || sh.block > 1024 || sh.block % 64 != 0)
        return set_error(SINCOS_EINVAL, std::string(who) + ": block must be a multiple of 64 in [64, 1024]");
    if (sh.unroll != 1 && sh.unroll != 2 && sh.unroll != 4 && sh.unroll != 8)
        return set_error(SINCOS_EINVAL, std::string(who) + ": unroll must be 1, 2, 4 or 8");
    if (sh.grid < 0)
        return set_error(SINCOS_EINVAL, std::string(who) + ": grid must be >= 0");
    if (sh.lds < 0 || sh.lds > 65536)
        return set_error(SINCOS_EINVAL, std::string(who) + ": lds must be in [0, 65536]");
    return SINCOS_OK;
}

namespace {

// Recursive-descent reader over a NUL-terminated string; every accessor
// checks for the terminator before it advances.
struct Reader {
    const char *p;
    std::string err;

    void ws()  // JSON whitespace only
    {
        while (*p == ' ' || *p == '\t' || *p == '\n' || *p == '\r')
            ++p;
    }
    bool fail(const std::string &m)
    {
        if (err.empty())
            err = m;
        return false;
    }
    bool expect(char ch)
    {
        ws();
        if (*p != ch)
            return fail(std::string("expected '") + ch + "'");
        ++p;
        return true;
    }
    bool key(std::string &out)
    {
        ws();
        if (*p != '"')
            return fail("expected a quoted key");
        ++p;
        out.clear();
        while (*p && *p != '"') {
            if (*p == '\\' || out.size() > 32)
                return fail("unsupported key");
            out.push_back(*p++);
        }
        if (*p != '"')
            return fail("unterminated key");
        ++p;
        return true;
    }
    bool integer(int &out)
    {
        ws();
        bool neg = false;
        if (*p == '-') {
            neg = true;
            ++p;
        }
        if (!std::isdigit((unsigned char)*p))
            return fail("expected an integer");
        if (p[0] == '0' && std::isdigit((unsigned char)p[1]))
            return fail("leading zero");
        long long v = 0;
        while (std::isdigit((unsigned char)*p)) {
            v = v * 10 + (*p++ - '0');
            if (v > (1LL << 31) || (!neg && v > INT_MAX))
                return fail("integer out of range");
        }
        if (*p == '.' || *p == 'e' || *p == 'E')
            return fail("expected an integer");
        out = (int)(neg ? -v : v);
        return true;
    }
    // {"block": B, "unroll": U, "grid": G, "lds": L}, any subset, any order
    bool shape(LaunchShape &sh)
    {
        if (!expect('{'))
            return false;
        ws();
        if (*p == '}') {
            ++p;
            return true;
        }
        bool seen[4] = {false, false, false, false};
        for (;;) {
            std::string k;
            int v = 0;
            if (!key(k) || !expect(':') || !integer(v))
                return false;
            const int f = k == "block" ? 0 : k == "unroll" ? 1 : k == "grid" ? 2 : k == "lds" ? 3 : -1;
            if (f < 0)
                return fail("unknown field \"" + k + "\"");
            if (seen[f])
                return fail("repeated field \"" + k + "\"");
            seen[f] = true;
            (f == 0 ? sh.block : f == 1 ? sh.unroll : f == 2 ? sh.grid : sh.lds) = v;
            ws();
            if (*p == ',') {
                ++p;
                continue;
            }
            return expect('}');
        }
    }
    bool document(LaunchShape out[2])
    {
        if (!expect('{'))
            return false;
        ws();
        if (*p == '}') {
            ++p;
        } else {
            bool seen[2] = {false, false};
            for (;;) {
                std::string k;
                if (!key(k) || !expect(':'))
                    return false;
                const int form = k == "plain" ? kFormPlain : k == "ragged" ? kFormRagged : -1;
                if (form < 0)
                    return fail("unknown form \"" + k + "\" (plain or ragged)");
                if (seen[form])
                    return fail("repeated form \"" + k + "\"");
                seen[form] = true;
                if (!shape(out[form]))
                    return false;
                ws();
                if (*p == ',') {
                    ++p;
                    continue;
                }
                if (!expect('}'))
                    return false;
                break;
            }
        }
        ws();
        if (*p)
            return fail("trailing text");
        return true;
    }
};

}  // namespace
}  // namespace mi355

using namespace mi355;

extern "C" int sincos_set_tuning(const char *json)
{
    clear_error();
    // built-in defaults; fields present in json override
    LaunchShape next[2] = {kBuiltinShape[kFormPlain], kBuiltinShape[kFormRagged]};
    if (json) {
        Reader r{json, {}};
        if (!r.document(next))
            return set_error(SINCOS_EINVAL, "sincos_set_tuning: " + r.err + " at offset " +
                                                std::to_string(r.p - json));
        int rc;
        if ((rc = validate_shape(next[kFormPlain], "sincos_set_tuning: plain")) != SINCOS_OK ||
            (rc = validate_shape(next[kFormRagged], "sincos_set_tuning: ragged")) != SINCOS_OK)
            return rc;
    }
    std::lock_guard<std::mutex> lk(g_tune_mu);
    g_tuned[kFormPlain] = next[kFormPlain];
    g_tuned[kFormRagged] = next[kFormRagged];
    return SINCOS_OK;
}

extern "C" int64_t sincos_get_tuning(char *buf, int64_t cap)
{
    clear_error();
    LaunchShape cur[2];
    {
        std::lock_guard<std::mutex> lk(g_tune_mu);
        cur[0] = g_tuned[0];
        cur[1] = g_tuned[1];
    }
    char text[256];
    const int len = std::snprintf(
        text, sizeof text,
        "{\"plain\": {\"block\": %d, \"unroll\": %d, \"grid\": %d, \"lds\": %d}, "
        "\"ragged\": {\"block\": %d, \"unroll\": %d, \"grid\": %d, \"lds\": %d}}",
        cur[0].block, cur[0].unroll, cur[0].grid, cur[0].lds, cur[1].block, cur[1].unroll,
        cur[1].grid, cur[1].lds);
    if (len < 0 || len >= (int)sizeof text)
        return set_error(SINCOS_EINVAL, "sincos_get_tuning: formatting failed");
    if (buf && cap > 0) {
        const int64_t n = std::min<int64_t>(len, cap - 1);
        std::memcpy(buf, text, (size_t)n);
        buf[n] = '\0';
    }
    return len;
}
