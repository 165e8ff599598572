// Host check of the autotuner cache's JSON reader and writer (gdi_tunecache.cpp), built
// with g++ under the address and undefined-behaviour sanitizers by test_tune_cache.py:
// round trips of generated tables, rejection of malformed texts (nothing merged), and
// every truncation and many single-byte mutations of a valid file (no crash, no
// out-of-bounds read; any accepted text is JSON of the format). No GPU.
#include <stdint.h>
#include <stdio.h>

#include <string>

#include "../paper_1908_00210_amd/csrc/gdi_tunecache.h"

using gdi_tunecache::Fields;
using gdi_tunecache::Table;

static int g_fail = 0;
#define CHECK(c)                                                   \
    do {                                                           \
        if (!(c)) {                                                \
            printf("FAIL line %d: %s\n", __LINE__, #c);            \
            ++g_fail;                                              \
        }                                                          \
    } while (0)

static uint64_t g_rng = 0x243F6A8885A308D3ull;
static uint64_t next()
{
    g_rng ^= g_rng << 13;
    g_rng ^= g_rng >> 7;
    g_rng ^= g_rng << 17;
    return g_rng;
}

int main()
{
    long checks = 0;
    // round trips of generated tables: integer fields, fractional times, odd keys
    for (int rep = 0; rep < 200; ++rep) {
        Table t;
        const int ne = (int)(next() % 6);
        for (int e = 0; e < ne; ++e) {
            std::string key = "gfx950/256cu|graph|n=" + std::to_string(next() % 100000);
            if (next() % 3 == 0) key += "\"q\\\x01\t\xc3\xa9";  // quote, backslash, controls, UTF-8
            Fields f;
            f["block"] = (double)(64 * (1 + next() % 16));
            f["tail_max"] = -1.0 + (double)(next() % 3);
            f["ms"] = (double)(next() % 1000000) / 977.0;
            t[key] = f;
        }
        Table back;
        std::string err;
        CHECK(gdi_tunecache::parse(gdi_tunecache::dump(t), &back, &err) == 0);
        CHECK(back == t);
        ++checks;
    }
    // malformed texts are rejected and leave the table unchanged
    const char *bad[] = {
        "",
        "[]",
        "{}",                                            // no format
        "{\"format\": \"gdi-tune-2\", \"entries\": {}}",  // unknown format
        "{\"format\": \"gdi-tune-1\", \"entries\": {\"k\": {\"block\": \"256\"}}}",
        "{\"format\": \"gdi-tune-1\", \"entries\": {\"k\": [1]}}",
        "{\"format\": \"gdi-tune-1\", \"entries\": {\"k\": {\"block\": 256,}}}",
        "{\"format\": \"gdi-tune-1\", \"entries\": {\"k\": {\"block\": 256}}} x",
        "{\"format\": \"gdi-tune-1\", \"entries\": {\"\\ud800\": {}}}",
        "{\"format\": \"gdi-tune-1\", \"entries\": {\"k\": {\"ms\": 1e999}}}",
        "{\"format\": \"gdi-tune-1\", \"entries\": {\"k\": {\"ms\": -}}}",
        "{\"format\": \"gdi-tune-1\", \"x\": [[[[[[[[[[[[[[[[[[[[[[[[[[[[[[[[[[[[1]]]]]]]]]]]]]]]]]]]]]]]]]]]]]]]]]]]}",
        "{\"format\": \"gdi-tune-1\", \"entries\": {\"k\": {\"block\": 256}}",
    };
    for (const char *b : bad) {
        Table t;
        t["keep"]["block"] = 1;
        const Table before = t;
        std::string err;
        CHECK(gdi_tunecache::parse(b, &t, &err) != 0);
        CHECK(!err.empty());
        CHECK(t == before);
        ++checks;
    }
    // accepted: unknown members skipped, entries merged over existing keys
    {
        Table t;
        t["a"]["block"] = 1;
        t["b"]["block"] = 2;
        std::string err;
        CHECK(gdi_tunecache::parse("{\"note\": [true, false, null, {\"x\": \"y\"}], \"format\": \"gdi-tune-1\", "
                                   "\"entries\": {\"b\": {\"block\": 512, \"ms\": 0.25}}}",
                                   &t, &err) == 0);
        CHECK(t.size() == 2 && t["a"]["block"] == 1 && t["b"]["block"] == 512 && t["b"]["ms"] == 0.25);
        ++checks;
    }
    // every truncation and random single-byte mutations of a valid text
    Table ref;
    ref["gfx950/256cu|batch|inst=320"]["block"] = 256;
    ref["gfx950/256cu|batch|inst=320"]["ms"] = 12.5;
    ref["gfx950/256cu|graph|n=7\\\"x"]["grid"] = 128;
    const std::string good = gdi_tunecache::dump(ref);
    for (size_t k = 0; k < good.size(); ++k) {
        Table t;
        std::string err;
        const int rc = gdi_tunecache::parse(good.substr(0, k), &t, &err);
        CHECK(rc != 0 || good.substr(k).find_first_not_of(" \n\t\r") == std::string::npos);
        ++checks;
    }
    for (int rep = 0; rep < 20000; ++rep) {
        std::string m = good;
        const int nmut = 1 + (int)(next() % 3);
        for (int j = 0; j < nmut; ++j) m[next() % m.size()] = (char)(next() & 0xFF);
        Table t;
        std::string err;
        if (gdi_tunecache::parse(m, &t, &err) == 0) {
            // what was accepted dumps and parses back to itself
            Table again;
            CHECK(gdi_tunecache::parse(gdi_tunecache::dump(t), &again, &err) == 0 && again == t);
        } else {
            CHECK(t.empty());
        }
        ++checks;
    }
    if (g_fail) {
        printf("FAILED %d\n", g_fail);
        return 1;
    }
    printf("OK %ld\n", checks);
    return 0;
}
