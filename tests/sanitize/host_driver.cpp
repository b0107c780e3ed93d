// Host-only checks built with AddressSanitizer and UndefinedBehaviorSanitizer: the prolate
// kernel tables for every support and oversampling the library accepts, and the autotuner's
// cache parser on crafted files (overlong lines, malformed and truncated records, keys at
// the buffer limit). Exits non-zero on a wrong result; the sanitizers abort on any error.
#include <cstdio>
#include <cstring>
#include <string>
#include <vector>

#include "internal.h"
#include "tune_cache.h"

int main(int argc, char **argv) {
    if (argc < 2) return 2;
    const std::string dir = argv[1];
    // kernel tables: every odd W in 1..15, O in 1..16, odd and even grid sizes
    for (int W = 1; W <= 15; W += 2)
        for (int O = 1; O <= 16; O++) {
            std::vector<float> tab, cx, cy;
            mwg::prolate_tables(W, O, 8 + 2 * O, 64 + W, tab, cx, cy);
            if ((int)tab.size() != O * W || (int)cx.size() != 8 + 2 * O || (int)cy.size() != 64 + W) return 3;
            for (int p = 0; p < O; p++) {
                double sum = 0;
                for (int t = 0; t < W; t++) sum += tab[(size_t)p * W + t];
                if (!(sum > 0.999 && sum < 1.001)) return 4;
            }
        }
    // tuner cache
    const std::string path = dir + "/cache.jsonl";
    FILE *f = std::fopen(path.c_str(), "w");
    if (!f) return 5;
    std::string longkey(300, 'k');
    std::string overlong(2000, 'x');
    std::fprintf(f, "%s\n", overlong.c_str());
    std::fprintf(f, "{\"key\": \"%s\", \"tile\": 1, \"split\": 2, \"wg_waves\": 3, \"order\": 4, \"variant\": 5, "
                    "\"flush\": 6, \"schedule\": 7, \"ms\": 1.0}\n", longkey.c_str());
    std::fprintf(f, "{\"key\": \"a/b\", \"tile\": 16, \"split\": 2048\n");  // malformed
    std::fprintf(f, "garbage without braces\n\n");
    std::fclose(f);
    mwg::tune_cache_store(path.c_str(), "a/b", mwg::TuneRecord{8, 4096, 4, 3, 4, 2, 1}, 0.5f);
    mwg::tune_cache_store(path.c_str(), "a/c", mwg::TuneRecord{16, 0, 8, 3, 4, 3, 1}, 0.25f);
    mwg::TuneRecord r{};
    if (!mwg::tune_cache_lookup(path.c_str(), "a/b", &r)) return 6;
    if (r.tile != 8 || r.split != 4096 || r.wg_waves != 4 || r.flush != 2) return 7;
    if (!mwg::tune_cache_lookup(path.c_str(), "a/c", &r) || r.tile != 16 || r.flush != 3) return 8;
    if (mwg::tune_cache_lookup(path.c_str(), "missing", &r)) return 9;
    if (mwg::tune_cache_lookup(path.c_str(), longkey.c_str(), &r)) return 10;  // its key does not fit
    // a file cut in the middle of its last record
    f = std::fopen(path.c_str(), "a");
    std::fprintf(f, "{\"key\": \"a/b\", \"tile\": 32, \"split\": 1, \"wg_waves\": 1");
    std::fclose(f);
    if (!mwg::tune_cache_lookup(path.c_str(), "a/b", &r) || r.tile != 8) return 11;
    if (mwg::tune_cache_lookup((dir + "/absent.jsonl").c_str(), "a/b", &r)) return 12;
    std::printf("host checks passed\n");
    return 0;
}
