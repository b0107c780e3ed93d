// The autotuner's result cache: a text file of one JSON object per line,
//   {"key": "...", "tile": T, "split": S, "wg_waves": W, "order": R, "variant": V,
//    "flush": F, "schedule": C, "ms": M}
// Host-only code with no HIP dependency, so that it can also be built on its own (the
// sanitizer tests parse crafted files with it).
#pragma once

#include <cstdio>
#include <cstring>

namespace mwg {

// Fields of one cache record, in file order.
struct TuneRecord {
    int tile, split, wg_waves, order, variant, flush, schedule;
};

// The last record of the file whose key equals key. Lines longer than the read buffer are
// skipped whole; malformed lines are ignored.
inline bool tune_cache_lookup(const char *path, const char *key, TuneRecord *out) {
    FILE *f = std::fopen(path, "r");
    if (!f) return false;
    char line[512];
    bool found = false, skipping = false;
    while (std::fgets(line, sizeof line, f)) {
        const size_t n = std::strlen(line);
        const bool whole = n > 0 && line[n - 1] == '\n';
        if (skipping) {  // the rest of an overlong line
            skipping = !whole;
            continue;
        }
        if (!whole) {  // the start of an overlong line, or a last line cut short: ignored
            skipping = true;
            continue;
        }
        char k[256];
        TuneRecord c;
        if (std::sscanf(line,
                        "{\"key\": \"%255[^\"]\", \"tile\": %d, \"split\": %d, \"wg_waves\": %d, "
                        "\"order\": %d, \"variant\": %d, \"flush\": %d, \"schedule\": %d",
                        k, &c.tile, &c.split, &c.wg_waves, &c.order, &c.variant, &c.flush, &c.schedule) == 8 &&
            std::strcmp(key, k) == 0) {
            *out = c;  // the last matching line wins
            found = true;
        }
    }
    std::fclose(f);
    return found;
}

inline void tune_cache_store(const char *path, const char *key, const TuneRecord &c, float ms) {
    FILE *f = std::fopen(path, "a");
    if (!f) return;
    std::fprintf(f,
                 "{\"key\": \"%s\", \"tile\": %d, \"split\": %d, \"wg_waves\": %d, \"order\": %d, "
                 "\"variant\": %d, \"flush\": %d, \"schedule\": %d, \"ms\": %.4f}\n",
                 key, c.tile, c.split, c.wg_waves, c.order, c.variant, c.flush, c.schedule, ms);
    std::fclose(f);
}

} // namespace mwg
