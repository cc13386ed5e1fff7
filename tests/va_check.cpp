// CPU check of agile::VaRanges against a granule map: random take/give sequences in granule
// units; every take must return the lowest start of a long-enough free run (found by scanning
// the map), stay inside the aperture and overlap nothing live, and first_fit must name the run
// it splits; merged must name the run each give forms; giving everything back must leave one
// free range covering the aperture.
#include <stdio.h>
#include <stdlib.h>

#include <random>
#include <vector>

#include "../paper_2606_06697_amd/csrc/va_ranges.h"

static int fail(const char* what, int step) {
    printf("FAIL %s at step %d\n", what, step);
    return 1;
}

int main() {
    std::mt19937_64 rng(7);
    for (int round = 0; round < 40; ++round) {
        const uint64_t G = 1ull << (12 + round % 10);            // granule
        const uint64_t lo = (1ull << 40) + G * (round * 37 % 101);
        const uint64_t ng = 64 + round * 13;                       // granules in the aperture
        agile::VaRanges va;
        va.reset(lo, lo + ng * G);
        std::vector<int> map(ng, 0);                               // 1 = taken
        std::vector<std::pair<uint64_t, uint64_t>> live;           // (start granule, count)
        for (int step = 0; step < 4000; ++step) {
            if (live.empty() || rng() % 3 != 0) {
                const uint64_t want = 1 + rng() % (rng() % 4 == 0 ? ng : 8);
                // lowest start of `want` free granules, by scan
                int64_t expect = -1;
                for (uint64_t g = 0; g + want <= ng && expect < 0; ++g) {
                    uint64_t k = 0;
                    while (k < want && !map[g + k]) ++k;
                    if (k == want) expect = (int64_t)g;
                }
                uint64_t fs = 0, fe = 0;
                const bool fit = va.first_fit(want * G, &fs, &fe);
                uint64_t addr = 0;
                const bool ok = va.take(want * G, &addr);
                if (fit != ok) return fail("first_fit agrees with take", step);
                if (ok && (fs != addr || fe < addr + want * G)) return fail("first_fit run", step);
                if (ok != (expect >= 0)) return fail("fit", step);
                if (!ok) continue;
                if (addr < lo || (addr - lo) % G) return fail("alignment", step);
                const uint64_t g0 = (addr - lo) / G;
                if ((int64_t)g0 != expect) return fail("lowest fit", step);
                if (g0 + want > ng) return fail("inside", step);
                for (uint64_t k = 0; k < want; ++k) {
                    if (map[g0 + k]) return fail("overlap", step);
                    map[g0 + k] = 1;
                }
                live.push_back({g0, want});
            } else {
                const size_t j = rng() % live.size();
                const auto [g0, cnt] = live[j];
                live[j] = live.back();
                live.pop_back();
                uint64_t ms = 0, me = 0;
                va.merged(lo + g0 * G, cnt * G, &ms, &me);
                va.give(lo + g0 * G, cnt * G);
                {
                    auto it = va.free_.find(ms);
                    if (it == va.free_.end() || it->second != me) return fail("merged run", step);
                }
                for (uint64_t k = 0; k < cnt; ++k) map[g0 + k] = 0;
            }
            // free ranges are maximal and match the map
            uint64_t prev_end = 0;
            bool first = true;
            for (const auto& [s, e] : va.free_) {
                if (s >= e || s < lo || e > lo + ng * G) return fail("free range bounds", step);
                if (!first && s <= prev_end) return fail("free ranges not maximal", step);
                for (uint64_t a = s; a < e; a += G)
                    if (map[(a - lo) / G]) return fail("free range covers a taken granule", step);
                prev_end = e;
                first = false;
            }
        }
        for (const auto& [g0, cnt] : live) va.give(lo + g0 * G, cnt * G);
        if (!va.whole()) return fail("not whole after giving everything back", -1);
    }
    printf("ok\n");
    return 0;
}
