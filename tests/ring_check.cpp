// CPU check of the serving loop's output ring (compiled with g++ by test_serving_host.py).
// Random alloc / free sequences against a brute-force byte map: live slices never overlap,
// stay inside the ring and are 256-byte aligned; an empty ring never refuses a slice that fits
// the ring; freeing everything reclaims the whole ring.
#include <cstdio>
#include <map>
#include <random>
#include <vector>

#include "../paper_2606_06697_amd/csrc/ring.h"

static int fails = 0;
#define CHECK(c, ...) do { if (!(c)) { if (fails++ < 10) { printf(__VA_ARGS__); printf("\n"); } } } while (0)

int main() {
    std::mt19937_64 rng(7);
    const uint64_t sizes[3] = {4096, 16384, 65536};
    for (int seed = 0; seed < 24; ++seed) {
        const uint64_t size = sizes[seed % 3];
        const uint64_t base = 0x7F0000000000ull;
        agile::Ring ring;
        ring.base = base;
        ring.size = size;
        std::map<uint64_t, std::pair<uint64_t, uint64_t>> live;  // start -> (addr, n)
        std::vector<int64_t> owner(size, -1);
        for (int step = 0; step < 4000; ++step) {
            if (!live.empty() && rng() % 100 < 45) {
                auto it = live.begin();
                std::advance(it, rng() % live.size());
                const uint64_t start = it->first, addr = it->second.first, n = it->second.second;
                for (uint64_t k = addr - base; k < addr - base + n; ++k) {
                    CHECK(owner[k] == (int64_t)start, "freed byte not owned by its slice");
                    owner[k] = -1;
                }
                live.erase(it);
                ring.free(start);
                continue;
            }
            const uint64_t wants[6] = {1, 100, 256, 1000, size / 8, size / 3};
            const uint64_t want = wants[rng() % 6];
            const uint64_t n = (want + 255) & ~255ull;
            uint64_t start, addr;
            if (!ring.alloc(want, &start, &addr)) {
                CHECK(!live.empty(), "an empty ring refused %llu of %llu bytes",
                      (unsigned long long)n, (unsigned long long)size);
                continue;
            }
            CHECK((addr - base) % 256 == 0 && addr >= base && addr + n <= base + size,
                  "slice outside the ring or unaligned");
            for (uint64_t k = addr - base; k < addr - base + n && k < size; ++k) {
                CHECK(owner[k] == -1, "overlapping slices (step %d)", step);
                owner[k] = (int64_t)start;
            }
            live[start] = {addr, n};
        }
        for (auto& l : live) ring.free(l.first);
        uint64_t s0, a0;
        CHECK(ring.live.empty() && ring.alloc(size, &s0, &a0) && a0 == base,
              "freeing everything did not reclaim the ring");
    }
    if (fails) {
        printf("%d failures\n", fails);
        return 1;
    }
    printf("ok\n");
    return 0;
}
