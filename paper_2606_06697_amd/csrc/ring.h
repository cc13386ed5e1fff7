// Output ring of one serving client (host code, also compiled by the CPU tests): bump
// allocation in 256-byte units, frees in any order, space reclaimed in allocation order; an
// empty ring starts over at its base.
#pragma once
#include <stdint.h>

#include <deque>

namespace agile {

struct Ring {
    uint64_t base = 0, size = 0, head = 0, tail = 0;
    struct Live {
        uint64_t start, n;
        bool freed;
    };
    std::deque<Live> live;

    // true with (start key, address) when `want` bytes fit now
    bool alloc(uint64_t want, uint64_t* start_out, uint64_t* addr_out) {
        const uint64_t n = (want + 255) & ~255ull;
        if (n == 0 || n > size) return false;
        uint64_t start = head;
        uint64_t off = start % size;
        if (off + n > size) {  // skip the wrap gap
            start += size - off;
            off = 0;
        }
        if (start + n - tail > size) return false;
        head = start + n;
        live.push_back(Live{start, n, false});
        *start_out = start;
        *addr_out = base + off;
        return true;
    }

    void free(uint64_t start) {
        for (auto& l : live)
            if (l.start == start) {
                l.freed = true;
                break;
            }
        while (!live.empty() && live.front().freed) {
            tail = live.front().start + live.front().n;
            live.pop_front();
        }
        if (live.empty()) head = tail = 0;
    }
};

}  // namespace agile
