// Address-space bookkeeping of one aperture (host code, also compiled by the CPU tests): the
// free parts of [lo, hi) as maximal ranges; a request takes the lowest-addressed free range
// that is long enough, from its start; a range given back merges with free neighbours.
#pragma once
#include <stdint.h>

#include <iterator>
#include <map>

namespace agile {

struct VaRanges {
    uint64_t lo = 0, hi = 0;
    std::map<uint64_t, uint64_t> free_;  // start -> end

    void reset(uint64_t l, uint64_t h) {
        lo = l;
        hi = h;
        free_.clear();
        if (h > l) free_[l] = h;
    }

    // Takes n > 0 bytes at the lowest start that fits; false when nothing fits.
    bool take(uint64_t n, uint64_t* out) {
        if (n == 0) return false;
        for (auto it = free_.begin(); it != free_.end(); ++it) {
            const uint64_t s = it->first, e = it->second;
            if (e - s < n) continue;
            free_.erase(it);
            if (s + n < e) free_[s + n] = e;
            *out = s;
            return true;
        }
        return false;
    }

    // Gives back [s, s + n), which an earlier take returned and nothing has given back.
    void give(uint64_t s, uint64_t n) {
        uint64_t e = s + n;
        auto nx = free_.lower_bound(s);
        if (nx != free_.end() && nx->first == e) {
            e = nx->second;
            nx = free_.erase(nx);
        }
        if (nx != free_.begin()) {
            auto pv = std::prev(nx);
            if (pv->second == s) {
                s = pv->first;
                free_.erase(pv);
            }
        }
        free_[s] = e;
    }

    // The free run that take(n) would split: [*s, *e); false when nothing fits.
    bool first_fit(uint64_t n, uint64_t* s, uint64_t* e) const {
        if (n == 0) return false;
        for (const auto& [fs, fe] : free_)
            if (fe - fs >= n) {
                *s = fs;
                *e = fe;
                return true;
            }
        return false;
    }

    // The free run that give(s, n) would form, merged with its free neighbours: [*ms, *me).
    void merged(uint64_t s, uint64_t n, uint64_t* ms, uint64_t* me) const {
        *ms = s;
        *me = s + n;
        auto nx = free_.lower_bound(s);
        if (nx != free_.end() && nx->first == s + n) *me = nx->second;
        if (nx != free_.begin()) {
            auto pv = std::prev(nx);
            if (pv->second == s) *ms = pv->first;
        }
    }

    bool whole() const { return free_.size() == 1 && free_.begin()->first == lo && free_.begin()->second == hi; }
};

}  // namespace agile
