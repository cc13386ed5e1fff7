// Guard arithmetic that decides whether an element access is allowed (host- and
// device-compilable, so its bounds properties can be checked on the CPU).
#pragma once
#include <stdint.h>

#if defined(__HIPCC__)
#define AGILE_HD __host__ __device__
#else
#define AGILE_HD
#endif

namespace agile {

struct Bind {
    uint64_t lo, hi;  // [lo, hi) of the USER range containing the pointer; lo == hi == 0 if none
};

// Number of leading elements of width w at p (p, p+w, ...) that lie inside binding bd, capped
// at n: allowed accesses of a pointer argument form a prefix, since p >= lo when bound.
AGILE_HD inline uint64_t clip_prefix(Bind bd, uint64_t p, uint64_t n, uint64_t w) {
    if (bd.hi <= bd.lo || p < bd.lo || p >= bd.hi) return 0;
    uint64_t k = (bd.hi - p) / w;
    return k < n ? k : n;
}

// Row-addressed operand (base + idx*rb + col*W): rows wholly inside the binding form the
// index interval [rlo, rhi]; other rows are checked per element with exact arithmetic.
struct RowGuard {
    int64_t rlo, rhi;  // rows wholly inside the binding
    uint64_t dlo, dhi; // base - lo and hi - base of the binding (exact per-element check)
    bool bound;
};

AGILE_HD inline RowGuard row_guard(Bind b, uint64_t base, uint64_t rb) {
    RowGuard g;
    g.bound = b.hi > b.lo && base >= b.lo && base < b.hi;
    if (!g.bound) {
        g.rlo = 1;
        g.rhi = 0;
        g.dlo = 0;
        g.dhi = 0;
        return g;
    }
    g.dlo = base - b.lo;
    g.dhi = b.hi - base;
    const uint64_t q = g.dlo / rb;
    g.rlo = q > (uint64_t)INT64_MAX ? INT64_MIN : -(int64_t)q;
    if (g.dhi >= rb) {
        const uint64_t h = (g.dhi - rb) / rb;
        g.rhi = h > (uint64_t)INT64_MAX ? INT64_MAX : (int64_t)h;
    } else {
        g.rhi = -1;
    }
    return g;
}

// Exact check of element `col` of row `iv` (address base + iv*rb + col*W) against the binding.
AGILE_HD inline bool elem_ok(const RowGuard& g, int64_t iv, uint64_t rb, uint64_t col, uint32_t W) {
    if (!g.bound) return false;
    const __int128 off = (__int128)iv * (__int128)rb + (__int128)(col * W);
    return off >= -(__int128)g.dlo && off + (__int128)W <= (__int128)g.dhi;
}

// Guard of a row kernel (gather, scatter, scatter-add), fixed for a launch: the readable prefix
// of the index array, the allowed element prefix of the contiguous operand (out or src), the
// number of leading rows that pass both (index readable and contiguous row wholly allowed),
// and the row interval of the row-addressed operand (table or dst).
struct RowsGuard {
    uint64_t ki, kc, nfast;
    RowGuard g;
};

AGILE_HD inline RowsGuard rows_guard(Bind bi, Bind bc, Bind br, uint64_t idx, uint64_t cptr,
                                     uint64_t rptr, uint64_t n, uint64_t rb, uint32_t W) {
    RowsGuard r;
    const uint64_t D = rb / W;
    r.ki = clip_prefix(bi, idx, n, 8);
    r.kc = clip_prefix(bc, cptr, n * D, W);
    const uint64_t crows = r.kc / D;
    r.nfast = r.ki < crows ? r.ki : crows;
    r.g = row_guard(br, rptr, rb);
    return r;
}

// The same shape with every access allowed (the unguarded twins).
AGILE_HD inline RowsGuard rows_open(uint64_t n, uint64_t rb, uint32_t W) {
    RowsGuard r;
    r.ki = n;
    r.kc = n * (rb / W);
    r.nfast = n;
    r.g.rlo = INT64_MIN;
    r.g.rhi = INT64_MAX;
    r.g.dlo = 0;
    r.g.dhi = 0;
    r.g.bound = true;
    return r;
}

}  // namespace agile
