// CPU property check of the guard's allow decisions (compiled with g++ by
// test_guard_arith.py). For random bindings, row sizes and hostile indices it verifies, with
// exact 128-bit arithmetic written out here, that every access the kernels' helpers allow lies
// inside the binding, and that everything inside is allowed.
#include <cstdio>
#include <cstdlib>
#include <random>

#include "../paper_2606_06697_amd/csrc/guard_arith.h"

using namespace agile;
typedef __int128 i128;

static std::mt19937_64 rng(12345);
static uint64_t pick_u64() {
    switch (rng() % 6) {
        case 0: return rng() % 4096;
        case 1: return ~0ull - rng() % 4096;
        case 2: return (1ull << 63) + (rng() % 8192) - 4096;
        default: return rng();
    }
}

static int fails = 0;
#define CHECK(c, ...) do { if (!(c)) { if (fails++ < 10) { printf(__VA_ARGS__); printf("\n"); } } } while (0)

int main() {
    const uint32_t widths[2] = {4, 8};
    for (int it = 0; it < 400000; ++it) {
        uint64_t lo = pick_u64(), hi = pick_u64();
        if (lo > hi) { uint64_t t = lo; lo = hi; hi = t; }
        if (rng() % 5 == 0) hi = lo + rng() % 5000;           // small allocations
        if (hi < lo) hi = ~0ull;
        Bind b{lo, hi};
        if (rng() % 10 == 0) b = Bind{0, 0};
        const uint32_t W = widths[rng() % 2];
        const uint64_t D = 1 + rng() % 9;
        const uint64_t rb = (rng() % 4 == 0) ? W * (1 + rng() % 300) : W * D;
        uint64_t base;
        switch (rng() % 4) {
            case 0: base = b.lo + (b.hi > b.lo ? rng() % (b.hi - b.lo) : 0); break;
            case 1: base = b.lo; break;
            case 2: base = b.hi - 1 - rng() % 8; break;
            default: base = pick_u64();
        }
        RowGuard g = row_guard(b, base, rb);
        const bool bound = b.hi > b.lo && base >= b.lo && base < b.hi;
        CHECK(g.bound == bound, "bound mismatch");
        // candidate indices: around the row interval and extremes
        int64_t cands[12] = {0, 1, -1, g.rlo, g.rlo - 1, g.rhi, g.rhi + 1, INT64_MIN, INT64_MAX,
                             (int64_t)rng(), (int64_t)(rng() % 1000) - 500,
                             g.rlo + (int64_t)(rng() % 50)};
        if (g.rlo == INT64_MIN) cands[4] = INT64_MIN;
        if (g.rhi == INT64_MAX) cands[6] = INT64_MAX;
        const uint64_t Dr = rb / W;
        for (int64_t iv : cands) {
            bool all_ok = bound;
            for (uint64_t col : {(uint64_t)0, Dr / 2, Dr - 1}) {
                const i128 A = (i128)base + (i128)iv * (i128)rb + (i128)(col * W);
                const bool inside = bound && A >= (i128)b.lo && A + W <= (i128)b.hi;
                CHECK(elem_ok(g, iv, rb, col, W) == inside, "elem_ok wrong iv=%lld col=%llu",
                      (long long)iv, (unsigned long long)col);
                all_ok = all_ok && inside;
            }
            const bool full = g.rlo <= iv && iv <= g.rhi;
            CHECK(full == all_ok, "row interval wrong: iv=%lld rlo=%lld rhi=%lld bound=%d",
                  (long long)iv, (long long)g.rlo, (long long)g.rhi, (int)bound);
        }
        // prefix clip of a contiguous operand
        const uint64_t p = (rng() % 2) ? base : pick_u64();
        const uint64_t n = rng() % 100000;
        const uint64_t w = (rng() % 3 == 0) ? 1 : W;
        const uint64_t k = clip_prefix(b, p, n, w);
        CHECK(k <= n, "clip > n");
        for (uint64_t i : {(uint64_t)0, k > 0 ? k - 1 : 0, k}) {
            if (i >= n) continue;
            const i128 A = (i128)p + (i128)(i * w);
            const bool inside = b.hi > b.lo && p >= b.lo && p < b.hi && A >= (i128)b.lo &&
                                A + (i128)w <= (i128)b.hi;
            CHECK(inside == (i < k), "clip wrong i=%llu k=%llu", (unsigned long long)i,
                  (unsigned long long)k);
        }
    }
    // rows that the row kernels take on their fast path: the index element and the whole
    // contiguous-operand row are inside their bindings for every row below nfast, and row
    // nfast (when < n) fails one of the two
    for (int it = 0; it < 200000; ++it) {
        auto mkbind = [&](uint64_t& p) {
            uint64_t lo = pick_u64(), hi = pick_u64();
            if (lo > hi) { uint64_t t = lo; lo = hi; hi = t; }
            if (rng() % 3 == 0) hi = lo + rng() % 100000;
            if (hi < lo) hi = ~0ull;
            Bind b{lo, hi};
            if (rng() % 10 == 0) b = Bind{0, 0};
            p = (rng() % 4 != 0 && b.hi > b.lo) ? b.lo + rng() % (b.hi - b.lo) : pick_u64();
            return b;
        };
        uint64_t pi, pc, pr;
        const Bind bi = mkbind(pi), bc = mkbind(pc), br = mkbind(pr);
        const uint32_t W = widths[rng() % 2];
        const uint64_t rb = W * (1 + rng() % 64);
        const uint64_t n = rng() % 50000;
        const RowsGuard r = rows_guard(bi, bc, br, pi, pc, pr, n, rb, W);
        CHECK(r.nfast <= n, "nfast > n");
        auto row_ok = [&](uint64_t i) {
            const i128 Ai = (i128)pi + (i128)(8 * i);
            const bool iok = bi.hi > bi.lo && pi >= bi.lo && pi < bi.hi && Ai >= (i128)bi.lo &&
                             Ai + 8 <= (i128)bi.hi;
            const i128 Ac = (i128)pc + (i128)i * (i128)rb;
            const bool cok = bc.hi > bc.lo && pc >= bc.lo && pc < bc.hi && Ac >= (i128)bc.lo &&
                             Ac + (i128)rb <= (i128)bc.hi;
            return iok && cok;
        };
        for (uint64_t i : {(uint64_t)0, r.nfast > 0 ? r.nfast - 1 : 0, r.nfast / 2}) {
            if (i < r.nfast) CHECK(row_ok(i), "row %llu below nfast not allowed", (unsigned long long)i);
        }
        if (r.nfast < n) CHECK(!row_ok(r.nfast), "row nfast=%llu allowed", (unsigned long long)r.nfast);
        const RowsGuard o = rows_open(n, rb, W);
        CHECK(o.nfast == n && o.ki == n && o.kc == n * (rb / W) && o.g.rlo == INT64_MIN &&
              o.g.rhi == INT64_MAX, "rows_open");
    }
    if (fails) { printf("FAILED %d\n", fails); return 1; }
    printf("ok\n");
    return 0;
}
