"""Guarded scatter-add on the sorted path (calls of at least 32,768 rows) against the oracle.

One device arena holds the destination table (USER), a protected canary right after it, an
unregistered hole, another USER allocation, the index buffer and the source rows. Source and
destination values are small integers, so every sum is exact in any order and the arena must
equal the oracle's memory byte for byte. Cases: hot and hostile indices (protected, hole,
other allocation, negative, huge), an index buffer and a source buffer that run out before n, an
interior destination pointer (negative indices allowed), a destination with no binding (no row
takes the sorted path), destinations of exactly 2^8 and 2^16 rows (the last row's key has every
sorted bit set, as the hostile rows' key has), and the unguarded twin on valid indices.
"""
import random

import numpy as np
import pytest

from gpu_util import Arena, Twin, log_matches, need_gpu
from oracle import guarded as G

pytestmark = pytest.mark.gpu

DST_ROWS = 3000
NMAX = 70001
# (4, 300) and (8, 70): rows wider than one column block of the reduce (256 floats in 16-byte
# chunks, 64 doubles one per lane), so each tile is walked once per block
CASES = [(4, 1), (4, 3), (4, 64), (4, 128), (8, 2), (8, 32), (4, 300), (8, 70)]


def layout(w, D, rows=DST_ROWS):
    rb = w * D
    off = {}
    o = 0
    for name, size in (("dst", rows * rb), ("prot", 4096), ("hole", 4096), ("other", 8192),
                       ("idx", NMAX * 8), ("src", NMAX * rb)):
        o = (o + 255) // 256 * 256
        off[name] = (o, o + size)
        o += size
    return off, (o + 4095) // 4096 * 4096


def setup(w, D, seed, rows=DST_ROWS):
    need_gpu()
    off, size = layout(w, D, rows)
    ar = Arena(size, seed)
    tw = Twin(16)
    kinds = {"dst": 0, "prot": 1, "other": 0, "idx": 0, "src": 0}
    for k, kind in kinds.items():
        lo, hi = off[k]
        tw.insert(ar.addr(lo), hi - lo, kind)
    dt = np.float32 if w == 4 else np.float64
    rng = np.random.default_rng(seed)
    for k in ("dst", "src", "other"):
        lo, hi = off[k]
        ar.write(lo, rng.integers(-50, 51, (hi - lo) // w).astype(dt))
    return ar, tw, off


def indices(rng, n, rows, extra, neg_ok=0):
    """Hot rows (Zipf-like), uniform rows and hostile values, shuffled."""
    hot = [rng.randrange(rows) for _ in range(5)]
    bad = [rows, rows + 1, -1 - neg_ok, 3 * rows, -(1 << 62), (1 << 62), -(1 << 63),
           (1 << 63) - 1, (1 << 40) + 3] + list(extra)
    vals = []
    for _ in range(n):
        u = rng.random()
        if u < 0.5:
            vals.append(hot[min(int(rng.expovariate(1.0)), 4)])
        elif u < 0.9:
            vals.append(rng.randrange(-neg_ok, rows))
        else:
            vals.append(rng.choice(bad))
    return np.array(vals, dtype=np.int64)


@pytest.mark.parametrize("w,D", CASES)
def test_sorted_scatter_add_against_oracle(w, D):
    ar, tw, off = setup(w, D, 40 + D + w)
    rb = w * D
    dtype = 0 if w == 4 else 1
    ol = G.FaultLog()
    rng = random.Random(1000 + D * 10 + w)
    base = ar.addr(off["dst"][0])
    hostile_rows = [(ar.addr(off["prot"][0]) - base) // rb + 1,
                    (ar.addr(off["hole"][0]) - base) // rb + 1,
                    (ar.addr(off["other"][0]) - base) // rb + 2]
    trials = [
        dict(dst=base, n=40000, idx_end=False, src_end=False, neg=0),
        dict(dst=base, n=NMAX, idx_end=True, src_end=True, neg=0),
        dict(dst=base + 100 * rb + w, n=32768, idx_end=False, src_end=False, neg=100),
        dict(dst=ar.addr(off["hole"][0]), n=33000, idx_end=False, src_end=False, neg=0),
    ]
    for t, tr in enumerate(trials):
        n = tr["n"]
        rows = DST_ROWS - 101 if tr["neg"] else DST_ROWS
        idx = indices(rng, n, rows, hostile_rows, tr["neg"])
        ilo, ihi = off["idx"]
        idx_ptr = ar.addr(ihi - 8 * (n - 700)) if tr["idx_end"] else ar.addr(ilo)
        ar.write(idx_ptr - ar.base, idx[:(ihi - (idx_ptr - ar.base)) // 8])
        slo, shi = off["src"]
        src = ar.addr(shi - rb * (n - 1234) - w) if tr["src_end"] else ar.addr(slo)
        tw.g.agile_guarded_scatter(tw.h, tr["dst"], rb, idx_ptr, src, n, dtype, 1)
        G.scatter_vec(tw.ot, ar.mem, ol, tw.next_seq(), tr["dst"], rb, idx_ptr, src, n, w, True)
        ar.check(f"scatter-add w={w} D={D} trial {t} n={n}")
        log_matches(tw, ol, f"scatter-add w={w} D={D} trial {t}")
    tw.close()


@pytest.mark.parametrize("w,D,rows,hostile", [(4, 4, 256, True), (4, 1, 65536, True),
                                              (8, 1, 256, True), (4, 4, 256, False),
                                              (4, 1, 65536, False)])
def test_sorted_scatter_add_last_row_of_a_power_of_two_table(w, D, rows, hostile):
    """Rows that fail the guard's fast test sort after every allowed row, also when the table has
    exactly 2^8 or 2^16 rows and its last row's key is all ones in the sorted bits: every update
    of the last row lands, hostile rows are dropped and logged, as in the oracle. Without hostile
    rows the sort's last pass sees one digit only and is skipped, and the reduce reads the
    previous pass's buffer."""
    ar, tw, off = setup(w, D, 300 + rows + w, rows=rows)
    rb = w * D
    dtype = 0 if w == 4 else 1
    rng = np.random.default_rng(rows + w)
    n = 40000
    u = rng.random(n)
    idx = rng.integers(0, rows, n)
    idx[u < 0.3] = rows - 1
    if hostile:
        bad = np.array([rows, rows + 5, -1, 1 << 40], dtype=np.int64)
        idx[u > 0.9] = bad[rng.integers(0, bad.size, int((u > 0.9).sum()))]
    ar.write(off["idx"][0], idx.astype(np.int64))
    base = ar.addr(off["dst"][0])
    ol = G.FaultLog()
    tw.g.agile_guarded_scatter(tw.h, base, rb, ar.addr(off["idx"][0]), ar.addr(off["src"][0]), n,
                               dtype, 1)
    G.scatter_vec(tw.ot, ar.mem, ol, tw.next_seq(), base, rb, ar.addr(off["idx"][0]),
                  ar.addr(off["src"][0]), n, w, True)
    ar.check(f"scatter-add into {rows} rows")
    log_matches(tw, ol, f"scatter-add into {rows} rows")
    tw.close()


@pytest.mark.parametrize("w,D", [(4, 64), (4, 3), (8, 2), (4, 300)])
def test_scatter_add_into_zeros(w, D):
    """accumulate == 2 (the destination's rows are +0.0 before the call, as for a fresh
    gradient): on the sorted path the rows are written without being read, and the arena and
    the log equal the oracle's scatter-add into the same zeroed destination byte for byte, with
    hot rows, hostile indices and an interior destination pointer (negative indices)."""
    ar, tw, off = setup(w, D, 500 + D + w)
    rb = w * D
    dtype = 0 if w == 4 else 1
    dt = np.float32 if w == 4 else np.float64
    ol = G.FaultLog()
    rng = random.Random(600 + D + w)
    base = ar.addr(off["dst"][0])
    hostile_rows = [(ar.addr(off["prot"][0]) - base) // rb + 1,
                    (ar.addr(off["other"][0]) - base) // rb + 2]
    for t, (dst, n, neg) in enumerate(((base, 40000, 0), (base + 100 * rb, 50001, 100))):
        ar.write(off["dst"][0], np.zeros(DST_ROWS * D, dtype=dt))
        rows = DST_ROWS - 101 if neg else DST_ROWS
        idx = indices(rng, n, rows, hostile_rows, neg)
        ar.write(off["idx"][0], idx)
        tw.g.agile_guarded_scatter(tw.h, dst, rb, ar.addr(off["idx"][0]), ar.addr(off["src"][0]),
                                   n, dtype, tw.g.SCATTER_ADD_INTO_ZEROS)
        G.scatter_vec(tw.ot, ar.mem, ol, tw.next_seq(), dst, rb, ar.addr(off["idx"][0]),
                      ar.addr(off["src"][0]), n, w, True)
        ar.check(f"scatter-add into zeros w={w} D={D} trial {t}")
        log_matches(tw, ol, f"scatter-add into zeros w={w} D={D} trial {t}")
    tw.close()


@pytest.mark.parametrize("w,D", [(4, 64), (8, 2)])
def test_unguarded_sorted_scatter_add_matches_guarded(w, D):
    ar, tw, off = setup(w, D, 77 + D)
    rb = w * D
    dtype = 0 if w == 4 else 1
    rng = random.Random(5 + D)
    n = 50001
    idx = indices(rng, n, DST_ROWS, [], 0)
    idx[(idx < 0) | (idx >= DST_ROWS)] = 7                  # valid rows only
    ar.write(off["idx"][0], idx)
    base = ar.addr(off["dst"][0])
    before = ar.dev.clone()
    tw.g.agile_guarded_scatter(tw.h, base, rb, ar.addr(off["idx"][0]), ar.addr(off["src"][0]), n,
                               dtype, 1)
    guarded = ar.dev.clone()
    ar.dev.copy_(before)
    tw.g.agile_unguarded_scatter(base, rb, ar.addr(off["idx"][0]), ar.addr(off["src"][0]), n,
                                 dtype, 1)
    assert bool((ar.dev == guarded).all())
    G.scatter_vec(tw.ot, ar.mem, G.FaultLog(), 0, base, rb, ar.addr(off["idx"][0]),
                  ar.addr(off["src"][0]), n, w, True)
    ar.check("unguarded sorted scatter-add")
    rc, f = tw.rt.fault_log(clear=True)
    assert f["count"] == 0
    tw.close()


def test_sorted_scatter_add_suppress_only_leaves_log_empty():
    """The SUPPRESS_ONLY policy on the sorted path: the same data as the oracle, no log entry,
    and the call still takes a sequence number (a later logged call records the next one)."""
    w, D = 4, 64
    ar, tw, off = setup(w, D, 91)
    rb = w * D
    rng = random.Random(91)
    base = ar.addr(off["dst"][0])
    n = 40000
    idx = indices(rng, n, DST_ROWS, [(ar.addr(off["prot"][0]) - base) // rb + 1])
    ar.write(off["idx"][0], idx)
    ol = G.FaultLog()
    tw.g.agile_guarded_scatter(tw.h, base, rb, ar.addr(off["idx"][0]), ar.addr(off["src"][0]), n,
                               0, 1, G.SUPPRESS_ONLY)
    G.scatter_vec(tw.ot, ar.mem, ol, tw.next_seq(), base, rb, ar.addr(off["idx"][0]),
                  ar.addr(off["src"][0]), n, w, True, G.SUPPRESS_ONLY)
    ar.check("sorted scatter-add, suppress only")
    log_matches(tw, ol, "sorted scatter-add, suppress only")
    tw.g.agile_guarded_scatter(tw.h, base, rb, ar.addr(off["idx"][0]), ar.addr(off["src"][0]), n,
                               0, 1)
    G.scatter_vec(tw.ot, ar.mem, ol, tw.next_seq(), base, rb, ar.addr(off["idx"][0]),
                  ar.addr(off["src"][0]), n, w, True)
    ar.check("sorted scatter-add, logged after suppress only")
    log_matches(tw, ol, "sorted scatter-add, logged after suppress only")
    tw.close()
