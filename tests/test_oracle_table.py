"""Pins for the oracle's allocation table and classification rule (CPU only).

The oracle is checked against things other than itself: a brute-force per-byte scan,
hand-derived verdicts on the paper's Table I layout, and boundary invariants.
"""
import os
import random

import numpy as np
import pytest

from oracle import (RangeTable, OverlapError, ALLOW, V_PROTECTED, V_STRADDLE, V_UNMAPPED,
                    V_INEXACT, USER, PROTECTED, MMIO, U64_MAX)
from oracle.brute import verdict_brute, dma_verdict_brute

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def load_fixture(name):
    steps = []
    with open(os.path.join(GOLDEN, name)) as f:
        for line in f:
            line = line.split("#")[0].strip()
            if not line:
                continue
            tok = line.split()
            steps.append((tok[0], [int(x, 0) for x in tok[1:]]))
    return steps


def test_table1_arithmetic():
    # Table I sizes: 64 GiB, 448 GiB and 1 TiB, contiguous apertures
    assert 0xF1000000000 - 0xF0000000000 == 64 << 30 == 1 << 36
    assert 0xF8000000000 - 0xF1000000000 == 448 << 30 == 7 << 36
    assert 0x108000000000 - 0xF8000000000 == 1 << 40
    assert 0x108000000000 < 1 << 45


def test_table1_fixture():
    t = RangeTable()
    n_q = 0
    for op, a in load_fixture("table1_layout.txt"):
        if op == "insert":
            t.insert(a[0], a[1], a[2])
        elif op == "remove":
            t.remove(a[0])
        else:
            got = t.verdict(a[0], a[1])
            assert got == (a[2], a[3]), (hex(a[0]), a[1], got)
            assert verdict_brute(t.entries(), a[0], a[1]) == got
            v, o = t.verdict_many(np.array([a[0]], np.uint64), np.array([a[1]], np.uint64))
            assert (int(v[0]), int(o[0])) == got
            n_q += 1
    assert n_q >= 20


def _random_table(rng, n, span=1 << 12, top=False):
    t = RangeTable()
    pos = rng.randrange(0, 64) if not top else U64_MAX - span * 4
    for _ in range(n):
        pos += rng.choice([0, 0, 1, 3, rng.randrange(0, 64)])
        size = rng.choice([1, 2, 3, 7, 16, rng.randrange(1, 200)])
        if pos + size > U64_MAX:
            break
        kind = rng.choice([USER, USER, USER, PROTECTED, MMIO])
        t.insert(pos, size, kind)
        pos += size
    return t


@pytest.mark.parametrize("seed", range(12))
def test_brute_force_exhaustive_boundaries(seed):
    rng = random.Random(seed)
    t = _random_table(rng, rng.randrange(1, 16), top=(seed % 4 == 3))
    ents = t.entries()
    addrs = set()
    for b, e, _, _ in ents:
        for x in (b - 2, b - 1, b, b + 1, e - 2, e - 1, e, e + 1):
            if 0 <= x <= U64_MAX:
                addrs.add(x)
    addrs |= {0, U64_MAX}
    lens = [0, 1, 2, 3, 5, 17, 255, 1 << 20, U64_MAX]
    A = []
    L = []
    for a in sorted(addrs):
        for ln in lens:
            want = verdict_brute(ents, a, ln)
            assert t.verdict(a, ln) == want, (a, ln)
            A.append(a)
            L.append(ln)
    v, o = t.verdict_many(np.array(A, np.uint64), np.array(L, np.uint64))
    for k in range(len(A)):
        assert (int(v[k]), int(o[k])) == t.verdict(A[k], L[k])


def test_boundary_invariants():
    t = RangeTable()
    u = t.insert(1000, 100, USER)
    p = t.insert(1100, 50, PROTECTED)      # adjacent to the user range
    m = t.insert(2000, 10, MMIO)
    assert t.verdict(999, 1) == (V_UNMAPPED, -1)           # base - 1
    assert t.verdict(1000, 1) == (ALLOW, u)                # base
    assert t.verdict(1099, 1) == (ALLOW, u)                # base + size - 1
    assert t.verdict(1099, 2) == (V_STRADDLE, u)           # crosses into the adjacent range
    assert t.verdict(1100, 1) == (V_PROTECTED, p)          # base + size = next entry
    assert t.verdict(1150, 1) == (V_UNMAPPED, -1)          # hole
    assert t.verdict(1000, 100) == (ALLOW, u)
    assert t.verdict(1000, 101) == (V_STRADDLE, u)
    assert t.verdict(1000, 0) == (ALLOW, u)                # zero length counts as one byte
    assert t.verdict(1100, 0) == (V_PROTECTED, p)
    assert t.verdict(2005, 1) == (V_PROTECTED, m)          # MMIO classifies as protected
    assert t.verdict(1050, U64_MAX) == (V_STRADDLE, u)     # addr + len overflows
    # protected and MMIO bytes are never ALLOW, whatever the length
    for a in range(1100, 1150):
        for ln in (0, 1, 8, 1 << 40):
            assert t.verdict(a, ln)[0] == V_PROTECTED
    t.remove(u)
    assert t.verdict(1000, 1) == (V_UNMAPPED, -1)          # freed range is a hole
    assert t.verdict(1099, 2) == (V_UNMAPPED, -1)
    with pytest.raises(KeyError):
        t.remove(u)
    nu = t.insert(1000, 100, USER)
    assert nu == 3                                          # ids are never reused
    assert t.verdict(1000, 1) == (ALLOW, nu)


def test_insert_rules():
    t = RangeTable()
    t.insert(100, 10, USER)
    with pytest.raises(OverlapError):
        t.insert(105, 2, USER)
    with pytest.raises(OverlapError):
        t.insert(95, 6, USER)
    with pytest.raises(OverlapError):
        t.insert(90, 30, PROTECTED)
    t.insert(110, 5, USER)            # adjacency is legal
    t.insert(90, 10, USER)
    with pytest.raises(ValueError):
        t.insert(200, 0, USER)
    with pytest.raises(ValueError):
        t.insert(U64_MAX - 4, 5, USER)   # end would be 2**64
    t.insert(U64_MAX - 5, 5, USER)       # ends at 2**64 - 1
    with pytest.raises(ValueError):
        t.insert(300, 1, 7)
    assert t.verdict(U64_MAX - 1, 1)[0] == ALLOW
    assert t.verdict(U64_MAX, 1) == (V_UNMAPPED, -1)


def test_binding():
    t = RangeTable()
    u = t.insert(4096, 4096, USER)
    t.insert(8192, 4096, PROTECTED)
    assert t.binding(4096) == (4096, 8192)
    assert t.binding(8191) == (4096, 8192)
    assert t.binding(8192) == (0, 0)
    assert t.binding(100) == (0, 0)
    assert u == 0


def test_generated_table_matches_brute_sample():
    from synth import make_table, make_queries
    tb = make_table(64, 16, 0)
    t = RangeTable()
    for b, s, k in zip(tb.base.tolist(), tb.size.tolist(), tb.kind.tolist()):
        t.insert(b, s, k)
    q = make_queries(tb, 4000, 0).numpy().astype(np.uint64)
    v, o = t.verdict_many(q[:, 0], q[:, 1])
    ents = t.entries()
    for k in range(0, 4000, 7):
        assert (int(v[k]), int(o[k])) == verdict_brute(ents, int(q[k, 0]), int(q[k, 1]))
    # the query mix hits every verdict class
    counts = np.bincount(v, minlength=4)
    assert counts[ALLOW] > 2000 and counts[V_PROTECTED] > 500
    assert counts[V_STRADDLE] > 100 and counts[V_UNMAPPED] > 300


# --- DMA registration: only an exact live user allocation (Section V-C) ---------------
@pytest.mark.parametrize("seed", range(8))
def test_dma_verdict_brute_force(seed):
    """Against the definition (some USER entry equals [addr, addr+len) exactly), on every
    boundary address and every length that reaches a boundary."""
    rng = random.Random(100 + seed)
    t = _random_table(rng, rng.randrange(1, 12), top=(seed % 4 == 3))
    ents = t.entries()
    A, L = [], []
    for b, e, _, _ in ents:
        for a in (b - 1, b, b + 1, e - 1):
            if not 0 <= a <= U64_MAX:
                continue
            lens = {0, 1, 2, U64_MAX}
            for b2, e2, _, _ in ents:
                for x in (e2 - 1, e2, e2 + 1):
                    if x >= a:
                        lens.add(x - a)
            for ln in sorted(lens):
                assert t.dma_verdict(a, ln) == dma_verdict_brute(ents, a, ln), (a, ln)
                A.append(a)
                L.append(ln)
    v, o = t.dma_verdict_many(np.array(A, np.uint64), np.array(L, np.uint64))
    for k in range(len(A)):
        assert (int(v[k]), int(o[k])) == t.dma_verdict(A[k], L[k])


def test_dma_verdict_invariants():
    t = RangeTable()
    u = t.insert(1000, 100, USER)
    p = t.insert(1100, 50, PROTECTED)
    v = t.insert(1150, 1, USER)
    assert t.dma_verdict(1000, 100) == (ALLOW, u)          # the whole allocation
    assert t.dma_verdict(1000, 99) == (V_INEXACT, u)       # a prefix
    assert t.dma_verdict(1001, 99) == (V_INEXACT, u)       # a suffix
    assert t.dma_verdict(1010, 10) == (V_INEXACT, u)       # an interior piece
    assert t.dma_verdict(1000, 0) == (V_INEXACT, u)        # zero length is never exact
    assert t.dma_verdict(1000, 101) == (V_STRADDLE, u)     # one byte too long
    assert t.dma_verdict(1100, 50) == (V_PROTECTED, p)     # exact, but protected
    assert t.dma_verdict(1150, 1) == (ALLOW, v)            # one-byte allocation
    assert t.dma_verdict(1150, 0) == (V_INEXACT, v)
    assert t.dma_verdict(999, 101) == (V_UNMAPPED, -1)
    t.remove(u)
    assert t.dma_verdict(1000, 100) == (V_UNMAPPED, -1)    # freed: no longer live
