"""Pins of the aperture classification oracle (CPU only).

* the Table I fixture (tests/golden/table1_apertures.txt), hand-derived from the layout;
* brute force: the three apertures entered as three ranges (I/O MMIO, module PROTECTED, user
  USER) and classified by the per-byte scan ``brute.verdict_brute``, on every address within
  two bytes of a boundary, with lengths that reach every boundary;
* the vectorized form equals the scalar one on random and boundary queries.
"""
import os

import numpy as np
import pytest

from oracle import aperture as AP
from oracle.brute import verdict_brute
from oracle.table import MMIO, PROTECTED, USER, U64_MAX

HERE = os.path.dirname(os.path.abspath(__file__))


def read_fixture():
    rows = []
    with open(os.path.join(HERE, "golden", "table1_apertures.txt")) as fh:
        lines = fh.readlines()
    for line in lines:
        line = line.split("#", 1)[0].split()
        if line:
            a, L, v, o = line
            rows.append((int(a, 0), int(L, 0), int(v), int(o)))
    return rows


def test_table1_apertures_fixture():
    rows = read_fixture()
    assert len(rows) >= 15
    for a, L, v, o in rows:
        assert AP.aperture_verdict(AP.TABLE1, a, L) == (v, o), hex(a)
    got_v, got_o = AP.aperture_verdict_many(AP.TABLE1, [r[0] for r in rows],
                                            [r[1] for r in rows])
    assert got_v.tolist() == [r[2] for r in rows]
    assert got_o.tolist() == [r[3] for r in rows]


def entries_of(bounds):
    b0, b1, b2, b3 = bounds
    return [(b0, b1, MMIO, AP.IO), (b1, b2, PROTECTED, AP.MODULE), (b2, b3, USER, AP.USER_AP)]


def boundary_queries(bounds):
    pts = set()
    for b in bounds:
        for d in range(-2, 3):
            if 0 <= b + d <= U64_MAX:
                pts.add(b + d)
    qs = []
    for a in sorted(pts):
        lens = {0, 1, 2, 3, 7}
        for b in bounds:
            if b > a:
                lens.update({b - a - 1, b - a, b - a + 1})
        qs.extend((a, L) for L in sorted(lens) if L >= 0)
    return qs


@pytest.mark.parametrize("seed", range(10))
def test_brute_force_on_the_apertures_as_ranges(seed):
    rng = np.random.default_rng(seed)
    if seed == 9:   # the user aperture ends at the top of the address space
        b3 = U64_MAX
        sizes = rng.integers(1, 40, 3)
        b2 = b3 - int(sizes[2])
        b1 = b2 - int(sizes[1])
        b0 = b1 - int(sizes[0])
    else:
        b0 = int(rng.integers(0, 50))
        s = rng.integers(1, 40, 3)
        b1, b2 = b0 + int(s[0]), b0 + int(s[0]) + int(s[1])
        b3 = b2 + int(s[2])
    bounds = (b0, b1, b2, b3)
    ents = entries_of(bounds)
    qs = boundary_queries(bounds)
    for a, L in qs:
        assert AP.aperture_verdict(bounds, a, L) == verdict_brute(ents, a, L), (bounds, a, L)
    v, o = AP.aperture_verdict_many(bounds, [q[0] for q in qs], [min(q[1], U64_MAX) for q in qs])
    assert v.tolist() == [verdict_brute(ents, a, L)[0] for a, L in qs]
    assert o.tolist() == [verdict_brute(ents, a, L)[1] for a, L in qs]


def test_vector_form_equals_scalar_on_random_queries():
    rng = np.random.default_rng(5)
    bounds = AP.TABLE1
    addr = rng.integers(0xE0000000000, 0x110000000000, 20000, dtype=np.uint64)
    length = rng.integers(0, 1 << 42, 20000, dtype=np.uint64)
    length[::7] = 0
    v, o = AP.aperture_verdict_many(bounds, addr, length)
    for i in range(0, 20000, 13):
        assert (int(v[i]), int(o[i])) == AP.aperture_verdict(bounds, int(addr[i]), int(length[i]))


def test_bounds_are_checked():
    for bad in ((5, 5, 6, 7), (0, 2, 1, 3), (0, 1, 2, 1 << 64)):
        with pytest.raises(ValueError):
            AP.aperture_verdict(bad, 0, 1)
