"""Batched pointer validation on the GPU against the oracle: bit-exact verdicts and owners."""
import os
import random

import numpy as np
import pytest
import torch

from gpu_util import Twin, need_gpu
from synth import make_table, make_queries
from oracle import U64_MAX

pytestmark = pytest.mark.gpu
GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def run_validate(tw, q_u64):
    """q_u64: numpy uint64 [n, 2] -> device verdicts/owners as numpy."""
    n = q_u64.shape[0]
    q = torch.from_numpy(q_u64.view(np.int64).copy()).cuda()
    v = torch.full((n,), 255, dtype=torch.uint8, device="cuda")
    o = torch.full((n,), -7, dtype=torch.int32, device="cuda")
    tw.g.agile_validate_ptrs(tw.h, q, n, v, o)
    torch.cuda.synchronize()
    return v.cpu().numpy(), o.cpu().numpy()


def assert_same(tw, q_u64, what=""):
    v, o = run_validate(tw, q_u64)
    ev, eo = tw.ot.verdict_many(q_u64[:, 0], q_u64[:, 1])
    bad = np.flatnonzero((v != ev) | (o != eo))
    assert bad.size == 0, (what, bad.size, [(hex(int(q_u64[k, 0])), int(q_u64[k, 1]), int(v[k]),
                                            int(o[k]), int(ev[k]), int(eo[k])) for k in bad[:5]])
    return ev


def test_table1_fixture():
    need_gpu()
    tw = Twin(64)
    qs, exp = [], []
    for line in open(os.path.join(GOLDEN, "table1_layout.txt")):
        tok = line.split("#")[0].split()
        if not tok:
            continue
        a = [int(x, 0) for x in tok[1:]]
        if tok[0] == "insert":
            tw.insert(a[0], a[1], a[2])
        elif tok[0] == "remove":
            q = np.array(qs, dtype=np.uint64)
            v, o = run_validate(tw, q)
            assert [(int(x), int(y)) for x, y in zip(v, o)] == exp
            qs, exp = [], []
            tw.remove(a[0])
        else:
            qs.append([a[0], a[1]])
            exp.append((a[2], a[3]))
    v, o = run_validate(tw, np.array(qs, dtype=np.uint64))
    assert [(int(x), int(y)) for x, y in zip(v, o)] == exp
    tw.close()


def test_small_guard_config_1e6_queries():
    """64-range table (48 USER log-uniform 256 B-1 MiB, 16 protected 4-64 KiB), 10^6 queries."""
    need_gpu()
    tb = make_table(64, 16, 0)
    tw = Twin(64)
    tw.insert_table(tb)
    q = make_queries(tb, 1_000_000, 0).numpy().view(np.uint64)
    ev = assert_same(tw, q, "c0")
    counts = np.bincount(ev, minlength=4)
    assert counts.min() > 0
    tw.close()


def _boundary_queries(ot, rng):
    qs = []
    ents = ot.entries()
    for b, e, _, _ in ents:
        for a in (b - 2, b - 1, b, b + 1, e - 2, e - 1, e, e + 1):
            if 0 <= a <= U64_MAX:
                for ln in (0, 1, 2, 3, 7, 4096, 1 << 40, U64_MAX):
                    qs.append([a, ln])
    for _ in range(200):
        qs.append([rng.getrandbits(64), rng.choice([0, 1, 5, U64_MAX])])
    qs += [[0, 0], [U64_MAX, 1], [U64_MAX, U64_MAX]]
    return np.array(qs, dtype=np.uint64)


@pytest.mark.parametrize("seed", range(8))
def test_exhaustive_boundaries_random_tables(seed, monkeypatch):
    """Byte-granular bases (uncompressed splitters), adjacency, kinds, top of address space."""
    need_gpu()
    monkeypatch.setenv("AGILE_WIDE_RECORDS", "1" if seed % 2 else "0")
    rng = random.Random(seed)
    tw = Twin(512)
    pos = rng.choice([0, 1 << 40, U64_MAX - (1 << 20)])
    for _ in range(rng.randrange(1, 300)):
        pos += rng.choice([0, 0, 1, 3, rng.randrange(0, 5000)])
        size = rng.choice([1, 2, 7, 64, rng.randrange(1, 9000)])
        if pos + size > U64_MAX:
            break
        tw.insert(pos, size, rng.choice([0, 0, 0, 1, 2]))
        pos += size
    assert_same(tw, _boundary_queries(tw.ot, rng), f"seed {seed}")
    # remove a third of the ranges: freed ranges become holes (lazy re-upload)
    ids = [e[3] for e in tw.ot.entries()]
    for rid in ids[::3]:
        tw.remove(rid)
    assert_same(tw, _boundary_queries(tw.ot, rng), f"seed {seed} after removal")
    tw.close()


def test_empty_table_and_zero_queries():
    need_gpu()
    tw = Twin(8)
    q = np.array([[0, 0], [12345, 1], [U64_MAX, U64_MAX]], dtype=np.uint64)
    v, o = run_validate(tw, q)
    assert (v == 3).all() and (o == -1).all()
    tw.g.agile_validate_ptrs(tw.h, 0, 0, 0, 0)   # n == 0 is a no-op
    tw.insert(100, 10, 0)
    assert_same(tw, q, "one entry")
    tw.close()


@pytest.mark.parametrize("budget", ["1024", "4096"])
def test_two_level_search_small_lds_budget(budget, monkeypatch):
    """Tables larger than the LDS budget search their last levels in global memory."""
    need_gpu()
    monkeypatch.setenv("AGILE_LDS_BUDGET", budget)
    tb = make_table(4096, 512, 11)
    tw = Twin(4096)
    tw.insert_table(tb)
    q = make_queries(tb, 300_001, 11).numpy().view(np.uint64)
    assert_same(tw, q, f"budget {budget}")
    tw.close()


@pytest.mark.parametrize("lift", ["2", "4", "6", "8"])
@pytest.mark.parametrize("n_ranges", [64, 4096])
def test_every_unrolled_search_depth(n_ranges, lift, monkeypatch):
    """The packed-record search is unrolled for 2, 4, 6 and 8 lifting levels and a table picks
    the depth its radix runs need; AGILE_MIN_LIFT raises the depth (deeper is still exact: the
    staged splitters are followed by sentinels), so each variant runs against the oracle."""
    need_gpu()
    monkeypatch.setenv("AGILE_MIN_LIFT", lift)
    tb = make_table(n_ranges, n_ranges // 8, 20 + int(lift))
    tw = Twin(n_ranges)
    tw.insert_table(tb)
    q = make_queries(tb, 200_003, 20 + int(lift)).numpy().view(np.uint64)
    assert_same(tw, q, f"{n_ranges} ranges, lift {lift}")
    tw.close()


@pytest.mark.parametrize("wide", ["0", "1"])
def test_large_table_ragged_queries(wide, monkeypatch):
    """65,536 ranges (8,192 protected) and a query count that is not a multiple of any tile,
    with the packed 16-byte bucket records and with the general 32-byte ones."""
    need_gpu()
    monkeypatch.setenv("AGILE_WIDE_RECORDS", wide)
    tb = make_table(65536, 8192, 1)
    tw = Twin(65536)
    tw.insert_table(tb)
    q = make_queries(tb, (1 << 22) + 77, 1).numpy().view(np.uint64)
    ev = assert_same(tw, q, "65536 ranges")
    assert np.bincount(ev, minlength=4).min() > 0
    tw.close()


def test_insert_remove_interleaved_with_validation():
    need_gpu()
    tw = Twin(256)
    rng = random.Random(5)
    live = []
    for step in range(40):
        if live and rng.random() < 0.3:
            tw.remove(live.pop(rng.randrange(len(live))))
        else:
            base = rng.randrange(0, 1 << 20) * 4096
            try:
                live.append(tw.insert(base, rng.randrange(1, 1 << 16), rng.choice([0, 1, 2])))
            except tw.g.AgileError as e:
                assert e.code == tw.g.AGILE_EOVERLAP      # both tables rejected it
        q = _boundary_queries(tw.ot, rng)
        assert_same(tw, q, f"step {step}")
    tw.close()
