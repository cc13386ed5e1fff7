"""DMA registration check on the GPU against the oracle: bit-exact verdicts and owners.

A module may register a user buffer for device DMA only when it is an exact live user
allocation (Section V-C); agile_validate_dma answers that for a batch of (addr, len) queries
with the validation kernel's search. Cases: the small-guard table with 10^6 DMA queries,
random tables with byte-granular bases (packed and general records) probed at every boundary
with lengths that reach every nearby boundary, the 65,536-range table with a ragged query
count, the two-level search, an empty table and removal (a freed allocation is not live).
"""
import random

import numpy as np
import pytest
import torch

from gpu_util import Twin, need_gpu
from synth import make_table
from synth.workloads import make_dma_queries
from oracle import U64_MAX, ALLOW, V_INEXACT

pytestmark = pytest.mark.gpu


def run_dma(tw, q_u64):
    n = q_u64.shape[0]
    q = torch.from_numpy(q_u64.view(np.int64).copy()).cuda()
    v = torch.full((n,), 255, dtype=torch.uint8, device="cuda")
    o = torch.full((n,), -7, dtype=torch.int32, device="cuda")
    tw.g.agile_validate_dma(tw.h, q, n, v, o)
    torch.cuda.synchronize()
    return v.cpu().numpy(), o.cpu().numpy()


def assert_same(tw, q_u64, what=""):
    v, o = run_dma(tw, q_u64)
    ev, eo = tw.ot.dma_verdict_many(q_u64[:, 0], q_u64[:, 1])
    bad = np.flatnonzero((v != ev) | (o != eo))
    assert bad.size == 0, (what, bad.size, [(hex(int(q_u64[k, 0])), int(q_u64[k, 1]), int(v[k]),
                                            int(o[k]), int(ev[k]), int(eo[k])) for k in bad[:5]])
    return ev


def test_small_guard_table_1e6_dma_queries():
    need_gpu()
    tb = make_table(64, 16, 0)
    tw = Twin(64)
    tw.insert_table(tb)
    q = make_dma_queries(tb, 1_000_000, 0).numpy().view(np.uint64)
    ev = assert_same(tw, q, "small table")
    counts = np.bincount(ev, minlength=6)
    assert counts[ALLOW] > 300_000 and counts[V_INEXACT] > 200_000
    tw.close()


def _boundary_dma_queries(ot, rng):
    ents = ot.entries()
    qs = []
    for k, (b, e, _, _) in enumerate(ents):
        near = ents[max(0, k - 2):k + 3]
        for a in (b - 1, b, b + 1, e - 1):
            if not 0 <= a <= U64_MAX:
                continue
            lens = {0, 1, 2, U64_MAX}
            for b2, e2, _, _ in near:
                for x in (b2, e2 - 1, e2, e2 + 1):
                    if x >= a:
                        lens.add(x - a)
            qs += [[a, ln] for ln in lens]
    for _ in range(200):
        qs.append([rng.getrandbits(64), rng.choice([0, 1, 5, U64_MAX])])
    return np.array(qs, dtype=np.uint64)


@pytest.mark.parametrize("seed", range(6))
def test_boundaries_random_tables(seed, monkeypatch):
    need_gpu()
    monkeypatch.setenv("AGILE_WIDE_RECORDS", "1" if seed % 2 else "0")
    rng = random.Random(300 + seed)
    tw = Twin(512)
    pos = rng.choice([0, 1 << 40, U64_MAX - (1 << 20)])
    for _ in range(rng.randrange(1, 300)):
        pos += rng.choice([0, 0, 1, 3, rng.randrange(0, 5000)])
        size = rng.choice([1, 2, 7, 64, rng.randrange(1, 9000)])
        if pos + size > U64_MAX:
            break
        tw.insert(pos, size, rng.choice([0, 0, 0, 1, 2]))
        pos += size
    assert_same(tw, _boundary_dma_queries(tw.ot, rng), f"seed {seed}")
    ids = [e[3] for e in tw.ot.entries()]
    for rid in ids[::3]:
        tw.remove(rid)
    assert_same(tw, _boundary_dma_queries(tw.ot, rng), f"seed {seed} after removal")
    tw.close()


@pytest.mark.parametrize("wide", ["0", "1"])
def test_large_table_ragged_dma_queries(wide, monkeypatch):
    need_gpu()
    monkeypatch.setenv("AGILE_WIDE_RECORDS", wide)
    tb = make_table(65536, 8192, 1)
    tw = Twin(65536)
    tw.insert_table(tb)
    q = make_dma_queries(tb, (1 << 21) + 77, 1).numpy().view(np.uint64)
    ev = assert_same(tw, q, "65536 ranges")
    assert np.bincount(ev, minlength=6)[[0, 1, 2, 3, 5]].min() > 0
    tw.close()


def test_two_level_search_dma(monkeypatch):
    need_gpu()
    monkeypatch.setenv("AGILE_LDS_BUDGET", "1024")
    tb = make_table(4096, 512, 11)
    tw = Twin(4096)
    tw.insert_table(tb)
    q = make_dma_queries(tb, 200_003, 11).numpy().view(np.uint64)
    assert_same(tw, q, "two-level search")
    tw.close()


def test_empty_table_and_removed_allocation():
    need_gpu()
    tw = Twin(8)
    q = np.array([[0, 0], [4096, 4096], [U64_MAX, 1]], dtype=np.uint64)
    v, o = run_dma(tw, q)
    assert (v == 3).all() and (o == -1).all()
    rid = tw.insert(4096, 4096, 0)
    assert_same(tw, q, "one entry")
    v, _ = run_dma(tw, q)
    assert int(v[1]) == ALLOW
    tw.remove(rid)
    v, o = run_dma(tw, q)
    assert int(v[1]) == 3 and int(o[1]) == -1
    tw.close()
