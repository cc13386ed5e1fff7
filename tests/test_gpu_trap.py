"""The trap policy on the device against the oracle: a violation retires the handle.

Reading of the paper's trap policy (Section V-E) with the retirement of a worker whose context
can no longer be trusted (Section IV-D): a TRAP call runs as under suppress-and-log, waits for
its stream, and if it denied an access the handle is retired. One arena holds a USER table A,
a protected canary P, a USER output C, an index buffer I and a USER source S; values are small
integers, so sums are exact in any order and the arena must equal the oracle's memory byte for
byte. Cases: a clean TRAP call, a violating TRAP gather, a violating TRAP scatter-add on the
sorted path, every later call of the retired handle (refused, nothing changes), revocation and
the log still readable, and violations under the other policies (no retirement).
"""
import random

import numpy as np
import pytest
import torch

from gpu_util import Arena, Twin, log_matches, need_gpu
from oracle import guarded as G

pytestmark = pytest.mark.gpu

ROWS, D = 4096, 4
RB = 4 * D
NIDX = 40000


def layout():
    off, o = {}, 0
    for name, size in (("A", ROWS * RB), ("P", 4096), ("C", ROWS * RB), ("I", NIDX * 8),
                       ("S", NIDX * RB)):
        o = (o + 255) // 256 * 256
        off[name] = (o, o + size)
        o += size
    return off, (o + 4095) // 4096 * 4096


def setup(seed):
    need_gpu()
    off, size = layout()
    ar = Arena(size, seed)
    tw = Twin(16)
    ids = {}
    for k in ("A", "P", "C", "I", "S"):
        lo, hi = off[k]
        ids[k] = tw.insert(ar.addr(lo), hi - lo, 1 if k == "P" else 0)
    rng = np.random.default_rng(seed)
    for k in ("A", "C", "S"):
        lo, hi = off[k]
        ar.write(lo, rng.integers(-50, 51, (hi - lo) // 4).astype(np.float32))
    return ar, tw, off, ids


def trapped(g, fn):
    with pytest.raises(g.AgileError) as e:
        fn()
    assert e.value.code == g.AGILE_ETRAPPED
    return True


def test_trap_retires_handle_after_a_violating_gather():
    ar, tw, off, ids = setup(11)
    g = tw.g
    A, C, I, S = (ar.addr(off[k][0]) for k in ("A", "C", "I", "S"))
    ol = G.FaultLog()
    # 1. clean TRAP calls: ordinary results, handle stays live
    tw.g.agile_guarded_copy(tw.h, C, A, 3000, g.POLICY_TRAP)
    assert G.guarded_call(G.copy_vec, tw.ot, ar.mem, ol, tw.next_seq(), C, A, 3000,
                          policy=G.TRAP) == G.OK
    idx = np.arange(0, 2000, dtype=np.int64) * 3 % ROWS
    ar.write(off["I"][0], idx)
    tw.g.agile_guarded_gather(tw.h, C, A, RB, I, 2000, 0, g.POLICY_TRAP)
    assert G.guarded_call(G.gather_vec, tw.ot, ar.mem, ol, tw.next_seq(), C, A, RB, I, 2000, 4,
                          policy=G.TRAP) == G.OK
    ar.check("clean trap-policy calls")
    log_matches(tw, ol, "clean trap-policy calls")
    # 2. a violating TRAP gather: rows into the canary and past the table
    bad = (ar.addr(off["P"][0]) - A) // RB + 1
    idx = np.arange(4000, dtype=np.int64) * 7 % ROWS
    idx[[7, 3000, 3999]] = [bad, ROWS + 3, -1]
    ar.write(off["I"][0], idx)
    trapped(g, lambda: g.agile_guarded_gather(tw.h, C, A, RB, I, 4000, 0, g.POLICY_TRAP))
    assert G.guarded_call(G.gather_vec, tw.ot, ar.mem, ol, tw.next_seq(), C, A, RB, I, 4000, 4,
                          policy=G.TRAP) == G.ETRAPPED
    ar.check("violating trap-policy gather")
    # 3. the retired handle refuses everything that would queue work; nothing changes
    q = torch.tensor([[A, 16]], dtype=torch.int64, device="cuda")
    verdict = torch.full((1,), 0xEE, dtype=torch.uint8, device="cuda")
    owner = torch.full((1,), -7, dtype=torch.int32, device="cuda")
    for pol in (g.POLICY_SUPPRESS_LOG, g.POLICY_SUPPRESS_ONLY, g.POLICY_TRAP):
        trapped(g, lambda: g.agile_guarded_copy(tw.h, C, S, 4096, pol))
        trapped(g, lambda: g.agile_guarded_triad(tw.h, C, S, A, 2.0, 1000, pol))
        trapped(g, lambda: g.agile_guarded_gather(tw.h, C, A, RB, I, 100, 0, pol))
        trapped(g, lambda: g.agile_guarded_scatter(tw.h, C, RB, I, S, NIDX, 0, 1, pol))
    trapped(g, lambda: g.agile_validate_ptrs(tw.h, q, 1, verdict, owner))
    trapped(g, lambda: tw.rt.insert(ar.addr(ar.n) + (1 << 20), 4096, 0))
    trapped(g, lambda: g.agile_rt_sync(tw.h))
    torch.cuda.synchronize()
    assert int(verdict.item()) == 0xEE and int(owner.item()) == -7
    ar.check("calls of the retired handle")
    # 4. the log still reads (ETRAPPED, the violating call's record); revocation still works
    rc, f = tw.rt.fault_log(clear=True)
    assert rc == g.AGILE_ETRAPPED
    o = ol.first
    assert f["count"] == ol.count == 3 * D
    assert (f["first_seq"], f["first_elem"], f["first_operand"], f["first_addr"],
            f["first_verdict"], f["first_owner"], f["first_op"]) == \
        (o["seq"], o["elem"], o["operand"], o["addr"], o["verdict"], o["owner"], o["op"])
    rc, f = tw.rt.fault_log()
    assert rc == g.AGILE_ETRAPPED and f["count"] == 0
    tw.remove(ids["S"])
    assert len(tw.rt) == 4
    tw.close()


def test_trap_on_the_sorted_scatter_add_path():
    """A violating TRAP scatter-add of 40,000 rows (the sorted path): the arena equals the
    oracle's suppress-and-log result, the call reports ETRAPPED and a queued batch naming the
    client is refused."""
    ar, tw, off, ids = setup(12)
    g = tw.g
    A, I, S = (ar.addr(off[k][0]) for k in ("A", "I", "S"))
    rng = random.Random(12)
    idx = np.array([rng.randrange(ROWS) for _ in range(NIDX)], dtype=np.int64)
    idx[[3, 20000]] = [ROWS, -(1 << 40)]
    ar.write(off["I"][0], idx)
    ol = G.FaultLog()
    trapped(g, lambda: g.agile_guarded_scatter(tw.h, A, RB, I, S, NIDX, 0, 1, g.POLICY_TRAP))
    assert G.guarded_call(G.scatter_vec, tw.ot, ar.mem, ol, tw.next_seq(), A, RB, I, S, NIDX, 4,
                          True, policy=G.TRAP) == G.ETRAPPED
    ar.check("violating trap-policy scatter-add")
    cs = g.agile_clients_create([tw.rt])
    try:
        reqs = np.zeros(1, dtype=g.REQUEST_DTYPE)
        reqs["copy_dst"], reqs["copy_src"], reqs["copy_bytes"] = A, S, 4096
        res = torch.zeros(72, dtype=torch.uint8, device="cuda")
        trapped(g, lambda: g.agile_batch_run(cs, reqs, None, 0, None, None, res))
    finally:
        g.agile_clients_destroy(cs)
    ar.check("batch naming a retired client")
    rc, f = tw.rt.fault_log()
    assert rc == g.AGILE_ETRAPPED and f["count"] == ol.count == 2 * D
    tw.close()


def test_violations_under_other_policies_do_not_retire():
    ar, tw, off, ids = setup(13)
    g = tw.g
    A, C, I = (ar.addr(off[k][0]) for k in ("A", "C", "I"))
    idx = np.array([1, ROWS + 1, 2], dtype=np.int64)
    ar.write(off["I"][0], idx)
    ol = G.FaultLog()
    for pol in (g.POLICY_SUPPRESS_LOG, g.POLICY_SUPPRESS_ONLY):
        g.agile_guarded_gather(tw.h, C, A, RB, I, 3, 0, pol)
        assert G.guarded_call(G.gather_vec, tw.ot, ar.mem, ol, tw.next_seq(), C, A, RB, I, 3, 4,
                              policy=pol) == G.OK
    g.agile_guarded_copy(tw.h, C, A, 64, g.POLICY_TRAP)
    assert G.guarded_call(G.copy_vec, tw.ot, ar.mem, ol, tw.next_seq(), C, A, 64,
                          policy=G.TRAP) == G.OK
    ar.check("violations under suppress policies, then a clean trap call")
    log_matches(tw, ol, "violations under suppress policies")
    tw.close()
