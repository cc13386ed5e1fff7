"""Table changes while launches that read the table are still running (stream order, two
device images).

Section V-C has the worker search the allocation table of the live allocations on every
request, and freed allocations must be refused from then on (Section IV-E). A table change is
built into the device image that is not current, so launches still reading the current image
are not waited for; a second change reuses the older image only after its readers finish.
Stream A queues many validations of 2^26 queries; meanwhile the host removes and inserts
ranges twice and stream B validates after each change; then A validates again. Every launch
must see the table exactly as it stood when the launch was made.
"""
import random

import numpy as np
import pytest
import torch

from gpu_util import Twin, need_gpu
from synth import make_table, make_queries

pytestmark = pytest.mark.gpu


def mutate(tw, rng, nrem, nins):
    """Remove nrem random ranges, then insert nins ranges into the holes they left."""
    ents = tw.ot.entries()
    gone = rng.sample(ents, nrem)
    for b, e, k, rid in gone:
        tw.remove(rid)
    for b, e, k, rid in gone[:nins]:
        size = max(1, (e - b) // 2)
        tw.insert(b + (e - b - size), size, rng.choice([0, 0, 1]))


def expect(tw, q):
    return tw.ot.verdict_many(q[:, 0], q[:, 1])


def test_changes_while_launches_are_in_flight():
    need_gpu()
    tb = make_table(65536, 8192, 1)
    tw = Twin(70000)
    tw.insert_table(tb)
    g = tw.g
    rng = random.Random(17)
    nbig, nsmall, nq = 1 << 26, 1 << 16, 100
    qbig = make_queries(tb, nbig, 1, device="cuda")
    qsmall = make_queries(tb, nsmall, 2, device="cuda")
    qs_host = qsmall.cpu().numpy().view(np.uint64)
    sample = np.sort(np.random.default_rng(3).choice(nbig, 1 << 18, replace=False))
    qb_sample = qbig[torch.from_numpy(sample).cuda()].cpu().numpy().view(np.uint64)
    A, B = torch.cuda.Stream(), torch.cuda.Stream()
    torch.cuda.synchronize()

    def validate(q, n, stream):
        with torch.cuda.stream(stream):
            v = torch.empty(n, dtype=torch.uint8, device="cuda")
            o = torch.empty(n, dtype=torch.int32, device="cuda")
            g.agile_validate_ptrs(tw.h, q, n, v, o, stream)
        return v, o

    want0 = expect(tw, qb_sample)
    vscr, oscr = validate(qbig, nbig, A)
    for _ in range(nq - 2):
        with torch.cuda.stream(A):
            g.agile_validate_ptrs(tw.h, qbig, nbig, vscr, oscr, A)
    vA0, oA0 = validate(qbig, nbig, A)
    doneA = torch.cuda.Event(enable_timing=True)
    doneA.record(A)
    mutate(tw, rng, 2000, 1000)
    vB1, oB1 = validate(qsmall, nsmall, B)
    doneB1 = torch.cuda.Event(enable_timing=True)
    doneB1.record(B)
    in_flight = not doneA.query()
    want1 = expect(tw, qs_host)
    mutate(tw, rng, 2000, 1000)
    vB2, oB2 = validate(qsmall, nsmall, B)
    want2 = expect(tw, qs_host)
    mutate(tw, rng, 500, 500)
    vA3, oA3 = validate(qbig, nbig, A)
    want3 = expect(tw, qb_sample)
    torch.cuda.synchronize()
    print(f"stream A still running at the first change: {in_flight}; "
          f"B's first launch done before A's queue: {doneB1.elapsed_time(doneA) > 0}")
    idx = torch.from_numpy(sample).cuda()
    for (v, o), (ev, eo), what in (((vA0[idx], oA0[idx]), want0, "A before the changes"),
                                   ((vscr[idx], oscr[idx]), want0, "A queue"),
                                   ((vB1, oB1), want1, "B after one change"),
                                   ((vB2, oB2), want2, "B after two changes"),
                                   ((vA3[idx], oA3[idx]), want3, "A after three changes")):
        v, o = v.cpu().numpy(), o.cpu().numpy()
        bad = np.flatnonzero((v != ev) | (o != eo))
        assert bad.size == 0, (what, bad.size)
    # the changes did change verdicts
    assert not np.array_equal(want1[0], expect(tw, qs_host)[0]) or \
        not np.array_equal(want0[0], want3[0])
    tw.close()
