"""Full-size parity: the workloads bench.py times, at their sizes and in the same launch
configuration, checked against the oracle on sampled outputs (the oracle computes each one
independently) and on properties that hold for every output.

* large table: 65,536 ranges (8,192 protected), 2^28 queries; guarded triad over 3 x 2^28 fp32;
  guarded gather of 2^26 indices over a 2^28-row fp32 table, 0.1% hostile;
* embedding: 1,048,576 x 256 fp32 table, 2^20 Zipf(1.1) indices, 0.01% aimed at a protected
  pad; forward rows bit-exact, gradient within 1e-5 relative (Frobenius) of an fp64 reference;
* batched launch: 16 clients x 4,096 ranges, 512 requests with up to 4,096 pointers and one
  4 KiB-64 MiB guarded copy each.
"""
import gc

import numpy as np
import pytest
import torch

from gpu_util import need_gpu, guard_mod
from oracle import guarded as G
from oracle.batched import batch_verdicts
from oracle.embedding import embedding_grad_ref
from oracle.table import RangeTable as OracleTable
from synth import (make_table, make_queries, uniform_f32, uniform_indices, zipf_indices,
                   make_batch_requests)

pytestmark = pytest.mark.gpu

SAMPLE = 1 << 20


def _free():
    gc.collect()
    torch.cuda.empty_cache()


def _oracle_table(tb):
    ot = OracleTable()
    for b, s, k in zip(tb.base.tolist(), tb.size.tolist(), tb.kind.tolist()):
        ot.insert(b, s, k)
    return ot


def _sample_positions(n, seed, k=SAMPLE):
    gen = torch.Generator().manual_seed(seed)
    pos = torch.randint(0, n, (k,), generator=gen)
    edges = torch.cat([torch.arange(0, 4096), torch.arange(n - 4096, n)])
    return torch.unique(torch.cat([pos, edges]))


def test_validate_2e28_queries_65536_ranges():
    need_gpu()
    g = guard_mod()
    n = 1 << 28
    tb = make_table(65536, 8192, 1, first_hi=2**44)
    rt = g.RangeTable(65536 + 16)
    rt.insert_many(tb.base, tb.size, tb.kind)
    q = make_queries(tb, n, 1, device="cuda")
    verdict = torch.full((n,), 255, dtype=torch.uint8, device="cuda")
    owner = torch.full((n,), -7, dtype=torch.int32, device="cuda")
    g.agile_validate_ptrs(rt.handle, q, n, verdict, owner)
    torch.cuda.synchronize()
    # every output: a verdict code, and owner == -1 exactly for UNMAPPED
    assert int(verdict.max()) <= 3
    assert bool(((owner == -1) == (verdict == 3)).all())
    assert bool((owner < 65536).all())
    # sampled outputs against the oracle
    pos = _sample_positions(n, 11).cuda()
    qs = q[pos].cpu().numpy().view(np.uint64)
    ev, eo = _oracle_table(tb).verdict_many(qs[:, 0], qs[:, 1])
    assert np.array_equal(verdict[pos].cpu().numpy(), ev)
    assert np.array_equal(owner[pos].cpu().numpy(), eo)
    # the mix shows up in the verdict histogram
    hist = torch.bincount(verdict.to(torch.int64), minlength=4).cpu().numpy() / n
    assert hist[0] > 0.5 and hist[1] > 0.15 and hist[2] > 0.04 and hist[3] > 0.05
    rt.close()
    del q, verdict, owner
    _free()


def test_triad_and_gather_large_table():
    need_gpu()
    g = guard_mod()
    N, ROWS, NI, PAD = 1 << 28, 1 << 28, 1 << 26, 64 << 10
    dt = g.RangeTable(64)
    ot = OracleTable()

    def reg(ptr, size, kind=0):
        rid = dt.insert(ptr, size, kind)
        assert rid == ot.insert(ptr, size, kind)
        return rid

    # triad a = b + 3*c
    a = torch.empty(N, dtype=torch.float32, device="cuda")
    b = uniform_f32(N, 1, device="cuda", stream=10)
    c = uniform_f32(N, 1, device="cuda", stream=11)
    ids = [reg(t.data_ptr(), t.numel() * 4) for t in (a, b, c)]
    g.agile_guarded_triad(dt.handle, a, b, c, 3.0, N)
    rc, f = dt.fault_log(clear=True)
    assert rc == g.AGILE_OK and f["count"] == 0
    pos = _sample_positions(N, 12).cuda()
    bs, cs = b[pos].cpu().numpy(), c[pos].cpu().numpy()
    want = (bs + np.float32(3.0) * cs).astype(np.float32)       # two float32 roundings
    assert np.array_equal(a[pos].cpu().numpy().view(np.uint32), want.view(np.uint32))
    for rid in ids:                                 # freed below: their bytes become holes
        dt.remove(rid)
        ot.remove(rid)
    del a, b, c
    _free()

    # gather with hostile indices into a protected pad and an unregistered hole
    gbuf = torch.empty(ROWS * 4 + 2 * PAD, dtype=torch.uint8, device="cuda")
    table = gbuf[:ROWS * 4].view(torch.float32)
    table.copy_(uniform_f32(ROWS, 1, device="cuda", stream=12))
    gbuf[ROWS * 4:].fill_(0xA5)
    prot_rows = (ROWS, ROWS + PAD // 4)
    hole_rows = (ROWS + PAD // 4, ROWS + PAD // 2)
    idx = uniform_indices(NI, ROWS, 1, device="cuda", bad_frac=0.001,
                          bad_ranges=(prot_rows, hole_rows))
    out = torch.full((NI,), 7.0, dtype=torch.float32, device="cuda")
    reg(idx.data_ptr(), NI * 8)
    reg(out.data_ptr(), NI * 4)
    reg(table.data_ptr(), ROWS * 4)
    reg(table.data_ptr() + ROWS * 4, PAD, 1)
    seq_before = 1                                  # the triad was this table's call 0
    g.agile_guarded_gather(dt.handle, out, table, 4, idx, NI)
    rc, f = dt.fault_log(clear=True)
    bad = (idx < 0) | (idx >= ROWS)
    nbad = int(bad.sum())
    assert nbad == round(NI * 0.001)
    assert rc == g.AGILE_EFAULTED and f["count"] == nbad
    # every suppressed row reads zero, the pad is untouched
    assert bool((out[bad] == 0).all())
    assert bool((gbuf[ROWS * 4:] == 0xA5).all())
    # sampled good rows: the table element, bit for bit
    pos = _sample_positions(NI, 13).cuda()
    ip = idx[pos].cpu().numpy()
    op = out[pos].cpu().numpy()
    okp = (ip >= 0) & (ip < ROWS)
    tv = table[torch.from_numpy(ip[okp]).cuda()].cpu().numpy()
    assert np.array_equal(op[okp].view(np.uint32), tv.view(np.uint32))
    assert (op[~okp] == 0).all()
    # first record: the smallest hostile i, operand 1 (table), reason from the oracle table
    i0 = int(torch.nonzero(bad)[0, 0])
    A = table.data_ptr() + int(idx[i0]) * 4
    v, o = G.reason(ot, A, 4)
    assert (f["first_seq"], f["first_elem"], f["first_operand"], f["first_addr"],
            f["first_width"], f["first_verdict"], f["first_owner"], f["first_op"]) == \
        (seq_before, i0, 1, A, 4, v, o, G.OP_GATHER)
    dt.close()
    del gbuf, table, idx, out
    _free()


def test_embedding_forward_backward_full_size():
    need_gpu()
    g = guard_mod()
    from paper_2606_06697_amd.embedding import guarded_embedding
    R, D, N, PAD = 1 << 20, 256, 1 << 20, 16
    buf = torch.empty((R + PAD) * D, dtype=torch.float32, device="cuda")
    buf[:R * D].copy_(uniform_f32(R * D, 2, device="cuda", stream=30))
    buf[R * D:].fill_(5.0)
    W = buf[:R * D].view(R, D)
    idx = zipf_indices(N, R, 1.1, 2, device="cuda", bad_frac=1e-4, bad_ranges=((R, R + PAD),))
    tab = g.RangeTable(64)
    tab.insert_tensor(W, g.KIND_USER)
    tab.insert(W.data_ptr() + R * D * 4, PAD * D * 4, g.KIND_PROTECTED)
    tab.insert_tensor(idx, g.KIND_USER)
    Wp = W.detach().requires_grad_()
    Y = guarded_embedding(Wp, idx, tab)
    good = (idx >= 0) & (idx < R)
    nbad = int((~good).sum())
    assert nbad == round(N * 1e-4)
    # forward: every row equals the selected table row (a plain index_select where allowed),
    # zero where suppressed; sampled rows against the oracle's definition as well
    assert bool((Y[~good] == 0).all())
    assert torch.equal(Y[good], W[idx[good]])
    dY = uniform_f32(N * D, 2, device="cuda", stream=31).view(N, D)
    Y.backward(dY)
    dW = Wp.grad
    rc, f = tab.fault_log(clear=True)
    assert f["count"] == 2 * nbad * D               # forward loads + backward stores
    assert bool((buf[R * D:] == 5.0).all())
    # backward against an fp64 reference over the whole table
    ref = torch.zeros((R, D), dtype=torch.float64, device="cuda")
    ref.index_add_(0, idx[good], dY[good].double())
    err = torch.linalg.vector_norm(dW.double() - ref) / torch.linalg.vector_norm(ref)
    assert float(err) <= 1e-5, float(err)
    # elementwise: within the worst-case bound of an fp32 sum of m terms in any order,
    # |error| <= m * 2^-24 * sum |terms| (m = the row's number of allowed indices)
    cnt = torch.bincount(idx[good], minlength=R).double()[:, None]
    absref = torch.zeros((R, D), dtype=torch.float64, device="cuda")
    absref.index_add_(0, idx[good], dY[good].abs().double())
    diff = (dW.double() - ref).abs()
    assert bool((diff <= cnt * 2.0**-24 * absref * 1.0001).all())
    big = ref.abs() > 1e-3 * ref.abs().max()
    rel = (diff[big] / ref.abs()[big]).max()
    print(f"embedding gradient: frobenius rel {float(err):.3e}, elementwise max rel over "
          f"|ref| > 1e-3 max {float(rel):.3e}")
    del absref, diff, cnt
    # sampled rows (the hottest ones, random ones, never-indexed ones) against the oracle
    ih = idx.cpu().numpy()
    gh = (ih >= 0) & (ih < R)
    u, cnt = np.unique(ih[gh], return_counts=True)
    rng = np.random.default_rng(3)
    rows = np.unique(np.concatenate([u[np.argsort(cnt)[-4:]], rng.choice(u, 60, replace=False),
                                     np.setdiff1d(rng.integers(0, R, 200), u)[:20]]))
    sel = np.flatnonzero(gh & np.isin(ih, rows))
    local = np.searchsorted(rows, ih[sel])
    dys = dY[torch.from_numpy(sel).cuda()].cpu().numpy()
    want = embedding_grad_ref(local, np.ones(sel.size, bool), dys, rows.size)
    got = dW[torch.from_numpy(rows).cuda()].cpu().numpy()
    num = np.linalg.norm(got.astype(np.float64) - want.astype(np.float64))
    assert num <= 1e-5 * np.linalg.norm(want.astype(np.float64))
    tab.close()
    del buf, W, Wp, Y, dY, dW, ref, idx
    _free()


def test_batched_launch_16_clients_512_requests():
    need_gpu()
    g = guard_mod()
    ncl, nreq = 16, 512
    tabs = [make_table(4096, 512, 300 + c, first_hi=2**44) for c in range(ncl)]
    spec = make_batch_requests(tabs, nreq, 3)
    rts, ots = [], []
    for tb in tabs:
        rt = g.RangeTable(4096 + nreq + 8)
        rt.insert_many(tb.base, tb.size, tb.kind)
        rts.append(rt)
        ots.append(_oracle_table(tb))
    client = spec["client"].numpy()
    cbytes = spec["copy_bytes"].numpy()
    gen = torch.Generator(device="cuda").manual_seed(5)
    src = [torch.randint(0, 256, (64 << 20,), dtype=torch.uint8, device="cuda", generator=gen)
           for _ in range(ncl)]
    for c in range(ncl):
        assert rts[c].insert_tensor(src[c]) == ots[c].insert(src[c].data_ptr(), 64 << 20, 0)
    dst_total = [int(((cbytes[client == c] + 255) // 256 * 256).sum()) for c in range(ncl)]
    dst = [torch.zeros(max(n, 256), dtype=torch.uint8, device="cuda") for n in dst_total]
    reqs = np.zeros(nreq, dtype=g.REQUEST_DTYPE)
    off = [0] * ncl
    rng = np.random.default_rng(5)
    for r in range(nreq):
        c, nb = int(client[r]), int(cbytes[r])
        d = dst[c].data_ptr() + off[c]
        assert rts[c].insert(d, nb, g.KIND_USER) == ots[c].insert(d, nb, 0)
        off[c] += (nb + 255) // 256 * 256
        reqs[r]["client"] = c
        reqs[r]["ptr_off"] = int(spec["ptr_off"][r])
        reqs[r]["nptr"] = int(spec["ptr_off"][r + 1] - spec["ptr_off"][r])
        reqs[r]["copy_dst"] = d
        reqs[r]["copy_src"] = src[c].data_ptr() + int(rng.integers(0, ((64 << 20) - nb) // 16 + 1)) * 16
        reqs[r]["copy_bytes"] = nb
    P = spec["ptrs"].cuda()
    nptrs = P.shape[0]
    pv = torch.full((nptrs,), 255, dtype=torch.uint8, device="cuda")
    po = torch.full((nptrs,), -7, dtype=torch.int32, device="cuda")
    res = torch.zeros(nreq * g.RESULT_DTYPE.itemsize, dtype=torch.uint8, device="cuda")
    cs = g.agile_clients_create(rts)
    g.agile_batch_run(cs, reqs, P, nptrs, pv, po, res)
    out = g.batch_results(res, nreq)
    ev, eo, rv, ra, ro = batch_verdicts(ots, client, spec["ptr_off"].numpy(),
                                        spec["ptrs"].numpy().view(np.uint64))
    assert np.array_equal(pv.cpu().numpy(), ev) and np.array_equal(po.cpu().numpy(), eo)
    assert np.array_equal(out["verdict"], rv) and np.array_equal(out["arg"], ra)
    assert np.array_equal(out["owner"], ro)
    assert (out["done"] == 1).all() and (out["count"] == 0).all()
    # every copy moved its bytes exactly (a fault-free guarded copy is a plain copy)
    for r in range(nreq):
        c, nb = int(client[r]), int(cbytes[r])
        s0 = int(reqs[r]["copy_src"]) - src[c].data_ptr()
        d0 = int(reqs[r]["copy_dst"]) - dst[c].data_ptr()
        assert torch.equal(dst[c][d0:d0 + nb], src[c][s0:s0 + nb]), r
    g.agile_clients_destroy(cs)
    for rt in rts:
        rt.close()
    del src, dst, P, pv, po, res
    _free()


def test_redirecting_policies_full_size_gather():
    """The bench's gather (2^26 indices over 2^28 rows, 0.1% aimed at a protected pad or an
    unregistered hole) under SINK (64 KiB quarantine), REPORT and REMAP. Every hostile row is
    checked: its target comes from the oracle's per-access rule and its value from the buffer
    that holds the target (zero when the access stays suppressed). Sampled allowed rows are the
    table element; the count and first record equal the suppress-and-log ones."""
    need_gpu()
    g = guard_mod()
    ROWS, NI, PAD, QS = 1 << 28, 1 << 26, 64 << 10, 1 << 16
    dt = g.RangeTable(16)
    ot = OracleTable()
    gbuf = torch.empty(ROWS * 4 + 2 * PAD, dtype=torch.uint8, device="cuda")
    table = gbuf[:ROWS * 4].view(torch.float32)
    table.copy_(uniform_f32(ROWS, 2, device="cuda", stream=12))
    gbuf[ROWS * 4:].fill_(0xA5)
    idx = uniform_indices(NI, ROWS, 2, device="cuda", bad_frac=0.001,
                          bad_ranges=((ROWS, ROWS + PAD // 4), (ROWS + PAD // 4, ROWS + PAD // 2)))
    out = torch.empty(NI, dtype=torch.float32, device="cuda")
    quar = uniform_f32(QS // 4, 3, device="cuda", stream=13)
    qh = quar.cpu().numpy()
    T = table.data_ptr()
    for ptr, size, kind in ((idx.data_ptr(), NI * 8, 0), (out.data_ptr(), NI * 4, 0),
                            (T, ROWS * 4, 0), (T + ROWS * 4, PAD, 1)):
        # all four are device memory (the pad is the tail of gbuf), so REPORT may touch them
        assert dt.insert(ptr, size, kind, backed=True) == ot.insert(ptr, size, kind, backed=True)
    g.agile_rt_set_quarantine(dt.handle, quar, QS)
    bad = (idx < 0) | (idx >= ROWS)
    ib = torch.nonzero(bad).flatten()
    bad_rows = idx[ib].cpu().numpy()
    nbad = bad_rows.size
    pos = _sample_positions(NI, 14).cuda()
    ip = idx[pos].cpu().numpy()
    okp = (ip >= 0) & (ip < ROWS)
    tv = table[torch.from_numpy(ip[okp]).cuda()].cpu().numpy()
    bind = ot.binding(T)
    first = None
    for seq, policy in enumerate((G.SUPPRESS_LOG, G.SINK, G.REPORT, G.REMAP)):
        out.fill_(7.0)
        g.agile_guarded_gather(dt.handle, out, table, 4, idx, NI, 0, policy)
        rc, f = dt.fault_log(clear=True)
        assert rc == g.AGILE_EFAULTED and f["count"] == nbad, policy
        rec = (f["first_elem"], f["first_operand"], f["first_addr"], f["first_verdict"],
               f["first_owner"])
        assert f["first_seq"] == seq
        first = first or rec
        assert rec == first, policy
        # every hostile row: the oracle's target, read from the buffer that holds it
        den = G._Denier(ot, G.FaultLog(), seq, G.OP_GATHER, policy, quarantine=(quar.data_ptr(), QS))
        want = np.zeros(nbad, dtype=np.uint32)
        tgt_rows = []
        for k, r in enumerate(bad_rows.tolist()):
            t = den.target(T + 4 * r, 4, bind)
            if t is None:
                continue
            if T <= t < T + ROWS * 4:
                tgt_rows.append((k, (t - T) // 4))
            elif T + ROWS * 4 <= t < T + ROWS * 4 + PAD:
                want[k] = 0xA5A5A5A5
            else:
                assert quar.data_ptr() <= t < quar.data_ptr() + QS
                want[k] = qh[(t - quar.data_ptr()) // 4].view(np.uint32)
        if tgt_rows:
            ks, rows_ = zip(*tgt_rows)
            vals = table[torch.tensor(rows_, device="cuda")].cpu().numpy().view(np.uint32)
            want[list(ks)] = vals
        got = out[ib].cpu().numpy().view(np.uint32)
        assert np.array_equal(got, want), (policy, int((got != want).sum()))
        op = out[pos].cpu().numpy()
        assert np.array_equal(op[okp].view(np.uint32), tv.view(np.uint32)), policy
        assert bool((gbuf[ROWS * 4:] == 0xA5).all())
    g.agile_rt_set_quarantine(dt.handle, 0, 0)
    dt.close()
    del gbuf, table, idx, out, quar
    _free()
