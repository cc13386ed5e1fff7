"""Serving loop: continuous batching of many clients' requests; each request's result in the
mix equals the same request run alone, and sampled outputs are the oracle's."""
import numpy as np
import pytest
import torch

from gpu_util import need_gpu, guard_mod

pytestmark = pytest.mark.gpu


def check_against_alone_and_oracle(srv, kept):
    """Every kept result equals the same request run alone; copies carry the source bytes and
    gathers the table rows (0 for a denied index, with the denial counted)."""
    for r, (res, out, pv, po, q) in kept.items():
        assert res["done"] == 1
        ares, aout, apv, apo = srv.run_alone(q)
        for k in ("verdict", "arg", "owner", "count", "first_elem", "first_operand",
                  "first_addr", "first_verdict", "first_owner"):
            assert ares[k] == res[k], (r, k)
        if out is not None:
            assert np.array_equal(aout, out), r
        if pv is not None:
            assert np.array_equal(apv, pv) and np.array_equal(apo, po), r
        c = int(q["client"])
        if q["copy_bytes"]:
            o = int(q["copy_src"]) - srv.csrc[c].data_ptr()
            assert np.array_equal(out, srv.csrc[c][o:o + int(q["copy_bytes"])].cpu().numpy())
            assert res["count"] == 0
        elif q["gather_n"]:
            i0 = (int(q["gather_idx"]) - srv.gidx[c].data_ptr()) // 8
            iv = srv.gidx[c][i0:i0 + int(q["gather_n"])].cpu().numpy()
            tab = srv.gtab[c].cpu().numpy()
            ok = (iv >= 0) & (iv < tab.size)
            want = np.zeros(iv.size, np.float32)
            want[ok] = tab[iv[ok]]
            assert np.array_equal(out.view(np.float32), want)
            assert res["count"] == int((~ok).sum())


def test_serving_mix_equals_alone():
    need_gpu()
    g = guard_mod()
    from paper_2606_06697_amd.serving import Server, ServeConfig
    from synth import make_serving_trace
    cfg = ServeConfig(n_clients=6, rate=20000.0, duration=0.3, ranges=(256, 1024),
                      gather_table_bytes=16 << 20, idx_pool=1 << 16, copy_src_bytes=2 << 20,
                      ptr_pool=1 << 13, ring_bytes=64 << 20, hbm_budget=1 << 30, max_batch=128,
                      copy_range=(4096, 2 << 20), gather_range=(1 << 12, 1 << 16))
    srv = Server(cfg)
    trace = make_serving_trace(cfg.n_clients, cfg.rate, cfg.duration, cfg.seed,
                               mix=cfg.mix, val_ptrs=cfg.val_ptrs, copy_range=cfg.copy_range,
                               gather_range=cfg.gather_range)
    n = trace["t"].numel()
    rng = np.random.default_rng(0)
    sample = set(rng.choice(n, size=min(150, n), replace=False).tolist())
    lat, stats, kept = srv.run(trace, record=sample)
    assert stats["requests"] == n and not np.isnan(lat).any()
    assert stats["launches"] < n                      # requests were batched
    assert stats["max_inflight_bytes"] <= cfg.hbm_budget
    assert len(kept) == len(sample)
    check_against_alone_and_oracle(srv, kept)
    srv.close()


def _copy_burst(budget, ring, copy_range, oversize=()):
    """400-odd copy requests from 6 clients arriving within 2 ms, at most 4 per launch and 4
    launches in flight; the requests at positions `oversize` copy 2 MiB, more than the budget
    or the ring can ever hold, and must be refused without a launch. Returns the server, the
    request count and the run's statistics."""
    from paper_2606_06697_amd.serving import Server, ServeConfig
    from synth import make_serving_trace
    cfg = ServeConfig(n_clients=6, rate=200000.0, duration=0.002, ranges=(256, 1024),
                      gather_table_bytes=16 << 20, idx_pool=1 << 16, copy_src_bytes=2 << 20,
                      ptr_pool=1 << 13, ring_bytes=ring, hbm_budget=budget, max_batch=4,
                      max_inflight=4, val_ptrs=(16, 256), copy_range=copy_range,
                      gather_range=(1 << 12, 1 << 16), mix=(0.0, 1.0, 0.0))
    srv = Server(cfg)
    trace = make_serving_trace(cfg.n_clients, cfg.rate, cfg.duration, cfg.seed,
                               mix=cfg.mix, val_ptrs=cfg.val_ptrs, copy_range=cfg.copy_range,
                               gather_range=cfg.gather_range)
    n = trace["t"].numel()
    assert n > 300
    big = np.zeros(n, dtype=bool)
    big[list(oversize)] = True
    trace["size"][torch.from_numpy(big)] = 2 << 20
    rng = np.random.default_rng(3)
    sample = set(rng.choice(np.flatnonzero(~big), size=100, replace=False).tolist())
    lat, stats, kept = srv.run(trace, record=sample)
    assert stats["requests"] == n - big.sum() and stats["refused"] == big.sum()   # served / refused
    assert np.array_equal(srv.refused, big) and not np.isnan(lat[~big]).any()
    arr = trace["t"].numpy()
    assert (srv.t_launch[~big] >= arr[~big]).all()
    # admitted as earlier launches returned their output space, not all at once
    assert (srv.t_launch[~big] > float(np.min(arr[~big] + lat[~big]))).sum() > n // 4
    check_against_alone_and_oracle(srv, kept)
    return srv, n, stats


def test_serving_admission_waits_for_the_hbm_budget():
    """Copies of 1-1.5 MiB against a 1.75 MiB budget for in-flight outputs (rings of 64 MiB):
    no two requests fit the budget together, so each launch carries one request, only one
    launch is ever in flight, and the FIFO head waits for the budget (counted per request)
    while the launch before it holds its bytes. Sampled results equal the request run alone
    and the oracle. Five 2 MiB copies, which no budget of 1.75 MiB can ever admit, are refused
    without a launch and do not hold up the requests behind them."""
    need_gpu()
    guard_mod()
    budget = 1792 << 10
    srv, n, stats = _copy_burst(budget, 64 << 20, (1 << 20, 1536 << 10),
                                oversize=(3, 50, 51, 200, 300))
    assert stats["budget_waits"] > 0 and stats["ring_waits"] == 0, stats
    assert 1 << 20 <= stats["max_inflight_bytes"] <= budget, stats
    assert stats["max_concurrent_launches"] == 1 and stats["launches"] == n - 5, stats
    srv.close()


def test_serving_admission_waits_for_ring_space():
    """Copies of 1.1-1.5 MiB into 2 MiB output rings per client (budget 1 GiB): a client's next
    request fits its ring only after the client's request in flight has completed, so the FIFO
    head waits for ring space (counted per request), while other clients' requests run in
    other launches at the same time. Sampled results equal the request run alone and the
    oracle."""
    need_gpu()
    guard_mod()
    ring = 2 << 20
    srv, n, stats = _copy_burst(1 << 30, ring, (1126 << 10, 1536 << 10))
    assert stats["ring_waits"] > 0 and stats["budget_waits"] == 0, stats
    assert 0 < stats["max_inflight_bytes"] <= 6 * ring, stats
    assert 2 <= stats["max_concurrent_launches"] <= 4, stats
    srv.close()


def test_serving_revocation_while_batches_are_in_flight():
    """A client is revoked at 0.12 s of a 0.3 s trace (every range of its table removed while
    other batches are on the device). Its requests launched before then give the results of the
    table they were launched with (oracle verdicts, source bytes); its later requests are refused
    without a launch; every other client's results equal the same request run alone; a request
    of the revoked client run after the revocation is denied everywhere."""
    need_gpu()
    g = guard_mod()
    from paper_2606_06697_amd.serving import Server, ServeConfig
    from synth import make_serving_trace
    from oracle import RangeTable as OT
    cfg = ServeConfig(n_clients=6, rate=20000.0, duration=0.3, ranges=(256, 1024),
                      gather_table_bytes=16 << 20, idx_pool=1 << 16, copy_src_bytes=2 << 20,
                      ptr_pool=1 << 13, ring_bytes=64 << 20, hbm_budget=1 << 30, max_batch=128,
                      copy_range=(4096, 2 << 20), gather_range=(1 << 12, 1 << 16))
    srv = Server(cfg)
    trace = make_serving_trace(cfg.n_clients, cfg.rate, cfg.duration, cfg.seed,
                               mix=cfg.mix, val_ptrs=cfg.val_ptrs, copy_range=cfg.copy_range,
                               gather_range=cfg.gather_range)
    victim = 2
    # the victim's table as built, in insertion order (so ids match)
    ot = OT()
    tb = srv.synth_tables[victim]
    for b, s, k in zip(tb.base.tolist(), tb.size.tolist(), tb.kind.tolist()):
        ot.insert(b, s, k)
    for t in (srv.gtab[victim], srv.gidx[victim], srv.csrc[victim], srv.ring_mem[victim]):
        ot.insert(t.data_ptr(), t.numel() * t.element_size(), 0)
    client = trace["client"].numpy()
    n = client.size
    rng = np.random.default_rng(1)
    others = np.flatnonzero(client != victim)
    sample = set(np.flatnonzero(client == victim).tolist())
    sample |= set(rng.choice(others, size=min(100, others.size), replace=False).tolist())
    lat, stats, kept = srv.run(trace, record=sample, revoke={victim: 0.12})
    t_rev = srv.revoked_at[victim]
    vic = client == victim
    arr = trace["t"].numpy()
    assert not srv.refused[~vic].any()
    assert srv.refused[vic & (arr > t_rev)].all()
    served = vic & ~srv.refused
    assert served.sum() > 10 and srv.refused.sum() > 10 and stats["refused"] == srv.refused.sum()
    assert (srv.t_launch[served] < t_rev).all()
    assert not np.isnan(lat[~srv.refused]).any()
    ptrs = srv.ptrs.cpu().numpy().view(np.uint64)
    for r, (res, out, pv, po, q) in kept.items():
        assert res["done"] == 1
        c = int(q["client"])
        if c != victim:
            ares, aout, apv, apo = srv.run_alone(q)
            for k in ("verdict", "arg", "owner", "count", "first_elem", "first_operand"):
                assert ares[k] == res[k], (r, k)
            if out is not None:
                assert np.array_equal(aout, out), r
            if pv is not None:
                assert np.array_equal(apv, pv) and np.array_equal(apo, po), r
            continue
        if q["nptr"]:
            a, e = int(q["ptr_off"]), int(q["ptr_off"] + q["nptr"])
            ev, eo = ot.verdict_many(ptrs[a:e, 0], ptrs[a:e, 1])
            assert np.array_equal(pv, ev) and np.array_equal(po, eo), r
        if q["copy_bytes"]:
            o = int(q["copy_src"]) - srv.csrc[c].data_ptr()
            assert np.array_equal(out, srv.csrc[c][o:o + int(q["copy_bytes"])].cpu().numpy())
            assert res["count"] == 0
        if q["gather_n"]:
            i0 = (int(q["gather_idx"]) - srv.gidx[c].data_ptr()) // 8
            iv = srv.gidx[c][i0:i0 + int(q["gather_n"])].cpu().numpy()
            tab = srv.gtab[c].cpu().numpy()
            ok = (iv >= 0) & (iv < tab.size)
            want = np.zeros(iv.size, np.float32)
            want[ok] = tab[iv[ok]]
            assert np.array_equal(out.view(np.float32), want) and res["count"] == int((~ok).sum())
    # after the revocation the victim's requests are denied on the device as well
    q = next(kept[r][4] for r in sorted(kept) if client[r] == victim and kept[r][4]["copy_bytes"])
    c0 = int(q["copy_dst"]) - srv.ring_mem[victim].data_ptr()
    before = srv.ring_mem[victim][c0:c0 + int(q["copy_bytes"])].cpu().numpy().copy()
    ares, aout, _, _ = srv.run_alone(q)
    assert ares["count"] == 2 * int(q["copy_bytes"])
    assert ares["first_verdict"] == g.V_UNMAPPED and np.array_equal(aout, before)
    srv.close()
