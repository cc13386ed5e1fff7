"""Serving loop: continuous batching of many clients' requests; each request's result in the
mix equals the same request run alone, and sampled outputs are the oracle's."""
import numpy as np
import pytest
import torch

from gpu_util import need_gpu, guard_mod

pytestmark = pytest.mark.gpu


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
    assert len(kept) == len(sample)
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
    srv.close()
