"""Benchmark of the range guard's hot path on one MI355X.

Workload (large table, bandwidth-bound guarded kernels): a 65,536-range table (8,192 of them
protected), 2^28 pointer queries with the 60/20/10/10 mix (inside USER / protected /
straddling / unmapped), a guarded fp32 triad a = b + 3*c over three 1 GiB buffers, and a
guarded gather of 2^26 int64 indices uniform over a 1 GiB fp32 table, 0.1% of them aimed at a
protected range registered right after the table or at an unregistered hole after that.

One step = validate all queries, run the guarded triad, run the guarded gather, then read and
clear the fault log (the synchronization point where denials surface). Inputs are resident in
HBM before timing starts. The unguarded twins of the triad and the gather are timed on the same
inputs for the guarded/unguarded ratio. The CPU oracle is timed on a bounded sample.

Prints one JSON line (see the "metric" and "roofline" keys).
"""
from __future__ import annotations

import argparse
import json
import os
import platform
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

PEAK_HBM_GBS = 8000.0
N_RANGES, N_PROT = 65536, 8192
N_QUERIES = 1 << 28
TRIAD_N = 1 << 28
GATHER_ROWS = 1 << 28
GATHER_N = 1 << 26
PAD_BYTES = 64 << 10          # protected range right after the table, then a hole
SEED = 1


def parse():
    p = argparse.ArgumentParser()
    p.add_argument("--gpus", type=int, default=1)
    p.add_argument("--steps", type=int, default=20)
    p.add_argument("--warmup", type=int, default=3)
    p.add_argument("--no-cpu-baseline", action="store_true")
    p.add_argument("--no-extras", action="store_true",
                   help="skip the embedding and batched-launch measurements")
    p.add_argument("--serve-seconds", type=float, default=60.0,
                   help="length of the serving-loop run (0 skips it)")
    p.add_argument("--counters-pass", action="store_true",
                   help="only launch each large-table kernel a few times, plus a plain 1 GiB copy "
                        "(the reference for scaling HBM counters), for a rocprofv3 --pmc run")
    p.add_argument("--extra", choices=("small_guard", "tokens", "embedding", "batch",
                                       "serving_capacity"),
                   help="run only this workload, then a plain 1 GiB copy (the reference for "
                        "scaling HBM counters), and print its JSON object")
    p.add_argument("--queries-log2", type=int, default=28, help=argparse.SUPPRESS)
    return p.parse_args()


def main():
    args = parse()
    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print("bench.py measures one GPU only: the library has no multi-GPU path "
              "(run with --gpus 1)", file=sys.stderr)
        sys.exit(2)
    import numpy as np
    import torch

    from paper_2606_06697_amd import guard as g
    if not os.path.exists(g.LIB_PATH):
        from paper_2606_06697_amd import _build
        _build.build()
    g.lib()
    from synth import make_table, make_queries, aperture_table, uniform_f32, uniform_indices

    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    if args.extra:
        fn = {"small_guard": bench_small_guard, "tokens": bench_tokens,
              "embedding": lambda g_: bench_embedding(g_, args),
              "batch": lambda g_: bench_batch(g_, args),
              "serving_capacity": lambda g_: bench_serving_capacity(g_, args)}[args.extra]
        out = fn(g)
        torch.cuda.empty_cache()
        ref_a = torch.empty(1 << 30, dtype=torch.uint8, device=dev)
        ref_b = torch.zeros(1 << 30, dtype=torch.uint8, device=dev)
        for _ in range(3):
            g.agile_unguarded_copy(ref_a, ref_b, 1 << 30)   # reference: 1 GiB in, 1 GiB out
        torch.cuda.synchronize()
        print(json.dumps({"extra": args.extra, **out}), flush=True)
        return
    nq = 1 << args.queries_log2

    # ---------------- inputs (resident before timing) ----------------
    tb = make_table(N_RANGES, N_PROT, SEED, first_hi=2**44)
    vt = g.RangeTable(N_RANGES + 16)
    vt.insert_many(tb.base, tb.size, tb.kind)
    q = make_queries(tb, nq, SEED, device=dev)
    verdict = torch.empty(nq, dtype=torch.uint8, device=dev)
    owner = torch.empty(nq, dtype=torch.int32, device=dev)

    a = torch.empty(TRIAD_N, dtype=torch.float32, device=dev)
    b = uniform_f32(TRIAD_N, SEED, device=dev, stream=10)
    c = uniform_f32(TRIAD_N, SEED, device=dev, stream=11)
    a_ref = torch.empty_like(a)

    gbuf = torch.empty(GATHER_ROWS * 4 + 2 * PAD_BYTES, dtype=torch.uint8, device=dev)
    table = gbuf[:GATHER_ROWS * 4].view(torch.float32)
    table.copy_(uniform_f32(GATHER_ROWS, SEED, device=dev, stream=12))
    gbuf[GATHER_ROWS * 4:].fill_(0xA5)
    prot_rows = (GATHER_ROWS, GATHER_ROWS + PAD_BYTES // 4)
    hole_rows = (GATHER_ROWS + PAD_BYTES // 4, GATHER_ROWS + 2 * PAD_BYTES // 4)
    idx = uniform_indices(GATHER_N, GATHER_ROWS, SEED, device=dev, bad_frac=0.001,
                          bad_ranges=(prot_rows, hole_rows))
    out = torch.empty(GATHER_N, dtype=torch.float32, device=dev)
    out_ref = torch.empty_like(out)

    # data table: the synthetic ranges plus the real buffers and the protected pad
    dt = g.RangeTable(N_RANGES + 64)
    dt.insert_many(tb.base, tb.size, tb.kind)
    for t in (a, b, c, idx, out):
        dt.insert_tensor(t)
    # the table and the protected pad after it are device memory (the synthetic ranges are not)
    dt.insert(table.data_ptr(), GATHER_ROWS * 4, g.KIND_USER, backed=True)
    dt.insert(table.data_ptr() + GATHER_ROWS * 4, PAD_BYTES, g.KIND_PROTECTED, backed=True)
    n_bad = int(((idx < 0) | (idx >= GATHER_ROWS)).sum())
    torch.cuda.synchronize()

    bytes_validate = nq * 21
    bytes_triad = TRIAD_N * 12
    bytes_gather = GATHER_N * 16
    step_bytes = bytes_validate + bytes_triad + bytes_gather

    if args.counters_pass:
        ap = g.agile_aperture_create(0, (64 << 30, 448 << 30, 1 << 40))
        qa = make_queries(aperture_table(g.agile_aperture_info(ap)[0]), nq, SEED, device=dev)
        for _ in range(3):
            g.agile_validate_aperture(ap, qa, nq, verdict, owner)
            g.agile_validate_ptrs(vt.handle, q, nq, verdict, owner)
            g.agile_guarded_triad(dt.handle, a, b, c, 3.0, TRIAD_N)
            g.agile_unguarded_triad(a_ref, b, c, 3.0, TRIAD_N)
            g.agile_guarded_gather(dt.handle, out, table, 4, idx, GATHER_N)
            g.agile_unguarded_gather(out_ref, table, 4, idx, GATHER_N)
            g.agile_unguarded_copy(a_ref, b, 4 * TRIAD_N)      # reference: 1 GiB in, 1 GiB out
        dt.fault_log(clear=True)
        torch.cuda.synchronize()
        g.agile_aperture_destroy(ap)
        print(json.dumps({"counters_pass": True, "bytes_per_launch": {
            "validate": nq * 21, "validate_aperture": nq * 21, "triad": TRIAD_N * 12,
            "gather": GATHER_N * 16,
            "copy_reference": {"read": 4 * TRIAD_N, "write": 4 * TRIAD_N}}}), flush=True)
        return

    ev = [torch.cuda.Event(enable_timing=True) for _ in range(4)]
    t_kern = {"validate": [], "triad": [], "gather": []}

    def step(timed):
        if timed:
            ev[0].record()
        g.agile_validate_ptrs(vt.handle, q, nq, verdict, owner)
        if timed:
            ev[1].record()
        g.agile_guarded_triad(dt.handle, a, b, c, 3.0, TRIAD_N)
        if timed:
            ev[2].record()
        g.agile_guarded_gather(dt.handle, out, table, 4, idx, GATHER_N)
        if timed:
            ev[3].record()
        rc, f = dt.fault_log(clear=True)       # synchronizes the stream
        if timed:
            t_kern["validate"].append(ev[0].elapsed_time(ev[1]))
            t_kern["triad"].append(ev[1].elapsed_time(ev[2]))
            t_kern["gather"].append(ev[2].elapsed_time(ev[3]))
        return rc, f

    for _ in range(args.warmup):
        rc, f = step(False)
    assert f["count"] == n_bad, (f["count"], n_bad)     # every hostile index denied once
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        step(True)
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    ms_step = elapsed * 1e3 / args.steps

    # guarded vs unguarded twins on the same inputs, each timed the same way (a block of
    # launches, one launch between two events); the hostile indices stay inside the gather buffer
    twin = time_blocks({
        "triad": lambda: g.agile_guarded_triad(dt.handle, a, b, c, 3.0, TRIAD_N),
        "triad_unguarded": lambda: g.agile_unguarded_triad(a_ref, b, c, 3.0, TRIAD_N),
        "gather": lambda: g.agile_guarded_gather(dt.handle, out, table, 4, idx, GATHER_N),
        "gather_unguarded": lambda: g.agile_unguarded_gather(out_ref, table, 4, idx, GATHER_N),
        "validate_dma": lambda: g.agile_validate_dma(vt.handle, q, nq, verdict, owner),
    }, args.warmup, args.steps)
    dt.fault_log(clear=True)
    torch.cuda.synchronize()
    # PyTorch's own ops on the same work, for context (no guard; out-of-range indices masked to
    # row 0 beforehand), into separate outputs
    a_t, out_t = torch.empty_like(a), torch.empty_like(out)
    idx_m = torch.where((idx < 0) | (idx >= GATHER_ROWS), torch.zeros_like(idx), idx)
    tref = time_blocks({
        "triad_torch": lambda: torch.add(b, c, alpha=3.0, out=a_t),
        "gather_torch": lambda: torch.index_select(table, 0, idx_m, out=out_t),
    }, args.warmup, args.steps)
    torch.cuda.synchronize()
    del a_t, out_t, idx_m
    ug = {"triad": twin["triad_unguarded"], "gather": twin["gather_unguarded"]}
    ok_triad = torch.equal(a.view(torch.int32), a_ref.view(torch.int32))
    good = (idx >= 0) & (idx < GATHER_ROWS)
    ok_gather = bool(torch.equal(out[good], out_ref[good])) and bool((out[~good] == 0).all())
    # the redirecting policies on the same gather (the guarded kernel, then the redirect pass)
    qbuf = torch.zeros(1 << 16, dtype=torch.uint8, device=dev)
    g.agile_rt_set_quarantine(dt.handle, qbuf, 1 << 16)
    pol = time_blocks({
        "gather_sink": lambda: g.agile_guarded_gather(dt.handle, out, table, 4, idx, GATHER_N, 0,
                                                      g.POLICY_SINK),
        "gather_report": lambda: g.agile_guarded_gather(dt.handle, out, table, 4, idx, GATHER_N,
                                                        0, g.POLICY_REPORT),
        "gather_remap": lambda: g.agile_guarded_gather(dt.handle, out, table, 4, idx, GATHER_N,
                                                       0, g.POLICY_REMAP),
    }, args.warmup, args.steps)
    dt.fault_log(clear=True)
    g.agile_rt_set_quarantine(dt.handle, 0, 0)
    torch.cuda.synchronize()
    # the coarse aperture check (Table I's sizes, no memory attached) on queries with the same
    # mix drawn relative to the three apertures, against the table validation above
    ap = g.agile_aperture_create(0, (64 << 30, 448 << 30, 1 << 40))
    ap_bounds, _, _ = g.agile_aperture_info(ap)
    qa = make_queries(aperture_table(ap_bounds), nq, SEED, device=dev)
    apt = time_blocks({"validate_aperture": lambda: g.agile_validate_aperture(ap, qa, nq, verdict,
                                                                              owner)},
                      args.warmup, args.steps)
    torch.cuda.synchronize()
    g.agile_aperture_destroy(ap)
    del qa
    # PyTorch's own formulation of the same validation, for context: searchsorted over the sorted
    # bases, then the end, kind and length tests as tensor ops; its verdicts and owners are
    # compared with the kernel's
    tbase, tend, tkind = tb.base.to(dev), (tb.base + tb.size).to(dev), tb.kind.to(dev)
    qad, qln = q[:, 0].contiguous(), q[:, 1].contiguous()

    def torch_validate():
        j = torch.searchsorted(tbase, qad, right=True) - 1
        jc = j.clamp_min(0)
        e = tend[jc]
        inside = (j >= 0) & (qad < e)
        ok = qln.clamp_min(1) <= e - qad
        v = torch.where(~inside, 3, torch.where(tkind[jc] != 0, 1, torch.where(ok, 0, 2)))
        return v.to(torch.uint8), torch.where(inside, jc, -1).to(torch.int32)

    tval = time_blocks({"validate_torch": torch_validate}, 1, max(3, args.steps // 4))
    v_t, o_t = torch_validate()
    g.agile_validate_ptrs(vt.handle, q, nq, verdict, owner)
    torch.cuda.synchronize()
    torch_equal = bool(torch.equal(v_t, verdict)) and bool(torch.equal(o_t, owner))
    del tbase, tend, tkind, qad, qln, v_t, o_t
    torch.cuda.empty_cache()

    def med(x):
        return float(np.median(np.array(x)))

    t_v, t_t, t_g = med(t_kern["validate"]), med(t_kern["triad"]), med(t_kern["gather"])
    gbs = {"validate": bytes_validate / t_v / 1e6, "triad": bytes_triad / t_t / 1e6,
           "gather": bytes_gather / t_g / 1e6}
    tw_t, tw_g = med(twin["triad"]), med(twin["gather"])
    gbs_twin = {"triad": bytes_triad / tw_t / 1e6, "gather": bytes_gather / tw_g / 1e6}
    ug_t, ug_g = med(ug["triad"]), med(ug["gather"])
    ugbs = {"triad": bytes_triad / ug_t / 1e6, "gather": bytes_gather / ug_g / 1e6}
    dominant = max(("validate", t_v), ("triad", t_t), ("gather", t_g), key=lambda x: x[1])[0]
    avg_ms = {"validate": float(np.mean(t_kern["validate"])),
              "triad": float(np.mean(t_kern["triad"])),
              "gather": float(np.mean(t_kern["gather"]))}
    per_launch = {"validate": bytes_validate, "triad": bytes_triad, "gather": bytes_gather}
    achieved = per_launch[dominant] / avg_ms[dominant] / 1e6
    value = step_bytes / (ms_step / 1e3) / 1e9

    result = {
        "metric": "guarded vs unguarded HBM GB/s (% overhead); ptr validations/s; "
                  "p50/p99 latency",
        "value": round(value, 2),
        "unit": "GB/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_step, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "u64",
        "data": "synthetic",
        "config": {"workload": "large table + bandwidth-bound guarded kernels: 65536 ranges "
                               "(8192 protected), 2^28 validation queries, guarded fp32 triad "
                               "3x1 GiB, guarded gather 2^26 int64 idx over 1 GiB fp32 "
                               "(0.1% hostile)",
                   "queries": nq, "ranges": N_RANGES, "triad_elems": TRIAD_N,
                   "gather_idx": GATHER_N, "gather_rows": GATHER_ROWS},
        "validations_per_s": round(nq / (t_v / 1e3), 1),
        "dma_checks_per_s": round(nq / (med(twin["validate_dma"]) / 1e3), 1),
        "validate_torch": {"formulation": "torch.searchsorted over the sorted bases, then the "
                                          "end, kind and length tests as tensor ops",
                           "kernel_ms": round(med(tval["validate_torch"]), 3),
                           "validations_per_s": round(nq / (med(tval["validate_torch"]) / 1e3), 1),
                           "results_equal": torch_equal},
        "kernel_ms": {"validate": round(t_v, 4), "validate_dma": round(med(twin["validate_dma"]), 4),
                      "triad": round(t_t, 4),
                      "gather": round(t_g, 4), "triad_unguarded": round(ug_t, 4),
                      "gather_sink": round(med(pol["gather_sink"]), 4),
                      "gather_report": round(med(pol["gather_report"]), 4),
                      "gather_remap": round(med(pol["gather_remap"]), 4),
                      "gather_unguarded": round(ug_g, 4),
                      "triad_torch": round(med(tref["triad_torch"]), 4),
                      "gather_torch": round(med(tref["gather_torch"]), 4)},
        "guarded_gbps": {k: round(v, 1) for k, v in gbs.items()},
        "unguarded_gbps": {k: round(v, 1) for k, v in ugbs.items()},
        "guarded_gbps_isolated": {k: round(v, 1) for k, v in gbs_twin.items()},
        "guarded_over_unguarded": {k: round(gbs_twin[k] / ugbs[k], 4) for k in ugbs},
        "overhead_pct": {k: round(100.0 * (ugbs[k] / gbs_twin[k] - 1.0), 2) for k in ugbs},
        "unguarded_frac_of_peak": {k: round(v / PEAK_HBM_GBS, 4) for k, v in ugbs.items()},
        "aperture_check": {
            "workload": f"{nq} queries, same mix, against Table I's three apertures "
                        "(64 GiB I/O, 448 GiB module, 1 TiB user)",
            "kernel_ms": round(med(apt["validate_aperture"]), 4),
            "validations_per_s": round(nq / (med(apt["validate_aperture"]) / 1e3), 1),
            "gbps": round(bytes_validate / med(apt["validate_aperture"]) / 1e6, 1),
            "frac_of_peak": round(bytes_validate / med(apt["validate_aperture"]) / 1e6
                                  / PEAK_HBM_GBS, 4),
            "table_validate_ms": round(t_v, 4),
            "table_over_aperture_time": round(t_v / med(apt["validate_aperture"]), 3)},
        "faults_per_step": n_bad,
        "twin_results_equal": {"triad": ok_triad, "gather": ok_gather},
        "latency_p50_ms": None,
        "latency_p99_ms": None,
        "roofline": {"bound": "hbm", "kernel": dominant, "achieved": round(achieved, 1),
                     "peak": PEAK_HBM_GBS, "unit": "GB/s",
                     "frac": round(achieved / PEAK_HBM_GBS, 4), "traffic": None,
                     "bytes_per_launch": per_launch[dominant]},
    }
    result["roofline"]["traffic"] = measured_traffic(dominant, per_launch[dominant])
    del q, verdict, owner, a, b, c, a_ref, gbuf, table, idx, out, out_ref, qbuf
    vt.close()
    dt.close()
    torch.cuda.empty_cache()
    if not args.no_extras:
        result["small_guard"] = bench_small_guard(g)
        result["table_build"] = bench_table_build(g, tb)
        result["tokens"] = bench_tokens(g)
        torch.cuda.empty_cache()
        result["embedding"] = bench_embedding(g, args)
        torch.cuda.empty_cache()
        result["batch"] = bench_batch(g, args)
        torch.cuda.empty_cache()
    if args.serve_seconds > 0:
        srv = bench_serving(g, args)
        result["serving"] = srv
        result["latency_p50_ms"] = srv["latency_p50_ms"]
        result["latency_p99_ms"] = srv["latency_p99_ms"]
        torch.cuda.empty_cache()
    if not args.no_cpu_baseline:
        result["cpu_baseline"] = cpu_baseline(tb, step_bytes, nq)
    print(json.dumps(result), flush=True)


def time_blocks(calls, warmup, reps):
    """Per callable: `warmup` untimed launches, then `reps` launches each bracketed by HIP events
    on the current stream; every callable gets the same treatment, one after another, so that
    none of them inherits a cache state set up by another."""
    import torch
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    out = {}
    for name, fn in calls.items():
        setup = None
        if isinstance(fn, tuple):  # (untimed set-up before each launch, the timed launch)
            setup, fn = fn
        ts = []
        for rep in range(warmup + reps):
            if setup is not None:
                setup()
            e0.record()
            fn()
            e1.record()
            e1.synchronize()
            if rep >= warmup:
                ts.append(e0.elapsed_time(e1))
        out[name] = ts
    return out


def _kernel_sources_digest(kernel):
    import hashlib
    csrc = os.path.join(ROOT, "paper_2606_06697_amd", "csrc")
    files = {"validate": ["k_validate.hip"], "triad": ["k_stream.hip"],
             "gather": ["k_gather.hip"]}[kernel] + ["guard_device.h", "guard_arith.h", "launch.h"]
    h = hashlib.sha256()
    for f in files:
        with open(os.path.join(csrc, f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()


def measured_traffic(kernel, algorithmic):
    """HBM bytes per launch of `kernel` from the committed counter summary, or None when there
    is none or the kernel's sources changed since the counters were taken."""
    path = os.path.join(ROOT, "profiles", f"traffic_{kernel}_large_table.md")
    if not os.path.exists(path):
        return None
    vals = {}
    with open(path) as fh:
        for line in fh:
            if line.startswith("- ") and ":" in line:
                k, v = line[2:].split(":", 1)
                vals[k.strip()] = v.strip().strip("`")
    if vals.get("kernel_sources_sha256") != _kernel_sources_digest(kernel):
        return None
    try:
        return int(vals["hbm_bytes_per_launch"])
    except (KeyError, ValueError):
        return None


def bench_small_guard(g):
    """Small guard: a 64-range table (16 protected), 10^6 validation queries with the same mix,
    and a guarded 16 MiB fp32 copy with no faults (inputs cache-resident), 50 launches each."""
    import numpy as np
    import torch
    from synth import make_table, make_queries, uniform_f32

    dev = torch.device("cuda:0")
    tb = make_table(64, 16, 0, first_hi=2**47)
    vt = g.RangeTable(64)
    vt.insert_many(tb.base, tb.size, tb.kind)
    n = 1_000_000
    q = make_queries(tb, n, 0, device=dev)
    v = torch.empty(n, dtype=torch.uint8, device=dev)
    o = torch.empty(n, dtype=torch.int32, device=dev)
    src = uniform_f32(1 << 22, 0, device=dev, stream=20)
    dst = torch.empty_like(src)
    dst_u = torch.empty_like(src)
    ct = g.RangeTable(8)                  # real buffers in a table of their own
    ct.insert_tensor(src)
    ct.insert_tensor(dst)
    ts = time_blocks({
        "validate": lambda: g.agile_validate_ptrs(vt.handle, q, n, v, o),
        "copy": lambda: g.agile_guarded_copy(ct.handle, dst, src, 16 << 20),
        "copy_unguarded": lambda: g.agile_unguarded_copy(dst_u, src, 16 << 20),
    }, 5, 50)
    rc, f = ct.fault_log(clear=True)
    assert f["count"] == 0 and torch.equal(dst, src)
    med = {k: float(np.median(x)) for k, x in ts.items()}
    vt.close()
    ct.close()
    return {"workload": "64 ranges (16 protected), 1e6 queries; guarded 16 MiB fp32 copy, "
                        "0 faults",
            "kernel_ms": {k: round(x, 4) for k, x in med.items()},
            "validations_per_s": round(n / (med["validate"] / 1e3), 1),
            "copy_gbps": round(2 * (16 << 20) / med["copy"] / 1e6, 1),
            "copy_unguarded_gbps": round(2 * (16 << 20) / med["copy_unguarded"] / 1e6, 1),
            "copy_guarded_over_unguarded": round(med["copy_unguarded"] / med["copy"], 4)}


def bench_table_build(g, tb):
    """Host-side table maintenance: a bulk build of the 65,536-range table plus its first device
    upload, and single inserts / removes through the C ABI followed by an upload."""
    import numpy as np
    import torch

    reps = []
    for _ in range(3):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        rt = g.RangeTable(N_RANGES + 16)
        rt.insert_many(tb.base, tb.size, tb.kind)
        g.agile_rt_sync(rt.handle)
        torch.cuda.synchronize()
        reps.append(time.perf_counter() - t0)
        rt.close()
    bulk_ms = float(np.median(reps)) * 1e3
    m = 4096
    base, size, kind = tb.base[:m].tolist(), tb.size[:m].tolist(), tb.kind[:m].tolist()
    rt = g.RangeTable(m + 16)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    ids = [rt.insert(b, s, k) for b, s, k in zip(base, size, kind)]
    t1 = time.perf_counter()
    for rid in ids[::4]:
        rt.remove(rid)
    t2 = time.perf_counter()
    g.agile_rt_sync(rt.handle)
    torch.cuda.synchronize()
    t3 = time.perf_counter()
    rt.close()
    return {"workload": "65536-range bulk build + upload; 4096 single inserts, 1024 removes, "
                        "one upload (Python calling the C ABI)",
            "bulk_build_upload_ms": round(bulk_ms, 3),
            "single_inserts_per_s": round(m / (t1 - t0), 1),
            "single_removes_per_s": round((m // 4) / (t2 - t1), 1),
            "upload_after_edits_ms": round((t3 - t2) * 1e3, 3)}


def bench_tokens(g):
    """Client handle tokens: a 2^20-slot table with 2^19 live tokens of 64 clients (a third of
    a further 2^18 released), and a batch of 2^26 presented tokens (live by their owner, by
    other clients, released, bit-flipped), one device check per launch, 20 launches."""
    import numpy as np
    import torch

    rng = np.random.default_rng(5)
    cap, nlive, nrel, n = 1 << 20, 1 << 19, 1 << 18, 1 << 26
    ts = g.TokenTable(cap, 0x5EED_0F_70CE_5)
    owners = rng.integers(0, 64, nlive + nrel)
    t0 = time.perf_counter()
    toks = np.array([ts.mint(int(o), 0) for o in owners.tolist()], np.uint64)
    mint_s = time.perf_counter() - t0
    for i in range(nlive, nlive + nrel, 3):
        ts.release(int(toks[i]), int(owners[i]))
    dev = torch.device("cuda:0")
    pick = torch.from_numpy(rng.integers(0, nlive + nrel, n)).to(dev)
    tok = torch.from_numpy(toks.view(np.int64)).to(dev)[pick]
    cli = torch.from_numpy(owners.astype(np.int32)).to(dev)[pick]
    flip = torch.rand(n, device=dev) < 0.05
    tok = torch.where(flip, tok ^ 1, tok)
    other = torch.rand(n, device=dev) < 0.1
    cli = torch.where(other, (cli + 1) % 64, cli)
    v = torch.empty(n, dtype=torch.uint8, device=dev)
    sl = torch.empty(n, dtype=torch.int32, device=dev)
    ts_ = time_blocks({"check": lambda: g.agile_tokens_check(ts.handle, tok, cli, None, n, v, sl)},
                      3, 20)
    med = float(np.median(ts_["check"]))
    counts = torch.bincount(v.long(), minlength=5).cpu().tolist()
    ts.close()
    return {"workload": "2^20 slots, 2^19 live tokens of 64 clients, 2^26 presented tokens",
            "kernel_ms": round(med, 4),
            "checks_per_s": round(n / (med / 1e3), 1),
            "algorithmic_gbps": round(n * 17 / med / 1e6, 1),
            "verdict_counts": counts,
            "host_mints_per_s": round((nlive + nrel) / mint_s, 1)}


def bench_embedding(g, args):
    """Guarded embedding (1,048,576 x 256 fp32 table, 2^20 Zipf(1.1) indices, 0.01% aimed at a
    protected range right after the table): forward gather and scatter-add backward, guarded
    and unguarded (same kernels with the guard compiled out), and PyTorch's index_select /
    index_add_ on the same work with the out-of-range indices masked, HIP-event medians."""
    import numpy as np
    import torch
    from synth import uniform_f32, zipf_indices

    R, D, N, PAD = 1 << 20, 256, 1 << 20, 16
    rb = D * 4
    dev = torch.device("cuda:0")
    Wbuf = torch.empty((R + PAD) * D, device=dev)
    Wbuf[:R * D].copy_(uniform_f32(R * D, 2, device=dev, stream=30))
    Wbuf[R * D:].fill_(0.0)
    W = Wbuf[:R * D]
    idx = zipf_indices(N, R, 1.1, 2, device=dev, bad_frac=1e-4, bad_ranges=((R, R + PAD),))
    Y = torch.empty(N * D, device=dev)
    dY = uniform_f32(N * D, 2, device=dev, stream=31)
    dWbuf = torch.zeros((R + PAD) * D, device=dev)
    dW = dWbuf[:R * D]
    t = g.RangeTable(16)
    t.insert(W.data_ptr(), R * rb, g.KIND_USER)
    t.insert(W.data_ptr() + R * rb, PAD * rb, g.KIND_PROTECTED)
    for x in (idx, Y, dY):
        t.insert_tensor(x, g.KIND_USER)
    t.insert(dW.data_ptr(), R * rb, g.KIND_USER)
    ih = idx.cpu().numpy()
    distinct = int(np.unique(ih[(ih >= 0) & (ih < R)]).size)
    # PyTorch's own ops on the same work, for context: indices outside the table masked to row 0
    # and their gradient rows zeroed beforehand (outside the timed region)
    bad = (idx < 0) | (idx >= R)
    idx_m = torch.where(bad, torch.zeros_like(idx), idx)
    dY_m = dY.view(N, D).masked_fill(bad[:, None], 0.0)
    W2, Y2, dW2 = W.view(R, D), Y.view(N, D), torch.zeros(R, D, device=dev)
    ts = time_blocks({
        "forward": lambda: g.agile_guarded_gather(t.handle, Y, W, rb, idx, N),
        "forward_unguarded": lambda: g.agile_unguarded_gather(Y, Wbuf, rb, idx, N),
        "backward": lambda: g.agile_guarded_scatter(t.handle, dW, rb, idx, dY, N, 0, 1),
        "backward_unguarded": lambda: g.agile_unguarded_scatter(dWbuf, rb, idx, dY, N, 0, 1),
        "torch_index_select": lambda: torch.index_select(W2, 0, idx_m, out=Y2),
        "torch_index_add": lambda: dW2.index_add_(0, idx_m, dY_m),
        # the autograd path: a zeroed gradient (zeroed before each launch, untimed), summed
        # into without reading its rows
        "backward_into_zeros": (dW.zero_, lambda: g.agile_guarded_scatter(
            t.handle, dW, rb, idx, dY, N, 0, g.SCATTER_ADD_INTO_ZEROS)),
    }, 2, 10)
    rc, f = t.fault_log(clear=True)
    nbad = int(((ih < 0) | (ih >= R)).sum())
    calls_guarded = 3 * 12
    assert int(f["count"]) == nbad * D * calls_guarded, (int(f["count"]), nbad)
    t.close()
    med = {k: float(np.median(v)) for k, v in ts.items()}
    # bytes that must cross HBM: the index, each distinct row once (repeated Zipf rows are
    # served by the caches), the output; backward: dY, the index, a read and a write of every
    # distinct destination row
    fwd_bytes = N * (8 + rb) + distinct * rb
    bwd_bytes = N * (8 + rb) + distinct * 2 * rb
    out = {"workload": "1048576x256 fp32 table, 2^20 Zipf(1.1) idx, 0.01% hostile",
           "kernel_ms": {k: round(v, 4) for k, v in med.items()},
           "forward_gbps": round(fwd_bytes / med["forward"] / 1e6, 1),
           "forward_unguarded_gbps": round(fwd_bytes / med["forward_unguarded"] / 1e6, 1),
           "forward_rows_per_s": round(N / (med["forward"] / 1e3), 1),
           "backward_gbps": round(bwd_bytes / med["backward"] / 1e6, 1),
           "backward_into_zeros_gbps": round((N * (8 + rb) + distinct * rb)
                                             / med["backward_into_zeros"] / 1e6, 1),
           "backward_unguarded_gbps": round(bwd_bytes / med["backward_unguarded"] / 1e6, 1),
           "distinct_rows": distinct, "hostile_idx": nbad,
           "faults_per_call": int(f["count"]) // calls_guarded}
    out["forward_guarded_over_unguarded"] = round(med["forward_unguarded"] / med["forward"], 4)
    out["backward_guarded_over_unguarded"] = round(med["backward_unguarded"] / med["backward"], 4)
    out["torch_index_select_over_forward_time"] = round(med["torch_index_select"] / med["forward"], 3)
    out["torch_index_add_over_backward_time"] = round(med["torch_index_add"] / med["backward"], 3)
    return out


def bench_batch(g, args):
    """One persistent launch of 512 requests from 16 clients (4,096-range tables each): pointer
    arguments (log-uniform 1-4,096 per request) plus one guarded copy per request (log-uniform
    4 KiB-64 MiB)."""
    import numpy as np
    import torch
    from synth import make_table, make_batch_requests

    ncl, nreq = 16, 512
    dev = torch.device("cuda:0")
    tabs = [make_table(4096, 512, 300 + c, first_hi=2**44) for c in range(ncl)]
    reqspec = make_batch_requests(tabs, nreq, 3)
    rts = []
    for tb in tabs:
        rt = g.RangeTable(4096 + nreq + 8)
        rt.insert_many(tb.base, tb.size, tb.kind)
        rts.append(rt)
    client = reqspec["client"].numpy()
    cbytes = reqspec["copy_bytes"].numpy()
    src = [torch.randint(0, 256, (64 << 20,), dtype=torch.uint8, device=dev) for _ in range(ncl)]
    for c in range(ncl):
        rts[c].insert_tensor(src[c], g.KIND_USER)
    dst_total = [int(((cbytes[client == c] + 255) // 256 * 256).sum()) for c in range(ncl)]
    dst = [torch.empty(max(n, 256), dtype=torch.uint8, device=dev) for n in dst_total]
    reqs = np.zeros(nreq, dtype=g.REQUEST_DTYPE)
    off = [0] * ncl
    rng = np.random.default_rng(5)
    for r in range(nreq):
        c = int(client[r])
        nb = int(cbytes[r])
        d = dst[c].data_ptr() + off[c]
        rts[c].insert(d, nb, g.KIND_USER)            # each request's output is its own allocation
        off[c] += (nb + 255) // 256 * 256
        reqs[r]["client"] = c
        reqs[r]["ptr_off"] = int(reqspec["ptr_off"][r])
        reqs[r]["nptr"] = int(reqspec["ptr_off"][r + 1] - reqspec["ptr_off"][r])
        reqs[r]["copy_dst"] = d
        reqs[r]["copy_src"] = src[c].data_ptr() + int(rng.integers(0, ((64 << 20) - nb) // 16 + 1)) * 16
        reqs[r]["copy_bytes"] = nb
    P = reqspec["ptrs"].to(dev)
    nptrs = P.shape[0]
    pv = torch.empty(nptrs, dtype=torch.uint8, device=dev)
    po = torch.empty(nptrs, dtype=torch.int32, device=dev)
    res = torch.empty(nreq * g.RESULT_DTYPE.itemsize, dtype=torch.uint8, device=dev)
    cs = g.agile_clients_create(rts)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    ts = []
    for rep in range(2 + 5):
        e0.record()
        g.agile_batch_run(cs, reqs, P, nptrs, pv, po, res)
        e1.record()
        e1.synchronize()
        if rep >= 2:
            ts.append(e0.elapsed_time(e1))
    out_res = g.batch_results(res, nreq)
    g.agile_clients_destroy(cs)
    for rt in rts:
        rt.close()
    ms = float(np.median(ts))
    moved = int(cbytes.sum()) * 2
    return {"workload": "16 clients x 4096 ranges, 512 requests/launch, 1-4096 ptrs + one "
                        "4 KiB-64 MiB guarded copy per request",
            "launch_ms": round(ms, 4), "pointers": int(nptrs), "copy_bytes": int(cbytes.sum()),
            "copy_gbps": round(moved / ms / 1e6, 1),
            "validations_per_s": round(nptrs / (ms / 1e3), 1),
            "requests_failing_validation": int((out_res["verdict"] != 0).sum()),
            "requests_done": int(out_res["done"].sum())}


def bench_serving(g, args):
    """64 clients, Poisson arrivals at 20,000 requests/s, 50% validate / 30% copy / 20% gather,
    per-client tables of 1,024-8,192 ranges, 32 GiB budget for in-flight outputs."""
    from paper_2606_06697_amd.serving import Server, ServeConfig
    from synth import make_serving_trace

    cfg = ServeConfig(duration=args.serve_seconds)
    srv = Server(cfg)
    trace = make_serving_trace(cfg.n_clients, cfg.rate, cfg.duration, cfg.seed, mix=cfg.mix,
                               val_ptrs=cfg.val_ptrs, copy_range=cfg.copy_range,
                               gather_range=cfg.gather_range)
    lat, stats, _ = srv.run(trace)
    srv.close()
    stats = {k: (round(v, 4) if isinstance(v, float) else v) for k, v in stats.items()}
    stats["workload"] = (f"64 clients, Poisson 20000 req/s for {cfg.duration:g} s, "
                         "50/30/20 validate/copy/gather")
    return stats


def bench_serving_capacity(g, args):
    """The serving workload's server (64 clients, same mix and tables) offered more load: 2 s
    Poisson traces at 20,000 to 1,600,000 requests/s. Completed requests/s stops following the
    offered rate where the loop saturates; latency is arrival to completion (host clock)."""
    from paper_2606_06697_amd.serving import Server, ServeConfig
    from synth import make_serving_trace

    cfg = ServeConfig(duration=2.0)
    srv = Server(cfg)
    rows = []
    for rate in (20000.0, 50000.0, 100000.0, 200000.0, 400000.0, 800000.0, 1600000.0):
        trace = make_serving_trace(cfg.n_clients, rate, cfg.duration, cfg.seed, mix=cfg.mix,
                                   val_ptrs=cfg.val_ptrs, copy_range=cfg.copy_range,
                                   gather_range=cfg.gather_range)
        _, st, _ = srv.run(trace)
        rows.append({"offered_per_s": rate, "requests": st["requests"],
                     "completed_per_s": round(st["requests_per_s"], 1),
                     "latency_p50_ms": round(st["latency_p50_ms"], 4),
                     "latency_p99_ms": round(st["latency_p99_ms"], 4),
                     "mean_batch": round(st["mean_batch"], 2), "launches": st["launches"],
                     "moved_gb_per_s": round(st["moved_gb_per_s"], 1), "refused": st["refused"]})
        print(json.dumps(rows[-1]), file=sys.stderr, flush=True)
    srv.close()
    return {"workload": "64 clients, 50/30/20 validate/copy/gather, 2 s Poisson traces at "
                        "increasing offered rates", "rates": rows}


def _pool_validate_worker(args):
    """One process of the pooled oracle validation: rebuild the table from its arrays, wait for
    the others, classify its slice of the shared query array."""
    import numpy as np
    from multiprocessing import shared_memory
    from oracle.table import RangeTable as OT
    shm_name, n, lo, hi, base, size, kind, barrier = args
    ot = OT()
    for bb, s, k in zip(base, size, kind):
        ot.insert(bb, s, k)
    shm = shared_memory.SharedMemory(name=shm_name)
    try:
        q = np.ndarray((n, 2), dtype=np.uint64, buffer=shm.buf)
        barrier.wait()
        t0 = time.perf_counter()
        ot.verdict_many(q[lo:hi, 0], q[lo:hi, 1])
        return time.perf_counter() - t0
    finally:
        del q
        shm.close()


def cpu_pool_validate(tb, qs, procs):
    """The oracle's validation of the same queries split over `procs` processes (spawned: they
    never touch the GPU); wall time from a common start."""
    import multiprocessing as mp
    from multiprocessing import shared_memory
    import numpy as np

    n = qs.shape[0]
    shm = shared_memory.SharedMemory(create=True, size=qs.nbytes)
    try:
        np.ndarray(qs.shape, dtype=qs.dtype, buffer=shm.buf)[:] = qs
        ctx = mp.get_context("spawn")
        with ctx.Manager() as man:
            barrier = man.Barrier(procs + 1)
            cuts = np.linspace(0, n, procs + 1).astype(np.int64)
            tab = (tb.base.tolist(), tb.size.tolist(), tb.kind.tolist())
            with ctx.Pool(procs) as pool:
                res = pool.map_async(_pool_validate_worker,
                                     [(shm.name, n, int(cuts[k]), int(cuts[k + 1]), *tab, barrier)
                                      for k in range(procs)])
                barrier.wait()
                t0 = time.perf_counter()
                res.get()
                wall = time.perf_counter() - t0
    finally:
        shm.close()
        shm.unlink()
    return wall


def cpu_model():
    """The host CPU's model name (from /proc/cpuinfo), or the machine type."""
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return platform.processor() or platform.machine()


def cpu_baseline(tb, step_bytes, nq):
    """Time the oracle (as it stands) on a bounded sample of the same workload (about 10 s of
    single-thread CPU work) and scale each part to its full size."""
    import numpy as np
    import torch

    from oracle.table import RangeTable as OT
    from oracle.memory import Memory
    from oracle import guarded as G
    from synth import make_queries, uniform_f32, uniform_indices

    ot = OT()
    for bb, s, k in zip(tb.base.tolist(), tb.size.tolist(), tb.kind.tolist()):
        ot.insert(bb, s, k)
    nsv = 1 << 26
    qs = make_queries(tb, nsv, SEED + 100).numpy().view(np.uint64)
    t0 = time.perf_counter()
    ot.verdict_many(qs[:, 0], qs[:, 1])
    tv = time.perf_counter() - t0

    nst = 1 << 25
    base = 1 << 40
    mt, tt = Memory(), OT()
    for k, arr in enumerate((np.zeros(nst, np.float32), uniform_f32(nst, 5).numpy(),
                             uniform_f32(nst, 6).numpy())):
        tt.insert(base + k * (1 << 30), 4 * nst, 0)
        mt.add(base + k * (1 << 30), arr.view(np.uint8))
    t0 = time.perf_counter()
    G.triad_vec(tt, mt, G.FaultLog(), 0, base, base + (1 << 30), base + (2 << 30), 3.0, nst)
    ttr = time.perf_counter() - t0

    nsg, rows = 1 << 21, 1 << 24
    mg, tg = Memory(), OT()
    idx = uniform_indices(nsg, rows, 7, bad_frac=0.001,
                          bad_ranges=((rows, rows + 16384), (rows + 16384, rows + 32768))).numpy()
    tg.insert(base, rows * 4, 0)
    tg.insert(base + rows * 4, PAD_BYTES, 1)
    mg.add(base, uniform_f32(rows, 8).numpy().view(np.uint8))
    tg.insert(base + (1 << 30), nsg * 8, 0)
    mg.add(base + (1 << 30), idx.view(np.uint8))
    tg.insert(base + (2 << 30), nsg * 4, 0)
    mg.add(base + (2 << 30), np.zeros(nsg * 4, np.uint8))
    t0 = time.perf_counter()
    G.gather_vec(tg, mg, G.FaultLog(), 0, base + (2 << 30), base, 4, base + (1 << 30), nsg)
    tgt = time.perf_counter() - t0

    procs = max(1, min(16, os.cpu_count() or 1))
    try:
        tpool = cpu_pool_validate(tb, qs, procs)
        pool = {"processes": procs, "seconds": round(tpool, 3),
                "validations_per_s": round(nsv / tpool, 1),
                "sample": f"the same {nsv} queries split over {procs} spawned processes"}
    except Exception as e:  # a host without process support still reports the single thread
        pool = {"error": str(e)[:200]}
    cpu_step = tv * nq / nsv + ttr * TRIAD_N / nst + tgt * GATHER_N / nsg
    return {"value": round(step_bytes / cpu_step / 1e9, 4), "unit": "GB/s", "cores": 1,
            "kind": "oracle",
            "sample": f"validate {nsv} queries on the same 65536-range table ({tv:.2f} s), "
                      f"triad {nst} elems ({ttr:.2f} s), gather {nsg} idx over {rows} rows "
                      f"({tgt:.2f} s); each scaled to its full size; host CPU "
                      f"{cpu_model()}, {os.cpu_count()} cpus visible, numpy single-threaded",
            "validations_per_s": round(nsv / tv, 1),
            "pool_validate": pool}


if __name__ == "__main__":
    main()
