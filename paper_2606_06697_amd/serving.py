"""Worker-side request serving with continuous batching: a thin Python front end over the
library's native serving loop (``agile_server_run``).

The paper's scheduler assigns clients to a worker that owns the device context and executes
their mediated requests (AgileOS Section IV-B); every pointer argument is checked against the
calling client's own allocations before the real work runs (Sections IV-C, IV-E). This module
sets up many clients in one process:

* every client keeps a device-resident range table (synthetic ranges plus its real buffers: a
  gather table, an index pool, a copy source and an output ring), gathered once into a client
  set;
* a trace gives each request's arrival time and operation (validate a slice of pointers,
  guarded copy, guarded gather).

The native loop (C++, host side) serves the trace open-loop: arrived requests wait in a FIFO; a
request is admitted when its output fits in its client's output ring and in the global HBM
budget for in-flight outputs and a launch slot (stream) is free; every poll retires finished
launches (their event completed: latencies are recorded, output space is returned) and launches
the admitted requests as one persistent batch on a free stream, so new work overlaps the
batches already on the device. Revocation (Section IV-D, lifetime and revocation): at a given
time every range of a client's table is removed while other batches are still on the device,
and its requests from then on are refused; launches made before keep the table they were made
with (the library's two table images).

Latency = completion seen by the loop minus arrival, on the host clock.
"""
from __future__ import annotations

from dataclasses import dataclass

import numpy as np
import torch

from . import guard as g

OP_VALIDATE, OP_COPY, OP_GATHER = 0, 1, 2


@dataclass
class ServeConfig:
    n_clients: int = 64
    rate: float = 20000.0
    duration: float = 60.0
    ranges: tuple = (1024, 8192)        # per-client synthetic ranges, log-uniform
    gather_table_bytes: int = 256 << 20
    idx_pool: int = 1 << 20
    copy_src_bytes: int = 16 << 20
    ptr_pool: int = 1 << 16
    ring_bytes: int = 512 << 20         # per-client output ring
    hbm_budget: int = 32 << 30          # in-flight output bytes, all clients
    max_batch: int = 512
    max_inflight: int = 4
    val_ptrs: tuple = (16, 1024)
    copy_range: tuple = (4096, 16 << 20)
    gather_range: tuple = (1 << 12, 1 << 20)
    mix: tuple = (0.5, 0.3, 0.2)
    bad_idx_frac: float = 0.001
    seed: int = 4


class Server:
    def __init__(self, cfg: ServeConfig, device="cuda"):
        from synth import make_table, make_queries, loguniform_int
        from synth.workloads import _gen

        self.cfg = cfg
        self.dev = torch.device(device)
        gen = _gen(cfg.seed, 20)
        nr = loguniform_int(cfg.ranges[0], cfg.ranges[1], cfg.n_clients, gen).tolist()
        self.tables, self.synth_tables = [], []
        self.gtab, self.gidx, self.csrc, self.ring_mem = [], [], [], []
        ptr_chunks = []
        for c in range(cfg.n_clients):
            tb = make_table(nr[c], max(1, nr[c] // 8), cfg.seed * 1000 + c, first_hi=2**44)
            rt = g.RangeTable(nr[c] + 16)
            rt.insert_many(tb.base, tb.size, tb.kind)
            gt = torch.rand(cfg.gather_table_bytes // 4, device=self.dev)
            rows = gt.numel()
            idx = torch.randint(0, rows, (cfg.idx_pool,), device=self.dev)
            nbad = int(cfg.idx_pool * cfg.bad_idx_frac)
            if nbad:
                pos = torch.randperm(cfg.idx_pool, device=self.dev)[:nbad]
                idx[pos] = rows + torch.arange(nbad, device=self.dev)   # past the table
            src = torch.randint(0, 256, (cfg.copy_src_bytes,), dtype=torch.uint8, device=self.dev)
            ring = torch.empty(cfg.ring_bytes, dtype=torch.uint8, device=self.dev)
            for t in (gt, idx, src, ring):
                rt.insert_tensor(t, g.KIND_USER)
            self.tables.append(rt)
            self.synth_tables.append(tb)
            self.gtab.append(gt)
            self.gidx.append(idx)
            self.csrc.append(src)
            self.ring_mem.append(ring)
            ptr_chunks.append(make_queries(tb, cfg.ptr_pool, cfg.seed * 7 + c, device=self.dev))
        self.ptrs = torch.cat(ptr_chunks, 0).contiguous()
        self.nptrs = self.ptrs.shape[0]
        self.pv = torch.empty(self.nptrs, dtype=torch.uint8, device=self.dev)
        self.po = torch.empty(self.nptrs, dtype=torch.int32, device=self.dev)
        self.cs = g.agile_clients_create(self.tables, self.dev.index or 0)
        self.revoked_at = {}
        self.sv = g.agile_server_create(
            self.cs, self.tables, [r.data_ptr() for r in self.ring_mem],
            [cfg.ring_bytes] * cfg.n_clients, cfg.max_batch, cfg.max_inflight, cfg.hbm_budget,
            self.ptrs, self.nptrs, self.pv, self.po, self.dev.index or 0)
        self.alone_stream = torch.cuda.Stream(device=self.dev)
        self.alone_result = torch.empty(g.RESULT_DTYPE.itemsize, dtype=torch.uint8,
                                        device=self.dev)
        torch.cuda.synchronize(self.dev)

    def close(self):
        torch.cuda.synchronize(self.dev)
        if getattr(self, "sv", None):
            g.agile_server_destroy(self.sv)
            self.sv = None
        if self.cs:
            g.agile_clients_destroy(self.cs)
            self.cs = None
        for rt in self.tables:
            rt.close()
        self.tables = []

    def revoke(self, client):
        """End a client's assignment between runs: remove every range of its table."""
        g.agile_rt_clear(self.tables[client].handle)

    # ------------------------------------------------------------------ requests
    def make_requests(self, trace):
        """Static part of every request of a trace (everything but the output address)."""
        cfg = self.cfg
        n = trace["t"].numel()
        rng = np.random.default_rng(cfg.seed + 99)
        client = trace["client"].numpy().astype(np.uint32)
        op = trace["op"].numpy()
        size = trace["size"].numpy().astype(np.int64)
        reqs = np.zeros(n, dtype=g.REQUEST_DTYPE)
        reqs["client"] = client
        v = op == OP_VALIDATE
        start = rng.integers(0, cfg.ptr_pool - cfg.val_ptrs[1], n)
        reqs["ptr_off"][v] = client[v].astype(np.uint64) * cfg.ptr_pool + start[v]
        reqs["nptr"][v] = size[v]
        cp = op == OP_COPY
        srcb = np.array([t.data_ptr() for t in self.csrc], dtype=np.uint64)
        room = np.maximum(cfg.copy_src_bytes - size, 0) // 16 + 1
        src_off = (rng.integers(0, 1 << 62, n) % room) * 16
        reqs["copy_src"][cp] = srcb[client[cp]] + src_off[cp].astype(np.uint64)
        reqs["copy_bytes"][cp] = size[cp]
        ga = op == OP_GATHER
        tb = np.array([t.data_ptr() for t in self.gtab], dtype=np.uint64)
        ib = np.array([t.data_ptr() for t in self.gidx], dtype=np.uint64)
        off = rng.integers(0, cfg.idx_pool, n) % np.maximum(cfg.idx_pool - size + 1, 1)
        reqs["gather_table"][ga] = tb[client[ga]]
        reqs["gather_idx"][ga] = ib[client[ga]] + (off[ga] * 8).astype(np.uint64)
        reqs["gather_n"][ga] = size[ga]
        reqs["gather_row_bytes"][ga] = 4
        out_bytes = np.where(cp, size, np.where(ga, size * 4, 0))
        return reqs, out_bytes

    # ------------------------------------------------------------------ the loop
    def run(self, trace, record=None, revoke=None):
        """Serve a trace with the native loop; returns (latency in s per request, stats, kept).

        record: optional set of request ids whose results and outputs (and, for validation, the
        pointer verdicts and owners) are copied to host at completion, kept[r] = (result,
        output bytes or None, verdicts or None, owners or None, request). revoke: optional
        {client: time in s}. Afterwards ``self.t_launch`` holds each request's launch time (NaN
        if refused), ``self.refused`` which requests were refused and ``self.revoked_at`` when
        each revocation took effect."""
        reqs, out_bytes = self.make_requests(trace)
        reqs = np.ascontiguousarray(reqs)
        arr = trace["t"].numpy().astype(np.float64)
        n = arr.size
        rec = rec_off = rec_buf = None
        if record:
            rec = np.zeros(n, np.uint8)
            ids = np.array(sorted(record), dtype=np.int64)
            rec[ids] = 1
            need = out_bytes.astype(np.uint64) + reqs["nptr"] * 5
            rec_off = np.zeros(n, np.uint64)
            rec_off[ids] = np.concatenate([[0], np.cumsum(need[ids])[:-1]]).astype(np.uint64)
            rec_buf = np.empty(int(need[ids].sum()) + 1, np.uint8)
        rcl = rts = None
        if revoke:
            rcl = np.array(list(revoke.keys()), np.uint32)
            rts = np.array([revoke[c] for c in revoke], np.float64)
        lat, t_launch, res, st = g.agile_server_run(self.sv, reqs, out_bytes, arr, rcl, rts, rec,
                                                    rec_buf, rec_off)
        self.t_launch = t_launch
        self.refused = np.isnan(t_launch)
        if revoke:
            self.revoked_at = {int(c): st.revoked_at_s[k] for k, c in enumerate(rcl.tolist())}
        kept = {}
        for r in (sorted(record) if record else []):
            if self.refused[r]:
                continue
            q = reqs[r].copy()
            o, nb, npt = int(rec_off[r]), int(out_bytes[r]), int(q["nptr"])
            out = rec_buf[o:o + nb].copy() if nb else None
            pv = po = None
            if npt:
                pv = rec_buf[o + nb:o + nb + npt].copy()
                po = rec_buf[o + nb + npt:o + nb + 5 * npt].copy().view(np.int32)
            kept[r] = (res[r].copy(), out, pv, po, q)
        ok = ~np.isnan(lat)
        served = ~self.refused
        moved = int(reqs["copy_bytes"][served].sum() * 2 + reqs["gather_n"][served].sum() * 16)
        stats = {
            "requests": int(ok.sum()),
            "elapsed_s": st.elapsed_s,
            "requests_per_s": float(ok.sum() / st.elapsed_s),
            "latency_p50_ms": float(np.percentile(lat[ok], 50) * 1e3) if ok.any() else None,
            "latency_p99_ms": float(np.percentile(lat[ok], 99) * 1e3) if ok.any() else None,
            "launches": int(st.launches),
            "mean_batch": float(ok.sum() / max(st.launches, 1)),
            "moved_gb_per_s": moved / st.elapsed_s / 1e9,
            "refused": int(st.refused),
            "max_inflight_bytes": int(st.max_inflight_bytes),
            "max_concurrent_launches": int(st.max_concurrent),
            "budget_waits": int(st.budget_waits),
            "ring_waits": int(st.ring_waits),
        }
        return lat, stats, kept

    def run_alone(self, q):
        """Run one request by itself (same output address) and return (result, out, pv, po)."""
        st = self.alone_stream
        one = np.array([q], dtype=g.REQUEST_DTYPE)
        g.agile_batch_run(self.cs, one, self.ptrs, self.nptrs, self.pv, self.po,
                          self.alone_result, stream=st)
        st.synchronize()
        res = g.batch_results(self.alone_result, 1)[0]
        c = int(q["client"])
        ring = self.ring_mem[c]
        base = ring.data_ptr()
        out = None
        if q["copy_bytes"]:
            o = int(q["copy_dst"]) - base
            out = ring[o:o + int(q["copy_bytes"])].cpu().numpy()
        elif q["gather_n"]:
            o = int(q["gather_out"]) - base
            out = ring[o:o + int(q["gather_n"]) * 4].cpu().numpy()
        pv = po = None
        if q["nptr"]:
            a, e = int(q["ptr_off"]), int(q["ptr_off"] + q["nptr"])
            pv, po = self.pv[a:e].cpu().numpy(), self.po[a:e].cpu().numpy()
        return res, out, pv, po
