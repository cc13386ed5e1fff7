"""Worker-side request loop with continuous batching over ``agile_batch_run``.

The paper's scheduler assigns clients to a worker that owns the device context and executes
their mediated requests (AgileOS Section IV-B); every pointer argument is checked against the
calling client's own allocations before the real work runs (Sections IV-C, IV-E). This loop
serves many clients from one process:

* every client keeps a device-resident range table (synthetic ranges plus its real buffers: a
  gather table, an index pool, a copy source and an output ring), gathered once into a client
  set;
* requests arrive open-loop at their trace times (validate a slice of pointers, guarded copy,
  guarded gather); arrived requests wait in a FIFO;
* admission: a request is admitted when its output fits in its client's output ring and in
  the global HBM budget for in-flight outputs, and a launch slot (stream) is free;
* every poll retires finished launches (their event completed: latencies are recorded, output
  space is returned) and launches the admitted requests as one persistent batch on a free
  stream, so new work overlaps the batches already on the device;
* revocation (Section IV-D, lifetime and revocation: a client's resources are revoked when its
  assignment ends): at a given time every range of the client's table is removed while other
  batches are still on the device, and its requests from then on are refused without a launch.
  Launches made before keep the table they were made with (the library's two table images).

Latency = completion seen by the loop minus arrival, on the host clock.
"""
from __future__ import annotations

import collections
import time
from dataclasses import dataclass, field

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


class _Ring:
    """Output ring of one client: bump allocation, frees in any order, space reclaimed in order."""

    def __init__(self, base, size):
        self.base, self.size = base, size
        self.head = 0      # next allocation offset (monotone, wraps by modulo)
        self.tail = 0      # oldest live byte
        self.live = collections.OrderedDict()  # alloc start -> [length, freed]

    def alloc(self, n):
        n = (n + 255) & ~255
        start = self.head
        off = start % self.size
        if off + n > self.size:                   # skip the wrap gap
            start += self.size - off
            off = 0
        if start + n - self.tail > self.size:
            return None
        self.head = start + n
        self.live[start] = [n, False]
        return start, self.base + off

    def free(self, start):
        self.live[start][1] = True
        while self.live:
            k, (n, freed) = next(iter(self.live.items()))
            if not freed:
                break
            self.live.popitem(last=False)
            self.tail = k + n
        if not self.live:
            self.head = self.tail = 0     # empty: start over at the ring's base


@dataclass
class _Inflight:
    event: object
    rids: np.ndarray
    allocs: list
    nbytes: int
    slot: int
    reqs: np.ndarray = field(default=None)


class Server:
    def __init__(self, cfg: ServeConfig, device="cuda"):
        from synth import make_table, make_queries, loguniform_int
        from synth.workloads import _gen

        self.cfg = cfg
        self.dev = torch.device(device)
        gen = _gen(cfg.seed, 20)
        nr = loguniform_int(cfg.ranges[0], cfg.ranges[1], cfg.n_clients, gen).tolist()
        self.tables, self.rings, self.range_ids, self.synth_tables = [], [], [], []
        self.gtab, self.gidx, self.csrc, self.ring_mem = [], [], [], []
        ptr_chunks = []
        for c in range(cfg.n_clients):
            tb = make_table(nr[c], max(1, nr[c] // 8), cfg.seed * 1000 + c, first_hi=2**44)
            rt = g.RangeTable(nr[c] + 16)
            ids = rt.insert_many(tb.base, tb.size, tb.kind).tolist()
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
                ids.append(rt.insert_tensor(t, g.KIND_USER))
            self.tables.append(rt)
            self.range_ids.append(ids)
            self.synth_tables.append(tb)
            self.gtab.append(gt)
            self.gidx.append(idx)
            self.csrc.append(src)
            self.ring_mem.append(ring)
            self.rings.append(_Ring(ring.data_ptr(), cfg.ring_bytes))
            ptr_chunks.append(make_queries(tb, cfg.ptr_pool, cfg.seed * 7 + c, device=self.dev))
        self.ptrs = torch.cat(ptr_chunks, 0).contiguous()
        self.nptrs = self.ptrs.shape[0]
        self.pv = torch.empty(self.nptrs, dtype=torch.uint8, device=self.dev)
        self.po = torch.empty(self.nptrs, dtype=torch.int32, device=self.dev)
        self.cs = g.agile_clients_create(self.tables, self.dev.index or 0)
        self.revoked_at = {}
        self.streams = [torch.cuda.Stream(device=self.dev) for _ in range(cfg.max_inflight)]
        self.results = [torch.empty(cfg.max_batch * g.RESULT_DTYPE.itemsize, dtype=torch.uint8,
                                    device=self.dev) for _ in range(cfg.max_inflight)]
        torch.cuda.synchronize(self.dev)

    def close(self):
        torch.cuda.synchronize(self.dev)
        if self.cs:
            g.agile_clients_destroy(self.cs)
            self.cs = None
        for rt in self.tables:
            rt.close()
        self.tables = []

    def revoke(self, client, when=0.0):
        """End a client's assignment: remove every range of its table (later launches see an
        empty table) and refuse its requests from now on."""
        rt = self.tables[client]
        for rid in self.range_ids[client]:
            rt.remove(rid)
        self.range_ids[client] = []
        self.revoked_at[client] = when

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
        """Serve a trace; returns latencies (s) per request, completion order and stats.

        record: optional set of request ids whose results and outputs are copied to host at
        completion (for identity checks). revoke: optional {client: time in s}; the client is
        revoked at the first poll at or after that trace time. Afterwards ``self.t_launch``
        holds each request's launch time (NaN if refused) and ``self.refused`` which requests
        were refused."""
        cfg = self.cfg
        reqs, out_bytes = self.make_requests(trace)
        arr = trace["t"].numpy()
        n = arr.size
        lat = np.full(n, np.nan)
        t_launch = np.full(n, np.nan)
        refused = np.zeros(n, dtype=bool)
        due = sorted((t, c) for c, t in (revoke or {}).items())
        kept = {}
        pending = collections.deque()
        inflight = []
        free_slots = list(range(cfg.max_inflight))
        inflight_bytes = 0
        nxt = 0
        done = 0
        launches = 0
        moved = 0
        t0 = time.perf_counter()
        while done < n:
            now = time.perf_counter() - t0
            # retire finished launches
            still = []
            for b in inflight:
                if b.event.query():
                    fin = time.perf_counter() - t0
                    lat[b.rids] = fin - arr[b.rids]
                    done += b.rids.size
                    if record is not None:
                        self._record(b, record, kept)
                    for c, start in b.allocs:
                        self.rings[c].free(start)
                    inflight_bytes -= b.nbytes
                    free_slots.append(b.slot)
                else:
                    still.append(b)
            inflight = still
            # revocations that are due, while other batches may still be on the device
            while due and due[0][0] <= now:
                self.revoke(due.pop(0)[1], now)
            # arrivals
            while nxt < n and arr[nxt] <= now:
                pending.append(nxt)
                nxt += 1
            # admission + launch
            if pending and free_slots:
                take, allocs, nbytes = [], [], 0
                while pending and len(take) < cfg.max_batch:
                    r = pending[0]
                    if int(reqs["client"][r]) in self.revoked_at:
                        pending.popleft()
                        refused[r] = True
                        done += 1
                        continue
                    need = int(out_bytes[r])
                    if inflight_bytes + nbytes + need > cfg.hbm_budget:
                        break
                    c = int(reqs["client"][r])
                    a = None
                    if need:
                        a = self.rings[c].alloc(need)
                        if a is None:
                            break
                        if reqs["copy_bytes"][r]:
                            reqs["copy_dst"][r] = a[1]
                        else:
                            reqs["gather_out"][r] = a[1]
                        allocs.append((c, a[0]))
                    take.append(pending.popleft())
                    nbytes += need
                if take:
                    slot = free_slots.pop()
                    rids = np.array(take, dtype=np.int64)
                    batch = reqs[rids]
                    st = self.streams[slot]
                    g.agile_batch_run(self.cs, batch, self.ptrs, self.nptrs, self.pv, self.po,
                                      self.results[slot], stream=st)
                    ev = torch.cuda.Event()
                    ev.record(st)
                    t_launch[rids] = now
                    inflight.append(_Inflight(ev, rids, allocs, nbytes, slot, batch))
                    inflight_bytes += nbytes
                    launches += 1
                    moved += int(batch["copy_bytes"].sum() * 2 + batch["gather_n"].sum() * 16)
                    continue
            if not inflight and not pending and nxt < n:
                # idle until the next arrival
                wait = arr[nxt] - (time.perf_counter() - t0)
                if wait > 0.0002:
                    time.sleep(wait - 0.0001)
        elapsed = time.perf_counter() - t0
        ok = ~np.isnan(lat)
        stats = {
            "requests": int(ok.sum()),
            "elapsed_s": elapsed,
            "requests_per_s": float(ok.sum() / elapsed),
            "latency_p50_ms": float(np.percentile(lat[ok], 50) * 1e3) if ok.any() else None,
            "latency_p99_ms": float(np.percentile(lat[ok], 99) * 1e3) if ok.any() else None,
            "launches": launches,
            "mean_batch": float(ok.sum() / max(launches, 1)),
            "moved_gb_per_s": moved / elapsed / 1e9,
            "refused": int(refused.sum()),
        }
        self.t_launch, self.refused = t_launch, refused
        return lat, stats, kept

    def _record(self, b, record, kept):
        res = g.batch_results(self.results[b.slot], b.rids.size)
        for k, r in enumerate(b.rids.tolist()):
            if r not in record:
                continue
            q = b.reqs[k]
            c = int(q["client"])
            ring = self.ring_mem[c]
            base = ring.data_ptr()
            out = None
            if q["copy_bytes"]:
                o = int(q["copy_dst"]) - base
                out = ring[o:o + int(q["copy_bytes"])].cpu().numpy().copy()
            elif q["gather_n"]:
                o = int(q["gather_out"]) - base
                out = ring[o:o + int(q["gather_n"]) * 4].cpu().numpy().copy()
            pv = po = None
            if q["nptr"]:
                a, e = int(q["ptr_off"]), int(q["ptr_off"] + q["nptr"])
                pv, po = self.pv[a:e].cpu().numpy().copy(), self.po[a:e].cpu().numpy().copy()
            kept[r] = (res[k].copy(), out, pv, po, q.copy())

    def run_alone(self, q):
        """Run one request by itself (same output address) and return (result, out, pv, po)."""
        st = self.streams[0]
        one = np.array([q], dtype=g.REQUEST_DTYPE)
        g.agile_batch_run(self.cs, one, self.ptrs, self.nptrs, self.pv, self.po, self.results[0],
                          stream=st)
        st.synchronize()
        res = g.batch_results(self.results[0], 1)[0]
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
