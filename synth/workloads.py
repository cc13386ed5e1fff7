"""Seeded generators for the range-guard workloads.

Every generator is a pure function of its seed (and device): a ``torch.Generator``
seeded from ``(seed, stream)`` drives each component, so the same call gives the same
tensors on the same device. Addresses are produced as int64 (all generated addresses
are below 2**48, so the int64 bit pattern equals the uint64 address); consumers
reinterpret them as uint64.

Recipes (the paper prints no workload; these follow the threat model of the paper's
Section III: valid, protected, straddling and unmapped pointers):

* Table: ``n`` disjoint ranges, ``n_protected`` of them protected (a quarter of those
  MMIO-like), kinds shuffled. USER sizes are log-uniform integers in [256 B, 1 MiB]
  (byte-granular ends), protected sizes uniform integers in [4 KiB, 64 KiB]. The first
  base is a random page in ``[first_lo, first_hi)``; each later base is the previous
  end rounded up to a 4 KiB page plus ``4096*G``, ``G ~ U{0..16}``. Generation order is
  address order, so insertion id ``i`` is the ``i``-th range by address.
* Queries ``(addr, len)``: 60% inside a USER range (len log-uniform in [1, min(4096,size)]),
  20% starting inside a protected range (len log-uniform in [1, 4096]), 10% straddling
  (half leave a USER range across its end, half enter a range from the hole below it),
  10% wholly inside a hole. Categories are shuffled.
"""
from __future__ import annotations

import math
from dataclasses import dataclass

import torch

PAGE = 4096
KIND_USER, KIND_PROTECTED, KIND_MMIO = 0, 1, 2


def _gen(seed: int, stream: int, device="cpu") -> torch.Generator:
    g = torch.Generator(device=device)
    g.manual_seed((int(seed) * 1_000_003 + int(stream)) & 0x7FFF_FFFF_FFFF_FFFF)
    return g


def loguniform_int(lo, hi, n: int, g: torch.Generator, device="cpu") -> torch.Tensor:
    """Integers in [lo, hi] (inclusive, elementwise if tensors) with log-uniform density."""
    lo_t = torch.as_tensor(lo, dtype=torch.float64, device=device)
    hi_t = torch.as_tensor(hi, dtype=torch.float64, device=device)
    u = torch.rand(n, generator=g, device=device, dtype=torch.float64)
    v = torch.exp(torch.log(lo_t) + u * (torch.log(hi_t + 1.0) - torch.log(lo_t)))
    v = torch.floor(v)
    v = torch.minimum(torch.maximum(v, lo_t), hi_t)
    return v.to(torch.int64)


def _uniform_below(m: torch.Tensor, g: torch.Generator) -> torch.Tensor:
    """Integers uniform in [0, m) elementwise (m >= 1, m < 2**52)."""
    u = torch.rand(m.shape, generator=g, device=m.device, dtype=torch.float64)
    r = torch.floor(u * m.to(torch.float64)).to(torch.int64)
    return torch.minimum(r, m - 1)


@dataclass
class Table:
    """A generated range table in insertion (= address) order."""
    base: torch.Tensor   # int64 [n]
    size: torch.Tensor   # int64 [n]
    kind: torch.Tensor   # uint8 [n]

    @property
    def n(self) -> int:
        return int(self.base.numel())

    @property
    def end(self) -> torch.Tensor:
        return self.base + self.size

    def to(self, device) -> "Table":
        return Table(self.base.to(device), self.size.to(device), self.kind.to(device))


def make_table(n: int, n_protected: int, seed: int, *, first_lo: int = 2**40,
               first_hi: int = 2**46, user_size=(256, 2**20), prot_size=(4096, 65536),
               max_gap_pages: int = 16, mmio_frac: float = 0.25) -> Table:
    """Draw ``n`` disjoint ranges (CPU tensors) as described in the module docstring."""
    if n <= 0:
        return Table(torch.zeros(0, dtype=torch.int64), torch.zeros(0, dtype=torch.int64),
                     torch.zeros(0, dtype=torch.uint8))
    g = _gen(seed, 1)
    kind = torch.zeros(n, dtype=torch.uint8)
    n_mmio = int(round(n_protected * mmio_frac))
    kind[:n_protected] = KIND_PROTECTED
    kind[:n_mmio] = KIND_MMIO
    kind = kind[torch.randperm(n, generator=g)]
    usize = loguniform_int(user_size[0], user_size[1], n, g)
    psize = prot_size[0] + _uniform_below(
        torch.full((n,), prot_size[1] - prot_size[0] + 1, dtype=torch.int64), g)
    size = torch.where(kind == KIND_USER, usize, psize)
    gaps = _uniform_below(torch.full((n,), max_gap_pages + 1, dtype=torch.int64), g) * PAGE
    first_pages = (first_hi - first_lo) // PAGE
    first = first_lo + int(_uniform_below(torch.tensor([first_pages]), g)[0]) * PAGE
    # base_{i+1} = roundup(base_i + size_i, PAGE) + gap_i, computed sequentially.
    base = torch.empty(n, dtype=torch.int64)
    b = first
    sz = size.tolist()
    gp = gaps.tolist()
    out = [0] * n
    for i in range(n):
        out[i] = b
        e = b + sz[i]
        b = ((e + PAGE - 1) // PAGE) * PAGE + gp[i]
    base = torch.tensor(out, dtype=torch.int64)
    assert int(base[-1] + size[-1]) < 2**48
    return Table(base, size, kind)


def make_queries(table: Table, n: int, seed: int, device="cpu",
                 mix=(0.6, 0.2, 0.1, 0.1), max_len: int = 4096,
                 min_len: int = 1) -> torch.Tensor:
    """``n`` pointer queries as an int64 tensor [n, 2] = (addr, len) on ``device``.

    Lengths are log-uniform in [min_len, max_len], clamped to what the category allows
    (a query inside a USER range is never longer than the range, one inside a hole never
    leaves the hole, a straddling query is at least 2 bytes long)."""
    g = _gen(seed, 2, device)
    t = table.to(device)
    base, size, kind = t.base, t.size, t.kind
    end = base + size
    user = torch.nonzero(kind == KIND_USER).flatten()
    prot = torch.nonzero(kind != KIND_USER).flatten()
    # holes: the gap below range i is [end_{i-1}, base_i) (only where non-empty)
    prev_end = torch.cat([base[:1] - 2 * PAGE, end[:-1]])
    gap = base - prev_end
    holed = torch.nonzero(gap > 0).flatten()

    n_user = int(round(n * mix[0]))
    n_prot = int(round(n * mix[1]))
    n_strad = int(round(n * mix[2]))
    n_hole = n - n_user - n_prot - n_strad
    if user.numel() == 0:
        n_prot += n_user; n_user = 0
    if prot.numel() == 0:
        n_user += n_prot; n_prot = 0
    out = torch.empty((n, 2), dtype=torch.int64, device=device)
    parts = []

    def pick(pool, m):
        return pool[_uniform_below(torch.full((m,), pool.numel(), dtype=torch.int64,
                                              device=device), g)]

    if n_user:
        r = pick(user, n_user)
        s = size[r]
        L = loguniform_int(torch.clamp(s, max=min_len), torch.clamp(s, max=max_len),
                           n_user, g, device)
        off = _uniform_below(s - L + 1, g)
        parts.append(torch.stack([base[r] + off, L], 1))
    if n_prot:
        r = pick(prot, n_prot)
        off = _uniform_below(size[r], g)
        L = loguniform_int(min_len, max_len, n_prot, g, device)
        parts.append(torch.stack([base[r] + off, L], 1))
    if n_strad:
        na = n_strad // 2 if user.numel() else 0
        nb = n_strad - na
        if na:
            r = pick(user, na)
            L = loguniform_int(max(2, min_len), max_len, na, g, device)
            d = 1 + _uniform_below(torch.minimum(L - 1, size[r]), g)
            parts.append(torch.stack([end[r] - d, L], 1))
        if nb:
            r = pick(holed, nb)
            L = loguniform_int(max(2, min_len), max_len, nb, g, device)
            d = 1 + _uniform_below(torch.minimum(L - 1, gap[r]), g)
            parts.append(torch.stack([base[r] - d, L], 1))
    if n_hole:
        r = pick(holed, n_hole)
        off = _uniform_below(gap[r], g)
        room = gap[r] - off
        L = loguniform_int(torch.clamp(room, max=min_len), torch.clamp(room, max=max_len),
                           n_hole, g, device)
        parts.append(torch.stack([prev_end[r] + off, L], 1))
    allq = torch.cat(parts, 0)
    perm = torch.randperm(n, generator=g, device=device)
    out[perm] = allq
    return out


def aperture_table(bounds) -> Table:
    """The three apertures ``[b0, b1)``, ``[b1, b2)``, ``[b2, b3)`` as a ``Table`` (I/O as MMIO,
    module as PROTECTED, user as USER), so that ``make_queries`` draws its mix relative to
    them."""
    b = [int(x) for x in bounds]
    return Table(torch.tensor(b[:3], dtype=torch.int64),
                 torch.tensor([b[1] - b[0], b[2] - b[1], b[3] - b[2]], dtype=torch.int64),
                 torch.tensor([KIND_MMIO, KIND_PROTECTED, KIND_USER], dtype=torch.uint8))


def make_dma_queries(table: Table, n: int, seed: int, device="cpu") -> torch.Tensor:
    """``n`` DMA registration queries [n, 2] = (addr, len): 40% the exact extent of a USER
    range, 10% one byte short of it (from its base, or from base + 1), 5% one byte too long,
    5% the exact extent of a protected range, 40% the pointer-query mix of ``make_queries``.
    Categories are shuffled."""
    g = _gen(seed, 9, device)
    t = table.to(device)
    base, size, kind = t.base, t.size, t.kind
    user = torch.nonzero(kind == KIND_USER).flatten()
    prot = torch.nonzero(kind != KIND_USER).flatten()
    out = make_queries(table, n, seed, device).clone()
    pick_n = lambda pool, m: pool[_uniform_below(torch.full((m,), pool.numel(), dtype=torch.int64,
                                                            device=device), g)]
    cut = torch.randperm(n, generator=g, device=device)
    k0, k1, k2, k3 = (int(round(n * f)) for f in (0.40, 0.50, 0.55, 0.60))
    if user.numel() and k1:
        r = pick_n(user, k1)
        a, L = base[r].clone(), size[r].clone()
        short = torch.arange(k1, device=device) >= k0
        from_next = short & (_uniform_below(torch.full((k1,), 2, dtype=torch.int64, device=device),
                                            g) == 1) & (L > 1)
        L = torch.where(short & (L > 1), L - 1, L)
        a = torch.where(from_next, a + 1, a)
        out[cut[:k1]] = torch.stack([a, L], 1)
    if user.numel() and k2 > k1:
        r = pick_n(user, k2 - k1)
        out[cut[k1:k2]] = torch.stack([base[r], size[r] + 1], 1)
    if prot.numel() and k3 > k2:
        r = pick_n(prot, k3 - k2)
        out[cut[k2:k3]] = torch.stack([base[r], size[r]], 1)
    return out


def uniform_f32(n: int, seed: int, device="cpu", stream: int = 3) -> torch.Tensor:
    """fp32 values uniform in [-1, 1)."""
    g = _gen(seed, stream, device)
    return torch.rand(n, generator=g, device=device, dtype=torch.float32) * 2.0 - 1.0


def uniform_indices(n: int, rows: int, seed: int, device="cpu", bad_frac: float = 0.0,
                    bad_ranges=(), stream: int = 4) -> torch.Tensor:
    """int64 indices uniform in [0, rows); a ``bad_frac`` share is replaced by indices drawn
    uniformly from the half-open index intervals in ``bad_ranges`` (chosen uniformly)."""
    g = _gen(seed, stream, device)
    idx = _uniform_below(torch.full((n,), rows, dtype=torch.int64, device=device), g)
    return _plant_bad(idx, g, bad_frac, bad_ranges)


def _plant_bad(idx, g, bad_frac, bad_ranges):
    n = idx.numel()
    nbad = int(round(n * bad_frac))
    if nbad == 0 or not bad_ranges:
        return idx
    dev = idx.device
    pos = torch.randperm(n, generator=g, device=dev)[:nbad]
    which = _uniform_below(torch.full((nbad,), len(bad_ranges), dtype=torch.int64,
                                      device=dev), g)
    lo = torch.tensor([r[0] for r in bad_ranges], dtype=torch.int64, device=dev)[which]
    hi = torch.tensor([r[1] for r in bad_ranges], dtype=torch.int64, device=dev)[which]
    idx[pos] = lo + _uniform_below(hi - lo, g)
    return idx


def zipf_indices(n: int, rows: int, s: float, seed: int, device="cpu", bad_frac: float = 0.0,
                 bad_ranges=(), stream: int = 5) -> torch.Tensor:
    """int64 row indices with Zipf(s) rank popularity over a finite support of ``rows``:
    rank k in [1, rows] has probability proportional to k**-s (inverse CDF), and rank k
    maps to row ``perm[k-1]`` for a seeded permutation so hot rows are scattered."""
    g = _gen(seed, stream, device)
    k = torch.arange(1, rows + 1, dtype=torch.float64, device=device)
    cdf = torch.cumsum(k.pow(-s), 0)
    cdf = cdf / cdf[-1]
    u = torch.rand(n, generator=g, device=device, dtype=torch.float64)
    rank = torch.searchsorted(cdf, u).clamp_(max=rows - 1)
    perm = torch.randperm(rows, generator=g, device=device)
    return _plant_bad(perm[rank], g, bad_frac, bad_ranges)


def make_batch_requests(tables, n_req: int, seed: int, *, max_ptrs: int = 4096,
                        len_range=(4, 64 << 20), copy_range=(4096, 64 << 20),
                        cross_frac: float = 0.05, mix=(0.6, 0.2, 0.1, 0.1)):
    """Requests for one batched multi-client launch.

    Returns a dict of CPU tensors: ``client`` [R] int32; ``ptr_off`` [R+1] int64 offsets into
    ``ptrs`` [P, 2] int64 (addr, len); ``copy_bytes`` [R] int64. Pointer counts are
    log-uniform in [1, max_ptrs]; each pointer follows the query mix over the request's own
    client table, except a ``cross_frac`` share taken from inside a USER range of another
    client's table. Pointer lengths are log-uniform in ``len_range`` (clamped to what the
    category allows). Copy sizes are log-uniform in ``copy_range``.
    """
    g = _gen(seed, 6)
    n_cl = len(tables)
    client = _uniform_below(torch.full((n_req,), n_cl, dtype=torch.int64), g)
    counts = loguniform_int(1, max_ptrs, n_req, g)
    off = torch.zeros(n_req + 1, dtype=torch.int64)
    off[1:] = torch.cumsum(counts, 0)
    ptrs = torch.empty((int(off[-1]), 2), dtype=torch.int64)
    for r in range(n_req):
        c = int(client[r])
        m = int(counts[r])
        q = make_queries(tables[c], m, seed * 7919 + r + 1, mix=mix,
                         min_len=len_range[0], max_len=len_range[1])
        ncross = int(round(m * cross_frac)) if n_cl > 1 else 0
        if ncross:
            other = (c + 1 + int(_uniform_below(torch.tensor([n_cl - 1]), g)[0])) % n_cl
            t = tables[other]
            users = torch.nonzero(t.kind == KIND_USER).flatten()
            rr = users[_uniform_below(torch.full((ncross,), users.numel(),
                                                 dtype=torch.int64), g)]
            pos = torch.randperm(m, generator=g)[:ncross]
            q[pos, 0] = t.base[rr]
            q[pos, 1] = torch.minimum(t.size[rr], torch.full((ncross,), 4096))
        ptrs[int(off[r]):int(off[r + 1])] = q
    copy_bytes = loguniform_int(copy_range[0], copy_range[1], n_req, g)
    return {"client": client.to(torch.int32), "ptr_off": off, "ptrs": ptrs,
            "copy_bytes": copy_bytes}


def make_serving_trace(n_clients: int, rate: float, duration: float, seed: int, *,
                       mix=(0.5, 0.3, 0.2), val_ptrs=(16, 1024), copy_range=(4096, 16 << 20),
                       gather_range=(1 << 12, 1 << 20)):
    """Open-loop arrivals for the serving loop (CPU tensors).

    Poisson arrivals at ``rate`` requests/s in aggregate over ``duration`` seconds; each
    request picks a client uniformly and an op by ``mix`` (0 validate, 1 copy, 2 gather)
    with a size log-uniform in the op's range (pointer count, bytes, or index count).
    """
    g = _gen(seed, 7)
    expect = int(rate * duration * 1.2 + 64)
    inter = -torch.log1p(-torch.rand(expect, generator=g, dtype=torch.float64)) / rate
    t = torch.cumsum(inter, 0)
    t = t[t < duration]
    n = t.numel()
    client = _uniform_below(torch.full((n,), n_clients, dtype=torch.int64), g)
    u = torch.rand(n, generator=g, dtype=torch.float64)
    op = torch.where(u < mix[0], 0, torch.where(u < mix[0] + mix[1], 1, 2)).to(torch.int64)
    size = torch.empty(n, dtype=torch.int64)
    for o, (lo, hi) in enumerate((val_ptrs, copy_range, gather_range)):
        m = op == o
        k = int(m.sum())
        if k:
            size[m] = loguniform_int(lo, hi, k, g)
    return {"t": t, "client": client, "op": op, "size": size}
