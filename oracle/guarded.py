"""Guarded kernels and the first-fault log (oracle; test infrastructure only).

The paper's kernel memory guard checks an application's global loads and stores against
the protected ranges before the access and then applies a policy (Section V-E, Fig. 2
caption): ``poison`` records a violation that surfaces at a later boundary, ``sink``
redirects the access to quarantine memory. This module restates that guard per access:

* Binding: each pointer argument ``p`` is bound once to ``[lo, hi)``, the USER allocation
  that contains ``p`` (the paper's API-time rule of Section IV-E / V-C applied to the
  argument), or to the empty interval when ``p`` is not inside a USER allocation.
  (Reading: the kernel guard is an allow-list of the argument's own allocation; it denies
  everything the paper's deny-list of protected intervals denies, and also cross-allocation
  accesses.)
* An access of width ``w`` bytes at the exact integer address ``A`` (no wrap-around) is
  allowed iff ``lo <= A`` and ``A + w <= hi``.
* Suppression (``sink`` with a zero page): a denied load yields all-zero bits; a denied
  store is dropped and the destination keeps its bytes.
* Logging (``poison``): every denied access adds one to ``count``; the log keeps the
  record with the smallest key ``(seq, elem, operand)`` where ``seq`` numbers the guarded
  calls of a table in program order, ``elem`` is the flat element index and ``operand``
  the operand's position in the access order. The record's reason is the classification
  of ``[A, A+w)`` with ALLOW replaced by CROSS_ALLOC, or UNMAPPED when ``A`` lies outside
  ``[0, 2**64)``.

Policies: ``SUPPRESS_LOG`` (the ``sink`` to a zero page plus the ``poison`` record),
``SUPPRESS_ONLY`` (the sink alone), ``TRAP``, ``SINK`` and ``REPORT``. Under ``SINK`` a denied
access is redirected to a caller-provided quarantine of ``qsize`` bytes (a power of two) at
``qbase``: the access of width ``w`` at ``A`` goes to ``qbase + ((A mod 2**64) mod qsize)``
rounded down to a multiple of ``w`` (loads read it, stores write it, scatter-add adds into
it). Under ``REPORT`` a denied access is performed at ``A`` itself when ``[A, A+w)`` lies inside
one registered range of any kind that was inserted as backed (the caller vouches that it is
mapped memory), and suppressed otherwise (memory outside every range, or in a range with no
such statement, may not be mapped). Under ``REMAP`` (the paper's ``remap_or``,
kept to the condition under which the paper calls it safe: the target is a live user
allocation) a denied access is rewritten into its own argument's allocation ``[lo, hi)``:
with ``lo'`` = lo rounded up to a multiple of ``w`` and ``m`` the largest multiple of ``w``
not above ``hi - lo'``, it goes to ``lo' + ((A - lo') mod m)`` rounded down to a multiple of
``w``; an argument without a binding (or with ``m == 0``) leaves it suppressed. All three log
every denial like ``SUPPRESS_LOG``. Only the per-access loops define them. The paper's ``trap`` stops at a violation and
may leave the worker's context unusable, so the worker is retired (Section V-E; Section IV-D,
lifetime and revocation). Restated per call (``guarded_call``): a call of a retired handle does
nothing and reports ``ETRAPPED``; a ``TRAP`` call runs as under ``SUPPRESS_LOG`` (the denied
access never happens and is logged), and if it denied anything the handle is retired and the
call reports ``ETRAPPED``.

Access widths and orders: copy - bytes, src(0) then dst(1); triad ``a = b + s*c`` - fp32
elements, b(0), c(1), a(2), computed as two float32 roundings (no fused multiply-add);
gather ``out[i,:] = T[idx[i],:]`` - the 8-byte index load (elem ``i*D``), then per column
the table element (1) and the out element (2); scatter ``dst[idx[i],:] = src[i,:]`` (or
``+=``) - idx(0), src(1), dst(2). ``D = row_bytes / w``. Scatter-add into a destination whose rows
are all +0.0 (the library's ``accumulate == 2``) is scatter-add on that destination: the oracle
takes any true ``accumulate`` as ``+=``, and its callers zero the destination first.

Each kernel comes twice: ``*_loop`` walks every access in program order (the definition,
for small inputs) and ``*_vec`` computes the same result with numpy masks (pinned against
the loop form by the tests).
"""
from __future__ import annotations

import numpy as np

from .table import ALLOW, V_CROSS_ALLOC, V_UNMAPPED, U64_MAX

OP_COPY, OP_TRIAD, OP_GATHER, OP_SCATTER, OP_SCATTER_ADD = 1, 2, 3, 4, 5
SUPPRESS_LOG, SUPPRESS_ONLY, TRAP, SINK, REPORT, REMAP = 0, 1, 2, 3, 4, 5
REDIRECTING = (SINK, REPORT, REMAP)
OK, ETRAPPED = 0, -8
_DT = {4: np.float32, 8: np.float64}


def reason(table, A: int, w: int):
    """Reason code and owner recorded for a denied access at exact address ``A``."""
    if A < 0 or A > U64_MAX:
        return V_UNMAPPED, -1
    v, owner = table.verdict(A, w)
    if v == ALLOW:
        v = V_CROSS_ALLOC
    return v, owner


class FaultLog:
    """Exact denial count plus the record with the smallest key."""

    def __init__(self):
        self.count = 0
        self.first = None
        self.retired = False          # set by a violation under TRAP; clearing keeps it

    def clear(self):
        self.count = 0
        self.first = None

    def key(self):
        f = self.first
        return None if f is None else (f["seq"], f["elem"], f["operand"])

    def offer(self, table, seq, elem, operand, A, w, op, n=1):
        """Account ``n`` denials whose smallest key is ``(seq, elem, operand)`` at ``A``."""
        self.count += int(n)
        k = (int(seq), int(elem), int(operand))
        if self.first is None or k < self.key():
            v, owner = reason(table, int(A), int(w))
            self.first = dict(seq=k[0], elem=k[1], operand=k[2], addr=int(A) % (1 << 64),
                              width=int(w), verdict=int(v), owner=int(owner), op=int(op))


def _allowed(bind, A, w):
    return bind[0] <= A and A + w <= bind[1]


class _Denier:
    def __init__(self, table, log, seq, op, policy, quarantine=None, loops=True):
        if policy not in (SUPPRESS_LOG, SUPPRESS_ONLY, TRAP) + REDIRECTING:
            raise ValueError("unknown policy")
        if policy in REDIRECTING and not loops:
            raise NotImplementedError("the redirecting policies are defined by the loop forms")
        if policy == SINK:
            qb, qs = quarantine
            if qs < 256 or qs & (qs - 1):
                raise ValueError("quarantine size must be a power of two >= 256")
        self.t, self.log, self.seq, self.op = table, log, seq, op
        self.policy, self.q = policy, quarantine
        self.on = policy != SUPPRESS_ONLY

    def __call__(self, elem, operand, A, w):
        if self.on:
            self.log.offer(self.t, self.seq, elem, operand, A, w, self.op)

    def target(self, A, w, bind=(0, 0)):
        """Where a denied access of width w at exact address A of the argument bound to
        ``bind`` goes (None: suppressed)."""
        if self.policy == REMAP:
            lo, hi = bind
            if hi <= lo:
                return None
            lo_a = -(-lo // w) * w
            m = (hi - lo_a) // w * w
            if m <= 0:
                return None
            return lo_a + ((A - lo_a) % m) // w * w
        if self.policy == SINK:
            qb, qs = self.q
            return qb + ((A % (1 << 64)) % qs) // w * w
        if self.policy == REPORT:
            if A < 0 or A + w > (1 << 64):
                return None
            ent = self.t.owner_entry(A)
            if ent is not None and A + w <= ent[1] and self.t.is_backed(ent[3]):
                return A
        return None

    def load(self, mem, A, w, bind=(0, 0)):
        """The bytes a denied load reads."""
        t = self.target(A, w, bind)
        return bytes(w) if t is None else mem.read(t, w)

    def store(self, mem, A, data, bind=(0, 0)):
        t = self.target(A, len(data), bind)
        if t is not None:
            mem.write(t, data)

    def add(self, mem, A, val, dt, bind=(0, 0)):
        t = self.target(A, dt().itemsize, bind)
        if t is not None:
            old = np.frombuffer(mem.read(t, dt().itemsize), dtype=dt)[0]
            mem.write(t, dt(old + val).tobytes())


def guarded_call(kernel, table, mem, log, seq, *args, policy=SUPPRESS_LOG, **kw):
    """One guarded call of a handle whose log is ``log``, under any policy; returns the status.

    ``kernel`` is one of the ``*_loop`` / ``*_vec`` functions below. A retired handle runs
    nothing. Under ``TRAP`` a call that denied at least one access retires the handle.
    """
    if log.retired:
        return ETRAPPED
    before = log.count
    kernel(table, mem, log, seq, *args, policy=policy, **kw)
    if policy == TRAP and log.count != before:
        log.retired = True
        return ETRAPPED
    return OK


# ------------------------------------------------------------------ per-access loops
def copy_loop(table, mem, log, seq, dst, src, n, policy=SUPPRESS_LOG, quarantine=None):
    deny = _Denier(table, log, seq, OP_COPY, policy, quarantine)
    bs, bd = table.binding(src), table.binding(dst)
    for k in range(n):
        A = src + k
        if _allowed(bs, A, 1):
            byte = mem.read(A, 1)
        else:
            byte = deny.load(mem, A, 1, bs)
            deny(k, 0, A, 1)
        A = dst + k
        if _allowed(bd, A, 1):
            mem.write(A, byte)
        else:
            deny.store(mem, A, byte, bd)
            deny(k, 1, A, 1)


def _f32(b: bytes):
    return np.frombuffer(b, dtype=np.float32)[0]


def triad_loop(table, mem, log, seq, a, b, c, s, n, policy=SUPPRESS_LOG, quarantine=None):
    deny = _Denier(table, log, seq, OP_TRIAD, policy, quarantine)
    ba, bb, bc = table.binding(a), table.binding(b), table.binding(c)
    s32 = np.float32(s)
    for i in range(n):
        vals = []
        for op_i, (p, bind) in enumerate(((b, bb), (c, bc))):
            A = p + 4 * i
            if _allowed(bind, A, 4):
                vals.append(_f32(mem.read(A, 4)))
            else:
                vals.append(_f32(deny.load(mem, A, 4, bind)))
                deny(i, op_i, A, 4)
        with np.errstate(over="ignore", invalid="ignore"):   # IEEE overflow to inf / NaN is the result
            prod = np.float32(s32 * vals[1])          # first rounding
            r = np.float32(vals[0] + prod)            # second rounding
        A = a + 4 * i
        if _allowed(ba, A, 4):
            mem.write(A, np.float32(r).tobytes())
        else:
            deny.store(mem, A, np.float32(r).tobytes(), ba)
            deny(i, 2, A, 4)


def _idx_load(mem, bind, idx_ptr, i, deny, elem):
    A = idx_ptr + 8 * i
    if _allowed(bind, A, 8):
        return int(np.frombuffer(mem.read(A, 8), dtype=np.int64)[0])
    deny(elem, 0, A, 8)
    return int(np.frombuffer(deny.load(mem, A, 8, bind), dtype=np.int64)[0])


def gather_loop(table, mem, log, seq, out, T, row_bytes, idx_ptr, n, w=4,
                policy=SUPPRESS_LOG, quarantine=None):
    deny = _Denier(table, log, seq, OP_GATHER, policy, quarantine)
    D = row_bytes // w
    bi, bt, bo = table.binding(idx_ptr), table.binding(T), table.binding(out)
    for i in range(n):
        iv = _idx_load(mem, bi, idx_ptr, i, deny, i * D)
        for col in range(D):
            e = i * D + col
            A = T + iv * row_bytes + col * w
            if _allowed(bt, A, w):
                val = mem.read(A, w)
            else:
                val = deny.load(mem, A, w, bt)
                deny(e, 1, A, w)
            A = out + i * row_bytes + col * w
            if _allowed(bo, A, w):
                mem.write(A, val)
            else:
                deny.store(mem, A, val, bo)
                deny(e, 2, A, w)


def scatter_loop(table, mem, log, seq, dst, row_bytes, idx_ptr, src, n, w=4, accumulate=False,
                 policy=SUPPRESS_LOG, quarantine=None):
    deny = _Denier(table, log, seq, OP_SCATTER_ADD if accumulate else OP_SCATTER, policy,
                   quarantine)
    D = row_bytes // w
    dt = _DT[w]
    bi, bs, bd = table.binding(idx_ptr), table.binding(src), table.binding(dst)
    for i in range(n):
        iv = _idx_load(mem, bi, idx_ptr, i, deny, i * D)
        for col in range(D):
            e = i * D + col
            A = src + i * row_bytes + col * w
            if _allowed(bs, A, w):
                val = mem.read(A, w)
            else:
                val = deny.load(mem, A, w, bs)
                deny(e, 1, A, w)
            A = dst + iv * row_bytes + col * w
            if _allowed(bd, A, w):
                if accumulate:
                    old = np.frombuffer(mem.read(A, w), dtype=dt)[0]
                    new = dt(old + np.frombuffer(val, dtype=dt)[0])
                    mem.write(A, new.tobytes())
                else:
                    mem.write(A, val)
            else:
                if accumulate:
                    deny.add(mem, A, np.frombuffer(val, dtype=dt)[0], dt, bd)
                else:
                    deny.store(mem, A, val, bd)
                deny(e, 2, A, w)


# ------------------------------------------------------------------ vectorized forms
_C = 1 << 62


def _window(p, bind):
    """Offsets ``off`` (relative to ``p``) of allowed width-``w`` accesses satisfy
    ``dlo <= off`` and ``off + w <= dhi``; clamped so int64 comparisons stay exact."""
    return max(-_C, min(_C, bind[0] - p)), max(-_C, min(_C, bind[1] - p))


def _cols(roff, D, w, dlo, dhi):
    """Per row with object-int row offsets ``roff``: allowed column range [c0, c1)."""
    c0 = np.array([min(D, -((r - dlo) // w)) if r < dlo else 0 for r in roff], dtype=np.int64) \
        if len(roff) else np.zeros(0, np.int64)
    c1 = np.array([min(D, (dhi - r - w) // w + 1) if dhi - r - w >= 0 else 0 for r in roff],
                  dtype=np.int64) if len(roff) else np.zeros(0, np.int64)
    return c0, np.maximum(c1, c0)


def _first_denied_col(c0, c1, D):
    """First denied column per row (D when the row has none)."""
    return np.where(c0 > 0, 0, np.where(c1 < D, c1, D))


def copy_vec(table, mem, log, seq, dst, src, n, policy=SUPPRESS_LOG):
    deny = _Denier(table, log, seq, OP_COPY, policy, loops=False)
    bs, bd = table.binding(src), table.binding(dst)
    ks = max(0, min(n, bs[1] - src)) if bs[0] <= src else 0
    kd = max(0, min(n, bd[1] - dst)) if bd[0] <= dst else 0
    kk = min(ks, kd)
    if kd > 0:
        darr, doff = mem.locate(dst, dst + kd)
        if kk > 0:
            sarr, soff = mem.locate(src, src + kk)
            darr[doff:doff + kk] = sarr[soff:soff + kk].copy()
        darr[doff + kk:doff + kd] = 0
    nden = (n - ks) + (n - kd)
    if nden and deny.on:
        if ks <= kd:
            log.offer(table, seq, ks, 0, src + ks, 1, OP_COPY, nden)
        else:
            log.offer(table, seq, kd, 1, dst + kd, 1, OP_COPY, nden)


def triad_vec(table, mem, log, seq, a, b, c, s, n, policy=SUPPRESS_LOG):
    deny = _Denier(table, log, seq, OP_TRIAD, policy, loops=False)
    i = np.arange(n, dtype=np.int64) * 4
    vals = []
    cands = []
    nden = 0
    for op_i, p in enumerate((b, c)):
        bind = table.binding(p)
        dlo, dhi = _window(p, bind)
        ok = (i >= dlo) & (i + 4 <= dhi)
        v = np.zeros(n, dtype=np.float32)
        if ok.any():
            arr, off = mem.locate(bind[0], bind[1])
            base = off + (p - bind[0])
            byte_idx = base + i[ok][:, None] + np.arange(4)[None, :]
            v[ok] = arr[byte_idx].reshape(-1).view(np.float32)
        vals.append(v)
        bad = np.flatnonzero(~ok)
        nden += bad.size
        if bad.size:
            cands.append((int(bad[0]), op_i, p + 4 * int(bad[0])))
    with np.errstate(over="ignore", invalid="ignore"):   # IEEE overflow to inf / NaN is the result
        r = (vals[0] + (np.float32(s) * vals[1]).astype(np.float32)).astype(np.float32)
    bind = table.binding(a)
    dlo, dhi = _window(a, bind)
    ok = (i >= dlo) & (i + 4 <= dhi)
    if ok.any():
        arr, off = mem.locate(bind[0], bind[1])
        base = off + (a - bind[0])
        byte_idx = base + i[ok][:, None] + np.arange(4)[None, :]
        arr[byte_idx.reshape(-1)] = r[ok].view(np.uint8)
    bad = np.flatnonzero(~ok)
    nden += bad.size
    if bad.size:
        cands.append((int(bad[0]), 2, a + 4 * int(bad[0])))
    if nden and deny.on:
        e, o, A = min(cands)
        log.offer(table, seq, e, o, A, 4, OP_TRIAD, nden)


def _read_idx_vec(table, mem, idx_ptr, n):
    """Index values (0 where the index load is denied) and the denial mask."""
    bind = table.binding(idx_ptr)
    dlo, dhi = _window(idx_ptr, bind)
    off = np.arange(n, dtype=np.int64) * 8
    ok = (off >= dlo) & (off + 8 <= dhi)
    iv = np.zeros(n, dtype=np.int64)
    if ok.any():
        arr, o = mem.locate(bind[0], bind[1])
        base = o + (idx_ptr - bind[0])
        byte_idx = base + off[ok][:, None] + np.arange(8)[None, :]
        iv[ok] = arr[byte_idx].reshape(-1).view(np.int64)
    return iv, ~ok


def _row_access(table, p, roff, D, w):
    """Allowed column ranges for accesses at ``p + roff[i] + col*w`` (roff object ints)."""
    bind = table.binding(p)
    dlo, dhi = bind[0] - p, bind[1] - p  # exact Python ints
    c0, c1 = _cols(roff, D, w, dlo, dhi)
    return bind, c0, c1


def _gather_bytes(mem, bind, p, roff, rows, c0, c1, D, w):
    """(len(rows), D*w) uint8 block with allowed columns filled and denied ones zero."""
    m = len(rows)
    out = np.zeros((m, D * w), dtype=np.uint8)
    if m == 0 or bind[1] <= bind[0]:
        return out
    arr, o = mem.locate(bind[0], bind[1])
    rel = np.array([int(roff[r]) + (p - bind[0]) + o if c1[r] > c0[r] else 0 for r in rows],
                   dtype=np.int64)
    full = (c0[rows] == 0) & (c1[rows] == D)
    for k in np.flatnonzero(full):
        out[k] = arr[rel[k]:rel[k] + D * w]
    for k in np.flatnonzero(~full):
        r = rows[k]
        for col in range(c0[r], c1[r]):
            s = rel[k] + col * w
            out[k, col * w:(col + 1) * w] = arr[s:s + w]
    return out


def _scatter_store(mem, bind, p, roff, rows, c0, c1, D, w, data, accumulate):
    """Store rows of ``data`` (uint8, D*w wide) at allowed columns, in row order."""
    if len(rows) == 0 or bind[1] <= bind[0]:
        return
    arr, o = mem.locate(bind[0], bind[1])
    dt = _DT[w]
    if accumulate:
        # Every allowed (row, column) contribution lands on one destination element; each
        # element becomes its old value plus the float64 sum of its contributions, rounded once
        # to the element type (the order of the float64 additions is not significant at the
        # tolerance the gradient is held to).
        offs, vals = [], []
        for k, r in enumerate(rows):
            base = int(roff[r]) + (p - bind[0]) + o
            cols = np.arange(c0[r], c1[r], dtype=np.int64)
            offs.append(base + cols * w)
            vals.append(data[k].view(dt)[c0[r]:c1[r]].astype(np.float64))
        if not offs:
            return
        offs = np.concatenate(offs)
        vals = np.concatenate(vals)
        order = np.argsort(offs, kind="stable")
        so, sv = offs[order], vals[order]
        starts = np.flatnonzero(np.r_[True, so[1:] != so[:-1]])
        uniq = so[starts]
        sums = np.add.reduceat(sv, starts)
        byte_idx = uniq[:, None] + np.arange(w, dtype=np.int64)[None, :]
        old = arr[byte_idx].reshape(-1).view(dt).astype(np.float64)
        arr[byte_idx] = (old + sums).astype(dt).view(np.uint8).reshape(-1, w)
        return
    for k, r in enumerate(rows):
        base = int(roff[r]) + (p - bind[0]) + o
        if c0[r] == 0 and c1[r] == D:
            arr[base:base + D * w] = data[k]
        else:
            for col in range(c0[r], c1[r]):
                s = base + col * w
                arr[s:s + w] = data[k, col * w:(col + 1) * w]


def _count_and_first(D, n, idx_bad, groups):
    """Total denials and smallest (elem, operand, row, col) over idx and row operands."""
    nden = int(idx_bad.sum())
    cands = []
    if idx_bad.any():
        i0 = int(np.flatnonzero(idx_bad)[0])
        cands.append((i0 * D, 0, i0, 0))
    for operand, c0, c1 in groups:
        nden += int((D - (c1 - c0)).sum())
        fc = _first_denied_col(c0, c1, D)
        rows = np.flatnonzero(fc < D)
        if rows.size:
            r = int(rows[0])
            cands.append((r * D + int(fc[r]), operand, r, int(fc[r])))
    return nden, (min(cands) if cands else None)


def gather_vec(table, mem, log, seq, out, T, row_bytes, idx_ptr, n, w=4, policy=SUPPRESS_LOG):
    deny = _Denier(table, log, seq, OP_GATHER, policy, loops=False)
    D = row_bytes // w
    iv, idx_bad = _read_idx_vec(table, mem, idx_ptr, n)
    roff_t = iv.astype(object) * row_bytes
    roff_o = np.arange(n, dtype=np.int64).astype(object) * row_bytes
    bt, t0, t1 = _row_access(table, T, roff_t, D, w)
    bo, o0, o1 = _row_access(table, out, roff_o, D, w)
    rows = np.flatnonzero(o1 > o0)
    data = _gather_bytes(mem, bt, T, roff_t, rows, t0, t1, D, w)
    _scatter_store(mem, bo, out, roff_o, rows, o0, o1, D, w, data, False)
    nden, first = _count_and_first(D, n, idx_bad, ((1, t0, t1), (2, o0, o1)))
    if nden and deny.on:
        e, operand, r, col = first
        A = (idx_ptr + 8 * r if operand == 0 else
             T + int(iv[r]) * row_bytes + col * w if operand == 1 else
             out + r * row_bytes + col * w)
        log.offer(table, seq, e, operand, A, 8 if operand == 0 else w, OP_GATHER, nden)


def scatter_vec(table, mem, log, seq, dst, row_bytes, idx_ptr, src, n, w=4, accumulate=False,
                policy=SUPPRESS_LOG):
    op = OP_SCATTER_ADD if accumulate else OP_SCATTER
    deny = _Denier(table, log, seq, op, policy, loops=False)
    D = row_bytes // w
    iv, idx_bad = _read_idx_vec(table, mem, idx_ptr, n)
    roff_s = np.arange(n, dtype=np.int64).astype(object) * row_bytes
    roff_d = iv.astype(object) * row_bytes
    bs, s0, s1 = _row_access(table, src, roff_s, D, w)
    bd, d0, d1 = _row_access(table, dst, roff_d, D, w)
    rows = np.flatnonzero(d1 > d0)
    data = _gather_bytes(mem, bs, src, roff_s, rows, s0, s1, D, w)
    _scatter_store(mem, bd, dst, roff_d, rows, d0, d1, D, w, data, accumulate)
    nden, first = _count_and_first(D, n, idx_bad, ((1, s0, s1), (2, d0, d1)))
    if nden and deny.on:
        e, operand, r, col = first
        A = (idx_ptr + 8 * r if operand == 0 else
             src + r * row_bytes + col * w if operand == 1 else
             dst + int(iv[r]) * row_bytes + col * w)
        log.offer(table, seq, e, operand, A, 8 if operand == 0 else w, op, nden)
