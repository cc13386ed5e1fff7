"""Pins for the oracle's guarded kernels and first-fault log (CPU only).

* vectorized forms against the per-access loops on hostile scenarios;
* every denial enumerated by a recording log: count exact, first = minimum key;
* no-fault copy / gather against plain library routines;
* triad against exact rational arithmetic with an independent round-to-nearest-even;
* scatter-add with unit gradients against integer counts (np.bincount);
* protected canary bytes never change; suppressed loads read zero.
"""
import copy
import random
from fractions import Fraction

import numpy as np
import pytest

from oracle import RangeTable, USER, PROTECTED, MMIO, ALLOW, V_PROTECTED, V_STRADDLE, \
    V_UNMAPPED, V_CROSS_ALLOC
from oracle.memory import Memory
from oracle import guarded as G


class RecordingLog(G.FaultLog):
    """Keeps every denial; pins FaultLog's count and minimum-key bookkeeping."""

    def __init__(self):
        super().__init__()
        self.all = []

    def offer(self, table, seq, elem, operand, A, w, op, n=1):
        assert n == 1
        self.all.append((seq, elem, operand, A, w, op))
        super().offer(table, seq, elem, operand, A, w, op, n)


BASE = 0x7000_0000


def scenario(seed):
    """A table with backed USER allocations A, B (adjacent), C, a protected canary P,
    an MMIO range M and holes; returns (table, memory, named addresses)."""
    rng = np.random.default_rng(seed)
    t = RangeTable()
    mem = Memory()
    addr = {}

    def user(name, base, size):
        t.insert(base, size, USER, backed=True)
        mem.add(base, rng.integers(0, 256, size, dtype=np.uint8))
        addr[name] = (base, base + size)

    user("A", BASE, 512)
    user("B", BASE + 512, 384)                    # adjacent to A
    t.insert(BASE + 896, 128, PROTECTED, backed=True)   # canary, backed so we can check it
    mem.add(BASE + 896, np.full(128, 0xA5, np.uint8))
    addr["P"] = (BASE + 896, BASE + 1024)
    user("C", BASE + 2048, 1000)                   # hole [1024, 2048) before it
    t.insert(BASE + 4096, 64, MMIO, backed=True)
    mem.add(BASE + 4096, np.full(64, 0x3C, np.uint8))    # backed (REPORT may touch it)
    addr["M"] = (BASE + 4096, BASE + 4160)
    user("I", BASE + 8192, 8 * 64)                 # index buffer
    # registered but not declared backed, and with no memory in the model: any read or write
    # there raises, so every policy must leave it alone
    t.insert(BASE + 6144, 256, PROTECTED)
    addr["U"] = (BASE + 6144, BASE + 6400)
    return t, mem, addr


def pointer_choices(addr):
    A, B, C, P, M = addr["A"], addr["B"], addr["C"], addr["P"], addr["M"]
    return [A[0], A[0] + 13, A[1] - 40, B[0], B[1] - 1, C[0] + 4, C[1] - 100,
            P[0] + 8, M[0], BASE + 1500, BASE - 64, 0]


def _same(memA, memB, addr):
    for k in ("A", "B", "C", "P", "I"):
        lo, hi = addr[k]
        assert memA.read(lo, hi - lo) == memB.read(lo, hi - lo), k


def _overlap(p, n, q, m):
    """Partially overlapping operands give order-dependent results (like memcpy); the
    API leaves them unspecified, so the pins skip them (identical pointers are fine for
    elementwise ops)."""
    return p != q and n > 0 and m > 0 and p < q + m and q < p + n


def _logs_equal(la, lb):
    assert la.count == lb.count
    assert la.first == lb.first


@pytest.mark.parametrize("seed", range(6))
def test_copy_vec_matches_loop(seed):
    t, mem, addr = scenario(seed)
    rng = random.Random(seed)
    ptrs = pointer_choices(addr)
    for trial in range(40):
        dst, src = rng.choice(ptrs), rng.choice(ptrs)
        n = rng.choice([0, 1, 7, 64, 300, 700])
        if _overlap(dst, n, src, n) or (dst == src and n):
            continue
        m1, m2 = copy.deepcopy(mem), copy.deepcopy(mem)
        l1, l2 = RecordingLog(), G.FaultLog()
        G.copy_loop(t, m1, l1, trial, dst, src, n)
        G.copy_vec(t, m2, l2, trial, dst, src, n)
        _same(m1, m2, addr)
        _logs_equal(l1, l2)
        assert l1.count == len(l1.all)
        if l1.all:
            assert min((a[0], a[1], a[2]) for a in l1.all) == l1.key()
        # protected canary never changes
        assert m1.read(*addr["P"][:1], 128) == bytes([0xA5]) * 128


def test_copy_no_fault_is_plain_copy():
    t, mem, addr = scenario(1)
    src = addr["C"][0]
    dst = addr["A"][0]
    want = mem.read(src, 500)
    log = G.FaultLog()
    G.copy_vec(t, mem, log, 0, dst, src, 500)
    assert mem.read(dst, 500) == want and log.count == 0 and log.first is None


def test_copy_partial_closed_form_values():
    t, mem, addr = scenario(2)
    src = addr["A"][1] - 10          # 10 readable bytes, then B (another allocation)
    dst = addr["C"][0]
    before = mem.read(dst, 40)
    want = mem.read(src, 10) + bytes(30)
    log = G.FaultLog()
    G.copy_vec(t, mem, log, 5, dst, src, 40)
    assert mem.read(dst, 40) == want
    assert before != want
    assert log.count == 30
    f = log.first
    assert (f["seq"], f["elem"], f["operand"]) == (5, 10, 0)
    assert f["addr"] == addr["B"][0] and f["verdict"] == V_CROSS_ALLOC and f["owner"] == 1
    # copy into the protected canary: every store dropped, reason PROTECTED
    log.clear()
    G.copy_vec(t, mem, log, 6, addr["P"][0], addr["A"][0], 16)
    assert log.count == 16 and log.first["verdict"] == V_PROTECTED
    assert log.first["operand"] == 1 and log.first["elem"] == 0
    assert mem.read(addr["P"][0], 16) == bytes([0xA5]) * 16


def test_suppress_only_policy_logs_nothing():
    t, mem, addr = scenario(3)
    log = G.FaultLog()
    G.copy_vec(t, mem, log, 0, addr["P"][0], addr["A"][0], 16, policy=G.SUPPRESS_ONLY)
    assert log.count == 0 and log.first is None
    with pytest.raises(ValueError):
        G.copy_vec(t, mem, log, 0, addr["A"][0], addr["A"][0], 16, policy=7)


# --- triad --------------------------------------------------------------------------
def round_f32(x: Fraction) -> Fraction:
    """Round a rational to the nearest binary32 value, ties to even (independent of numpy)."""
    if x == 0:
        return Fraction(0)
    sgn = -1 if x < 0 else 1
    a = abs(x)
    e = a.numerator.bit_length() - a.denominator.bit_length()
    if Fraction(2) ** e > a:
        e -= 1
    while Fraction(2) ** (e + 1) <= a:
        e += 1
    q = Fraction(2) ** (max(e, -126) - 23)
    m = a / q
    fl = m.numerator // m.denominator
    rem = m - fl
    if rem > Fraction(1, 2) or (rem == Fraction(1, 2) and fl % 2 == 1):
        fl += 1
    r = fl * q
    if r >= Fraction(2) ** 128:
        return Fraction(sgn) * (Fraction(2) ** 200)   # stands for infinity
    return sgn * r


def _rand_f32(rng, n):
    kind = rng.integers(0, 4, n)
    mant = rng.uniform(-2, 2, n)
    exp = np.where(kind == 0, rng.integers(-10, 10, n),
                   np.where(kind == 1, rng.integers(-140, -120, n),
                            np.where(kind == 2, rng.integers(20, 60, n), 0)))
    return (mant * np.exp2(exp)).astype(np.float32)


def test_triad_matches_exact_rational_rounding():
    rng = np.random.default_rng(7)
    n = 3000
    b = _rand_f32(rng, n)
    c = _rand_f32(rng, n)
    for s in (np.float32(3.0), np.float32(-1.7), np.float32(1e-30), np.float32(0.0)):
        t = RangeTable()
        mem = Memory()
        for k, arr in enumerate((np.zeros(n, np.float32), b, c)):
            t.insert(BASE + k * (1 << 20), 4 * n, USER)
            mem.add(BASE + k * (1 << 20), arr.view(np.uint8))
        log = G.FaultLog()
        G.triad_vec(t, mem, log, 0, BASE, BASE + (1 << 20), BASE + (2 << 20), float(s), n)
        got = np.frombuffer(mem.read(BASE, 4 * n), dtype=np.float32)
        assert log.count == 0
        for i in range(n):
            p = round_f32(Fraction(float(s)) * Fraction(float(c[i])))
            r = round_f32(Fraction(float(b[i])) + p)
            assert Fraction(float(got[i])) == r, (i, b[i], c[i], s, got[i])


@pytest.mark.parametrize("seed", range(4))
def test_triad_vec_matches_loop(seed):
    t, mem, addr = scenario(seed)
    rng = random.Random(seed)
    ptrs = [p - (p % 4) for p in pointer_choices(addr)]
    for trial in range(30):
        a, b, c = rng.choice(ptrs), rng.choice(ptrs), rng.choice(ptrs)
        n = rng.choice([0, 1, 5, 33, 150])
        s = rng.choice([3.0, -0.5, 1.25])
        if _overlap(a, 4 * n, b, 4 * n) or _overlap(a, 4 * n, c, 4 * n):
            continue
        m1, m2 = copy.deepcopy(mem), copy.deepcopy(mem)
        l1, l2 = RecordingLog(), G.FaultLog()
        G.triad_loop(t, m1, l1, trial, a, b, c, s, n)
        G.triad_vec(t, m2, l2, trial, a, b, c, s, n)
        _same(m1, m2, addr)
        _logs_equal(l1, l2)
        if l1.all:
            assert min((x[0], x[1], x[2]) for x in l1.all) == l1.key()


# --- gather / scatter ----------------------------------------------------------------
def _write_idx(mem, addr, vals):
    lo = addr["I"][0]
    arr = np.array(vals, dtype=np.int64)
    mem.write(lo, arr.tobytes())
    return lo


def hostile_indices(rng, rows, k):
    choices = [0, 1, rows - 1, rows, rows + 1, -1, -2, rows * 3, -(1 << 62), (1 << 62),
               -(1 << 63), (1 << 63) - 1]
    return [rng.choice(choices + [rng.randrange(0, max(rows, 1))] * 6) for _ in range(k)]


@pytest.mark.parametrize("seed", range(6))
@pytest.mark.parametrize("w,D", [(4, 1), (4, 3), (8, 2)])
def test_gather_vec_matches_loop(seed, w, D):
    t, mem, addr = scenario(seed)
    rng = random.Random(seed * 31 + D)
    rb = w * D
    for trial in range(20):
        T = rng.choice([addr["A"][0], addr["A"][0] + rng.randrange(0, 40), addr["C"][0] + 4,
                        addr["P"][0], BASE + 1500])
        rows = max(1, (addr["A"][1] - T) // rb) if T < addr["A"][1] else 8
        n = rng.choice([0, 1, 9, 40])
        idx_ptr = _write_idx(mem, addr, hostile_indices(rng, rows, 64))
        if rng.random() < 0.2:
            idx_ptr = rng.choice([addr["I"][1] - 8 * 3, addr["P"][0]])
        out = rng.choice([addr["C"][0], addr["C"][1] - rb * 5 - 2, addr["B"][0], addr["P"][0]])
        if t.binding(out) != (0, 0) and t.binding(out) in (t.binding(T), t.binding(idx_ptr)):
            continue      # output aliasing an input: order-dependent, unspecified
        m1, m2 = copy.deepcopy(mem), copy.deepcopy(mem)
        l1, l2 = RecordingLog(), G.FaultLog()
        G.gather_loop(t, m1, l1, trial, out, T, rb, idx_ptr, n, w)
        G.gather_vec(t, m2, l2, trial, out, T, rb, idx_ptr, n, w)
        _same(m1, m2, addr)
        _logs_equal(l1, l2)
        assert l1.count == len(l1.all)
        if l1.all:
            assert min((x[0], x[1], x[2]) for x in l1.all) == l1.key()
        assert m1.read(addr["P"][0], 128) == bytes([0xA5]) * 128


@pytest.mark.parametrize("seed", range(6))
@pytest.mark.parametrize("accumulate", [False, True])
def test_scatter_vec_matches_loop(seed, accumulate):
    t, mem, addr = scenario(seed)
    rng = random.Random(seed + 100)
    w, D = 4, 2
    rb = w * D
    # integer-valued float32 sources so that accumulation order cannot matter
    for k in ("A", "C"):
        lo, hi = addr[k]
        vals = np.array([rng.randrange(-8, 9) for _ in range((hi - lo) // 4)], np.float32)
        mem.write(lo, vals.tobytes() + bytes((hi - lo) % 4))
    for trial in range(20):
        dst = rng.choice([addr["A"][0], addr["A"][0] + 8, addr["P"][0], addr["C"][0]])
        rows = 20
        n = rng.choice([0, 1, 9, 30])
        if accumulate:
            iv = hostile_indices(rng, rows, 64)
        else:
            pool = list(range(rows)) + [rows + 5, -3, 1 << 40]
            rng.shuffle(pool)
            iv = pool[:min(n, len(pool))] + [0] * 64
        idx_ptr = _write_idx(mem, addr, iv[:64])
        src = rng.choice([addr["C"][0], addr["C"][1] - rb * 4, addr["P"][0], addr["B"][0]])
        if t.binding(dst) != (0, 0) and t.binding(dst) in (t.binding(src), t.binding(idx_ptr)):
            continue      # destination aliasing an input: order-dependent, unspecified
        m1, m2 = copy.deepcopy(mem), copy.deepcopy(mem)
        l1, l2 = RecordingLog(), G.FaultLog()
        G.scatter_loop(t, m1, l1, trial, dst, rb, idx_ptr, src, n, w, accumulate)
        G.scatter_vec(t, m2, l2, trial, dst, rb, idx_ptr, src, n, w, accumulate)
        _same(m1, m2, addr)
        _logs_equal(l1, l2)
        if l1.all:
            assert min((x[0], x[1], x[2]) for x in l1.all) == l1.key()
        assert m1.read(addr["P"][0], 128) == bytes([0xA5]) * 128


def test_gather_no_fault_is_take():
    rng = np.random.default_rng(0)
    rows, D, n = 300, 5, 1000
    W = rng.standard_normal((rows, D)).astype(np.float32)
    idx = rng.integers(0, rows, n).astype(np.int64)
    t, mem = RangeTable(), Memory()
    for k, arr in enumerate((W, idx, np.zeros((n, D), np.float32))):
        t.insert(BASE + k * (1 << 20), arr.nbytes, USER)
        mem.add(BASE + k * (1 << 20), arr.view(np.uint8).reshape(-1))
    log = G.FaultLog()
    G.gather_vec(t, mem, log, 0, BASE + (2 << 20), BASE, 4 * D, BASE + (1 << 20), n)
    got = np.frombuffer(mem.read(BASE + (2 << 20), n * D * 4), np.float32).reshape(n, D)
    assert np.array_equal(got, np.take(W, idx, axis=0)) and log.count == 0


def test_scatter_add_unit_gradient_counts():
    rng = np.random.default_rng(1)
    rows, D, n = 50, 3, 2000
    idx = rng.integers(0, rows, n).astype(np.int64)
    idx[::97] = rows + 7          # out of bounds: dropped and logged
    t, mem = RangeTable(), Memory()
    for k, arr in enumerate((np.zeros((rows, D), np.float32), idx, np.ones((n, D), np.float32))):
        t.insert(BASE + k * (1 << 20), arr.nbytes, USER)
        mem.add(BASE + k * (1 << 20), arr.view(np.uint8).reshape(-1))
    log = G.FaultLog()
    G.scatter_vec(t, mem, log, 0, BASE, 4 * D, BASE + (1 << 20), BASE + (2 << 20), n,
                  accumulate=True)
    got = np.frombuffer(mem.read(BASE, rows * D * 4), np.float32).reshape(rows, D)
    ok = idx < rows
    want = np.bincount(idx[ok], minlength=rows).astype(np.float32)
    assert np.array_equal(got, np.repeat(want[:, None], D, 1))
    assert log.count == int((~ok).sum()) * D
    assert log.first["elem"] == 0 and log.first["operand"] == 2
    assert log.first["verdict"] in (V_UNMAPPED, V_CROSS_ALLOC, V_PROTECTED, V_STRADDLE)


def test_fault_reason_codes():
    t, mem, addr = scenario(0)
    log = G.FaultLog()
    # index past the table end into the adjacent allocation B -> CROSS_ALLOC, owner 1
    idx_ptr = _write_idx(mem, addr, [512 // 4])
    G.gather_vec(t, mem, log, 9, addr["C"][0], addr["A"][0], 4, idx_ptr, 1)
    f = log.first
    assert (f["verdict"], f["owner"], f["operand"], f["addr"]) == (V_CROSS_ALLOC, 1, 1,
                                                                   addr["B"][0])
    # into the protected canary -> PROTECTED with its owner id
    log.clear()
    idx_ptr = _write_idx(mem, addr, [(addr["P"][0] - addr["A"][0]) // 4])
    G.gather_vec(t, mem, log, 10, addr["C"][0], addr["A"][0], 4, idx_ptr, 1)
    assert log.first["verdict"] == V_PROTECTED and log.first["owner"] == 2
    # into the hole -> UNMAPPED; below address zero -> UNMAPPED with owner -1
    for iv in [(BASE + 1500 - addr["A"][0]) // 4, -(1 << 62)]:
        log.clear()
        idx_ptr = _write_idx(mem, addr, [iv])
        G.gather_vec(t, mem, log, 11, addr["C"][0], addr["A"][0], 4, idx_ptr, 1)
        assert log.first["verdict"] == V_UNMAPPED and log.first["owner"] == -1
    # an access running over the allocation end -> STRADDLE on the own allocation
    log.clear()
    idx_ptr = _write_idx(mem, addr, [0])
    G.gather_vec(t, mem, log, 12, addr["C"][0], addr["A"][1] - 2, 4, idx_ptr, 1)
    assert log.first["verdict"] == V_STRADDLE and log.first["owner"] == 0
    # suppressed loads read zero
    assert mem.read(addr["C"][0], 4) == bytes(4)
    assert ALLOW == 0


def test_access_straddling_the_allocation_end_is_denied():
    """The whole access must lie inside the binding (reading S9): an element whose first byte
    is inside the allocation but whose last byte is not is denied, for triad and gather, and
    its reason is STRADDLE on the own allocation. Values are derived by hand."""
    t, mem = RangeTable(), Memory()
    # b: a 10-byte allocation; elements at b+4 .. b+7 fit, b+8 .. b+11 runs past its end
    t.insert(BASE, 10, USER)
    mem.add(BASE, np.arange(10, dtype=np.uint8))
    bvals = np.frombuffer(bytes(range(10)) + bytes(2), np.float32)
    c = np.array([2.0, 3.0], np.float32)
    t.insert(BASE + 64, 8, USER)
    mem.add(BASE + 64, c.view(np.uint8))
    t.insert(BASE + 128, 8, USER)
    mem.add(BASE + 128, np.zeros(8, np.uint8))
    for fn in (G.triad_loop, G.triad_vec):
        log = RecordingLog() if fn is G.triad_loop else G.FaultLog()
        mem.write(BASE + 128, bytes(8))
        fn(t, mem, log, 5, BASE + 128, BASE + 4, BASE + 64, 1.0, 2)
        got = np.frombuffer(mem.read(BASE + 128, 8), np.float32)
        assert got[0] == np.float32(bvals[1] + np.float32(2.0))
        assert got[1] == np.float32(3.0)                     # b[1] denied: reads 0
        assert log.count == 1
        f = log.first
        assert (f["elem"], f["operand"], f["addr"], f["width"], f["verdict"], f["owner"]) == \
            (1, 0, BASE + 8, 4, V_STRADDLE, 0)
    # gather: the table's last row runs past the allocation end by two bytes
    idx = np.array([0, 1, 2], np.int64)
    t.insert(BASE + 256, 24, USER)
    mem.add(BASE + 256, idx.view(np.uint8))
    t.insert(BASE + 512, 12, USER)
    mem.add(BASE + 512, np.zeros(12, np.uint8))
    for fn in (G.gather_loop, G.gather_vec):
        log = G.FaultLog()
        mem.write(BASE + 512, bytes(12))
        fn(t, mem, log, 6, BASE + 512, BASE + 1, 4, BASE + 256, 3, 4)
        got = mem.read(BASE + 512, 12)
        # rows [1,5) and [5,9) are inside the 10-byte allocation, row [9,13) runs past its end
        assert got == bytes([1, 2, 3, 4]) + bytes([5, 6, 7, 8]) + bytes(4)
        f = log.first
        assert log.count == 1
        assert (f["elem"], f["operand"], f["addr"], f["verdict"], f["owner"]) == \
            (2, 1, BASE + 9, V_STRADDLE, 0)


# --- trap policy ----------------------------------------------------------------------
def test_trap_policy_retires_on_a_violation_only():
    """Reading of the paper's trap policy (Section V-E) with retirement of the worker whose
    context can no longer be trusted (Section IV-D): a TRAP call without a denial is an
    ordinary call; a violating TRAP call has exactly the suppress-and-log effect (the denied
    access never happens), retires the handle and reports ETRAPPED; every later call of the
    handle, under any policy, changes nothing and reports ETRAPPED; clearing the log does not
    bring the handle back."""
    t, mem, addr = scenario(4)
    ref = copy.deepcopy(mem)
    log, rlog = G.FaultLog(), G.FaultLog()
    A, B, C, P = addr["A"], addr["B"], addr["C"], addr["P"]
    assert G.guarded_call(G.copy_vec, t, mem, log, 0, C[0], A[0], 100, policy=G.TRAP) == G.OK
    G.copy_vec(t, ref, rlog, 0, C[0], A[0], 100)
    _same(mem, ref, addr)
    assert not log.retired and log.count == 0
    assert mem.read(C[0], 100) == mem.read(A[0], 100)
    bad = (P[0] - A[0]) // 4 + 1                   # row inside the protected canary
    for m in (mem, ref):
        idx_ptr = _write_idx(m, addr, [3, bad, 5])
    rc = G.guarded_call(G.gather_vec, t, mem, log, 1, C[0] + 200, A[0], 4, idx_ptr, 3,
                        policy=G.TRAP)
    G.gather_vec(t, ref, rlog, 1, C[0] + 200, A[0], 4, idx_ptr, 3)
    assert rc == G.ETRAPPED and log.retired
    _same(mem, ref, addr)
    _logs_equal(log, rlog)
    assert log.count == 1 and log.first["verdict"] == V_PROTECTED
    assert mem.read(C[0] + 200, 12) == mem.read(A[0] + 12, 4) + bytes(4) + mem.read(A[0] + 20, 4)
    # the calls below would change C if they ran
    probe = copy.deepcopy(mem)
    G.copy_vec(t, probe, G.FaultLog(), 2, C[0], B[0], 50)
    assert probe.read(C[0], 50) != mem.read(C[0], 50)
    snap = copy.deepcopy(mem)
    for pol in (G.SUPPRESS_LOG, G.SUPPRESS_ONLY, G.TRAP):
        assert G.guarded_call(G.copy_vec, t, mem, log, 2, C[0], B[0], 50, policy=pol) == G.ETRAPPED
        assert G.guarded_call(G.triad_vec, t, mem, log, 3, C[0], B[0], C[0] + 64, 2.0, 16,
                              policy=pol) == G.ETRAPPED
        assert G.guarded_call(G.scatter_vec, t, mem, log, 4, C[0], 4, idx_ptr, B[0], 3, 4, True,
                              policy=pol) == G.ETRAPPED
    _same(mem, snap, addr)
    _logs_equal(log, rlog)
    log.clear()
    assert log.retired and log.count == 0
    # a violation under the other policies never retires
    log2 = G.FaultLog()
    for pol in (G.SUPPRESS_LOG, G.SUPPRESS_ONLY):
        assert G.guarded_call(G.gather_vec, t, mem, log2, 5, C[0] + 200, A[0], 4, idx_ptr, 3,
                              policy=pol) == G.OK
    assert not log2.retired and log2.count == 1


# --- redirecting policies: sink to a quarantine, report ---------------------------------
Q_BASE, Q_SIZE = 0x5000_0000, 256


def _with_quarantine(mem, fill=0):
    mem.add(Q_BASE, np.full(Q_SIZE, fill, np.uint8) if np.isscalar(fill)
            else np.asarray(fill, np.uint8))
    return (Q_BASE, Q_SIZE)


@pytest.mark.parametrize("seed", range(4))
def test_redirecting_policies_log_like_suppress_for_copy_and_triad(seed):
    """Copy and triad deny by position only, so their logs under SINK and REPORT equal the
    SUPPRESS_LOG log exactly."""
    t, mem, addr = scenario(seed)
    rng = random.Random(seed)
    ptrs = pointer_choices(addr)
    for trial in range(25):
        dst, src, c = rng.choice(ptrs), rng.choice(ptrs), rng.choice(ptrs)
        n = rng.choice([1, 7, 64, 300])
        if _overlap(dst, n, src, n) or dst == src:
            continue
        ref = RecordingLog()
        G.copy_loop(t, copy.deepcopy(mem), ref, trial, dst, src, n)
        for pol in G.REDIRECTING:
            m = copy.deepcopy(mem)
            q = _with_quarantine(m, 7)
            log = G.FaultLog()
            G.copy_loop(t, m, log, trial, dst, src, n, pol, quarantine=q)
            _logs_equal(log, ref)
        if _overlap(dst, 4 * n, src, 4 * n) or _overlap(dst, 4 * n, c, 4 * n) or dst % 4:
            continue
        ref = RecordingLog()
        G.triad_loop(t, copy.deepcopy(mem), ref, trial, dst, src, c, 2.0, n)
        for pol in G.REDIRECTING:
            m = copy.deepcopy(mem)
            log = G.FaultLog()
            G.triad_loop(t, m, log, trial, dst, src, c, 2.0, n, pol,
                         quarantine=_with_quarantine(m))
            _logs_equal(log, ref)


def test_sink_by_hand():
    """A 16-byte copy whose source runs 6 bytes past its allocation into a hole and whose
    destination runs 4 bytes past its own: the denied source bytes read the quarantine at
    (address mod 256), the denied destination bytes land there. Values derived by hand."""
    t, mem = RangeTable(), Memory()
    src, dst = BASE + 0x100 - 10, BASE + 0x400 - 12        # 10 readable, 12 writable bytes
    t.insert(BASE, 0x100, USER)
    mem.add(BASE, np.arange(0x100, dtype=np.uint8))
    t.insert(BASE + 0x300, 0x100, USER)
    mem.add(BASE + 0x300, np.zeros(0x100, np.uint8))
    mem.add(BASE + 0x100, np.zeros(0x40, np.uint8))         # backed but unregistered
    mem.add(BASE + 0x400, np.full(0x40, 0xEE, np.uint8))
    q = _with_quarantine(mem, np.arange(Q_SIZE, dtype=np.uint8) ^ 0x5A)
    log = G.FaultLog()
    G.copy_loop(t, mem, log, 0, dst, src, 16, G.SINK, quarantine=q)
    got = mem.read(dst, 12)
    # bytes 0..9 from the source (0xF6..0xFF), bytes 10, 11 from the quarantine slots of
    # src + 10 = BASE + 0x100 and src + 11 (offsets 0x00, 0x01 mod 256)
    assert got == bytes(range(0xF6, 0x100)) + bytes([0x00 ^ 0x5A, 0x01 ^ 0x5A])
    # destination bytes 12..15 (addresses BASE + 0x400 .. 0x403) go to quarantine 0x00..0x03,
    # carrying source bytes 12..15, which themselves came from quarantine 0x02..0x05
    assert mem.read(Q_BASE, 4) == bytes([0x02 ^ 0x5A, 0x03 ^ 0x5A, 0x04 ^ 0x5A, 0x05 ^ 0x5A])
    assert mem.read(BASE + 0x400, 4) == bytes([0xEE] * 4)   # never written
    assert log.count == 6 + 4


def test_sink_aligns_the_slot_to_the_access_width():
    t, mem = RangeTable(), Memory()
    t.insert(BASE, 64, USER)
    mem.add(BASE, np.zeros(64, np.uint8))
    idx = np.array([0, 16 + 3], np.int64)        # row 19 of 4-byte rows: 12 bytes past the end
    t.insert(BASE + 0x1000, 16, USER)
    mem.add(BASE + 0x1000, idx.view(np.uint8))
    t.insert(BASE + 0x2000, 8, USER)
    mem.add(BASE + 0x2000, np.zeros(8, np.uint8))
    q = _with_quarantine(mem, np.arange(Q_SIZE, dtype=np.uint8))
    # a table pointer 2 bytes into the allocation (the oracle takes any pointer; the library
    # requires element alignment, where the rounding changes nothing)
    G.gather_loop(t, mem, G.FaultLog(), 0, BASE + 0x2000, BASE + 2, 4, BASE + 0x1000, 2, 4,
                  G.SINK, quarantine=q)
    # row 19 is at BASE + 78: (BASE + 78) mod 256 = 78, rounded down to the width: slot 76
    assert mem.read(BASE + 0x2004, 4) == bytes([76, 77, 78, 79])


def test_report_performs_only_inside_registered_ranges():
    """Under REPORT a denied access into another registered range (any kind) happens, exactly
    as an unguarded read or write of that address would; one into unregistered memory is
    suppressed, exactly as under SUPPRESS_LOG; both are logged like SUPPRESS_LOG."""
    t, mem, addr = scenario(5)
    A0, P0 = addr["A"][0], addr["P"][0]
    rows = [3, (addr["B"][0] - A0) // 4 + 2, (P0 - A0) // 4 + 1, (BASE + 1500 - A0) // 4]
    for pol in (G.REPORT, G.SUPPRESS_LOG):
        m = copy.deepcopy(mem)
        idx_ptr = _write_idx(m, addr, rows)
        log = RecordingLog()
        G.gather_loop(t, m, log, 0, addr["C"][0], A0, 4, idx_ptr, len(rows), 4, pol)
        got = [m.read(addr["C"][0] + 4 * k, 4) for k in range(len(rows))]
        plain = [m.read(A0 + 4 * r, 4) for r in rows[:3]]   # an unguarded gather's reads
        if pol == G.REPORT:
            assert got[:3] == plain and got[3] == bytes(4)      # row 3: an unbacked hole
            rep_log = (log.count, log.first)
        else:
            assert got == [plain[0], bytes(4), bytes(4), bytes(4)]
            assert (log.count, log.first) == rep_log
    # a denied store into the protected canary happens under REPORT
    m = copy.deepcopy(mem)
    G.copy_loop(t, m, G.FaultLog(), 0, P0, A0, 8, G.REPORT)
    assert m.read(P0, 8) == m.read(A0, 8) != bytes([0xA5] * 8)


def test_report_leaves_a_range_not_declared_backed_alone():
    """A registered range that was not inserted as backed may have no memory behind it: under
    REPORT a denied load there reads 0 and a denied store there is dropped (the memory model
    holds nothing at U, so touching it would raise), with the log of SUPPRESS_LOG."""
    t, mem, addr = scenario(8)
    A0, U0 = addr["A"][0], addr["U"][0]
    rows = [1, (U0 - A0) // 4 + 3, 7, (U0 - A0) // 4 + 60]
    logs = []
    for pol in (G.REPORT, G.SUPPRESS_LOG):
        m = copy.deepcopy(mem)
        idx_ptr = _write_idx(m, addr, rows)
        log = RecordingLog()
        G.gather_loop(t, m, log, 0, addr["C"][0], A0, 4, idx_ptr, len(rows), 4, pol)
        got = [m.read(addr["C"][0] + 4 * k, 4) for k in range(len(rows))]
        assert got[1] == got[3] == bytes(4)
        assert got[0] == m.read(A0 + 4, 4) and got[2] == m.read(A0 + 28, 4)
        logs.append((log.count, log.first))
    assert logs[0] == logs[1] and logs[0][0] == 2
    # a copy into U and out of U: both directions suppressed, the log counts every byte
    for dst, src in ((U0 + 16, A0), (A0 + 64, U0 + 8)):
        m = copy.deepcopy(mem)
        before = m.read(A0, 512)
        log = G.FaultLog()
        G.copy_loop(t, m, log, 0, dst, src, 8, G.REPORT)
        assert log.count == 8                   # one denied access per byte
        if dst == A0 + 64:
            assert m.read(A0 + 64, 8) == bytes(8)
        else:
            assert m.read(A0, 512) == before


def test_sink_with_a_zero_quarantine_and_no_denied_store_equals_suppress():
    """Denied loads that read an all-zero quarantine give the suppressed value."""
    t, mem, addr = scenario(6)
    rng = random.Random(6)
    rows = hostile_indices(rng, 128, 40)
    D = 2
    m1, m2 = copy.deepcopy(mem), copy.deepcopy(mem)
    for m in (m1, m2):
        idx_ptr = _write_idx(m, addr, rows)
    G.gather_loop(t, m1, G.FaultLog(), 0, addr["C"][0], addr["A"][0], 4 * D, idx_ptr, 40, 4)
    G.gather_loop(t, m2, G.FaultLog(), 0, addr["C"][0], addr["A"][0], 4 * D, idx_ptr, 40, 4,
                  G.SINK, quarantine=_with_quarantine(m2))
    _same(m1, m2, addr)


def test_sink_scatter_add_accumulates_in_the_quarantine():
    t, mem = RangeTable(), Memory()
    t.insert(BASE, 16, USER)                                  # dst: 4 fp32 rows of 1
    mem.add(BASE, np.zeros(4, np.float32).view(np.uint8))
    idx = np.array([1, 4, 4, 9], np.int64)                    # rows 4 and 9 are past the end
    t.insert(BASE + 0x1000, 32, USER)
    mem.add(BASE + 0x1000, idx.view(np.uint8))
    src = np.array([1.0, 2.0, 3.0, 4.0], np.float32)
    t.insert(BASE + 0x2000, 16, USER)
    mem.add(BASE + 0x2000, src.view(np.uint8))
    q = _with_quarantine(mem)
    G.scatter_loop(t, mem, G.FaultLog(), 0, BASE, 4, BASE + 0x1000, BASE + 0x2000, 4, 4, True,
                   G.SINK, quarantine=q)
    dst = np.frombuffer(mem.read(BASE, 16), np.float32)
    assert dst.tolist() == [0.0, 1.0, 0.0, 0.0]
    quar = np.frombuffer(mem.read(Q_BASE, Q_SIZE), np.float32)
    # row 4 -> BASE + 16 (slot 16 / 4 = 4), row 9 -> BASE + 36 (slot 9)
    assert quar[4] == 5.0 and quar[9] == 4.0 and quar.sum() == 9.0


def test_remap_copy_from_a_short_allocation_repeats_it():
    """A copy of 1000 bytes from a 37-byte allocation under REMAP reads byte k at k mod 37:
    numpy's tiled repetition of the source."""
    t, mem = RangeTable(), Memory()
    src = np.arange(37, dtype=np.uint8) * 3
    t.insert(BASE + 3, 37, USER)
    mem.add(BASE + 3, src)
    t.insert(BASE + 0x1000, 1000, USER)
    mem.add(BASE + 0x1000, np.zeros(1000, np.uint8))
    log = G.FaultLog()
    G.copy_loop(t, mem, log, 0, BASE + 0x1000, BASE + 3, 1000, G.REMAP)
    assert mem.read(BASE + 0x1000, 1000) == np.resize(src, 1000).tobytes()
    assert log.count == 1000 - 37


@pytest.mark.parametrize("D", [1, 3])
def test_remap_gather_wraps_rows_like_take(D):
    """A table allocation of rows*rb + 2 bytes: REMAP wraps whole elements, so every index
    (past the end or negative) reads row idx mod rows, as np.take(..., mode='wrap')."""
    rng = np.random.default_rng(D)
    rows, n = 37, 200
    W = rng.integers(-50, 50, (rows, D)).astype(np.float32)
    idx = rng.integers(-500, 500, n).astype(np.int64)
    t, mem = RangeTable(), Memory()
    t.insert(BASE, W.nbytes + 2, USER)
    mem.add(BASE, np.concatenate([W.view(np.uint8).reshape(-1), np.zeros(2, np.uint8)]))
    t.insert(BASE + (1 << 20), idx.nbytes, USER)
    mem.add(BASE + (1 << 20), idx.view(np.uint8))
    t.insert(BASE + (2 << 20), n * D * 4, USER)
    mem.add(BASE + (2 << 20), np.zeros(n * D * 4, np.uint8))
    G.gather_loop(t, mem, G.FaultLog(), 0, BASE + (2 << 20), BASE, 4 * D, BASE + (1 << 20), n,
                  4, G.REMAP)
    got = np.frombuffer(mem.read(BASE + (2 << 20), n * D * 4), np.float32).reshape(n, D)
    assert np.array_equal(got, np.take(W, idx, axis=0, mode="wrap"))


def test_remap_without_a_binding_suppresses():
    t, mem, addr = scenario(7)
    m1, m2 = copy.deepcopy(mem), copy.deepcopy(mem)
    G.copy_loop(t, m1, G.FaultLog(), 0, addr["P"][0], addr["A"][0], 64, G.REMAP)
    G.copy_loop(t, m2, G.FaultLog(), 0, addr["P"][0], addr["A"][0], 64)
    _same(m1, m2, addr)
    assert m1.read(addr["P"][0], 64) == bytes([0xA5] * 64)
