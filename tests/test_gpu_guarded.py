"""Guarded copy / triad / gather / scatter(-add) on the GPU against the oracle.

A device arena holds USER allocations A, B (adjacent), C, I (indices), O (outputs), a
protected canary P, an MMIO range M and an unregistered hole; a far protected range is
registered without backing. Hostile pointers and indices are drawn from all of them. After
every call the whole arena must equal the oracle's memory model byte for byte, and the fault
log (count and first record) must equal the oracle's.
"""
import random

import numpy as np
import pytest
import torch

from gpu_util import Arena, Twin, log_matches, need_gpu
from oracle import guarded as G

pytestmark = pytest.mark.gpu

REG = {"A": (0x0000, 0x4000, 0), "B": (0x4000, 0x6000, 0), "P": (0x6000, 0x7000, 1),
       "C": (0x8000, 0x10000, 0), "M": (0x10000, 0x10400, 2), "I": (0x11000, 0x13000, 0),
       "O": (0x14000, 0x1C000, 0)}
ARENA = 0x20000
FAR = 1 << 40


def setup(seed):
    need_gpu()
    ar = Arena(ARENA, seed)
    tw = Twin(64)
    for k, (lo, hi, kind) in REG.items():
        tw.insert(ar.addr(lo), hi - lo, kind)
    tw.insert(FAR, 4096, 1)
    return ar, tw


def fill_floats(ar, rng, dtype=np.float32, integer=False):
    for k in ("A", "B", "C", "O"):
        lo, hi, _ = REG[k]
        n = (hi - lo) // np.dtype(dtype).itemsize
        if integer:
            v = rng.integers(-50, 51, n).astype(dtype)
        else:
            v = (rng.standard_normal(n) * np.exp2(rng.integers(-20, 20, n))).astype(dtype)
            v[::97] = dtype(0.0)
            v[1::101] = -dtype(0.0)
            v[2::89] = np.array(1e-40 if dtype == np.float32 else 1e-310, dtype=dtype)
        ar.write(lo, v)


def pointer_pool(ar, align):
    pts = []
    for k, (lo, hi, _) in REG.items():
        for off in (0, align, 3 * align, 16, (hi - lo) // 2, hi - lo - 4 * align, hi - lo - align):
            pts.append(ar.addr(lo + off - (off % align)))
    pts += [ar.addr(0x7000), ar.addr(0x7800), FAR, FAR + 64, 0, ar.addr(ARENA - 64)]
    return pts


def _overlap(p, n, q, m):
    return n > 0 and m > 0 and p < q + m and q < p + n


def test_copy_random_cases():
    ar, tw = setup(1)
    rng = random.Random(1)
    ol = G.FaultLog()
    pool = pointer_pool(ar, 1) + [ar.addr(0x8001), ar.addr(0x8003), ar.addr(0x400d)]
    ran = 0
    for trial in range(160):
        dst, src = rng.choice(pool), rng.choice(pool)
        n = rng.choice([0, 1, 3, 15, 16, 17, 31, 64, 100, 1000, 4096, 9000, 20000, 40000])
        if _overlap(dst, n, src, n):
            continue
        policy = G.SUPPRESS_ONLY if trial % 11 == 5 else G.SUPPRESS_LOG
        tw.g.agile_guarded_copy(tw.h, dst, src, n, policy)
        G.copy_vec(tw.ot, ar.mem, ol, tw.next_seq(), dst, src, n, policy)
        ar.check(f"copy trial {trial} dst={dst - ar.base:#x} src={src - ar.base:#x} n={n}")
        log_matches(tw, ol, f"copy trial {trial}")
        ran += 1
    assert ran > 100
    tw.close()


def test_copy_16mib_fp32_no_faults():
    """16 MiB of fp32 uniform[-1,1] between two registered buffers: bit-exact, empty log."""
    need_gpu()
    from synth import uniform_f32
    src = uniform_f32(4 << 20, 0, device="cuda")
    dst = torch.zeros_like(src)
    tw = Twin(8)
    tw.insert(src.data_ptr(), src.numel() * 4, 0)
    tw.insert(dst.data_ptr(), dst.numel() * 4, 0)
    tw.g.agile_guarded_copy(tw.h, dst, src, src.numel() * 4)
    torch.cuda.synchronize()
    assert torch.equal(dst.view(torch.int32), src.view(torch.int32))
    rc, f = tw.rt.fault_log()
    assert rc == tw.g.AGILE_OK and f["count"] == 0 and f["first_seq"] == tw.g.NO_SEQ
    out2 = torch.zeros_like(src)
    tw.g.agile_unguarded_copy(out2, src, src.numel() * 4)
    torch.cuda.synchronize()
    assert torch.equal(out2, dst)
    tw.close()


def test_triad_random_cases():
    ar, tw = setup(2)
    rng = random.Random(2)
    fill_floats(ar, np.random.default_rng(2))
    ol = G.FaultLog()
    pool = pointer_pool(ar, 4)
    ran = 0
    for trial in range(120):
        a, b, c = rng.choice(pool), rng.choice(pool), rng.choice(pool)
        n = rng.choice([0, 1, 3, 4, 5, 17, 100, 1000, 2048, 5000])
        if (a != b and _overlap(a, 4 * n, b, 4 * n)) or (a != c and _overlap(a, 4 * n, c, 4 * n)):
            continue
        s = rng.choice([3.0, -1.5, 1e-30, 0.0])
        tw.g.agile_guarded_triad(tw.h, a, b, c, s, n)
        G.triad_vec(tw.ot, ar.mem, ol, tw.next_seq(), a, b, c, s, n)
        ar.check(f"triad trial {trial} n={n}")
        log_matches(tw, ol, f"triad trial {trial}")
        ran += 1
    assert ran > 80
    tw.close()


def hostile_indices(rng, rows, n, extra_rows=()):
    base = [0, 1, rows - 1, rows, rows + 1, -1, -2, 3 * rows, -(1 << 62), (1 << 62),
            -(1 << 63), (1 << 63) - 1, (1 << 40) + 3] + list(extra_rows)
    vals = []
    for _ in range(n):
        if rng.random() < 0.75:
            vals.append(rng.randrange(0, max(rows, 1)))
        else:
            vals.append(rng.choice(base))
    return np.array(vals, dtype=np.int64)


# row shapes for every gather/scatter path: narrow rows (<= 16 B), rows of a part of a wave, rows of a
# whole wave in 16-byte chunks (1 KiB), and rows of a whole wave in element-wide chunks (a row whose
# size is not a multiple of 16 bytes and spans more than 64 elements: (4, 67), (8, 33)); (4, 100)
# leaves 7 of its 32 lanes idle
ROWS_CASES = [(4, 1), (4, 2), (4, 3), (4, 4), (4, 8), (4, 64), (4, 256), (8, 1), (8, 2), (8, 32),
              (4, 67), (8, 33), (4, 100)]


@pytest.mark.parametrize("w,D", ROWS_CASES)
def test_gather_random_cases(w, D):
    ar, tw = setup(3 + D + w)
    rng = random.Random(D * 10 + w)
    ol = G.FaultLog()
    rb = w * D
    dtype = 0 if w == 4 else 1
    ran = 0
    for trial in range(25):
        tname = rng.choice(["A", "A", "C", "B", "P", "hole", "far", "Aoff", "Cend"])
        if tname == "hole":
            T = ar.addr(0x7000)
        elif tname == "far":
            T = FAR
        elif tname == "Aoff":
            T = ar.addr(REG["A"][0] + w * rng.randrange(1, 9))
        elif tname == "Cend":
            T = ar.addr(REG["C"][1] - rb * 3 - w)
        else:
            T = ar.addr(REG[tname][0])
        lo, hi = tw.ot.binding(T)
        rows = max(1, (hi - T) // rb) if hi > lo else 16
        # indices that land in P (protected) and B (another allocation) from table A
        extra = [(ar.addr(0x6000) - T) // rb, (ar.addr(0x4000) - T) // rb + 1]
        n = rng.choice([0, 1, 2, 7, 33, 100, 257, 1024])
        idx = hostile_indices(rng, rows, max(n, 1), extra)
        ar.write(REG["I"][0], idx)
        idx_ptr = ar.addr(REG["I"][0])
        if rng.random() < 0.15:
            idx_ptr = ar.addr(REG["I"][1] - 8 * rng.randrange(1, 5))   # index buffer runs out
        out = rng.choice([ar.addr(REG["O"][0]), ar.addr(REG["O"][1] - rb * 5 - w),
                          ar.addr(REG["P"][0]), FAR])
        tw.g.agile_guarded_gather(tw.h, out, T, rb, idx_ptr, n, dtype)
        G.gather_vec(tw.ot, ar.mem, ol, tw.next_seq(), out, T, rb, idx_ptr, n, w)
        ar.check(f"gather w={w} D={D} trial {trial} T={tname} n={n}")
        log_matches(tw, ol, f"gather w={w} D={D} trial {trial} T={tname} n={n}")
        ran += 1
    tw.close()


@pytest.mark.parametrize("w,D", ROWS_CASES)
@pytest.mark.parametrize("accumulate", [0, 1])
def test_scatter_random_cases(w, D, accumulate):
    ar, tw = setup(5 + D + w + accumulate)
    rng = random.Random(D * 100 + w + accumulate)
    fill_floats(ar, np.random.default_rng(D + w), np.float32 if w == 4 else np.float64,
                integer=True)
    ol = G.FaultLog()
    rb = w * D
    dtype = 0 if w == 4 else 1
    for trial in range(20):
        dname = rng.choice(["A", "A", "C", "P", "hole", "Aoff"])
        if dname == "hole":
            dst = ar.addr(0x7000)
        elif dname == "Aoff":
            dst = ar.addr(REG["A"][0] + w * rng.randrange(1, 9))
        else:
            dst = ar.addr(REG[dname][0])
        lo, hi = tw.ot.binding(dst)
        rows = max(1, (hi - dst) // rb) if hi > lo else 16
        n = rng.choice([0, 1, 5, 33, 200])
        if accumulate:
            idx = hostile_indices(rng, rows, max(n, 1), [(ar.addr(0x6000) - dst) // rb])
        else:
            pool = list(range(rows)) + [rows, rows + 3, -1, 1 << 40, -(1 << 62)]
            rng.shuffle(pool)
            idx = np.array((pool * (1 + max(n, 1) // len(pool)))[:max(n, 1)], dtype=np.int64)
            if len(set(idx.tolist())) < idx.size:     # plain scatter needs unique indices
                continue
        ar.write(REG["I"][0], idx)
        idx_ptr = ar.addr(REG["I"][0])
        src = rng.choice([ar.addr(REG["O"][0]), ar.addr(REG["O"][1] - rb * 3),
                          ar.addr(REG["P"][0])])
        tw.g.agile_guarded_scatter(tw.h, dst, rb, idx_ptr, src, n, dtype, accumulate)
        G.scatter_vec(tw.ot, ar.mem, ol, tw.next_seq(), dst, rb, idx_ptr, src, n, w,
                      bool(accumulate))
        ar.check(f"scatter acc={accumulate} w={w} D={D} trial {trial} n={n}")
        log_matches(tw, ol, f"scatter acc={accumulate} w={w} D={D} trial {trial}")
    tw.close()


def test_log_accumulates_and_policies():
    """count adds up over calls, the earliest faulting call keeps the record, SUPPRESS_ONLY
    calls take a sequence number but record nothing, clearing empties the log."""
    ar, tw = setup(9)
    ol = G.FaultLog()
    A, P, C = ar.addr(0x0000), ar.addr(0x6000), ar.addr(0x8000)
    calls = [(C, A, 100, G.SUPPRESS_LOG), (P, A, 10, G.SUPPRESS_ONLY), (P, A, 20, G.SUPPRESS_LOG),
             (C, ar.addr(0x3FF0), 64, G.SUPPRESS_LOG)]
    for dst, src, n, pol in calls:
        tw.g.agile_guarded_copy(tw.h, dst, src, n, pol)
        G.copy_vec(tw.ot, ar.mem, ol, tw.next_seq(), dst, src, n, pol)
    ar.check("log sequence")
    rc, f = tw.rt.fault_log(clear=False)
    # call 2: 20 dropped stores into P; call 4: 48 src bytes past A's end (dst C is fine)
    assert rc == tw.g.AGILE_EFAULTED and f["count"] == ol.count == 20 + 48
    assert f["first_seq"] == 2 and f["first_verdict"] == 1    # the protected store of call 2
    log_matches(tw, ol, "log sequence")
    rc, f = tw.rt.fault_log()
    assert rc == tw.g.AGILE_OK and f["count"] == 0
    tw.close()


def test_unguarded_twins_match_guarded_on_valid_inputs():
    need_gpu()
    g = Twin(8)
    n = (1 << 20) + 3
    b = torch.randn(n, device="cuda")
    c = torch.randn(n, device="cuda")
    a1 = torch.empty_like(b)
    a2 = torch.empty_like(b)
    for t in (a1, b, c):
        g.insert(t.data_ptr(), t.numel() * 4, 0)
    g.g.agile_guarded_triad(g.h, a1, b, c, 3.0, n)
    g.g.agile_unguarded_triad(a2, b, c, 3.0, n)
    torch.cuda.synchronize()
    assert torch.equal(a1.view(torch.int32), a2.view(torch.int32))
    ref = (b.cpu().numpy() + np.float32(3.0) * c.cpu().numpy()).astype(np.float32)
    assert np.array_equal(a1.cpu().numpy().view(np.int32), ref.view(np.int32))
    W = torch.randn(1000, 64, device="cuda")
    idx = torch.randint(0, 1000, (5000,), device="cuda")
    o1 = torch.empty(5000, 64, device="cuda")
    o2 = torch.empty_like(o1)
    for t in (W, idx, o1):
        g.insert(t.data_ptr(), t.numel() * t.element_size(), 0)
    g.g.agile_guarded_gather(g.h, o1, W, 256, idx, 5000)
    g.g.agile_unguarded_gather(o2, W, 256, idx, 5000)
    torch.cuda.synchronize()
    assert torch.equal(o1, o2) and torch.equal(o1, W[idx])
    rc, f = g.rt.fault_log()
    assert rc == g.g.AGILE_OK
    g.close()


def test_elements_straddling_an_allocation_end():
    """Allocations whose ends fall inside an element: the element that straddles the end is
    denied as a whole (its first bytes are inside), for triad, gather, scatter and
    scatter-add, on both row kernels' fast and exact paths."""
    need_gpu()
    ar = Arena(1 << 16, 77)
    tw = Twin(16)
    X = (0x100, 0x100 + 1026)        # 256.5 floats
    Y = (0x1000, 0x1000 + 4094)
    Z = (0x3000, 0x3000 + 4096)
    I = (0x5000, 0x5000 + 2048)
    for lo, hi in (X, Y, Z, I):
        tw.insert(ar.addr(lo), hi - lo, 0)
    rng = np.random.default_rng(5)
    for lo, hi in (X, Y, Z):
        ar.write(lo, rng.integers(-50, 51, (hi - lo) // 4).astype(np.float32))
    ol = G.FaultLog()
    # triad: b runs out inside element 256
    for n in (256, 257, 300):
        tw.g.agile_guarded_triad(tw.h, ar.addr(Z[0]), ar.addr(X[0]), ar.addr(Y[0]), 2.0, n)
        G.triad_vec(tw.ot, ar.mem, ol, tw.next_seq(), ar.addr(Z[0]), ar.addr(X[0]),
                    ar.addr(Y[0]), 2.0, n)
        ar.check(f"triad straddle n={n}")
        log_matches(tw, ol, f"triad straddle n={n}")
    # gather / scatter / scatter-add with rows of 8 bytes over X: row 128 straddles the end
    idx = np.array([0, 127, 128, 5, 128, 129, -1, 64], dtype=np.int64)
    ar.write(I[0], idx)
    for D, dtype, w in ((2, 0, 4), (1, 1, 8), (4, 0, 4)):
        rb = w * D
        tw.g.agile_guarded_gather(tw.h, ar.addr(Z[0]), ar.addr(X[0]), rb, ar.addr(I[0]),
                                  idx.size, dtype)
        G.gather_vec(tw.ot, ar.mem, ol, tw.next_seq(), ar.addr(Z[0]), ar.addr(X[0]), rb,
                     ar.addr(I[0]), idx.size, w)
        ar.check(f"gather straddle D={D} w={w}")
        log_matches(tw, ol, f"gather straddle D={D} w={w}")
        for acc in (0, 1):
            uniq = idx if acc else np.array([0, 127, 128, 5, 129, -1, 64, 3], dtype=np.int64)
            ar.write(I[0], uniq)
            tw.g.agile_guarded_scatter(tw.h, ar.addr(X[0]), rb, ar.addr(I[0]), ar.addr(Y[0]),
                                       uniq.size, dtype, acc)
            G.scatter_vec(tw.ot, ar.mem, ol, tw.next_seq(), ar.addr(X[0]), rb, ar.addr(I[0]),
                          ar.addr(Y[0]), uniq.size, w, bool(acc))
            ar.check(f"scatter straddle D={D} w={w} acc={acc}")
            log_matches(tw, ol, f"scatter straddle D={D} w={w} acc={acc}")
        ar.write(I[0], idx)
    tw.close()
