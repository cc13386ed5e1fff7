"""The redirecting guard policies on the device against the oracle's per-access definition.

SINK sends every denied access to a caller-provided quarantine (slot = address mod its size,
rounded down to the width); REPORT performs a denied access when it lies inside a registered
range of any kind and suppresses it otherwise; REMAP rewrites it into the USER range of its own
pointer argument, modulo that range's size (Section V-E, sink, report and remap_or). One arena
holds:
a USER table/destination A, a protected canary P, an unregistered hole H, another USER
allocation X, an index buffer I, a source S, an output C and the quarantine Q (not
registered). Every registered range lies in the arena and is inserted as backed, so REPORT only
ever touches arena bytes; one case registers P without that statement, and REPORT must then
leave it alone. Values are small integers, so sums are exact in any order, and the whole arena,
quarantine included, must equal the oracle's memory byte for byte. Within one call the denied
accesses that reach the same quarantine slot or address are either all loads or all adds
(their order is unspecified, as for duplicate indices of a plain scatter); under REMAP the
layouts keep rewritten stores off every address that an allowed access of the same call reads
or writes.
"""
import numpy as np
import pytest

from gpu_util import Arena, Twin, log_matches, need_gpu
from oracle import guarded as G

pytestmark = pytest.mark.gpu

QSIZE = 4096
ROWS, NMAX = 1024, 40000


def layout(rb):
    off, o = {}, 0
    for name, size in (("A", ROWS * rb), ("P", 4096), ("H", 4096), ("X", 8192),
                       ("I", NMAX * 8), ("S", NMAX * rb), ("C", NMAX * rb), ("Q", QSIZE)):
        o = (o + 4095) // 4096 * 4096
        off[name] = (o, o + size)
        o += size
    return off, (o + 4095) // 4096 * 4096


def setup(w, D, seed, backed_p=True):
    need_gpu()
    rb = w * D
    off, size = layout(rb)
    ar = Arena(size, seed)
    tw = Twin(16)
    for k, kind in (("A", 0), ("P", 1), ("X", 0), ("I", 0), ("S", 0), ("C", 0)):
        lo, hi = off[k]
        tw.insert(ar.addr(lo), hi - lo, kind, backed=backed_p or k != "P")
    dt = np.float32 if w == 4 else np.float64
    rng = np.random.default_rng(seed)
    for k in ("A", "P", "H", "X", "S", "C"):
        lo, hi = off[k]
        ar.write(lo, rng.integers(-20, 21, (hi - lo) // w).astype(dt))
    q0 = off["Q"][0]
    tw.g.agile_rt_set_quarantine(tw.h, ar.addr(q0), QSIZE)
    return ar, tw, off, dt, rng


def run_both(tw, ar, fn_dev, fn_or, ol, what):
    fn_dev()
    fn_or()
    ar.check(what)
    log_matches(tw, ol, what)


@pytest.mark.parametrize("policy", [G.SINK, G.REPORT, G.REMAP])
@pytest.mark.parametrize("w,D", [(4, 1), (4, 4), (8, 2)])
def test_gather_and_scatter_redirected(policy, w, D):
    ar, tw, off, dt, rng = setup(w, D, 11 + w + D + policy)
    g = tw.g
    rb = w * D
    A, I, S, C, Q = (ar.addr(off[k][0]) for k in ("A", "I", "S", "C", "Q"))
    quar = (Q, QSIZE)
    # quarantine: small valid row numbers as int64 (read by denied index loads) and values
    qv = np.zeros(QSIZE // 8, np.int64)
    qv[:] = rng.integers(0, ROWS, qv.size)
    ar.write(off["Q"][0], qv)
    ol = G.FaultLog()
    past = [ROWS + k for k in range(0, (4096 + 4096 + 8192) // rb, 7)]   # into P, H and X
    before = [-1, -2, -(1 << 40)]
    n = 600
    # 1. denied table loads only (rows past the table and before it), all outputs allowed
    idx = rng.integers(0, ROWS, n).astype(np.int64)
    pos = rng.choice(n, len(past) + len(before), replace=False)
    idx[pos] = past + before
    ar.write(off["I"][0], idx)
    run_both(tw, ar, lambda: g.agile_guarded_gather(tw.h, C, A, rb, I, n, 0 if w == 4 else 1,
                                                    policy),
             lambda: G.gather_loop(tw.ot, ar.mem, ol, tw.next_seq(), C, A, rb, I, n, w, policy,
                                   quarantine=quar), ol, "gather, denied loads")
    # 2. denied index loads: the index buffer ends 100 rows before n (SINK reads the row
    #    numbers from the quarantine; under REPORT they lie in the unregistered padding after I
    #    and read as 0)
    i_end = off["I"][1]
    Iend = ar.addr(i_end - 8 * (n - 100))
    ar.write(i_end - 8 * (n - 100), rng.integers(0, ROWS, n - 100).astype(np.int64))
    run_both(tw, ar, lambda: g.agile_guarded_gather(tw.h, C, A, rb, Iend, n, 0 if w == 4 else 1,
                                                    policy),
             lambda: G.gather_loop(tw.ot, ar.mem, ol, tw.next_seq(), C, A, rb, Iend, n, w,
                                   policy, quarantine=quar), ol, "gather, denied index loads")
    # 3. denied output stores: the output runs 50 rows past C's end (into the next buffer)
    ar.write(off["I"][0], rng.integers(0, ROWS, n).astype(np.int64))
    Cend = ar.addr(off["C"][1] - rb * (n - 50))
    run_both(tw, ar, lambda: g.agile_guarded_gather(tw.h, Cend, A, rb, I, n, 0 if w == 4 else 1,
                                                    policy),
             lambda: G.gather_loop(tw.ot, ar.mem, ol, tw.next_seq(), Cend, A, rb, I, n, w,
                                   policy, quarantine=quar), ol, "gather, denied stores")
    # 4. scatter with destination rows past the end of A (distinct rows: stores only). Under
    #    SINK they stay within 4 KiB (P), so that no two of them share a quarantine slot; under
    #    REMAP (row r goes to row r mod ROWS) the allowed rows avoid every rewritten one.
    idx = rng.permutation(ROWS)[:n].astype(np.int64)
    past_st = [r for r in past if (r - ROWS) * rb < 4096] if policy == G.SINK else past
    if policy == G.REMAP:
        past_st = past[::5]
        hit = {r % ROWS for r in past_st}
        assert len(hit) == len(past_st)
        idx = rng.permutation([r for r in range(ROWS) if r not in hit])[:n].astype(np.int64)
    pos = rng.choice(n, len(past_st), replace=False)
    idx[pos] = past_st
    ar.write(off["I"][0], idx)
    run_both(tw, ar, lambda: g.agile_guarded_scatter(tw.h, A, rb, I, S, n, 0 if w == 4 else 1, 0,
                                                     policy),
             lambda: G.scatter_loop(tw.ot, ar.mem, ol, tw.next_seq(), A, rb, I, S, n, w, False,
                                    policy, quarantine=quar), ol, "scatter")
    tw.close()


@pytest.mark.parametrize("policy", [G.SINK, G.REPORT, G.REMAP])
@pytest.mark.parametrize("n", [600, NMAX])
def test_scatter_add_redirected(policy, n):
    """Duplicate destination rows, rows past the end (into P, H, X) and before it, and a
    source that runs out 30 rows early; NMAX rows take the sorted path."""
    w, D = 4, 2
    ar, tw, off, dt, rng = setup(w, D, 50 + n + policy)
    g = tw.g
    rb = w * D
    A, I, S, Q = (ar.addr(off[k][0]) for k in ("A", "I", "S", "Q"))
    ol = G.FaultLog()
    ar.write(off["Q"][0], np.zeros(QSIZE // 4, np.float32))
    idx = rng.integers(0, 64, n).astype(np.int64)
    bad = rng.choice(n, 200, replace=False)
    # quarantine slots of these rows (A + 8 r mod 4096: 0, 24, 3200, 3808, 4088, 4040) stay
    # clear of those of the source's denied loads (S's end + 8 k: 512 .. 752)
    idx[bad] = rng.choice([ROWS, ROWS + 3, ROWS + 400, ROWS + 1500, -1, -7], 200)
    ar.write(off["I"][0], idx)
    Send = ar.addr(off["S"][1] - rb * (n - 30))
    run_both(tw, ar, lambda: g.agile_guarded_scatter(tw.h, A, rb, I, Send, n, 0, 1, policy),
             lambda: G.scatter_loop(tw.ot, ar.mem, ol, tw.next_seq(), A, rb, I, Send, n, w, True,
                                    policy, quarantine=(Q, QSIZE)), ol, f"scatter-add n={n}")
    tw.close()


@pytest.mark.parametrize("policy", [G.SINK, G.REPORT, G.REMAP])
def test_copy_and_triad_redirected(policy):
    w, D = 4, 1
    ar, tw, off, dt, rng = setup(w, D, 70 + policy)
    g = tw.g
    A, X, C, Q = (ar.addr(off[k][0]) for k in ("A", "X", "C", "Q"))
    quar = (Q, QSIZE)
    ar.write(off["Q"][0], rng.integers(-20, 21, QSIZE // 4).astype(np.float32))
    ol = G.FaultLog()
    a_end = off["A"][1]
    # copy: the source runs 1000 bytes past A into P (loads), then the destination runs 1000
    # bytes past A (stores)
    src = ar.addr(a_end - 3000)
    run_both(tw, ar, lambda: g.agile_guarded_copy(tw.h, C, src, 4000, policy),
             lambda: G.copy_loop(tw.ot, ar.mem, ol, tw.next_seq(), C, src, 4000, policy,
                                 quarantine=quar), ol, "copy, denied loads")
    run_both(tw, ar, lambda: g.agile_guarded_copy(tw.h, src, C, 4000, policy),
             lambda: G.copy_loop(tw.ot, ar.mem, ol, tw.next_seq(), src, C, 4000, policy,
                                 quarantine=quar), ol, "copy, denied stores")
    # triad: b runs 200 elements past A, then a runs 200 elements past A
    bb = ar.addr(a_end - 4 * 300)
    run_both(tw, ar, lambda: g.agile_guarded_triad(tw.h, C, bb, X, 2.0, 500, policy),
             lambda: G.triad_loop(tw.ot, ar.mem, ol, tw.next_seq(), C, bb, X, 2.0, 500, policy,
                                  quarantine=quar), ol, "triad, denied loads")
    run_both(tw, ar, lambda: g.agile_guarded_triad(tw.h, bb, C, X, 2.0, 500, policy),
             lambda: G.triad_loop(tw.ot, ar.mem, ol, tw.next_seq(), bb, C, X, 2.0, 500, policy,
                                  quarantine=quar), ol, "triad, denied stores")
    tw.close()


def test_sink_without_quarantine_is_refused():
    need_gpu()
    tw = Twin(4)
    g = tw.g
    g.agile_rt_set_quarantine(tw.h, 0, 0)
    with pytest.raises(g.AgileError) as e:
        g.agile_guarded_copy(tw.h, 0, 0, 16, G.SINK)
    assert e.value.code == g.AGILE_EINVAL
    for bad in ((1 << 20, 300), (1 << 20, 4096 + 256), ((1 << 20) + 8, 4096)):
        with pytest.raises(g.AgileError):
            g.agile_rt_set_quarantine(tw.h, *bad)
    tw.close()


def test_remap_rounds_an_unaligned_binding_up():
    """REMAP with a USER range that starts at an odd address and has an odd size: rewritten
    accesses go to lo' = lo rounded up to 4 plus a multiple of 4 below m = the largest multiple
    of 4 not above hi - lo'. Denied loads (b runs past the range) and denied stores (a runs
    past it) against the oracle; the rewritten stores land below the allowed ones."""
    need_gpu()
    ar = Arena(1 << 16, 91)
    tw = Twin(8)
    g = tw.g
    U0, U1 = 1, 1 + 4001
    tw.insert(ar.addr(U0), U1 - U0, 0)
    tw.insert(ar.addr(8192), 4096, 0)     # C
    tw.insert(ar.addr(16384), 4096, 0)    # X
    rng = np.random.default_rng(91)
    for off, size in ((0, 1 << 14), (16384, 4096)):
        ar.write(off, rng.integers(-20, 21, size // 4).astype(np.float32))
    ol = G.FaultLog()
    C, X = ar.addr(8192), ar.addr(16384)
    b = ar.addr(4)                          # inside U, 4-aligned; elements 999.. are denied
    run_both(tw, ar, lambda: g.agile_guarded_triad(tw.h, C, b, X, 2.0, 1024, G.REMAP),
             lambda: G.triad_loop(tw.ot, ar.mem, ol, tw.next_seq(), C, b, X, 2.0, 1024, G.REMAP),
             ol, "remap, unaligned binding, denied loads")
    a = ar.addr(2000)                       # elements 500.. are denied stores
    run_both(tw, ar, lambda: g.agile_guarded_triad(tw.h, a, C, X, 2.0, 600, G.REMAP),
             lambda: G.triad_loop(tw.ot, ar.mem, ol, tw.next_seq(), a, C, X, 2.0, 600, G.REMAP),
             ol, "remap, unaligned binding, denied stores")
    tw.close()


@pytest.mark.parametrize("w,D", [(4, 1), (8, 2)])
def test_report_leaves_a_range_not_declared_backed_alone(w, D):
    """P is registered as protected but not as backed: under REPORT denied loads from it read 0
    and denied stores into it are dropped (P keeps its bytes), exactly as the oracle says; the
    other registered ranges are still reported through."""
    ar, tw, off, dt, rng = setup(w, D, 91 + w, backed_p=False)
    g = tw.g
    rb = w * D
    A, I, S, C = (ar.addr(off[k][0]) for k in ("A", "I", "S", "C"))
    ol = G.FaultLog()
    n = 500
    into_p = [ROWS + k for k in range(0, 4096 // rb, 9)]           # rows inside P
    into_x = [ROWS + 8192 // rb + k for k in range(0, 8192 // rb, 13)]   # rows inside X
    idx = rng.integers(0, ROWS, n).astype(np.int64)
    pos = rng.choice(n, len(into_p) + len(into_x), replace=False)
    idx[pos] = into_p + into_x
    ar.write(off["I"][0], idx)
    run_both(tw, ar, lambda: g.agile_guarded_gather(tw.h, C, A, rb, I, n, 0 if w == 4 else 1,
                                                    G.REPORT),
             lambda: G.gather_loop(tw.ot, ar.mem, ol, tw.next_seq(), C, A, rb, I, n, w,
                                   G.REPORT), ol, "report gather, P not backed")
    # scatter into P (dropped) and into X (performed), distinct rows
    idx = rng.permutation(ROWS)[:n].astype(np.int64)
    pos = rng.choice(n, len(into_p) + len(into_x), replace=False)
    idx[pos] = into_p + into_x
    ar.write(off["I"][0], idx)
    run_both(tw, ar, lambda: g.agile_guarded_scatter(tw.h, A, rb, I, S, n, 0 if w == 4 else 1, 0,
                                                     G.REPORT),
             lambda: G.scatter_loop(tw.ot, ar.mem, ol, tw.next_seq(), A, rb, I, S, n, w, False,
                                    G.REPORT), ol, "report scatter, P not backed")
    tw.close()
