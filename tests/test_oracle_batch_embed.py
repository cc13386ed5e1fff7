"""Pins for the oracle's batched verdicts and embedding gradient (CPU only)."""
import numpy as np
import pytest

from oracle import RangeTable, ALLOW, V_UNMAPPED, USER
from oracle.batched import batch_verdicts
from oracle.brute import verdict_brute
from oracle.embedding import embedding_grad_ref, embedding_forward_ref
from synth import make_table, make_batch_requests


def _oracle_tables(gen_tables):
    out = []
    for tb in gen_tables:
        t = RangeTable()
        for b, s, k in zip(tb.base.tolist(), tb.size.tolist(), tb.kind.tolist()):
            t.insert(b, s, k)
        out.append(t)
    return out


def test_batch_verdicts_against_brute():
    gts = [make_table(40, 10, 100 + c) for c in range(3)]
    tabs = _oracle_tables(gts)
    req = make_batch_requests(gts, 12, 3, max_ptrs=40)
    pv, po, rv, ra, ro = batch_verdicts(tabs, req["client"].numpy(), req["ptr_off"].numpy(),
                                        req["ptrs"].numpy())
    off = req["ptr_off"].tolist()
    ptrs = req["ptrs"].tolist()
    for r in range(12):
        ents = tabs[int(req["client"][r])].entries()
        first = None
        for k in range(off[r], off[r + 1]):
            v, o = verdict_brute(ents, ptrs[k][0], ptrs[k][1])
            assert (pv[k], po[k]) == (v, o)
            if v != ALLOW and first is None:
                first = (v, k - off[r], o)
        if first is None:
            assert (rv[r], ra[r], ro[r]) == (ALLOW, -1, -1)
        else:
            assert (rv[r], ra[r], ro[r]) == first


def test_cross_client_pointer_rejected():
    a, b = RangeTable(), RangeTable()
    ia = a.insert(1 << 40, 4096, USER)
    b.insert(1 << 41, 4096, USER)
    ptrs = np.array([[(1 << 40) + 8, 16], [(1 << 41) + 8, 16]], dtype=np.uint64)
    _, _, rv, ra, _ = batch_verdicts([a, b], [0, 1], [0, 2, 4],
                                     np.concatenate([ptrs, ptrs]))
    assert (rv[0], ra[0]) == (V_UNMAPPED, 1)      # b's pointer is unknown to client a
    assert (rv[1], ra[1]) == (V_UNMAPPED, 0)
    assert ia == 0


def test_embedding_grad_adjoint_identity():
    """<gather(W, idx), dY> equals <W, dW>: the gradient is the adjoint of the lookup."""
    rng = np.random.default_rng(0)
    rows, D, n = 64, 8, 200
    W = rng.standard_normal((rows, D))
    idx = rng.integers(0, rows, n)
    allowed = rng.random(n) > 0.1
    dY = rng.standard_normal((n, D))
    Y = embedding_forward_ref(W, idx, allowed)
    dW = embedding_grad_ref(idx, allowed, dY, rows, np.float64)
    lhs = float((Y * dY).sum())
    rhs = float((W * dW).sum())
    assert abs(lhs - rhs) <= 1e-12 * max(1.0, abs(lhs))


def test_embedding_grad_finite_differences():
    rng = np.random.default_rng(1)
    rows, D, n = 16, 4, 40
    W = rng.standard_normal((rows, D))
    idx = rng.integers(0, rows, n)
    allowed = np.ones(n, bool)
    allowed[::7] = False
    dY = rng.standard_normal((n, D))
    dW = embedding_grad_ref(idx, allowed, dY, rows, np.float64)
    h = 1e-6
    for r in range(rows):
        for c in range(D):
            Wp, Wm = W.copy(), W.copy()
            Wp[r, c] += h
            Wm[r, c] -= h
            fd = ((embedding_forward_ref(Wp, idx, allowed) * dY).sum()
                  - (embedding_forward_ref(Wm, idx, allowed) * dY).sum()) / (2 * h)
            assert fd == pytest.approx(dW[r, c], rel=1e-7, abs=1e-8)


def test_embedding_grad_unit_counts():
    rng = np.random.default_rng(2)
    rows, n = 100, 5000
    idx = rng.integers(0, rows, n)
    allowed = rng.random(n) > 0.05
    dW = embedding_grad_ref(idx, allowed, np.ones((n, 3), np.float32), rows)
    cnt = np.bincount(idx[allowed], minlength=rows).astype(np.float32)
    assert np.array_equal(dW, np.repeat(cnt[:, None], 3, 1))
