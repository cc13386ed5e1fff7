"""Guarded embedding (forward gather, sorted guarded scatter-add backward: radix-sorted for
large calls, chunk-sorted for small ones) against the oracle."""
import numpy as np
import pytest
import torch

from gpu_util import need_gpu, guard_mod
from oracle.embedding import embedding_grad_ref, embedding_forward_ref
from synth import zipf_indices, uniform_f32

pytestmark = pytest.mark.gpu


def _setup(rows, D, dtype, pad_rows=16, device="cuda"):
    g = guard_mod()
    from paper_2606_06697_amd.embedding import guarded_embedding
    buf = torch.zeros((rows + pad_rows) * D, dtype=dtype, device=device)
    W = buf[:rows * D].view(rows, D)
    canary = buf[rows * D:]
    tab = g.RangeTable(64)
    tab.insert_tensor(W, g.KIND_USER)
    tab.insert_tensor(canary, g.KIND_PROTECTED)
    return g, guarded_embedding, buf, W, canary, tab


def test_gradcheck_fp64_with_suppressed_index():
    need_gpu()
    g, emb, buf, W, canary, tab = _setup(64, 8, torch.float64)
    W.copy_(torch.randn(64, 8, dtype=torch.float64, device="cuda"))
    canary.fill_(7.0)
    idx = torch.randint(0, 64, (32,), device="cuda")
    idx[5] = 66                                   # aimed at the protected canary
    tab.insert_tensor(idx, g.KIND_USER)
    Wl = W.detach().requires_grad_()
    assert torch.autograd.gradcheck(lambda w: emb(w, idx, tab), (Wl,), eps=1e-6, atol=1e-7)
    y = emb(Wl, idx, tab)
    assert torch.all(y[5] == 0) and torch.equal(y[3], W[idx[3]])
    assert torch.all(canary == 7.0)
    rc, f = tab.fault_log(clear=True)
    assert rc == g.AGILE_EFAULTED and f["count"] > 0 and f["first_verdict"] == g.V_PROTECTED


@pytest.mark.parametrize("rows,D,n", [(1000, 64, 5000), (4096, 256, 30001), (300, 3, 7777)])
def test_forward_backward_against_oracle(rows, D, n):
    need_gpu()
    g, emb, buf, W, canary, tab = _setup(rows, D, torch.float32)
    W.copy_(uniform_f32(rows * D, 1, device="cuda").view(rows, D))
    canary.fill_(3.0)
    idx = zipf_indices(n, rows, 1.1, 2, device="cuda", bad_frac=0.01,
                       bad_ranges=((rows, rows + 16), (-5, 0), (1 << 40, (1 << 40) + 9)))
    tab.insert_tensor(idx, g.KIND_USER)
    Wl = W.detach().requires_grad_()
    y = emb(Wl, idx, tab)
    dY = uniform_f32(n * D, 3, device="cuda").view(n, D)
    y.backward(dY)
    torch.cuda.synchronize()
    ih = idx.cpu().numpy()
    allowed = (ih >= 0) & (ih < rows)
    Wh = W.cpu().numpy()
    assert np.array_equal(y.detach().cpu().numpy().view(np.uint32),
                          embedding_forward_ref(Wh, ih, allowed).view(np.uint32))
    ref = embedding_grad_ref(ih, allowed, dY.cpu().numpy(), rows, np.float64)
    got = Wl.grad.double().cpu().numpy()
    rel = np.linalg.norm(got - ref) / np.linalg.norm(ref)
    assert rel <= 1e-5, rel
    big = np.abs(ref) > 1e-3 * np.abs(ref).max()
    assert np.max(np.abs(got - ref)[big] / np.abs(ref)[big]) <= 1e-4
    assert torch.all(canary == 3.0)
    rc, f = tab.fault_log(clear=True)
    nbad = int((~allowed).sum())
    assert f["count"] == 2 * nbad * D            # forward table loads + backward dW updates


def test_unit_gradient_gives_exact_counts():
    need_gpu()
    g, emb, buf, W, canary, tab = _setup(5000, 16, torch.float32)
    idx = zipf_indices(200_000, 5000, 1.1, 4, device="cuda")
    tab.insert_tensor(idx, g.KIND_USER)
    Wl = W.detach().requires_grad_()
    emb(Wl, idx, tab).backward(torch.ones(200_000, 16, device="cuda"))
    cnt = np.bincount(idx.cpu().numpy(), minlength=5000).astype(np.float32)
    assert np.array_equal(Wl.grad.cpu().numpy(), np.repeat(cnt[:, None], 16, 1))
    assert tab.fault_log()[1]["count"] == 0


def test_sgd_training_matches_the_unguarded_embedding():
    """Eight SGD steps of a small model (guarded embedding, fixed linear head, squared error)
    against the same model on ``torch.nn.functional.embedding``, from the same weights and the
    same batches of 50,000 indices (the backward takes the radix-sorted path). 1% of each
    batch's indices point past the table: the guard reads zeros for them and drops their
    gradient, and the reference masks the same rows. Losses and weights stay within 1e-5
    relative of the reference after every step; the log counts every hostile load and store."""
    need_gpu()
    g = guard_mod()
    from paper_2606_06697_amd.embedding import GuardedEmbedding
    R, D, B, steps = 4096, 32, 50_000, 8
    tab = g.RangeTable(64)
    torch.manual_seed(0)
    emb = GuardedEmbedding(R, D, tab)
    Wr = emb.weight.detach().clone().requires_grad_()
    gen = torch.Generator(device="cuda").manual_seed(1)
    head = torch.randn(D, 1, device="cuda", generator=gen)
    opt = torch.optim.SGD([emb.weight], lr=0.5)
    opt_r = torch.optim.SGD([Wr], lr=0.5)
    nbad_total = 0
    for s in range(steps):
        idx = zipf_indices(B, R, 1.1, 100 + s, device="cuda", bad_frac=0.01,
                           bad_ranges=((R, R + 16),))
        y = torch.randn(B, 1, device="cuda", generator=gen)
        rid = tab.insert_tensor(idx, g.KIND_USER)
        loss = ((emb(idx) @ head - y) ** 2).mean()
        opt.zero_grad()
        loss.backward()
        opt.step()
        tab.remove(rid)
        valid = (idx >= 0) & (idx < R)
        xr = torch.nn.functional.embedding(idx.clamp(0, R - 1), Wr) * valid[:, None]
        loss_r = ((xr @ head - y) ** 2).mean()
        opt_r.zero_grad()
        loss_r.backward()
        opt_r.step()
        nbad_total += int((~valid).sum())
        assert abs(loss.item() - loss_r.item()) <= 1e-5 * abs(loss_r.item()), s
        rel = float((emb.weight.detach() - Wr.detach()).norm() / Wr.detach().norm())
        assert rel <= 1e-5, (s, rel)
    rc, f = tab.fault_log(clear=True)
    assert rc == g.AGILE_EFAULTED and f["count"] == 2 * nbad_total * D
    tab.close()
