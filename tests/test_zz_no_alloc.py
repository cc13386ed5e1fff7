"""The scatter-add without allocation (agile_guarded_scatter_add_noalloc) against the allocating
call (agile_guarded_scatter, accumulate = 1) on the same inputs, through the C ABI: two calls in
a row, the second smaller, both on the sorted path (the fixed scratch), then a small call on
the chunk path, a call past the row limit that must be refused before any work, and an
embedding-sized call checked against the fp64-accumulated reference."""
import numpy as np
import pytest
import torch

from gpu_util import guard_mod, need_gpu
from oracle.embedding import embedding_grad_ref
from synth import uniform_f32, zipf_indices

pytestmark = pytest.mark.gpu


def _case(g, R, D, N, seed, integer):
    """A table with two destinations (one per call), the index, the source and a protected pad
    after each destination; 0.05% of the indices aim at the pad."""
    dev = torch.device("cuda:0")
    PAD = 8
    rb = D * 4
    bufs = [torch.zeros((R + PAD) * D, device=dev) for _ in range(2)]
    idx = zipf_indices(N, R, 1.1, seed, device=dev, bad_frac=5e-4, bad_ranges=((R, R + PAD),))
    if integer:
        src = torch.randint(-8, 9, (N * D,), device=dev).float()
    else:
        src = uniform_f32(N * D, seed, device=dev, stream=40)
    rt = g.RangeTable(16)
    for b in bufs:
        rt.insert(b.data_ptr(), R * rb, g.KIND_USER)
        rt.insert(b.data_ptr() + R * rb, PAD * rb, g.KIND_PROTECTED)
    rt.insert_tensor(idx)
    rt.insert_tensor(src)
    return rt, bufs, idx, src, rb


def _compare(g, R, D, N, seed, integer):
    rt, (a, b), idx, src, rb = _case(g, R, D, N, seed, integer)
    g.agile_guarded_scatter(rt.handle, a, rb, idx, src, N, 0, 1)
    rc1, f1 = rt.fault_log(clear=True)
    g.agile_guarded_scatter_add_noalloc(rt.handle, b, rb, idx, src, N, 0)
    rc2, f2 = rt.fault_log(clear=True)
    torch.cuda.synchronize()
    nbad = int(((idx < 0) | (idx >= R)).sum())
    assert rc1 == rc2 and f1["count"] == f2["count"] == nbad * D
    for k in ("first_elem", "first_operand", "first_verdict", "first_width", "first_op"):
        assert f1[k] == f2[k], k
    if nbad:
        # the first denied access is the destination store of the same row, each call into
        # its own destination buffer (whose pad gives the owner id)
        assert f1["first_operand"] == 2
        assert f1["first_addr"] - a.data_ptr() == f2["first_addr"] - b.data_ptr()
        assert (f1["first_owner"], f2["first_owner"]) == (1, 3)
    ra, rb_ = a[:R * D].cpu().numpy(), b[:R * D].cpu().numpy()
    assert (a[R * D:] == 0).all() and (b[R * D:] == 0).all()      # the pads are untouched
    if integer:
        assert np.array_equal(ra, rb_)                               # exact sums in any order
    else:
        rel = np.linalg.norm(ra.astype(np.float64) - rb_) / np.linalg.norm(ra.astype(np.float64))
        assert rel <= 1e-5, rel
    rt.close()
    return idx, src, b


def test_noalloc_scatter_add_equals_the_allocating_call():
    need_gpu()
    g = guard_mod()
    print("noalloc: 2^20 rows, 2^17 x 64 destination, integer values", flush=True)
    _compare(g, 1 << 17, 64, 1 << 20, 1, integer=True)
    print("noalloc: 40,000 rows, 5,000 x 16 destination (second call, smaller)", flush=True)
    _compare(g, 5000, 16, 40000, 2, integer=True)
    print("noalloc: 3,000 rows (chunk path, no scratch)", flush=True)
    _compare(g, 700, 8, 3000, 3, integer=True)
    print("noalloc: 2^19 rows of 1 KiB, uniform values", flush=True)
    idx, src, b = _compare(g, 1 << 16, 256, 1 << 19, 4, integer=False)
    ih = idx.cpu().numpy()
    ref = embedding_grad_ref(ih, (ih >= 0) & (ih < (1 << 16)), src.cpu().numpy().reshape(-1, 256),
                             1 << 16, out_dtype=np.float64)
    got = b[:(1 << 16) * 256].cpu().numpy().reshape(-1, 256).astype(np.float64)
    assert np.linalg.norm(got - ref) / np.linalg.norm(ref) <= 1e-5


def test_noalloc_refuses_more_rows_than_its_scratch_holds():
    need_gpu()
    g = guard_mod()
    n = g.NOALLOC_MAX_ROWS + 1
    rt = g.RangeTable(8)
    dst = torch.zeros(64, device="cuda")
    idx = torch.zeros(n, dtype=torch.int64, device="cuda")
    src = torch.ones(n, device="cuda")
    for t in (dst, idx, src):
        rt.insert_tensor(t)
    rc = g.lib().agile_guarded_scatter_add_noalloc(rt.handle, dst.data_ptr(), 4, idx.data_ptr(),
                                                   src.data_ptr(), n, 0, 0, None)
    assert rc == g.AGILE_E2BIG
    torch.cuda.synchronize()
    assert (dst == 0).all()
    assert rt.fault_log()[0] == g.AGILE_OK
    rt.close()
