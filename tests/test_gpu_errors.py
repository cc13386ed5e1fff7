"""Argument errors with a live table: every call below is refused on the host with its status
code before anything is queued, leaves its out-parameters and every device buffer untouched, and
leaves the fault log empty; the table keeps working afterwards."""
import ctypes

import pytest
import torch

from gpu_util import need_gpu, guard_mod

pytestmark = pytest.mark.gpu


def _setup():
    g = guard_mod()
    L = g.lib()
    rt = g.RangeTable(4)
    a = torch.arange(1024, dtype=torch.float32, device="cuda")
    b = torch.full((1024,), 2.0, dtype=torch.float32, device="cuda")
    c = torch.full((1024,), 3.0, dtype=torch.float32, device="cuda")
    idx = torch.zeros(16, dtype=torch.int64, device="cuda")
    for t in (a, b, c, idx):
        rt.insert_tensor(t, g.KIND_USER)
    return g, L, rt, a, b, c, idx


def test_table_edits_refused_with_their_codes():
    need_gpu()
    g, L, rt, a, b, c, idx = _setup()
    h = rt.handle
    out = ctypes.c_int32(-77)
    assert L.agile_rt_insert(h, 1 << 44, 4096, 0, ctypes.byref(out)) == g.AGILE_ENOSPC  # capacity 4
    assert out.value == -77
    # size 0, an unknown kind, and an end past 2^64 are invalid (checked before the capacity)
    assert L.agile_rt_insert(h, 1 << 44, 0, 0, ctypes.byref(out)) == g.AGILE_EINVAL
    assert L.agile_rt_insert(h, 1 << 44, 16, 3, ctypes.byref(out)) == g.AGILE_EINVAL
    assert L.agile_rt_insert(h, (1 << 64) - 8, 16, 0, ctypes.byref(out)) == g.AGILE_EINVAL
    assert out.value == -77
    # unknown and already removed ids (a, b, c and idx were given ids 0 to 3)
    assert L.agile_rt_remove(h, 12345) == g.AGILE_ENOENT
    n = ctypes.c_uint32()
    assert L.agile_rt_count(h, ctypes.byref(n)) == g.AGILE_OK and n.value == 4
    rt.remove(0)
    assert L.agile_rt_remove(h, 0) == g.AGILE_ENOENT
    assert L.agile_rt_count(h, ctypes.byref(n)) == g.AGILE_OK and n.value == 3
    # with room again: a range overlapping the end of b is refused; one starting at the largest
    # end of the registered ranges (adjacent, never overlapping) is accepted and gets id 4
    bb = b.data_ptr()
    assert L.agile_rt_insert(h, bb + 4092, 8, 0, ctypes.byref(out)) == g.AGILE_EOVERLAP
    assert out.value == -77
    top = max(t.data_ptr() + t.numel() * t.element_size() for t in (b, c, idx))
    assert L.agile_rt_insert(h, top, 64, 1, ctypes.byref(out)) == g.AGILE_OK and out.value == 4
    assert L.agile_rt_count(h, ctypes.byref(n)) == g.AGILE_OK and n.value == 4
    rc, f = rt.fault_log()
    assert rc == g.AGILE_OK and f["count"] == 0
    rt.close()


def test_guarded_calls_refused_before_any_launch():
    need_gpu()
    g, L, rt, a, b, c, idx = _setup()
    h = rt.handle
    s = torch.cuda.current_stream().cuda_stream
    a0, idx0 = a.clone(), idx.clone()
    A, B, C, I = a.data_ptr(), b.data_ptr(), c.data_ptr(), idx.data_ptr()
    E = g.AGILE_EINVAL
    # unknown policy; the sink policy without a quarantine buffer
    assert L.agile_guarded_copy(h, A, B, 64, 99, s) == E
    assert L.agile_guarded_copy(h, A, B, 64, g.POLICY_SINK, s) == E
    assert L.agile_guarded_triad(h, A, B, C, 1.0, 16, -1, s) == E
    # misaligned fp32 operands, and an element count whose byte size overflows
    assert L.agile_guarded_triad(h, A + 2, B, C, 1.0, 16, 0, s) == E
    assert L.agile_guarded_triad(h, A, B, C, 1.0, 1 << 62, 0, s) == E
    # gather: unknown dtype, zero / non-multiple / huge row size, misaligned out, table or idx,
    # and n rows whose element count overflows
    assert L.agile_guarded_gather(h, A, B, 16, I, 4, 7, 0, s) == E
    assert L.agile_guarded_gather(h, A, B, 0, I, 4, g.DTYPE_F32, 0, s) == E
    assert L.agile_guarded_gather(h, A, B, 6, I, 4, g.DTYPE_F32, 0, s) == E
    assert L.agile_guarded_gather(h, A, B, 12, I, 4, g.DTYPE_F64, 0, s) == E
    assert L.agile_guarded_gather(h, A, B, (1 << 40) + 4, I, 4, g.DTYPE_F32, 0, s) == E
    assert L.agile_guarded_gather(h, A + 2, B, 16, I, 4, g.DTYPE_F32, 0, s) == E
    assert L.agile_guarded_gather(h, A, B + 2, 16, I, 4, g.DTYPE_F32, 0, s) == E
    assert L.agile_guarded_gather(h, A, B, 16, I + 4, 4, g.DTYPE_F32, 0, s) == E
    assert L.agile_guarded_gather(h, A, B, 1 << 32, I, 1 << 32, g.DTYPE_F32, 0, s) == E
    # scatter: accumulate outside 0..2, and the same row checks
    for acc in (-1, 3):
        assert L.agile_guarded_scatter(h, A, 16, I, B, 4, g.DTYPE_F32, acc, 0, s) == E
    assert L.agile_guarded_scatter(h, A, 6, I, B, 4, g.DTYPE_F32, 1, 0, s) == E
    assert L.agile_guarded_scatter(h, A, 16, I + 4, B, 4, g.DTYPE_F32, 1, 0, s) == E
    # the allocation-free scatter-add refuses more rows than its fixed scratch holds
    assert L.agile_guarded_scatter_add_noalloc(h, A, 16, I, B, g.NOALLOC_MAX_ROWS + 1,
                                               g.DTYPE_F32, 0, s) == g.AGILE_E2BIG
    # validation: misaligned queries; a quarantine that is not a power of two
    v = torch.zeros(4, dtype=torch.uint8, device="cuda")
    o = torch.zeros(4, dtype=torch.int32, device="cuda")
    assert L.agile_validate_ptrs(h, I + 8, 4, v.data_ptr(), o.data_ptr(), s) == E
    assert L.agile_validate_dma(h, I + 8, 4, v.data_ptr(), o.data_ptr(), s) == E
    assert L.agile_rt_set_quarantine(h, A, 1000) == E
    torch.cuda.synchronize()
    assert torch.equal(a, a0) and torch.equal(idx, idx0)
    assert torch.count_nonzero(v) == 0 and torch.count_nonzero(o) == 0
    rc, f = rt.fault_log()
    assert rc == g.AGILE_OK and f["count"] == 0
    # and the handle still works: a plain guarded copy of b into a
    g.agile_guarded_copy(h, a, b, 4096)
    torch.cuda.synchronize()
    assert torch.equal(a, b)
    assert rt.fault_log()[1]["count"] == 0
    rt.close()
