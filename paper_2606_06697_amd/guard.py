"""Python binding of libagile_guard.so (argument marshalling only).

Every function here has the name of the C entry point it forwards to (see
``include/agile_guard.h`` and ``include/agile_aperture.h``); pointers may be given as torch tensors (their ``data_ptr()``) or
as raw integer addresses, streams as ``torch.cuda.Stream``, raw handles or ``None`` (the
current torch stream). Nothing is computed in Python: all guard work runs in the library's
HIP kernels, and if the library is missing every call raises.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np
import torch

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libagile_guard.so")

AGILE_OK, AGILE_EINVAL, AGILE_ENOMEM, AGILE_EOVERLAP = 0, -1, -2, -3
AGILE_ENOENT, AGILE_ENOSPC, AGILE_EDEVICE, AGILE_EFAULTED = -4, -5, -6, -7
AGILE_ETRAPPED, AGILE_ENOTSUP, AGILE_E2BIG = -8, -9, -10
NOALLOC_MAX_ROWS = 1 << 20
AP_IO, AP_MODULE, AP_USER = 0, 1, 2
KIND_USER, KIND_PROTECTED, KIND_MMIO = 0, 1, 2
RANGE_BACKED = 0x80                     # OR-ed into a kind: the range is mapped memory
ALLOW, V_PROTECTED, V_STRADDLE, V_UNMAPPED, V_CROSS_ALLOC, V_INEXACT = 0, 1, 2, 3, 4, 5
(POLICY_SUPPRESS_LOG, POLICY_SUPPRESS_ONLY, POLICY_TRAP, POLICY_SINK, POLICY_REPORT,
 POLICY_REMAP) = 0, 1, 2, 3, 4, 5
OP_COPY, OP_TRIAD, OP_GATHER, OP_SCATTER, OP_SCATTER_ADD = 1, 2, 3, 4, 5
DTYPE_F32, DTYPE_F64 = 0, 1
# agile_guarded_scatter's `accumulate`: plain scatter, scatter-add, scatter-add into a destination
# whose rows are all +0.0 before the call (same result, the sorted path skips reading the rows)
SCATTER, SCATTER_ADD, SCATTER_ADD_INTO_ZEROS = 0, 1, 2
TOKEN_VALID, TOKEN_FORGED, TOKEN_STALE, TOKEN_CROSS_CLIENT, TOKEN_WRONG_KIND = 0, 1, 2, 3, 4
TOKEN_ANY_KIND = 255
NO_SEQ = (1 << 64) - 1


class AgileError(RuntimeError):
    def __init__(self, code: int, where: str):
        self.code = code
        super().__init__(f"{where}: {strerror(code)} ({code})")


class agile_fault(ctypes.Structure):
    _fields_ = [("count", ctypes.c_uint64), ("first_seq", ctypes.c_uint64),
                ("first_elem", ctypes.c_uint64), ("first_addr", ctypes.c_uint64),
                ("first_width", ctypes.c_uint32), ("first_op", ctypes.c_uint32),
                ("first_operand", ctypes.c_uint32), ("first_verdict", ctypes.c_uint32),
                ("first_owner", ctypes.c_int32), ("reserved", ctypes.c_uint32)]

    def as_dict(self):
        d = {k: getattr(self, k) for k, _ in self._fields_ if k != "reserved"}
        return d


_u64, _u32, _i32, _int, _vp = (ctypes.c_uint64, ctypes.c_uint32, ctypes.c_int32, ctypes.c_int,
                               ctypes.c_void_p)
SERVER_MAX_REVOKE = 16


class agile_server_config(ctypes.Structure):
    _fields_ = [("max_batch", ctypes.c_uint32), ("max_inflight", ctypes.c_uint32),
                ("hbm_budget", ctypes.c_uint64)]


class agile_server_stats(ctypes.Structure):
    _fields_ = [("elapsed_s", ctypes.c_double), ("launches", ctypes.c_uint64),
                ("served", ctypes.c_uint64), ("refused", ctypes.c_uint64),
                ("max_inflight_bytes", ctypes.c_uint64), ("max_concurrent", ctypes.c_uint64),
                ("budget_waits", ctypes.c_uint64), ("ring_waits", ctypes.c_uint64),
                ("revoked_at_s", ctypes.c_double * SERVER_MAX_REVOKE)]

_SIGS = {
    "agile_strerror": (ctypes.c_char_p, [_int]),
    "agile_rt_create": (_int, [ctypes.POINTER(_vp), _u32, _int]),
    "agile_rt_destroy": (_int, [_vp]),
    "agile_rt_insert": (_int, [_vp, _u64, _u64, _u32, ctypes.POINTER(_i32)]),
    "agile_rt_insert_many": (_int, [_vp, _vp, _vp, _vp, _u32, _vp]),
    "agile_rt_remove": (_int, [_vp, _i32]),
    "agile_rt_count": (_int, [_vp, ctypes.POINTER(_u32)]),
    "agile_rt_sync": (_int, [_vp, _vp]),
    "agile_validate_ptrs": (_int, [_vp, _vp, _u64, _vp, _vp, _vp]),
    "agile_validate_dma": (_int, [_vp, _vp, _u64, _vp, _vp, _vp]),
    "agile_guarded_copy": (_int, [_vp, _vp, _vp, _u64, _int, _vp]),
    "agile_guarded_triad": (_int, [_vp, _vp, _vp, _vp, ctypes.c_float, _u64, _int, _vp]),
    "agile_guarded_gather": (_int, [_vp, _vp, _vp, _u64, _vp, _u64, _int, _int, _vp]),
    "agile_guarded_scatter": (_int, [_vp, _vp, _u64, _vp, _vp, _u64, _int, _int, _int, _vp]),
    "agile_guarded_scatter_add_noalloc": (_int, [_vp, _vp, _u64, _vp, _vp, _u64, _int, _int, _vp]),
    "agile_fault_log_read": (_int, [_vp, ctypes.POINTER(agile_fault), _int, _vp]),
    "agile_unguarded_copy": (_int, [_vp, _vp, _u64, _vp]),
    "agile_unguarded_triad": (_int, [_vp, _vp, _vp, ctypes.c_float, _u64, _vp]),
    "agile_unguarded_gather": (_int, [_vp, _vp, _u64, _vp, _u64, _int, _vp]),
    "agile_unguarded_scatter": (_int, [_vp, _u64, _vp, _vp, _u64, _int, _int, _vp]),
    "agile_clients_create": (_int, [ctypes.POINTER(_vp), _vp, _u32, _int]),
    "agile_clients_destroy": (_int, [_vp]),
    "agile_batch_run": (_int, [_vp, _vp, _u32, _vp, _u64, _vp, _vp, _vp, _vp]),
    "agile_tokens_create": (_int, [ctypes.POINTER(_vp), _u32, _u64, _int]),
    "agile_tokens_destroy": (_int, [_vp]),
    "agile_token_mint": (_int, [_vp, _u32, _u32, ctypes.POINTER(_u64)]),
    "agile_token_release": (_int, [_vp, _u64, _u32]),
    "agile_tokens_check": (_int, [_vp, _vp, _vp, _vp, _u64, _vp, _vp, _vp]),
    "agile_rt_clear": (_int, [_vp]),
    "agile_rt_set_quarantine": (_int, [_vp, _vp, _u64]),
    "agile_server_create": (_int, [ctypes.POINTER(_vp), _vp, _vp, _u32, _vp, _vp,
                                   ctypes.POINTER(agile_server_config), _vp, _u64, _vp, _vp,
                                   _int]),
    "agile_server_destroy": (_int, [_vp]),
    "agile_aperture_create": (_int, [ctypes.POINTER(_vp), _int, _vp, _vp, _u64]),
    "agile_aperture_destroy": (_int, [_vp]),
    "agile_aperture_info": (_int, [_vp, _vp, _vp, ctypes.POINTER(_u64)]),
    "agile_aperture_alloc": (_int, [_vp, _int, _u64, _vp, ctypes.POINTER(_vp),
                                    ctypes.POINTER(_i32)]),
    "agile_aperture_free": (_int, [_vp, _vp]),
    "agile_validate_aperture": (_int, [_vp, _vp, _u64, _vp, _vp, _vp]),
    "agile_server_run": (_int, [_vp, _vp, _vp, _vp, _u64, _vp, _vp, _u32, _vp, _vp, _vp, _vp,
                                _vp, _vp, ctypes.POINTER(agile_server_stats)]),
}

# numpy mirrors of agile_request (96 bytes) and agile_req_result (72 bytes)
REQUEST_DTYPE = np.dtype([
    ("client", "<u4"), ("reserved0", "<u4"), ("ptr_off", "<u8"), ("nptr", "<u8"),
    ("copy_dst", "<u8"), ("copy_src", "<u8"), ("copy_bytes", "<u8"), ("gather_out", "<u8"),
    ("gather_table", "<u8"), ("gather_idx", "<u8"), ("gather_n", "<u8"),
    ("gather_row_bytes", "<u4"), ("reserved1", "<u4"), ("reserved2", "<u8")])
RESULT_DTYPE = np.dtype([
    ("verdict", "<u4"), ("arg", "<i4"), ("owner", "<i4"), ("done", "<u4"), ("count", "<u8"),
    ("first_seq", "<u8"), ("first_elem", "<u8"), ("first_addr", "<u8"),
    ("first_width", "<u4"), ("first_op", "<u4"), ("first_operand", "<u4"),
    ("first_verdict", "<u4"), ("first_owner", "<i4"), ("reserved", "<u4")])
assert REQUEST_DTYPE.itemsize == 96 and RESULT_DTYPE.itemsize == 72

_lib = None


def lib():
    """The loaded library (raises if it has not been built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is missing: build it with __graft_entry__.build() "
                               "(there is no fallback path)")
        L = ctypes.CDLL(LIB_PATH, mode=ctypes.RTLD_GLOBAL)
        for name, (res, args) in _SIGS.items():
            f = getattr(L, name)
            f.restype = res
            f.argtypes = args
        _lib = L
    return _lib


def agile_strerror(code: int) -> str:
    return lib().agile_strerror(int(code)).decode()


strerror = agile_strerror


def _ptr(x) -> int:
    if x is None:
        return 0
    if isinstance(x, torch.Tensor):
        return x.data_ptr()
    return int(x) & ((1 << 64) - 1)


def _stream(s):
    if s is None:
        return torch.cuda.current_stream().cuda_stream
    if isinstance(s, torch.cuda.Stream):
        return s.cuda_stream
    return int(s)


def _check(rc: int, where: str, ok=(AGILE_OK,)):
    if rc not in ok:
        raise AgileError(rc, where)
    return rc


# ---- C entry points ----------------------------------------------------------------------
def agile_rt_create(capacity: int, device: int = 0) -> int:
    h = _vp()
    _check(lib().agile_rt_create(ctypes.byref(h), capacity, device), "agile_rt_create")
    return h.value


def agile_rt_destroy(rt: int) -> None:
    _check(lib().agile_rt_destroy(rt), "agile_rt_destroy")


def agile_rt_insert(rt: int, base: int, size: int, kind: int) -> int:
    out = _i32()
    _check(lib().agile_rt_insert(rt, base & ((1 << 64) - 1), size, kind, ctypes.byref(out)),
           "agile_rt_insert")
    return out.value


def agile_rt_insert_many(rt: int, base, size, kind) -> "torch.Tensor":
    """base/size: int64 or uint64 CPU tensors (bit patterns), kind: uint8; returns int32 ids."""
    base = torch.as_tensor(base).contiguous().cpu()
    size = torch.as_tensor(size).contiguous().cpu()
    kind = torch.as_tensor(kind).to(torch.uint8).contiguous().cpu()
    n = base.numel()
    ids = torch.empty(n, dtype=torch.int32)
    _check(lib().agile_rt_insert_many(rt, base.data_ptr(), size.data_ptr(), kind.data_ptr(), n,
                                      ids.data_ptr()), "agile_rt_insert_many")
    return ids


def agile_rt_remove(rt: int, rid: int) -> None:
    _check(lib().agile_rt_remove(rt, rid), "agile_rt_remove")


def agile_rt_count(rt: int) -> int:
    out = _u32()
    _check(lib().agile_rt_count(rt, ctypes.byref(out)), "agile_rt_count")
    return out.value


def agile_rt_sync(rt: int, stream=None) -> None:
    _check(lib().agile_rt_sync(rt, _stream(stream)), "agile_rt_sync")


def agile_validate_ptrs(rt: int, q, n: int, verdict, owner, stream=None) -> None:
    _check(lib().agile_validate_ptrs(rt, _ptr(q), n, _ptr(verdict), _ptr(owner), _stream(stream)),
           "agile_validate_ptrs")


def agile_validate_dma(rt: int, q, n: int, verdict, owner, stream=None) -> None:
    _check(lib().agile_validate_dma(rt, _ptr(q), n, _ptr(verdict), _ptr(owner), _stream(stream)),
           "agile_validate_dma")


def agile_guarded_copy(rt: int, dst, src, nbytes: int, policy: int = 0, stream=None) -> None:
    _check(lib().agile_guarded_copy(rt, _ptr(dst), _ptr(src), nbytes, policy, _stream(stream)),
           "agile_guarded_copy")


def agile_guarded_triad(rt: int, a, b, c, s: float, n: int, policy: int = 0, stream=None) -> None:
    _check(lib().agile_guarded_triad(rt, _ptr(a), _ptr(b), _ptr(c), s, n, policy,
                                     _stream(stream)), "agile_guarded_triad")


def agile_guarded_gather(rt: int, out, table, row_bytes: int, idx, n: int, dtype: int = 0,
                         policy: int = 0, stream=None) -> None:
    _check(lib().agile_guarded_gather(rt, _ptr(out), _ptr(table), row_bytes, _ptr(idx), n, dtype,
                                      policy, _stream(stream)), "agile_guarded_gather")


def agile_guarded_scatter(rt: int, dst, row_bytes: int, idx, src, n: int, dtype: int = 0,
                          accumulate: int = 0, policy: int = 0, stream=None) -> None:
    _check(lib().agile_guarded_scatter(rt, _ptr(dst), row_bytes, _ptr(idx), _ptr(src), n, dtype,
                                       accumulate, policy, _stream(stream)),
           "agile_guarded_scatter")


def agile_guarded_scatter_add_noalloc(rt: int, dst, row_bytes: int, idx, src, n: int,
                                      dtype: int = 0, policy: int = 0, stream=None) -> None:
    _check(lib().agile_guarded_scatter_add_noalloc(rt, _ptr(dst), row_bytes, _ptr(idx), _ptr(src),
                                                   n, dtype, policy, _stream(stream)),
           "agile_guarded_scatter_add_noalloc")


def agile_fault_log_read(rt: int, clear: bool = False, stream=None):
    """Returns (status, record dict); status is AGILE_OK, AGILE_EFAULTED or AGILE_ETRAPPED."""
    f = agile_fault()
    rc = _check(lib().agile_fault_log_read(rt, ctypes.byref(f), int(bool(clear)),
                                           _stream(stream)), "agile_fault_log_read",
                ok=(AGILE_OK, AGILE_EFAULTED, AGILE_ETRAPPED))
    return rc, f.as_dict()


def agile_unguarded_copy(dst, src, nbytes: int, stream=None) -> None:
    _check(lib().agile_unguarded_copy(_ptr(dst), _ptr(src), nbytes, _stream(stream)),
           "agile_unguarded_copy")


def agile_unguarded_triad(a, b, c, s: float, n: int, stream=None) -> None:
    _check(lib().agile_unguarded_triad(_ptr(a), _ptr(b), _ptr(c), s, n, _stream(stream)),
           "agile_unguarded_triad")


def agile_unguarded_gather(out, table, row_bytes: int, idx, n: int, dtype: int = 0,
                           stream=None) -> None:
    _check(lib().agile_unguarded_gather(_ptr(out), _ptr(table), row_bytes, _ptr(idx), n, dtype,
                                        _stream(stream)), "agile_unguarded_gather")


def agile_unguarded_scatter(dst, row_bytes: int, idx, src, n: int, dtype: int = 0,
                            accumulate: int = 0, stream=None) -> None:
    _check(lib().agile_unguarded_scatter(_ptr(dst), row_bytes, _ptr(idx), _ptr(src), n, dtype,
                                         accumulate, _stream(stream)), "agile_unguarded_scatter")


def agile_clients_create(tables, device: int = 0) -> int:
    """Client set from table handles (ints) or RangeTable objects, client i = tables[i]."""
    hs = [t.handle if isinstance(t, RangeTable) else int(t) for t in tables]
    arr = (_vp * len(hs))(*hs)
    h = _vp()
    _check(lib().agile_clients_create(ctypes.byref(h), arr, len(hs), device),
           "agile_clients_create")
    return h.value


def agile_clients_destroy(cs: int) -> None:
    _check(lib().agile_clients_destroy(cs), "agile_clients_destroy")


def agile_batch_run(cs: int, reqs: np.ndarray, ptrs, nptrs: int, ptr_verdict, ptr_owner, result,
                    stream=None) -> None:
    """reqs: numpy array of REQUEST_DTYPE (host); ptrs: device int64 [nptrs, 2]; ptr_verdict
    (uint8) / ptr_owner (int32): device [nptrs]; result: device buffer of len(reqs) * 72 bytes."""
    reqs = np.ascontiguousarray(reqs, dtype=REQUEST_DTYPE)
    _check(lib().agile_batch_run(cs, reqs.ctypes.data, len(reqs), _ptr(ptrs), nptrs,
                                 _ptr(ptr_verdict), _ptr(ptr_owner), _ptr(result),
                                 _stream(stream)), "agile_batch_run")


def batch_results(result: torch.Tensor, nreq: int) -> np.ndarray:
    """Copy a device result buffer to host as a RESULT_DTYPE array (synchronizes)."""
    return result[:nreq * RESULT_DTYPE.itemsize].cpu().numpy().view(RESULT_DTYPE).copy()


def agile_rt_set_quarantine(rt: int, quarantine, nbytes: int) -> None:
    _check(lib().agile_rt_set_quarantine(rt, _ptr(quarantine), nbytes), "agile_rt_set_quarantine")


def agile_rt_clear(rt: int) -> None:
    _check(lib().agile_rt_clear(rt), "agile_rt_clear")


def agile_server_create(cs: int, tables, ring_base, ring_bytes, max_batch: int,
                        max_inflight: int, hbm_budget: int, ptrs, nptrs: int, ptr_verdict,
                        ptr_owner, device: int = 0) -> int:
    """tables: table handles (ints) or RangeTable objects, client i = tables[i];
    ring_base / ring_bytes: per-client output rings (device addresses, bytes)."""
    hs = [t.handle if isinstance(t, RangeTable) else int(t) for t in tables]
    arr = (_vp * len(hs))(*hs)
    rb = np.ascontiguousarray(ring_base, dtype=np.uint64)
    rs = np.ascontiguousarray(ring_bytes, dtype=np.uint64)
    cfg = agile_server_config(max_batch, max_inflight, hbm_budget)
    h = _vp()
    _check(lib().agile_server_create(ctypes.byref(h), cs, arr, len(hs), rb.ctypes.data,
                                     rs.ctypes.data, ctypes.byref(cfg), _ptr(ptrs), nptrs,
                                     _ptr(ptr_verdict), _ptr(ptr_owner), device),
           "agile_server_create")
    return h.value


def agile_server_destroy(sv: int) -> None:
    _check(lib().agile_server_destroy(sv), "agile_server_destroy")


def agile_server_run(sv: int, reqs: np.ndarray, out_bytes, arrival_s, revoke_client=None,
                     revoke_s=None, record=None, rec_buf=None, rec_off=None):
    """reqs: REQUEST_DTYPE array (in/out: output addresses are filled in). Returns
    (latency_s, launch_s, results, stats) as numpy arrays and an agile_server_stats."""
    assert reqs.dtype == REQUEST_DTYPE and reqs.flags.c_contiguous
    n = len(reqs)
    ob = np.ascontiguousarray(out_bytes, dtype=np.uint64)
    ar = np.ascontiguousarray(arrival_s, dtype=np.float64)
    rc_ = np.ascontiguousarray(revoke_client if revoke_client is not None else [], np.uint32)
    rt_ = np.ascontiguousarray(revoke_s if revoke_s is not None else [], np.float64)
    lat = np.empty(n, np.float64)
    lau = np.empty(n, np.float64)
    res = np.zeros(n, RESULT_DTYPE)
    st = agile_server_stats()
    rec = None if record is None else np.ascontiguousarray(record, np.uint8)
    roff = None if rec_off is None else np.ascontiguousarray(rec_off, np.uint64)
    _check(lib().agile_server_run(sv, reqs.ctypes.data, ob.ctypes.data, ar.ctypes.data, n,
                                  rc_.ctypes.data, rt_.ctypes.data, len(rc_),
                                  None if rec is None else rec.ctypes.data,
                                  None if rec_buf is None else rec_buf.ctypes.data,
                                  None if roff is None else roff.ctypes.data,
                                  lat.ctypes.data, lau.ctypes.data, res.ctypes.data,
                                  ctypes.byref(st)), "agile_server_run")
    return lat, lau, res, st


def agile_tokens_create(capacity: int, key: int, device: int = 0) -> int:
    h = _vp()
    _check(lib().agile_tokens_create(ctypes.byref(h), capacity, key & ((1 << 64) - 1), device),
           "agile_tokens_create")
    return h.value


def agile_tokens_destroy(ts: int) -> None:
    _check(lib().agile_tokens_destroy(ts), "agile_tokens_destroy")


def agile_token_mint(ts: int, client: int, kind: int) -> int:
    out = _u64()
    _check(lib().agile_token_mint(ts, client, kind, ctypes.byref(out)), "agile_token_mint")
    return out.value


def agile_token_release(ts: int, token: int, client: int) -> None:
    _check(lib().agile_token_release(ts, token & ((1 << 64) - 1), client), "agile_token_release")


def agile_tokens_check(ts: int, tokens, clients, kinds, n: int, verdict, slot,
                       stream=None) -> None:
    """tokens: device int64 [n] (bit patterns), clients: int32 [n], kinds: uint8 [n] or None,
    verdict: uint8 [n], slot: int32 [n]."""
    _check(lib().agile_tokens_check(ts, _ptr(tokens), _ptr(clients), _ptr(kinds), n,
                                    _ptr(verdict), _ptr(slot), _stream(stream)),
           "agile_tokens_check")


class TokenTable:
    """Owning wrapper of one token slot table."""

    def __init__(self, capacity: int, key: int, device: int = 0):
        self.handle = agile_tokens_create(capacity, key, device)

    def close(self):
        if getattr(self, "handle", None):
            agile_tokens_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def mint(self, client: int, kind: int) -> int:
        return agile_token_mint(self.handle, client, kind)

    def release(self, token: int, client: int) -> None:
        agile_token_release(self.handle, token, client)

    def check(self, tokens, clients, kinds=None, stream=None):
        """Device tensors in, (verdict uint8, slot int32) device tensors out."""
        n = tokens.numel()
        v = torch.empty(n, dtype=torch.uint8, device=tokens.device)
        s = torch.empty(n, dtype=torch.int32, device=tokens.device)
        agile_tokens_check(self.handle, tokens, clients, kinds, n, v, s, stream)
        return v, s


class RangeTable:
    """Owning wrapper of one table handle (destroyed on close or garbage collection)."""

    def __init__(self, capacity: int, device: int = 0):
        self.handle = agile_rt_create(capacity, device)

    def close(self):
        if getattr(self, "handle", None):
            agile_rt_destroy(self.handle)
            self.handle = None

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def insert(self, base: int, size: int, kind: int = KIND_USER, backed: bool = False) -> int:
        return agile_rt_insert(self.handle, base, size, kind | (RANGE_BACKED if backed else 0))

    def insert_tensor(self, t: torch.Tensor, kind: int = KIND_USER) -> int:
        """Register a tensor's bytes as one range (backed: a tensor's storage is mapped
        device memory)."""
        return self.insert(t.data_ptr(), t.numel() * t.element_size(), kind, backed=True)

    def insert_many(self, base, size, kind, backed: bool = False):
        if backed:
            kind = torch.as_tensor(kind).to(torch.uint8) | RANGE_BACKED
        return agile_rt_insert_many(self.handle, base, size, kind)

    def remove(self, rid: int) -> None:
        agile_rt_remove(self.handle, rid)

    def __len__(self):
        return agile_rt_count(self.handle)

    def fault_log(self, clear: bool = False, stream=None):
        return agile_fault_log_read(self.handle, clear, stream)


# ---- fixed address apertures (include/agile_aperture.h) -----------------------------------
def agile_aperture_create(device: int, sizes, budget=None, base_hint: int = 0) -> int:
    """sizes / budget: three byte counts (I/O, module, user); budget None: no limit."""
    sz = (ctypes.c_uint64 * 3)(*[int(x) for x in sizes])
    bk = (ctypes.c_uint64 * 3)(*[int(x) for x in budget]) if budget is not None else None
    h = _vp()
    _check(lib().agile_aperture_create(ctypes.byref(h), device, ctypes.cast(sz, _vp),
                                       ctypes.cast(bk, _vp) if bk is not None else None,
                                       base_hint), "agile_aperture_create")
    return h.value


def agile_aperture_destroy(ap: int) -> None:
    _check(lib().agile_aperture_destroy(ap), "agile_aperture_destroy")


def agile_aperture_info(ap: int):
    """Returns ((io start, module start, user start, user end), mapped bytes per aperture,
    granularity)."""
    b = (ctypes.c_uint64 * 4)()
    k = (ctypes.c_uint64 * 3)()
    g = _u64()
    _check(lib().agile_aperture_info(ap, ctypes.cast(b, _vp), ctypes.cast(k, _vp),
                                     ctypes.byref(g)), "agile_aperture_info")
    return tuple(int(x) for x in b), tuple(int(x) for x in k), g.value


def agile_aperture_alloc(ap: int, region: int, nbytes: int, rt: int = 0):
    """Returns (address, range id or -1)."""
    p, rid = _vp(), _i32()
    _check(lib().agile_aperture_alloc(ap, region, nbytes, rt or None, ctypes.byref(p),
                                      ctypes.byref(rid)), "agile_aperture_alloc")
    return p.value, rid.value


def agile_aperture_free(ap: int, ptr: int) -> None:
    _check(lib().agile_aperture_free(ap, _ptr(ptr)), "agile_aperture_free")


def agile_validate_aperture(ap: int, q, n: int, verdict, region, stream=None) -> None:
    _check(lib().agile_validate_aperture(ap, _ptr(q), n, _ptr(verdict), _ptr(region),
                                         _stream(stream)), "agile_validate_aperture")
