"""The C-ABI library loads and exports every entry point its header declares (CPU only:
no call here reaches the GPU; argument errors are rejected before any device work)."""
import ctypes
import glob
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_functions():
    names = set()
    for h in glob.glob(os.path.join(ROOT, "include", "*.h")):
        with open(h) as fh:
            text = fh.read()
        text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
        for m in re.finditer(r"^\s*(?:const\s+)?\w+\s*\*?\s*(agile_\w+)\s*\(", text, re.M):
            names.add(m.group(1))
    return sorted(names)


@pytest.fixture(scope="module")
def L():
    from paper_2606_06697_amd import guard
    if not os.path.exists(guard.LIB_PATH):
        from paper_2606_06697_amd import _build
        _build.build()
    return guard.lib()


def test_header_declares_the_boundary():
    names = declared_functions()
    for must in ("agile_rt_create", "agile_rt_insert", "agile_rt_remove", "agile_validate_ptrs",
                 "agile_guarded_copy", "agile_guarded_gather", "agile_guarded_scatter",
                 "agile_fault_log_read"):
        assert must in names
    assert len(names) >= 18


def test_library_exports_every_declared_symbol(L):
    for name in declared_functions():
        assert hasattr(L, name), name


def test_binding_covers_every_symbol():
    from paper_2606_06697_amd import guard
    for name in declared_functions():
        assert hasattr(guard, name), name


def test_argument_errors_fail_closed(L):
    from paper_2606_06697_amd import guard as g
    assert g.strerror(g.AGILE_EOVERLAP).startswith("range overlaps")
    assert "trap policy" in g.strerror(g.AGILE_ETRAPPED)
    h = ctypes.c_void_p()
    assert L.agile_rt_create(ctypes.byref(h), 0, 0) == g.AGILE_EINVAL
    assert L.agile_rt_create(None, 16, 0) == g.AGILE_EINVAL
    assert L.agile_rt_insert(None, 0, 1, 0, None) == g.AGILE_EINVAL
    assert L.agile_rt_remove(None, 0) == g.AGILE_EINVAL
    assert L.agile_validate_ptrs(None, 0, 1, 0, 0, 0) == g.AGILE_EINVAL
    assert L.agile_validate_dma(None, 0, 1, 0, 0, 0) == g.AGILE_EINVAL
    assert L.agile_rt_set_quarantine(None, 0, 0) == g.AGILE_EINVAL
    assert L.agile_tokens_create(None, 16, 1, 0) == g.AGILE_EINVAL
    assert L.agile_tokens_create(ctypes.byref(h), 0, 1, 0) == g.AGILE_EINVAL
    assert L.agile_tokens_create(ctypes.byref(h), (1 << 24) + 1, 1, 0) == g.AGILE_EINVAL
    assert L.agile_token_mint(None, 0, 0, None) == g.AGILE_EINVAL
    assert L.agile_token_release(None, 0, 0) == g.AGILE_EINVAL
    assert L.agile_tokens_check(None, 0, 0, 0, 1, 0, 0, 0) == g.AGILE_EINVAL
    assert L.agile_tokens_destroy(None) == g.AGILE_OK
    assert L.agile_guarded_copy(None, 0, 0, 16, 0, 0) == g.AGILE_EINVAL
    assert L.agile_guarded_gather(None, 0, 0, 4, 0, 1, 0, 0, 0) == g.AGILE_EINVAL
    assert L.agile_fault_log_read(None, None, 0, 0) == g.AGILE_EINVAL
    assert L.agile_rt_destroy(None) == g.AGILE_OK
    # unknown dtype / zero or misaligned row size are rejected before any launch
    assert L.agile_unguarded_gather(0, 0, 4, 0, 1, 9, 0) == g.AGILE_EINVAL
    assert L.agile_unguarded_gather(0, 0, 0, 0, 1, 0, 0) == g.AGILE_EINVAL
    assert L.agile_unguarded_gather(0, 0, 6, 0, 1, 0, 0) == g.AGILE_EINVAL
    assert L.agile_unguarded_scatter(0, 4, 0, 0, 1, 0, 3, 0) == g.AGILE_EINVAL
    # apertures: null handles and empty apertures are rejected before any HIP call
    assert "virtual memory" in g.strerror(g.AGILE_ENOTSUP)
    ok3 = (ctypes.c_uint64 * 3)(1, 1, 1)
    assert L.agile_aperture_create(None, 0, ok3, None, 0) == g.AGILE_EINVAL
    assert L.agile_aperture_create(ctypes.byref(h), 0, None, None, 0) == g.AGILE_EINVAL
    for bad in ((0, 1, 1), (1, 1, (1 << 48) + 1)):
        assert L.agile_aperture_create(ctypes.byref(h), 0, (ctypes.c_uint64 * 3)(*bad), None,
                                       0) == g.AGILE_EINVAL
    assert L.agile_aperture_info(None, None, None, None) == g.AGILE_EINVAL
    assert L.agile_aperture_alloc(None, 2, 16, None, None, None) == g.AGILE_EINVAL
    assert L.agile_aperture_free(None, None) == g.AGILE_EINVAL
    assert L.agile_validate_aperture(None, 0, 1, 0, 0, 0) == g.AGILE_EINVAL
    assert L.agile_aperture_destroy(None) == g.AGILE_OK
