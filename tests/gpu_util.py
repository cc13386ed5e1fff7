"""Helpers for the GPU parity tests: a device table kept in step with an oracle table, and a
device arena whose bytes are mirrored into the oracle's memory model."""
import os

import numpy as np
import pytest
import torch

from oracle.memory import Memory
from oracle.table import RangeTable as OracleTable


def need_gpu():
    if not torch.cuda.is_available():
        pytest.skip("needs a GPU")


def guard_mod():
    from paper_2606_06697_amd import guard
    if not os.path.exists(guard.LIB_PATH):
        from paper_2606_06697_amd import _build
        _build.build()
    guard.lib()
    return guard


class Twin:
    """A device range table and an oracle table fed the same inserts and removes."""

    def __init__(self, capacity=1024):
        g = guard_mod()
        self.g = g
        self.rt = g.RangeTable(capacity)
        self.ot = OracleTable()
        self.seq = 0

    @property
    def h(self):
        return self.rt.handle

    def insert(self, base, size, kind, backed=False):
        try:
            a = self.rt.insert(base, size, kind, backed)
        except self.g.AgileError:
            with pytest.raises(ValueError):   # the oracle rejects it too (OverlapError et al.)
                self.ot.insert(base, size, kind, backed)
            raise
        b = self.ot.insert(base, size, kind, backed)
        assert a == b
        return a

    def insert_table(self, tb):
        """Insert a synth.Table (bulk path on the device, one by one in the oracle)."""
        ids = self.rt.insert_many(tb.base, tb.size, tb.kind)
        for b, s, k in zip(tb.base.tolist(), tb.size.tolist(), tb.kind.tolist()):
            self.ot.insert(b, s, k)
        return ids

    def remove(self, rid):
        self.rt.remove(rid)
        self.ot.remove(rid)

    def next_seq(self):
        s = self.seq
        self.seq += 1
        return s

    def close(self):
        self.rt.close()


class Arena:
    """Device bytes (random) plus their mirror in an oracle Memory backing."""

    def __init__(self, nbytes, seed):
        gen = torch.Generator().manual_seed(seed)
        host = torch.randint(0, 256, (nbytes,), dtype=torch.uint8, generator=gen)
        self.dev = host.cuda()
        self.base = self.dev.data_ptr()
        self.mem = Memory()
        self.mem.add(self.base, host.numpy())
        self.n = nbytes

    def addr(self, off):
        return self.base + off

    def write(self, off, arr):
        b = np.ascontiguousarray(arr).view(np.uint8).reshape(-1)
        self.dev[off:off + b.size] = torch.from_numpy(b.copy()).cuda()
        self.mem.buffer(self.base)[off:off + b.size] = b

    def check(self, what=""):
        torch.cuda.synchronize()
        got = self.dev.cpu().numpy()
        want = self.mem.buffer(self.base)
        if not np.array_equal(got, want):
            bad = np.flatnonzero(got != want)
            raise AssertionError(f"{what}: {bad.size} bytes differ, first at arena offset "
                                 f"{bad[0]} (got {got[bad[0]]}, want {want[bad[0]]})")


def log_matches(twin, olog, what=""):
    """Compare (and clear) the device fault log with the oracle log."""
    g = twin.g
    rc, f = twin.rt.fault_log(clear=True)
    assert f["count"] == olog.count, (what, f, olog.count, olog.first)
    if olog.count == 0:
        assert rc == g.AGILE_OK and f["first_seq"] == g.NO_SEQ, (what, f)
    else:
        assert rc == g.AGILE_EFAULTED
        o = olog.first
        got = dict(seq=f["first_seq"], elem=f["first_elem"], operand=f["first_operand"],
                   addr=f["first_addr"], width=f["first_width"], verdict=f["first_verdict"],
                   owner=f["first_owner"], op=f["first_op"])
        assert got == o, (what, got, o)
    olog.clear()
