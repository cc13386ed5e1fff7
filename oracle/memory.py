"""Byte-addressed model of device memory for the oracle (test infrastructure only).

Only allocations that hold data are modelled; a guarded access that the guard allows
always lies inside one USER allocation, so the oracle never needs the contents of
protected ranges or holes (the guard never touches them: Section V-E's policies either
stop or redirect such an access).
"""
from __future__ import annotations

import bisect

import numpy as np


class Memory:
    def __init__(self):
        self._bases: list[int] = []
        self._bufs: dict[int, np.ndarray] = {}

    def add(self, base: int, data) -> np.ndarray:
        """Back ``[base, base + len(data))`` with a uint8 copy of ``data`` (bytes-like or array)."""
        arr = np.frombuffer(bytes(np.ascontiguousarray(data).tobytes()), dtype=np.uint8).copy()
        base = int(base)
        k = bisect.bisect_right(self._bases, base)
        if k > 0 and self._bases[k - 1] + self._bufs[self._bases[k - 1]].size > base:
            raise ValueError("backed allocations overlap")
        if k < len(self._bases) and self._bases[k] < base + arr.size:
            raise ValueError("backed allocations overlap")
        self._bases.insert(k, base)
        self._bufs[base] = arr
        return arr

    def buffer(self, base: int) -> np.ndarray:
        return self._bufs[int(base)]

    def locate(self, lo: int, hi: int):
        """(array, offset of ``lo`` in it) for the backed allocation covering [lo, hi)."""
        k = bisect.bisect_right(self._bases, int(lo)) - 1
        if k < 0:
            raise KeyError("address not backed")
        b = self._bases[k]
        arr = self._bufs[b]
        if int(hi) > b + arr.size:
            raise KeyError("range not backed")
        return arr, int(lo) - b

    def read(self, addr: int, w: int) -> bytes:
        arr, off = self.locate(addr, addr + w)
        return arr[off:off + w].tobytes()

    def write(self, addr: int, data: bytes) -> None:
        arr, off = self.locate(addr, addr + len(data))
        arr[off:off + len(data)] = np.frombuffer(data, dtype=np.uint8)
