"""Allocation table and pointer classification (oracle; test infrastructure only).

Follows the paper's memory model: every user allocation is recorded as (base, live size)
(Section V-A, V-C); protected module memory and the MMIO aperture are separate ranges
(Section IV-E, Table I); a client pointer is resolved against the table and the requested
byte range must stay inside one live user allocation, while pointers into protected or
MMIO ranges, freed allocations and unknown addresses are rejected (Section IV-E and V-C).

Readings where the paper is silent:

* verdict codes: ALLOW=0, PROTECTED=1, STRADDLE=2, UNMAPPED=3 (CROSS_ALLOC=4 is only used
  as a fault reason by the kernel guard); the owner of the first byte decides the code.
* owner index = the stable insertion id (0, 1, 2, ... per table, never reused).
* a zero length is checked as length 1 (the pointer itself must be inside an allocation).
* the length test is ``max(len,1) <= end - addr`` (no overflow of ``addr + len``).
* ranges are half-open ``[base, base+size)`` with ``size >= 1`` and ``base + size <= 2**64-1``.
* MMIO and module-protected ranges both classify as PROTECTED.
* DMA registration (Section V-C: accepted only for an exact live user allocation) uses the
  same classification, except that an allowed range which is not the whole allocation
  (``addr != base`` or ``len != size``, the length taken as given, so zero is never exact)
  gets the code INEXACT=5.
"""
from __future__ import annotations

import bisect

import numpy as np

ALLOW, V_PROTECTED, V_STRADDLE, V_UNMAPPED, V_CROSS_ALLOC = 0, 1, 2, 3, 4
V_INEXACT = 5
USER, PROTECTED, MMIO = 0, 1, 2
U64_MAX = (1 << 64) - 1


class OverlapError(ValueError):
    pass


class RangeTable:
    """A set of disjoint half-open ranges with stable insertion ids."""

    def __init__(self):
        self._bases: list[int] = []          # sorted
        self._by_base: dict[int, tuple] = {}  # base -> (end, kind, id)
        self._by_id: dict[int, int] = {}      # id -> base
        self._backed: set[int] = set()        # ids of ranges declared backed (mapped memory)
        self._next_id = 0

    def __len__(self):
        return len(self._bases)

    def insert(self, base: int, size: int, kind: int, backed: bool = False) -> int:
        """Add [base, base+size) of ``kind``; ``backed`` records the caller's statement that the
        range is mapped memory (read only by the ``report`` policy)."""
        base, size, kind = int(base), int(size), int(kind)
        if kind not in (USER, PROTECTED, MMIO):
            raise ValueError("unknown kind")
        if size < 1 or base < 0 or base + size > U64_MAX:
            raise ValueError("range must satisfy size >= 1 and base + size <= 2**64 - 1")
        end = base + size
        k = bisect.bisect_right(self._bases, base)
        if k > 0:
            pb = self._bases[k - 1]
            if self._by_base[pb][0] > base:
                raise OverlapError("overlaps the range below")
        if k < len(self._bases) and self._bases[k] < end:
            raise OverlapError("overlaps the range above")
        rid = self._next_id
        self._next_id += 1
        self._bases.insert(k, base)
        self._by_base[base] = (end, kind, rid)
        self._by_id[rid] = base
        if backed:
            self._backed.add(rid)
        return rid

    def is_backed(self, rid: int) -> bool:
        return int(rid) in self._backed

    def remove(self, rid: int) -> None:
        """Free a range: its bytes become a hole (freed allocations are rejected)."""
        base = self._by_id.pop(int(rid))  # KeyError for unknown or already-removed ids
        del self._by_base[base]
        self._backed.discard(int(rid))
        self._bases.pop(bisect.bisect_left(self._bases, base))

    def entries(self):
        """(base, end, kind, id) tuples in address order."""
        return [(b, *self._by_base[b]) for b in self._bases]

    def arrays(self):
        """Sorted uint64 bases and ends, uint8 kinds, int32 ids."""
        e = self.entries()
        base = np.array([x[0] for x in e], dtype=np.uint64)
        end = np.array([x[1] for x in e], dtype=np.uint64)
        kind = np.array([x[2] for x in e], dtype=np.uint8)
        ids = np.array([x[3] for x in e], dtype=np.int32)
        return base, end, kind, ids

    # ---- classification -------------------------------------------------------------
    def owner_entry(self, addr: int):
        """The entry (base, end, kind, id) with base <= addr < end, or None."""
        k = bisect.bisect_right(self._bases, int(addr)) - 1
        if k < 0:
            return None
        b = self._bases[k]
        end, kind, rid = self._by_base[b]
        if int(addr) < end:
            return (b, end, kind, rid)
        return None

    def verdict(self, addr: int, length: int):
        """Classify the byte range [addr, addr + max(length,1)) -> (verdict, owner id)."""
        addr, length = int(addr), int(length)
        ent = self.owner_entry(addr)
        if ent is None:
            return V_UNMAPPED, -1
        _, end, kind, rid = ent
        if kind != USER:
            return V_PROTECTED, rid
        if max(length, 1) <= end - addr:
            return ALLOW, rid
        return V_STRADDLE, rid

    def verdict_many(self, addr: np.ndarray, length: np.ndarray):
        """Vectorized ``verdict`` over uint64 arrays (same rules, numpy searchsorted)."""
        addr = np.asarray(addr, dtype=np.uint64)
        length = np.asarray(length, dtype=np.uint64)
        base, end, kind, ids = self.arrays()
        v = np.full(addr.shape, V_UNMAPPED, dtype=np.uint8)
        owner = np.full(addr.shape, -1, dtype=np.int32)
        if base.size == 0:
            return v, owner
        j = np.searchsorted(base, addr, side="right").astype(np.int64) - 1
        jc = np.maximum(j, 0)
        inside = (j >= 0) & (addr < end[jc])
        prot = inside & (kind[jc] != USER)
        L = np.maximum(length, np.uint64(1))
        room = end[jc] - np.where(inside, addr, end[jc])  # end - addr where inside
        fits = inside & ~prot & (L <= room)
        strad = inside & ~prot & ~fits
        v[prot] = V_PROTECTED
        v[fits] = ALLOW
        v[strad] = V_STRADDLE
        owner[inside] = ids[jc[inside]]
        return v, owner

    def dma_verdict(self, addr: int, length: int):
        """DMA registration check -> (verdict, owner id): ALLOW only when [addr, addr+length)
        is exactly a live USER allocation."""
        v, rid = self.verdict(addr, length)
        if v == ALLOW:
            b, end, _, _ = self.owner_entry(addr)
            if int(addr) != b or int(length) != end - b:
                v = V_INEXACT
        return v, rid

    def dma_verdict_many(self, addr: np.ndarray, length: np.ndarray):
        """Vectorized ``dma_verdict``."""
        addr = np.asarray(addr, dtype=np.uint64)
        length = np.asarray(length, dtype=np.uint64)
        v, owner = self.verdict_many(addr, length)
        base, end, _, _ = self.arrays()
        if base.size:
            jc = np.maximum(np.searchsorted(base, addr, side="right").astype(np.int64) - 1, 0)
            exact = (addr == base[jc]) & (length == end[jc] - base[jc])
            v[(v == ALLOW) & ~exact] = V_INEXACT
        return v, owner

    def binding(self, p: int):
        """Kernel-argument binding: the USER allocation containing pointer ``p`` as
        ``(lo, hi)``, or the empty interval ``(0, 0)`` when ``verdict(p, 1) != ALLOW``."""
        v, _ = self.verdict(p, 1)
        if v != ALLOW:
            return (0, 0)
        b, end, _, _ = self.owner_entry(p)
        return (b, end)
