"""Aperture classification on the fixed virtual-address layout (oracle; test infrastructure
only: the product path never imports it).

Section IV-E (Table I) lays the GPU address space out as three fixed apertures, in this order
and back to back: a protected I/O aperture for MMIO mappings, a protected aperture for
kernel/module and imported service memory, and the user aperture that every user allocation
is carved from. Section V-A reserves them with the VMM API and maps physical memory into them
on demand. The Fig. 2 guard tests an address against the protected apertures alone, so its
cost does not depend on the number of allocations.

The classification here is the pointer rule of ``table.RangeTable.verdict`` applied to the
three apertures as three ranges (I/O as MMIO, module as PROTECTED, user as USER):

* the aperture holding the first byte decides; outside all three the range is UNMAPPED;
* in a protected aperture it is PROTECTED, whatever its length;
* in the user aperture it is ALLOW when ``max(len, 1)`` bytes fit before the aperture's end,
  STRADDLE otherwise.

The owner reported is the aperture's index (0 I/O, 1 module, 2 user), -1 outside.

Readings where the paper is silent:

* ``bounds = (b0, b1, b2, b3)``: I/O is ``[b0, b1)``, module ``[b1, b2)``, user ``[b2, b3)``,
  each non-empty, with ``b3 <= 2**64 - 1`` (the same end rule as table ranges);
* the check knows nothing of individual allocations: a hole inside the user aperture, or a
  freed allocation, still reads ALLOW. The allocation table stays the authority for the
  API-time rule of Section V-C; the aperture check is the coarse, size-independent one.
"""
from __future__ import annotations

import numpy as np

from .table import ALLOW, V_PROTECTED, V_STRADDLE, V_UNMAPPED, U64_MAX

IO, MODULE, USER_AP = 0, 1, 2

# Table I: 64 GiB I/O, 448 GiB kernel/module, 1 TiB user
TABLE1 = (0xF0000000000, 0xF1000000000, 0xF8000000000, 0x108000000000)


def check_bounds(bounds):
    b0, b1, b2, b3 = (int(x) for x in bounds)
    if not (0 <= b0 < b1 < b2 < b3 <= U64_MAX):
        raise ValueError("apertures must be non-empty, ordered and end below 2**64 - 1")
    return b0, b1, b2, b3


def aperture_verdict(bounds, addr: int, length: int):
    """Classify [addr, addr + max(length, 1)) -> (verdict, aperture index)."""
    b0, b1, b2, b3 = check_bounds(bounds)
    addr, length = int(addr), int(length)
    if addr < b0 or addr >= b3:
        return V_UNMAPPED, -1
    if addr < b1:
        return V_PROTECTED, IO
    if addr < b2:
        return V_PROTECTED, MODULE
    if max(length, 1) <= b3 - addr:
        return ALLOW, USER_AP
    return V_STRADDLE, USER_AP


def aperture_verdict_many(bounds, addr, length):
    """Vectorized ``aperture_verdict`` over uint64 arrays (same rules)."""
    b0, b1, b2, b3 = (np.uint64(x) for x in check_bounds(bounds))
    addr = np.asarray(addr, dtype=np.uint64)
    length = np.asarray(length, dtype=np.uint64)
    v = np.full(addr.shape, V_UNMAPPED, dtype=np.uint8)
    ap = np.full(addr.shape, -1, dtype=np.int32)
    io = (addr >= b0) & (addr < b1)
    mod = (addr >= b1) & (addr < b2)
    usr = (addr >= b2) & (addr < b3)
    room = b3 - np.where(usr, addr, b3)
    fits = usr & (np.maximum(length, np.uint64(1)) <= room)
    v[io | mod] = V_PROTECTED
    v[fits] = ALLOW
    v[usr & ~fits] = V_STRADDLE
    ap[io], ap[mod], ap[usr] = IO, MODULE, USER_AP
    return v, ap
