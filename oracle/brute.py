"""Brute-force classification used to pin ``oracle.table`` (test infrastructure only).

No search, no subtraction trick: the owner of every byte is found by scanning all
entries, and a range is accepted only if every one of its bytes has the same USER owner
(the one-allocation rule of the paper's Section V-C). Meant for tables of a few dozen
entries and short lengths; longer lengths are checked through their first and last byte,
which is equivalent because entries are intervals.
"""
from __future__ import annotations

from .table import ALLOW, V_PROTECTED, V_STRADDLE, V_UNMAPPED, V_INEXACT, USER, U64_MAX


def owner_scan(entries, a: int):
    """Entry containing byte ``a`` by linear scan over (base, end, kind, id) tuples."""
    hit = None
    for e in entries:
        if e[0] <= a < e[1]:
            assert hit is None, "entries overlap"
            hit = e
    return hit


def verdict_brute(entries, addr: int, length: int):
    first = owner_scan(entries, addr)
    if first is None:
        return V_UNMAPPED, -1
    if first[2] != USER:
        return V_PROTECTED, first[3]
    L = length if length > 0 else 1
    last = addr + L - 1
    if last > U64_MAX:
        return V_STRADDLE, first[3]
    probe = range(addr, last + 1) if L <= 256 else (addr, last)
    for a in probe:
        if owner_scan(entries, a) is not first:
            return V_STRADDLE, first[3]
    return ALLOW, first[3]


def dma_verdict_brute(entries, addr: int, length: int):
    """DMA registration by its definition: accepted iff some USER entry is exactly
    [addr, addr + length); otherwise the pointer verdict, with ALLOW reported as INEXACT."""
    for b, e, kind, rid in entries:
        if kind == USER and b == addr and e - b == length:
            return ALLOW, rid
    v, rid = verdict_brute(entries, addr, length)
    return (V_INEXACT if v == ALLOW else v), rid
