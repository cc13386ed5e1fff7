"""CPU oracle for the protected-memory range guard. TEST INFRASTRUCTURE ONLY.

Only ``tests/``, ``__graft_entry__.smoke()`` and the ``cpu_baseline`` leg of ``bench.py``
may import this package. The product path (the HIP library and its Python binding)
never calls it, and it shares no code with that path.

It is a plain, slow, obviously-correct restatement of what the paper's memory model
computes (AgileOS, Section IV-C on client handles; Section IV-E "Protected GPU Memory
Model", Table I; Section V-A on the virtual-memory layout; Section V-C "Pointer Metadata and
DMA Registration"; Section V-E "PTX Processing and Kernel Memory Guard"):

* ``table``    - the allocation table and the pointer classification rule.
* ``brute``    - linear-scan / per-byte classification used to pin ``table``.
* ``memory``   - a byte-addressed model of device memory (backed allocations).
* ``guarded``  - per-access guarded copy / triad / gather / scatter(-add) and the
                 first-fault log, as vectorized masks and as per-access loops.
* ``batched``  - per-request verdicts for a multi-client batch.
* ``embedding``- guarded embedding forward and its fp64-accumulated gradient.
* ``tokens``   - client handle tokens (slot table, SplitMix64 tags) and their history model.
* ``aperture`` - the coarse check against Table I's three fixed apertures.

Where the paper is silent the readings are stated in the docstrings (verdict codes,
zero-length queries, overflow, adjacency, access width, suppression values, the order
that decides which fault is "first").
"""
from .table import (  # noqa: F401
    RangeTable, OverlapError, ALLOW, V_PROTECTED, V_STRADDLE, V_UNMAPPED, V_CROSS_ALLOC,
    V_INEXACT,
    USER, PROTECTED, MMIO, U64_MAX,
)
