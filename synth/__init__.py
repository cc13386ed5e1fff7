"""Seeded synthetic inputs shared by the oracle tests, the GPU parity tests and the bench.

This package draws range tables, pointer queries, data buffers and index streams.
It holds none of the guard's arithmetic (no verdicts, no bounds checks, no copies):
both the CPU oracle and the HIP library only ever receive what it produces.
"""
from .workloads import (  # noqa: F401
    PAGE, KIND_USER, KIND_PROTECTED, KIND_MMIO,
    Table, make_table, make_queries, aperture_table, uniform_f32, loguniform_int,
    uniform_indices, zipf_indices, make_batch_requests, make_serving_trace,
)
