"""Per-request verdicts for a batch of mediated requests (oracle; test infrastructure only).

The paper's worker checks every pointer argument of a mediated request (a CUDA handler
or a trusted library adapter call) against the calling client's own allocations before
the real call, and rejects the request otherwise (Section IV-E, IV-F, V-C); a pointer
that is valid for another client is not valid for this one (Section III, cross-client
pointers). Reading for a request with several arguments: the request's verdict is the
verdict of its lowest-index argument that is not ALLOW (ALLOW if there is none).
"""
from __future__ import annotations

import numpy as np

from .table import ALLOW


def batch_verdicts(tables, client, ptr_off, ptrs):
    """Per-pointer (verdict, owner) and per-request (verdict, failing arg index, owner).

    ``tables`` - one ``RangeTable`` per client; ``client`` [R]; ``ptr_off`` [R+1] offsets
    into ``ptrs`` [P, 2] = (addr, len) as uint64-compatible integers.
    """
    client = np.asarray(client)
    ptr_off = np.asarray(ptr_off, dtype=np.int64)
    ptrs = np.asarray(ptrs).astype(np.uint64)
    R = client.size
    P = ptrs.shape[0]
    pv = np.zeros(P, dtype=np.uint8)
    po = np.zeros(P, dtype=np.int32)
    rv = np.zeros(R, dtype=np.uint8)
    ra = np.full(R, -1, dtype=np.int32)
    ro = np.full(R, -1, dtype=np.int32)
    for r in range(R):
        a, b = int(ptr_off[r]), int(ptr_off[r + 1])
        v, o = tables[int(client[r])].verdict_many(ptrs[a:b, 0], ptrs[a:b, 1])
        pv[a:b] = v
        po[a:b] = o
        bad = np.flatnonzero(v != ALLOW)
        if bad.size:
            k = int(bad[0])
            rv[r], ra[r], ro[r] = v[k], k, o[k]
    return pv, po, rv, ra, ro
