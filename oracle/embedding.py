"""Guarded embedding lookup and its gradient (oracle; test infrastructure only).

The forward pass is the guarded gather of ``oracle.guarded`` (rows of the weight table
selected by an index vector; a denied row reads zeros and is logged). Its gradient with
respect to the table is the transpose of that selection: every allowed output row adds its
upstream gradient into the table row it was read from, ``dW[r] = sum over allowed i with
idx[i] = r of dY[i]``. The reference accumulates in float64 in index order and rounds
once to the table's dtype; the order of an fp32 sum is otherwise unspecified.
"""
from __future__ import annotations

import numpy as np


def embedding_grad_ref(idx, allowed, dY, rows, out_dtype=np.float32):
    """``dW`` [rows, D] from int64 ``idx`` [n], bool ``allowed`` [n] and ``dY`` [n, D]."""
    idx = np.asarray(idx, dtype=np.int64)
    allowed = np.asarray(allowed, dtype=bool)
    dY = np.asarray(dY)
    acc = np.zeros((rows, dY.shape[1]), dtype=np.float64)
    np.add.at(acc, idx[allowed], dY[allowed].astype(np.float64))
    return acc.astype(out_dtype)


def embedding_forward_ref(W, idx, allowed):
    """``Y[i] = W[idx[i]]`` for allowed rows, zeros otherwise (W [rows, D] array)."""
    idx = np.asarray(idx, dtype=np.int64)
    allowed = np.asarray(allowed, dtype=bool)
    Y = np.zeros((idx.size, W.shape[1]), dtype=W.dtype)
    Y[allowed] = W[idx[allowed]]
    return Y
