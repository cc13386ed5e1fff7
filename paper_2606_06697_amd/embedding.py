"""Guarded embedding lookup with a guarded backward, behind ``torch.autograd.Function``.

Forward: ``Y[i, :] = W[idx[i], :]`` through ``agile_guarded_gather``: a row whose address falls
outside W's own allocation (a hostile index aimed at a protected range, a hole, or another
allocation) reads zeros and is counted in the table's fault log. Backward:
``dW[r, :] = sum of dY[i, :] over allowed i with idx[i] = r`` through ``agile_guarded_scatter``
with accumulation (calls of 32,768 rows or more radix-sort their destination rows and sum each
run of equal rows once; smaller calls sort chunks of 2,048 rows in LDS and add each run with one
atomic row update); contributions aimed outside dW are dropped and counted. Both run on the current torch stream.

The guard binds every pointer argument to its own USER range, so the temporaries this function
creates (the output Y, the incoming gradient dY and the gradient dW) are registered in the
caller's table for the duration of the launch and removed right after; W and idx must already
be registered by the caller. Each call therefore changes the table, which is re-uploaded (in
stream order) by the next launch.
"""
from __future__ import annotations

import torch

from . import guard as g

_DTYPES = {torch.float32: g.DTYPE_F32, torch.float64: g.DTYPE_F64}


def _registered(table, tensors):
    ids = []
    try:
        for t in tensors:
            ids.append(table.insert_tensor(t, g.KIND_USER))
    except Exception:
        for rid in ids:
            table.remove(rid)
        raise
    return ids


class GuardedEmbeddingFunction(torch.autograd.Function):
    @staticmethod
    def forward(ctx, weight, idx, table, policy=g.POLICY_SUPPRESS_LOG):
        if weight.dim() != 2 or weight.dtype not in _DTYPES or not weight.is_contiguous():
            raise ValueError("weight must be a contiguous 2-D float32/float64 tensor")
        if idx.dtype != torch.int64 or not idx.is_contiguous():
            raise ValueError("idx must be a contiguous int64 tensor")
        n, D = idx.numel(), weight.shape[1]
        rb = D * weight.element_size()
        out = torch.empty((n, D), dtype=weight.dtype, device=weight.device)
        ids = _registered(table, [out])
        try:
            g.agile_guarded_gather(table.handle, out, weight, rb, idx, n, _DTYPES[weight.dtype],
                                   policy)
        finally:
            for rid in ids:
                table.remove(rid)
        ctx.save_for_backward(idx)
        ctx.table, ctx.policy = table, policy
        ctx.wshape, ctx.wdtype = weight.shape, weight.dtype
        return out

    @staticmethod
    def backward(ctx, dY):
        (idx,) = ctx.saved_tensors
        table = ctx.table
        dY = dY.contiguous()
        D = ctx.wshape[1]
        dW = torch.zeros(ctx.wshape, dtype=ctx.wdtype, device=dY.device)
        rb = D * dW.element_size()
        ids = _registered(table, [dW, dY])
        try:
            # dW was just zeroed: its rows are summed into without being read
            g.agile_guarded_scatter(table.handle, dW, rb, idx, dY, idx.numel(),
                                    _DTYPES[ctx.wdtype], g.SCATTER_ADD_INTO_ZEROS, ctx.policy)
        finally:
            for rid in ids:
                table.remove(rid)
        return dW, None, None, None


def guarded_embedding(weight, idx, table, policy=g.POLICY_SUPPRESS_LOG):
    """``weight[idx]`` with the kernel memory guard on the lookup and on its gradient."""
    return GuardedEmbeddingFunction.apply(weight, idx, table, policy)


class GuardedEmbedding(torch.nn.Module):
    """An embedding table whose storage is registered as one USER range of ``table``."""

    def __init__(self, num, dim, table, dtype=torch.float32, device="cuda"):
        super().__init__()
        self.weight = torch.nn.Parameter(torch.empty(num, dim, dtype=dtype, device=device))
        torch.nn.init.normal_(self.weight)
        self.table = table
        self._rid = table.insert_tensor(self.weight.data, g.KIND_USER)

    def forward(self, idx):
        return guarded_embedding(self.weight, idx, self.table)
