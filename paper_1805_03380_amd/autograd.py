"""torch.autograd.Function over the CSC product: forward Y = A.X (spm_csc_spmm), backward
dX = A^T.G and dvalues = G.X^T sampled on A's pattern (spm_csc_spmm_backward), both hand
written kernels.  Gradients are taken with respect to the stored CSC values and X; the
pattern (col_ptr, row_idx) is constant.
"""
from __future__ import annotations

import torch

from . import ops


class CscSpmm(torch.autograd.Function):
    """Y = A(values) . X  with A's pattern fixed by ``A`` (an ops.CSCMatrix)."""

    @staticmethod
    def forward(ctx, values: torch.Tensor, X: torch.Tensor, A: ops.CSCMatrix):
        ctx.A = A
        ctx.save_for_backward(values, X)
        return ops.spmm(A, X, values=values)

    @staticmethod
    def backward(ctx, G: torch.Tensor):
        values, X = ctx.saved_tensors
        A = ctx.A
        need_v, need_x = ctx.needs_input_grad[0], ctx.needs_input_grad[1]
        if not (need_v or need_x):
            return None, None, None
        G = G.to(X.dtype) if G.dtype != X.dtype else G
        dX, dval = ops.spmm_backward(A, G.contiguous(), X, values=values, need_dX=need_x,
                                     need_dval=need_v, dx_dtype=X.dtype,
                                     dval_dtype=values.dtype)
        if dval is not None:
            dval = dval[: values.shape[0]]
        return dval, dX, None


def csc_spmm(A: ops.CSCMatrix, values: torch.Tensor, X: torch.Tensor) -> torch.Tensor:
    """Differentiable Y = A(values) . X."""
    return CscSpmm.apply(values, X, A)
