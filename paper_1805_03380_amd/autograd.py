"""torch.autograd.Functions over the CSC product, every step in hand-written kernels.

CscSpmm: forward Y = A.X (spm_csc_spmm), backward dX = A^T.G and dvalues = G.X^T sampled on
A's pattern (spm_csc_spmm_backward); gradients with respect to the stored CSC values and X,
the pattern (col_ptr, row_idx) constant.

CooSpmm: assembly and product together, Y = assemble(row, col, val).X; the backward runs the
adjoint once (dX and the dvalues) and gives every input triplet the dvalue of its location
(spm_coo_triplet_grad_csc), duplicates and locations that summed to zero included.
"""
from __future__ import annotations

import torch

from . import ops


def _grad_dtype(dt: torch.dtype) -> torch.dtype:
    """Element type the adjoint writes a gradient in: binary64 or binary32."""
    return torch.float64 if dt == torch.float64 else torch.float32


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
        # G keeps the element type it arrives in (Y's: binary64 with binary64 values); the
        # adjoint reads it as such.  A bfloat16 X gets its gradient in binary32 (autograd
        # rounds it to X's type).
        dX, dval = ops.spmm_backward(A, G.contiguous(), X, values=values, need_dX=need_x,
                                     need_dval=need_v, dx_dtype=_grad_dtype(X.dtype),
                                     dval_dtype=values.dtype)
        if dval is not None:
            dval = dval[: values.shape[0]]
        return dval, dX, None


def csc_spmm(A: ops.CSCMatrix, values: torch.Tensor, X: torch.Tensor) -> torch.Tensor:
    """Differentiable Y = A(values) . X."""
    return CscSpmm.apply(values, X, A)


class CooSpmm(torch.autograd.Function):
    """Y = assemble(row, col, val) . X, differentiable in the triplet values and X."""

    @staticmethod
    def forward(ctx, val: torch.Tensor, X: torch.Tensor, row: torch.Tensor, col: torch.Tensor,
                shape):
        A = ops.coo_to_csc(row, col, val, shape)
        ctx.A, ctx.shape = A, (int(shape[0]), int(shape[1]))
        ctx.val_dtype = val.dtype
        ctx.save_for_backward(row, col, X)
        return ops.spmm(A, X)

    @staticmethod
    def backward(ctx, G: torch.Tensor):
        row, col, X = ctx.saved_tensors
        need_v, need_x = ctx.needs_input_grad[0], ctx.needs_input_grad[1]
        G = G.contiguous()  # in its own element type, never narrowed to X's
        if not (need_v or need_x):
            return None, None, None, None, None
        # one adjoint pass gives dX and the dvalues; each triplet then reads its location's
        # dvalue (the dot product only where the location summed to zero)
        dX, dslot = ops.spmm_backward(ctx.A, G, X, need_dX=need_x, need_dval=need_v,
                                      dx_dtype=_grad_dtype(X.dtype), dval_dtype=torch.float64)
        dval = None
        if need_v:
            dval = ops.triplet_grad_csc(row, col, ctx.A, dslot, G, X,
                                        out_dtype=_grad_dtype(ctx.val_dtype))
        return dval, dX, None, None, None


def coo_spmm(row: torch.Tensor, col: torch.Tensor, val: torch.Tensor, X: torch.Tensor,
             shape) -> torch.Tensor:
    """Differentiable Y = assemble(row, col, val) . X (gradients per input triplet)."""
    return CooSpmm.apply(val, X, row, col, shape)
