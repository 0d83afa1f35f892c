"""Torch-facing wrappers of the C ABI: device tensors in, device tensors out.

PyTorch supplies device memory and the current HIP stream; every computation is a libspm.so
kernel.  Functions raise if the library is missing, if no GPU is present, or when the library
reports an error (IndexError for out-of-range triplets, ValueError for bad arguments).
"""
from __future__ import annotations

from dataclasses import dataclass, field

import torch

from . import _lib

_DT = {torch.float64: _lib.F64, torch.float32: _lib.F32, torch.bfloat16: _lib.BF16}


def _dtype_code(t: torch.dtype) -> int:
    if t not in _DT:
        raise ValueError("unsupported element type %s" % t)
    return _DT[t]


def _ptr(t):
    return None if t is None else t.data_ptr()


def _stream(device) -> int:
    return torch.cuda.current_stream(device).cuda_stream


def _require_cuda(*tensors):
    if not torch.cuda.is_available():
        raise RuntimeError("libspm needs a GPU: torch.cuda.is_available() is False")
    for t in tensors:
        if t is not None and not t.is_cuda:
            raise ValueError("expected a device tensor, got one on %s" % t.device)


def _workspace(nbytes: int, device) -> torch.Tensor:
    return torch.empty(max(int(nbytes), 256), dtype=torch.uint8, device=device)


@dataclass
class CSCMatrix:
    """CSC arrays of Section 3.1 on the device.  ``row_idx`` / ``values`` have capacity
    ``nnz_cap``; the first ``nnz`` entries are the matrix."""
    n_rows: int
    n_cols: int
    col_ptr: torch.Tensor
    row_idx_buf: torch.Tensor
    values_buf: torch.Tensor
    info: torch.Tensor
    _nnz: int | None = None
    _plan: torch.Tensor | None = field(default=None, repr=False)

    @property
    def nnz_cap(self) -> int:
        return int(self.row_idx_buf.shape[0])

    @property
    def device(self):
        return self.col_ptr.device

    def sync(self) -> "CSCMatrix":
        """Read the device info words once (the only host synchronisation of assembly)."""
        if self._nnz is None:
            info = self.info.cpu()
            _lib.check(int(info[1]), "spm_coo_to_csc (device)")
            self._nnz = int(info[0])
        return self

    @property
    def nnz(self) -> int:
        return self.sync()._nnz

    @property
    def row_idx(self) -> torch.Tensor:
        return self.row_idx_buf[: self.nnz]

    @property
    def values(self) -> torch.Tensor:
        return self.values_buf[: self.nnz]

    def plan(self) -> torch.Tensor:
        """Row index of the pattern (built once, cached)."""
        if self._plan is None:
            self._plan = build_plan(self)
        return self._plan


def coo_to_csc(row: torch.Tensor, col: torch.Tensor, val: torch.Tensor, shape,
               out_dtype: torch.dtype | None = None, sync: bool = True) -> CSCMatrix:
    """Assemble COO triplets into CSC on the current stream (spm_coo_to_csc)."""
    _require_cuda(row, col, val)
    n_rows, n_cols = int(shape[0]), int(shape[1])
    row = row.contiguous()
    col = col.contiguous()
    val = val.contiguous()
    if row.dtype != torch.int32 or col.dtype != torch.int32:
        raise ValueError("row and col must be int32")
    nnz_in = int(row.numel())
    if col.numel() != nnz_in or val.numel() != nnz_in:
        raise ValueError("row, col and val must have the same length")
    if out_dtype is None:
        out_dtype = torch.float64 if val.dtype == torch.float64 else torch.float32
    lib = _lib.load()
    dev = row.device
    ws_bytes = _lib.ctypes.c_size_t(0)
    _lib.check(lib.spm_coo_to_csc_workspace(n_rows, n_cols, nnz_in, _lib.ctypes.byref(ws_bytes)),
               "spm_coo_to_csc_workspace")
    ws = _workspace(ws_bytes.value, dev)
    col_ptr = torch.empty(n_cols + 1, dtype=torch.int32, device=dev)
    row_idx = torch.empty(max(nnz_in, 1), dtype=torch.int32, device=dev)
    vout = torch.empty(max(nnz_in, 1), dtype=out_dtype, device=dev)
    info = torch.empty(2, dtype=torch.int32, device=dev)
    st = lib.spm_coo_to_csc(n_rows, n_cols, nnz_in, _ptr(row), _ptr(col), _ptr(val),
                            _dtype_code(val.dtype), _ptr(col_ptr), _ptr(row_idx), _ptr(vout),
                            _dtype_code(out_dtype), _ptr(info), _ptr(ws), ws.numel(),
                            _stream(dev))
    _lib.check(st, "spm_coo_to_csc")
    A = CSCMatrix(n_rows, n_cols, col_ptr, row_idx[:nnz_in] if nnz_in else row_idx[:0],
                  vout[:nnz_in] if nnz_in else vout[:0], info)
    A._ws = ws  # keep the workspace alive until the stream has consumed it
    if sync:
        A.sync()
    return A


def coo_to_csc_plan(row: torch.Tensor, col: torch.Tensor, val: torch.Tensor, shape,
                    out_dtype: torch.dtype | None = None, values_plan: bool = True,
                    sync: bool = True):
    """Assembly and plan in one call (spm_coo_to_csc_plan).  Returns (A, values_plan) where
    A carries its plan (A.plan()) and values_plan holds the assembled values in plan order
    (None with values_plan=False); the same results as coo_to_csc + build_plan."""
    _require_cuda(row, col, val)
    n_rows, n_cols = int(shape[0]), int(shape[1])
    row = row.contiguous()
    col = col.contiguous()
    val = val.contiguous()
    if row.dtype != torch.int32 or col.dtype != torch.int32:
        raise ValueError("row and col must be int32")
    nnz_in = int(row.numel())
    if col.numel() != nnz_in or val.numel() != nnz_in:
        raise ValueError("row, col and val must have the same length")
    if out_dtype is None:
        out_dtype = torch.float64 if val.dtype == torch.float64 else torch.float32
    lib = _lib.load()
    dev = row.device
    pb = _lib.ctypes.c_size_t(0)
    wb = _lib.ctypes.c_size_t(0)
    _lib.check(lib.spm_coo_to_csc_plan_size(n_rows, n_cols, nnz_in, _lib.ctypes.byref(pb),
                                            _lib.ctypes.byref(wb)), "spm_coo_to_csc_plan_size")
    ws = _workspace(wb.value, dev)
    plan = torch.empty(max(pb.value, 256), dtype=torch.uint8, device=dev)
    col_ptr = torch.empty(n_cols + 1, dtype=torch.int32, device=dev)
    row_idx = torch.empty(max(nnz_in, 1), dtype=torch.int32, device=dev)
    vout = torch.empty(max(nnz_in, 1), dtype=out_dtype, device=dev)
    vplan = torch.empty(max(nnz_in, 1), dtype=out_dtype, device=dev) if values_plan else None
    info = torch.empty(2, dtype=torch.int32, device=dev)
    plan_info = torch.empty(2, dtype=torch.int32, device=dev)
    st = lib.spm_coo_to_csc_plan(n_rows, n_cols, nnz_in, _ptr(row), _ptr(col), _ptr(val),
                                 _dtype_code(val.dtype), _ptr(col_ptr), _ptr(row_idx),
                                 _ptr(vout), _dtype_code(out_dtype), _ptr(info), _ptr(plan),
                                 plan.numel(), _ptr(vplan), _ptr(plan_info), _ptr(ws),
                                 ws.numel(), _stream(dev))
    _lib.check(st, "spm_coo_to_csc_plan")
    A = CSCMatrix(n_rows, n_cols, col_ptr, row_idx[:nnz_in] if nnz_in else row_idx[:0],
                  vout[:nnz_in] if nnz_in else vout[:0], info)
    A._ws = ws
    A._plan = plan
    A.plan_info = plan_info
    if sync:
        A.sync()
        _lib.check(int(plan_info.cpu()[1]), "spm_coo_to_csc_plan (device)")
    if vplan is not None:
        vplan = vplan[:nnz_in] if nnz_in else vplan[:0]
    return A, vplan


def csc_insert(A: CSCMatrix, row: torch.Tensor, col: torch.Tensor, val: torch.Tensor,
               out_dtype: torch.dtype | None = None, sync: bool = True) -> CSCMatrix:
    """Batch insertion of triplets into A (spm_csc_insert): a new CSC in which every location
    holds A's value (if any) plus the new values in input order, zero sums dropped.  `val`
    must have A's value type (float32 or float64)."""
    _require_cuda(row, col, val, A.col_ptr)
    row = row.contiguous()
    col = col.contiguous()
    val = val.contiguous()
    if row.dtype != torch.int32 or col.dtype != torch.int32:
        raise ValueError("row and col must be int32")
    if val.dtype != A.values_buf.dtype:
        raise ValueError("new values must have the matrix's value type %s" % A.values_buf.dtype)
    nnz_t = int(row.numel())
    if col.numel() != nnz_t or val.numel() != nnz_t:
        raise ValueError("row, col and val must have the same length")
    if out_dtype is None:
        out_dtype = A.values_buf.dtype
    lib = _lib.load()
    dev = row.device
    cap_a = A.nnz_cap
    wb = _lib.ctypes.c_size_t(0)
    _lib.check(lib.spm_csc_insert_workspace(A.n_rows, A.n_cols, cap_a, nnz_t,
                                            _lib.ctypes.byref(wb)), "spm_csc_insert_workspace")
    ws = _workspace(wb.value, dev)
    cap = cap_a + nnz_t
    col_ptr = torch.empty(A.n_cols + 1, dtype=torch.int32, device=dev)
    row_idx = torch.empty(max(cap, 1), dtype=torch.int32, device=dev)
    vout = torch.empty(max(cap, 1), dtype=out_dtype, device=dev)
    info = torch.empty(2, dtype=torch.int32, device=dev)
    st = lib.spm_csc_insert(A.n_rows, A.n_cols, cap_a, _ptr(A.col_ptr),
                            _ptr(A.row_idx_buf) if cap_a else None,
                            _ptr(A.values_buf) if cap_a else None, nnz_t, _ptr(row), _ptr(col),
                            _ptr(val), _dtype_code(val.dtype), _ptr(col_ptr), _ptr(row_idx),
                            _ptr(vout), _dtype_code(out_dtype), _ptr(info), _ptr(ws),
                            ws.numel(), _stream(dev))
    _lib.check(st, "spm_csc_insert")
    B = CSCMatrix(A.n_rows, A.n_cols, col_ptr, row_idx[:cap] if cap else row_idx[:0],
                  vout[:cap] if cap else vout[:0], info)
    B._ws = ws
    if sync:
        B.sync()
    return B


def csc_add(A: CSCMatrix, B: CSCMatrix, out_dtype: torch.dtype | None = None,
            sync: bool = True) -> CSCMatrix:
    """A + B (spm_csc_add): B's stored elements inserted into A, a shared location holding A's
    value plus B's, zero sums dropped.  A and B share one shape and value type."""
    _require_cuda(A.col_ptr, B.col_ptr)
    if (A.n_rows, A.n_cols) != (B.n_rows, B.n_cols):
        raise ValueError("A is %dx%d, B is %dx%d" % (A.n_rows, A.n_cols, B.n_rows, B.n_cols))
    if A.values_buf.dtype != B.values_buf.dtype:
        raise ValueError("A and B must share one value type")
    if out_dtype is None:
        out_dtype = A.values_buf.dtype
    lib = _lib.load()
    dev = A.device
    ca, cb = A.nnz_cap, B.nnz_cap
    wb = _lib.ctypes.c_size_t(0)
    _lib.check(lib.spm_csc_add_workspace(A.n_rows, A.n_cols, ca, cb, _lib.ctypes.byref(wb)),
               "spm_csc_add_workspace")
    ws = _workspace(wb.value, dev)
    cap = ca + cb
    col_ptr = torch.empty(A.n_cols + 1, dtype=torch.int32, device=dev)
    row_idx = torch.empty(max(cap, 1), dtype=torch.int32, device=dev)
    vout = torch.empty(max(cap, 1), dtype=out_dtype, device=dev)
    info = torch.empty(2, dtype=torch.int32, device=dev)
    st = lib.spm_csc_add(A.n_rows, A.n_cols, ca, _ptr(A.col_ptr),
                         _ptr(A.row_idx_buf) if ca else None, _ptr(A.values_buf) if ca else None,
                         cb, _ptr(B.col_ptr), _ptr(B.row_idx_buf) if cb else None,
                         _ptr(B.values_buf) if cb else None, _dtype_code(A.values_buf.dtype),
                         _ptr(col_ptr), _ptr(row_idx), _ptr(vout), _dtype_code(out_dtype),
                         _ptr(info), _ptr(ws), ws.numel(), _stream(dev))
    _lib.check(st, "spm_csc_add")
    C = CSCMatrix(A.n_rows, A.n_cols, col_ptr, row_idx[:cap] if cap else row_idx[:0],
                  vout[:cap] if cap else vout[:0], info)
    C._ws = ws
    if sync:
        h = info.cpu()
        _lib.check(int(h[1]), "spm_csc_add (device)")
        C._nnz = int(h[0])
    return C


def csc_transpose(A: CSCMatrix, sync: bool = True) -> CSCMatrix:
    """A^T as a CSC (spm_csc_transpose; X.t() of Table 1)."""
    _require_cuda(A.col_ptr)
    lib = _lib.load()
    dev = A.device
    cap = A.nnz_cap
    wb = _lib.ctypes.c_size_t(0)
    _lib.check(lib.spm_csc_transpose_workspace(A.n_rows, A.n_cols, cap, _lib.ctypes.byref(wb)),
               "spm_csc_transpose_workspace")
    ws = _workspace(wb.value, dev)
    t_cp = torch.empty(A.n_rows + 1, dtype=torch.int32, device=dev)
    t_ri = torch.empty(max(cap, 1), dtype=torch.int32, device=dev)
    t_v = torch.empty(max(cap, 1), dtype=A.values_buf.dtype, device=dev)
    info = torch.empty(2, dtype=torch.int32, device=dev)
    st = lib.spm_csc_transpose(A.n_rows, A.n_cols, cap, _ptr(A.col_ptr),
                               _ptr(A.row_idx_buf) if cap else None,
                               _ptr(A.values_buf) if cap else None,
                               _dtype_code(A.values_buf.dtype), _ptr(t_cp), _ptr(t_ri),
                               _ptr(t_v), _ptr(info), _ptr(ws), ws.numel(), _stream(dev))
    _lib.check(st, "spm_csc_transpose")
    T = CSCMatrix(A.n_cols, A.n_rows, t_cp, t_ri[:cap] if cap else t_ri[:0],
                  t_v[:cap] if cap else t_v[:0], info)
    T._ws = ws
    if sync:
        h = info.cpu()
        _lib.check(int(h[1]), "spm_csc_transpose (device)")
        T._nnz = int(h[0])
    return T


def trace_atb(A: CSCMatrix, B: CSCMatrix, sync: bool = True):
    """trace(A^T B) without forming A^T or the product (spm_csc_trace_atb; Section 2, Table 1).
    With sync, returns (trace as a Python float, number of locations stored in both); without,
    the device tensors (out float64[1], info int32[2]) with the call only enqueued."""
    _require_cuda(A.col_ptr, B.col_ptr)
    if (A.n_rows, A.n_cols) != (B.n_rows, B.n_cols):
        raise ValueError("A is %dx%d, B is %dx%d" % (A.n_rows, A.n_cols, B.n_rows, B.n_cols))
    if A.values_buf.dtype != B.values_buf.dtype:
        raise ValueError("A and B must share one value type")
    lib = _lib.load()
    dev = A.device
    wb = _lib.ctypes.c_size_t(0)
    _lib.check(lib.spm_csc_trace_atb_workspace(A.n_cols, _lib.ctypes.byref(wb)),
               "spm_csc_trace_atb_workspace")
    ws = _workspace(wb.value, dev)
    out = torch.empty(1, dtype=torch.float64, device=dev)
    info = torch.empty(2, dtype=torch.int32, device=dev)
    ca, cb = A.nnz_cap, B.nnz_cap
    st = lib.spm_csc_trace_atb(A.n_rows, A.n_cols, ca, _ptr(A.col_ptr),
                               _ptr(A.row_idx_buf) if ca else None,
                               _ptr(A.values_buf) if ca else None, cb, _ptr(B.col_ptr),
                               _ptr(B.row_idx_buf) if cb else None,
                               _ptr(B.values_buf) if cb else None,
                               _dtype_code(A.values_buf.dtype), _ptr(out), _ptr(info), _ptr(ws),
                               ws.numel(), _stream(dev))
    _lib.check(st, "spm_csc_trace_atb")
    if not sync:
        out._ws = ws
        return out, info
    h = info.cpu()
    _lib.check(int(h[1]), "spm_csc_trace_atb (device)")
    return float(out.item()), int(h[0])


def triplet_grad(row: torch.Tensor, col: torch.Tensor, G: torch.Tensor, X: torch.Tensor, shape,
                 val_dtype: torch.dtype = torch.float32,
                 out_dtype: torch.dtype | None = None) -> torch.Tensor:
    """dL/dv_t = G[row_t, :] . X[col_t, :] for every input triplet of an assembly followed by
    Y = A.X (spm_coo_triplet_grad): duplicates share it, a location that summed to zero still
    has it, a triplet outside the matrix gets 0.  `val_dtype` is the assembled values' type
    (it picks the accumulation, as for the adjoint)."""
    n_rows, n_cols = int(shape[0]), int(shape[1])
    G2 = G.reshape(-1, 1) if G.dim() == 1 else G
    X2 = X.reshape(-1, 1) if X.dim() == 1 else X
    _require_cuda(row, col, G2, X2)
    if G2.shape[0] != n_rows or X2.shape[0] != n_cols or G2.shape[1] != X2.shape[1]:
        raise ValueError("G %s and X %s do not fit a %dx%d matrix" % (tuple(G2.shape),
                         tuple(X2.shape), n_rows, n_cols))
    if G2.stride(1) != 1:
        G2 = G2.contiguous()
    if X2.stride(1) != 1:
        X2 = X2.contiguous()
    if row.dtype != torch.int32 or col.dtype != torch.int32:
        raise ValueError("row and col must be int32")
    n = int(row.shape[0])
    if out_dtype is None:
        out_dtype = val_dtype if val_dtype in (torch.float32, torch.float64) else torch.float32
    dv = torch.empty(max(n, 1), dtype=out_dtype, device=row.device)
    lib = _lib.load()
    st = lib.spm_coo_triplet_grad(n_rows, n_cols, n, int(X2.shape[1]), _ptr(row), _ptr(col),
                                  _dtype_code(val_dtype), _ptr(G2), G2.stride(0),
                                  _dtype_code(G2.dtype), _ptr(X2), X2.stride(0),
                                  _dtype_code(X2.dtype), _ptr(dv),
                                  _dtype_code(out_dtype), _stream(row.device))
    _lib.check(st, "spm_coo_triplet_grad")
    return dv[:n]


def triplet_grad_csc(row: torch.Tensor, col: torch.Tensor, A: CSCMatrix, dval: torch.Tensor,
                     G: torch.Tensor, X: torch.Tensor,
                     out_dtype: torch.dtype | None = None) -> torch.Tensor:
    """The gradient per input triplet read from the adjoint's dvalues `dval` of the CSC `A`
    assembled from these triplets (spm_coo_triplet_grad_csc): dv[t] = dval[slot of t], the dot
    product only where the location was dropped."""
    G2 = G.reshape(-1, 1) if G.dim() == 1 else G
    X2 = X.reshape(-1, 1) if X.dim() == 1 else X
    _require_cuda(row, col, A.col_ptr, dval, G2, X2)
    if G2.shape[0] != A.n_rows or X2.shape[0] != A.n_cols or G2.shape[1] != X2.shape[1]:
        raise ValueError("G %s and X %s do not fit a %dx%d matrix" % (tuple(G2.shape),
                         tuple(X2.shape), A.n_rows, A.n_cols))
    if G2.stride(1) != 1:
        G2 = G2.contiguous()
    if X2.stride(1) != 1:
        X2 = X2.contiguous()
    if row.dtype != torch.int32 or col.dtype != torch.int32:
        raise ValueError("row and col must be int32")
    n = int(row.shape[0])
    cap = A.nnz_cap
    if out_dtype is None:
        out_dtype = dval.dtype
    dv = torch.empty(max(n, 1), dtype=out_dtype, device=row.device)
    lib = _lib.load()
    st = lib.spm_coo_triplet_grad_csc(A.n_rows, A.n_cols, n, int(X2.shape[1]), _ptr(row),
                                      _ptr(col), cap, _ptr(A.col_ptr),
                                      _ptr(A.row_idx_buf) if cap else None,
                                      _ptr(dval) if cap else None, _dtype_code(dval.dtype),
                                      _dtype_code(A.values_buf.dtype), _ptr(G2), G2.stride(0),
                                      _dtype_code(G2.dtype), _ptr(X2), X2.stride(0),
                                      _dtype_code(X2.dtype), _ptr(dv),
                                      _dtype_code(out_dtype), _stream(row.device))
    _lib.check(st, "spm_coo_triplet_grad_csc")
    return dv[:n]


def rowvec_spmm(V: torch.Tensor, A: CSCMatrix, out_dtype: torch.dtype | None = None):
    """W = V.A for row vectors V (n_rows, or m x n_rows for m of them): the product of Section
    3's use case (iv) written as in Fig. 1.  It is the column walk of the adjoint with the
    vectors as its upstream operand (spm_csc_spmm_backward, dX only), so W[i] sums column i of
    A in increasing row order."""
    V2 = V.reshape(1, -1) if V.dim() == 1 else V
    Vt = V2.t().contiguous()  # n_rows x m
    X_dummy = torch.zeros(A.n_cols, Vt.shape[1], dtype=Vt.dtype, device=Vt.device)
    dX, _ = spmm_backward(A, Vt, X_dummy, need_dval=False, dx_dtype=out_dtype)
    W = dX.t()
    return W.reshape(-1) if V.dim() == 1 else W


def plan_size(n_rows: int, n_cols: int, nnz_cap: int):
    lib = _lib.load()
    pb = _lib.ctypes.c_size_t(0)
    wb = _lib.ctypes.c_size_t(0)
    _lib.check(lib.spm_csc_plan_size(n_rows, n_cols, nnz_cap, _lib.ctypes.byref(pb),
                                     _lib.ctypes.byref(wb)), "spm_csc_plan_size")
    return pb.value, wb.value


def build_plan(A: CSCMatrix, check: bool = True, values: torch.Tensor | None = None,
               values_plan: torch.Tensor | None = None) -> torch.Tensor:
    """Row index of A's pattern (spm_csc_plan_build), as a uint8 device buffer.  With
    `values` (CSC order) and `values_plan` (same type and capacity), the values are also
    written in plan order (for spmm(..., order="plan"))."""
    _require_cuda(A.col_ptr)
    if (values is None) != (values_plan is None):
        raise ValueError("values and values_plan go together")
    if values is not None and values.dtype != values_plan.dtype:
        raise ValueError("values and values_plan must share one element type")
    lib = _lib.load()
    cap = A.nnz_cap
    pb, wb = plan_size(A.n_rows, A.n_cols, cap)
    plan = torch.empty(max(pb, 256), dtype=torch.uint8, device=A.device)
    ws = _workspace(wb, A.device)
    info = torch.empty(2, dtype=torch.int32, device=A.device)
    vt = _dtype_code(values.dtype) if values is not None else _lib.F32
    st = lib.spm_csc_plan_build(A.n_rows, A.n_cols, cap, _ptr(A.col_ptr),
                                _ptr(A.row_idx_buf) if cap else None, _ptr(values), vt,
                                _ptr(plan), plan.numel(), _ptr(values_plan), _ptr(info),
                                _ptr(ws), ws.numel(), _stream(A.device))
    _lib.check(st, "spm_csc_plan_build")
    plan._ws = ws
    if check:
        h = info.cpu()
        _lib.check(int(h[1]), "spm_csc_plan_build (device)")
    return plan


def plan_arrays(plan: torch.Tensor, n_rows: int, nnz_cap: int):
    """(row_ptr, col_t, perm) int32 views of a plan buffer (layout of include/spm.h)."""
    def a256(x):
        return (x + 255) & ~255
    rp_bytes = a256(4 * (n_rows + 1))
    ct_bytes = a256(4 * nnz_cap)
    row_ptr = plan[:4 * (n_rows + 1)].view(torch.int32)
    col_t = plan[rp_bytes:rp_bytes + 4 * nnz_cap].view(torch.int32)
    perm = plan[rp_bytes + ct_bytes:rp_bytes + ct_bytes + 4 * nnz_cap].view(torch.int32)
    return row_ptr, col_t, perm


def _out_type(vt: torch.dtype, xt: torch.dtype) -> torch.dtype:
    return torch.float64 if torch.float64 in (vt, xt) else torch.float32


def spmm(A: CSCMatrix, X: torch.Tensor, values: torch.Tensor | None = None,
         out_dtype: torch.dtype | None = None, plan: torch.Tensor | None = None,
         out: torch.Tensor | None = None, order: str = "csc") -> torch.Tensor:
    """Y = A.X (spm_csc_spmm).  X is n_cols x k (or a vector of length n_cols).  `order`
    says whether `values` are in CSC order ("csc") or plan order ("plan", from
    build_plan(..., values_plan=...))."""
    if order not in ("csc", "plan"):
        raise ValueError("order must be 'csc' or 'plan'")
    if order == "plan" and values is None:
        raise ValueError("plan-order values must be passed explicitly")
    vec = X.dim() == 1
    X2 = X.reshape(-1, 1) if vec else X
    _require_cuda(X2, A.col_ptr)
    if X2.shape[0] != A.n_cols:
        raise ValueError("X has %d rows, A has %d columns" % (X2.shape[0], A.n_cols))
    if X2.stride(1) != 1:
        X2 = X2.contiguous()
    v = A.values_buf if values is None else values
    k = int(X2.shape[1])
    if out_dtype is None:
        out_dtype = _out_type(v.dtype, X2.dtype)
    if plan is None:
        plan = A.plan()
    Y = out if out is not None else torch.empty(A.n_rows, k, dtype=out_dtype, device=X2.device)
    lib = _lib.load()
    st = lib.spm_csc_spmm(A.n_rows, A.n_cols, A.nnz_cap, k, _ptr(plan), _ptr(v),
                          _dtype_code(v.dtype),
                          _lib.ORDER_PLAN if order == "plan" else _lib.ORDER_CSC, _ptr(X2),
                          X2.stride(0), _dtype_code(X2.dtype), _ptr(Y), Y.stride(0),
                          _dtype_code(Y.dtype), _stream(X2.device))
    _lib.check(st, "spm_csc_spmm")
    return Y.reshape(-1) if vec else Y


def spmm_backward(A: CSCMatrix, G: torch.Tensor, X: torch.Tensor,
                  values: torch.Tensor | None = None, need_dX: bool = True,
                  need_dval: bool = True, dx_dtype: torch.dtype | None = None,
                  dval_dtype: torch.dtype | None = None):
    """(dX, dval) of Y = A.X for dL/dY = G (spm_csc_spmm_backward); None where not needed.
    G and X keep their own element types (G usually arrives in Y's type)."""
    vec = X.dim() == 1
    X2 = X.reshape(-1, 1) if vec else X
    G2 = G.reshape(-1, 1) if G.dim() == 1 else G
    _require_cuda(X2, G2, A.col_ptr)
    if X2.stride(1) != 1:
        X2 = X2.contiguous()
    if G2.stride(1) != 1:
        G2 = G2.contiguous()
    v = A.values_buf if values is None else values
    k = int(X2.shape[1])
    if G2.shape != (A.n_rows, k) or X2.shape[0] != A.n_cols:
        raise ValueError("shape mismatch: G %s, X %s, A %dx%d" % (tuple(G2.shape),
                         tuple(X2.shape), A.n_rows, A.n_cols))
    if dx_dtype is None:
        dx_dtype = X2.dtype if X2.dtype != torch.bfloat16 else torch.float32
    if dval_dtype is None:
        dval_dtype = v.dtype
    dev = X2.device
    dX = torch.empty(A.n_cols, k, dtype=dx_dtype, device=dev) if need_dX else None
    dval = torch.empty(max(A.nnz_cap, 1), dtype=dval_dtype, device=dev) if need_dval else None
    lib = _lib.load()
    st = lib.spm_csc_spmm_backward(A.n_rows, A.n_cols, A.nnz_cap, k, _ptr(A.col_ptr),
                                   _ptr(A.row_idx_buf) if A.nnz_cap else None,
                                   _ptr(v) if A.nnz_cap else None, _dtype_code(v.dtype),
                                   _ptr(G2), G2.stride(0), _dtype_code(G2.dtype), _ptr(X2),
                                   X2.stride(0), _dtype_code(X2.dtype), _ptr(dX),
                                   dX.stride(0) if dX is not None else k,
                                   _dtype_code(dx_dtype), _ptr(dval), _dtype_code(dval_dtype),
                                   _stream(dev))
    _lib.check(st, "spm_csc_spmm_backward")
    if dval is not None:
        dval = dval[: A.nnz]
    if vec and dX is not None:
        dX = dX.reshape(-1)
    return dX, dval
