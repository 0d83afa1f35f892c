"""A preallocated assemble -> plan -> forward -> adjoint pipeline over the C ABI.

All buffers (outputs, plan, workspaces) are allocated once for a given problem size, so a
step enqueues only library calls on one stream, with no allocation and no host
synchronisation: spm_coo_to_csc_plan (assembly and plan in one call; with fused=False
spm_coo_to_csc then spm_csc_plan_build), spm_csc_spmm, spm_csc_spmm_backward.
The CSC capacity is nnz_in; kernels read the true nnz from col_ptr[n_cols] on the device.
The plan build also writes the assembled values in plan order (they are fixed for the step),
so the forward product reads them contiguously (SPM_ORDER_PLAN).
"""
from __future__ import annotations

import ctypes

import torch

from . import _lib
from .ops import CSCMatrix, _DT, plan_size

PHASES = ("assemble", "plan", "forward", "backward")
FUSED_PHASES = ("assemble_plan", "forward", "backward")


class Pipeline:
    def __init__(self, n_rows: int, n_cols: int, nnz_in: int, k: int,
                 val_dtype=torch.float32, x_dtype=torch.float32, csc_dtype=None,
                 device="cuda:0", fused=True):
        self.lib = _lib.load()
        self.fused = fused
        self.phases = FUSED_PHASES if fused else PHASES
        self.n_rows, self.n_cols, self.nnz_in, self.k = n_rows, n_cols, nnz_in, k
        self.device = torch.device(device)
        self.val_dtype, self.x_dtype = val_dtype, x_dtype
        self.csc_dtype = csc_dtype or (torch.float64 if val_dtype == torch.float64
                                       else torch.float32)
        self.y_dtype = torch.float64 if torch.float64 in (self.csc_dtype, x_dtype) \
            else torch.float32
        self.dx_dtype = x_dtype if x_dtype != torch.bfloat16 else torch.float32
        d = self.device
        if not fused:
            ws = ctypes.c_size_t(0)
            _lib.check(self.lib.spm_coo_to_csc_workspace(n_rows, n_cols, nnz_in,
                                                         ctypes.byref(ws)),
                       "spm_coo_to_csc_workspace")
            self.asm_ws = torch.empty(max(ws.value, 256), dtype=torch.uint8, device=d)
        cap = max(nnz_in, 1)
        self.col_ptr = torch.empty(n_cols + 1, dtype=torch.int32, device=d)
        self.row_idx = torch.empty(cap, dtype=torch.int32, device=d)
        self.values = torch.empty(cap, dtype=self.csc_dtype, device=d)
        self.info = torch.zeros(2, dtype=torch.int32, device=d)
        if fused:
            pb_, wb_ = ctypes.c_size_t(0), ctypes.c_size_t(0)
            _lib.check(self.lib.spm_coo_to_csc_plan_size(n_rows, n_cols, nnz_in,
                                                         ctypes.byref(pb_), ctypes.byref(wb_)),
                       "spm_coo_to_csc_plan_size")
            pb, wb = pb_.value, wb_.value
            self.asm_ws = torch.empty(max(wb, 256), dtype=torch.uint8, device=d)
            self.plan_ws = self.asm_ws
        else:
            pb, wb = plan_size(n_rows, n_cols, nnz_in)
            self.plan_ws = torch.empty(max(wb, 256), dtype=torch.uint8, device=d)
        self.plan = torch.empty(max(pb, 256), dtype=torch.uint8, device=d)
        self.plan_info = torch.zeros(2, dtype=torch.int32, device=d)
        self.values_plan = torch.empty(cap, dtype=self.csc_dtype, device=d)
        self.Y = torch.empty(n_rows, k, dtype=self.y_dtype, device=d)
        self.dX = torch.empty(n_cols, k, dtype=self.dx_dtype, device=d)
        self.dval = torch.empty(cap, dtype=self.csc_dtype, device=d)

    def step(self, row, col, val, X, G, stream=None, events=None):
        """Enqueue the calls of one step.  `events`, if given, is a list of
        len(self.phases) + 1 HIP events recorded between the phases on the same stream."""
        lib = self.lib
        s = stream if stream is not None else torch.cuda.current_stream(self.device)
        h = s.cuda_stream
        n_rows, n_cols, nnz, k = self.n_rows, self.n_cols, self.nnz_in, self.k
        if events is not None:
            events[0].record(s)
        self._assemble_plan(row, col, val, h, s, events)
        if events is not None:
            events[-3].record(s)
        _lib.check(lib.spm_csc_spmm(n_rows, n_cols, nnz, k, self.plan.data_ptr(),
                                    self.values_plan.data_ptr(), _DT[self.csc_dtype],
                                    _lib.ORDER_PLAN, X.data_ptr(), X.stride(0), _DT[X.dtype],
                                    self.Y.data_ptr(), self.Y.stride(0), _DT[self.y_dtype], h),
                   "spm_csc_spmm")
        if events is not None:
            events[-2].record(s)
        _lib.check(lib.spm_csc_spmm_backward(n_rows, n_cols, nnz, k, self.col_ptr.data_ptr(),
                                             self.row_idx.data_ptr(), self.values.data_ptr(),
                                             _DT[self.csc_dtype], G.data_ptr(), G.stride(0),
                                             _DT[G.dtype], X.data_ptr(), X.stride(0),
                                             _DT[X.dtype],
                                             self.dX.data_ptr(), self.dX.stride(0),
                                             _DT[self.dx_dtype], self.dval.data_ptr(),
                                             _DT[self.csc_dtype], h), "spm_csc_spmm_backward")
        if events is not None:
            events[-1].record(s)

    def _assemble_plan(self, row, col, val, h, s, events=None):
        lib = self.lib
        n_rows, n_cols, nnz = self.n_rows, self.n_cols, self.nnz_in
        if self.fused:
            _lib.check(lib.spm_coo_to_csc_plan(
                n_rows, n_cols, nnz, row.data_ptr(), col.data_ptr(), val.data_ptr(),
                _DT[val.dtype], self.col_ptr.data_ptr(), self.row_idx.data_ptr(),
                self.values.data_ptr(), _DT[self.csc_dtype], self.info.data_ptr(),
                self.plan.data_ptr(), self.plan.numel(), self.values_plan.data_ptr(),
                self.plan_info.data_ptr(), self.asm_ws.data_ptr(), self.asm_ws.numel(), h),
                "spm_coo_to_csc_plan")
            return
        _lib.check(lib.spm_coo_to_csc(n_rows, n_cols, nnz, row.data_ptr(), col.data_ptr(),
                                      val.data_ptr(), _DT[val.dtype], self.col_ptr.data_ptr(),
                                      self.row_idx.data_ptr(), self.values.data_ptr(),
                                      _DT[self.csc_dtype], self.info.data_ptr(),
                                      self.asm_ws.data_ptr(), self.asm_ws.numel(), h),
                   "spm_coo_to_csc")
        if events is not None:
            events[1].record(s)
        _lib.check(lib.spm_csc_plan_build(n_rows, n_cols, nnz, self.col_ptr.data_ptr(),
                                          self.row_idx.data_ptr(), self.values.data_ptr(),
                                          _DT[self.csc_dtype], self.plan.data_ptr(),
                                          self.plan.numel(), self.values_plan.data_ptr(),
                                          self.plan_info.data_ptr(), self.plan_ws.data_ptr(),
                                          self.plan_ws.numel(), h),
                   "spm_csc_plan_build")

    def step_assemble_plan(self, row, col, val, stream=None):
        """Only assembly and plan."""
        s = stream if stream is not None else torch.cuda.current_stream(self.device)
        self._assemble_plan(row, col, val, s.cuda_stream, s)

    def step_spmm(self, X, G, stream=None):
        """Only the products (forward and adjoint) on the current CSC and plan."""
        s = stream if stream is not None else torch.cuda.current_stream(self.device)
        h = s.cuda_stream
        lib = self.lib
        n_rows, n_cols, nnz, k = self.n_rows, self.n_cols, self.nnz_in, self.k
        _lib.check(lib.spm_csc_spmm(n_rows, n_cols, nnz, k, self.plan.data_ptr(),
                                    self.values_plan.data_ptr(), _DT[self.csc_dtype],
                                    _lib.ORDER_PLAN, X.data_ptr(), X.stride(0), _DT[X.dtype],
                                    self.Y.data_ptr(), self.Y.stride(0), _DT[self.y_dtype], h),
                   "spm_csc_spmm")
        _lib.check(lib.spm_csc_spmm_backward(n_rows, n_cols, nnz, k, self.col_ptr.data_ptr(),
                                             self.row_idx.data_ptr(), self.values.data_ptr(),
                                             _DT[self.csc_dtype], G.data_ptr(), G.stride(0),
                                             _DT[G.dtype], X.data_ptr(), X.stride(0),
                                             _DT[X.dtype],
                                             self.dX.data_ptr(), self.dX.stride(0),
                                             _DT[self.dx_dtype], self.dval.data_ptr(),
                                             _DT[self.csc_dtype], h), "spm_csc_spmm_backward")

    def capture(self, row, col, val, X, G, warmup: int = 1):
        """Record one step into a HIP graph (torch.cuda.CUDAGraph) over these tensors, so that
        graph.replay() submits the step's kernels at once.  The step holds no host
        synchronisation, allocation or memset, so it captures as it runs.  The tensors'
        addresses are part of the graph: to change the data, refill the same tensors."""
        dev = self.device
        s = torch.cuda.Stream(dev)
        s.wait_stream(torch.cuda.current_stream(dev))
        with torch.cuda.stream(s):
            for _ in range(warmup):
                self.step(row, col, val, X, G, stream=s)
        torch.cuda.current_stream(dev).wait_stream(s)
        g = torch.cuda.CUDAGraph()
        with torch.cuda.graph(g, stream=s):
            self.step(row, col, val, X, G, stream=s)
        torch.cuda.synchronize(dev)
        return g

    def status(self):
        """(nnz_out, assembly status, plan status) -- synchronises."""
        a = self.info.cpu()
        b = self.plan_info.cpu()
        return int(a[0]), int(a[1]), int(b[1])

    def csc(self) -> CSCMatrix:
        A = CSCMatrix(self.n_rows, self.n_cols, self.col_ptr, self.row_idx[: self.nnz_in],
                      self.values[: self.nnz_in], self.info)
        A._plan = self.plan
        return A.sync()

