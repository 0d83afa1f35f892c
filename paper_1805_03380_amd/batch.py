"""Batched assembly + SpMM over the C ABI: many independent matrices packed into flat device
arrays, run either by the batched entry point (spm_batch_run: a grouping launch, then the
product launches) or as per-matrix calls of the four
single-matrix entry points (for comparison; same kernels' device functions, bitwise-equal
results)."""
from __future__ import annotations

import ctypes

import numpy as np
import torch

from . import _lib
from .ops import _DT, plan_size, plan_arrays


def _off(counts):
    o = np.zeros(len(counts) + 1, dtype=np.int64)
    np.cumsum(counts, out=o[1:])
    return o


class PackedBatch:
    """Host problems (synth.COOProblem with n_rows x n_cols, X n_cols x k, G n_rows x k) packed
    into device arrays, plus preallocated outputs for both execution modes."""

    def __init__(self, problems, val_dtype=torch.float32, x_dtype=torch.float32,
                 device="cuda:0", workers: int = 0):
        self.lib = _lib.load()
        self.device = torch.device(device)
        self.B = len(problems)
        self.k = int(problems[0].X.shape[1])
        self.val_dtype, self.x_dtype = val_dtype, x_dtype
        n_r = np.array([p.n_rows for p in problems], np.int64)
        n_c = np.array([p.n_cols for p in problems], np.int64)
        nnz = np.array([p.nnz_in for p in problems], np.int64)
        k = self.k
        self.n_r, self.n_c, self.nnz = n_r, n_c, nnz
        self.trip_off = _off(nnz)
        self.colptr_off = _off(n_c + 1)
        self.rowptr_off = _off(n_r + 1)
        self.x_off = _off(n_c * k)
        self.g_off = _off(n_r * k)
        items = (_lib.BatchItem * self.B)()
        for b in range(self.B):
            it = items[b]
            it.n_rows, it.n_cols, it.nnz_in, it.reserved = int(n_r[b]), int(n_c[b]), int(nnz[b]), 0
            it.trip_off = int(self.trip_off[b])
            it.colptr_off = int(self.colptr_off[b])
            it.rowptr_off = int(self.rowptr_off[b])
            it.x_off = int(self.x_off[b])
            it.g_off = int(self.g_off[b])
        self.items_host = items
        order = (ctypes.c_int32 * self.B)()
        _lib.check(self.lib.spm_batch_schedule(ctypes.byref(items), self.B, k, order),
                   "spm_batch_schedule")
        self.order_host = np.frombuffer(order, dtype=np.int32).copy()
        d = self.device
        raw = bytes(items)
        self.items = torch.frombuffer(bytearray(raw), dtype=torch.uint8).to(d)
        self.order = torch.from_numpy(self.order_host).to(d)

        def cat(arrs, dt):
            return torch.from_numpy(np.ascontiguousarray(np.concatenate(arrs))).to(d).to(dt)

        self.row = cat([p.row for p in problems], torch.int32)
        self.col = cat([p.col for p in problems], torch.int32)
        self.val = cat([p.val.astype(np.float32) for p in problems], torch.float32).to(val_dtype)
        self.X = cat([p.X.reshape(-1).astype(np.float32) for p in problems],
                     torch.float32).to(x_dtype)
        self.G = cat([p.G.reshape(-1).astype(np.float32) for p in problems],
                     torch.float32).to(x_dtype)
        self.max_dim = int(max(n_r.max(), n_c.max())) if self.B else 0
        self.max_nnz = int(nnz.max()) if self.B else 0
        self.workers = workers
        ws = ctypes.c_size_t(0)
        _lib.check(self.lib.spm_batch_workspace(self.max_dim, self.max_nnz, workers,
                                                ctypes.byref(ws)), "spm_batch_workspace")
        self.ws = torch.empty(ws.value, dtype=torch.uint8, device=d)
        self.out = self._outputs()
        # per-matrix mode: workspaces at the largest sizes, reused call after call
        aws = ctypes.c_size_t(0)
        _lib.check(self.lib.spm_coo_to_csc_workspace(self.max_dim, self.max_dim, self.max_nnz,
                                                     ctypes.byref(aws)), "workspace")
        self.asm_ws = torch.empty(max(aws.value, 256), dtype=torch.uint8, device=d)
        pb, wb = plan_size(self.max_dim, self.max_dim, self.max_nnz)
        self.plan = torch.empty(max(pb, 256), dtype=torch.uint8, device=d)
        self.plan_ws = torch.empty(max(wb, 256), dtype=torch.uint8, device=d)
        self.plan_info = torch.zeros(2, dtype=torch.int32, device=d)

    def _outputs(self):
        d = self.device
        T = int(self.trip_off[-1])
        return dict(
            col_ptr=torch.zeros(int(self.colptr_off[-1]), dtype=torch.int32, device=d),
            row_idx=torch.zeros(max(T, 1), dtype=torch.int32, device=d),
            val_out=torch.zeros(max(T, 1), dtype=torch.float32, device=d),
            row_ptr=torch.zeros(int(self.rowptr_off[-1]), dtype=torch.int32, device=d),
            col_t=torch.zeros(max(T, 1), dtype=torch.int32, device=d),
            perm=torch.zeros(max(T, 1), dtype=torch.int32, device=d),
            Y=torch.zeros(max(int(self.g_off[-1]), 1), dtype=torch.float32, device=d),
            dX=torch.zeros(max(int(self.x_off[-1]), 1), dtype=torch.float32, device=d),
            dval=torch.zeros(max(T, 1), dtype=torch.float32, device=d),
            info=torch.zeros(2 * max(self.B, 1), dtype=torch.int32, device=d))

    def new_outputs(self):
        return self._outputs()

    def _ensure_workspace(self):
        """The workspace grows with the number of persistent workgroups (a tuning value)."""
        ws = ctypes.c_size_t(0)
        _lib.check(self.lib.spm_batch_workspace(self.max_dim, self.max_nnz, self.workers,
                                                ctypes.byref(ws)), "spm_batch_workspace")
        if ws.value > self.ws.numel():
            self.ws = torch.empty(ws.value, dtype=torch.uint8, device=self.device)

    def run_batched(self, out=None, stream=None, tune_key: str | None = None):
        """All matrices: the grouping launch, then the product launches (spm_batch_run; with a
        named tuning, spm_batch_coo_to_csc_spmm with that key for this call)."""
        if tune_key is not None:  # the workspace follows the tuning the call will run with
            _lib.select_tuning(tune_key)
            try:
                self._ensure_workspace()
            finally:
                _lib.select_tuning(None)
        else:
            self._ensure_workspace()
        o = self.out if out is None else out
        s = stream if stream is not None else torch.cuda.current_stream(self.device)
        args = [self.B, self.k, self.items.data_ptr(), self.order.data_ptr(), self.row.data_ptr(),
                self.col.data_ptr(), self.val.data_ptr(), _DT[self.val_dtype],
                self.X.data_ptr(), self.G.data_ptr(), _DT[self.x_dtype],
                o["col_ptr"].data_ptr(), o["row_idx"].data_ptr(), o["val_out"].data_ptr(),
                o["row_ptr"].data_ptr(), o["col_t"].data_ptr(), o["perm"].data_ptr(),
                o["Y"].data_ptr(), o["dX"].data_ptr(), o["dval"].data_ptr(),
                o["info"].data_ptr(), self.max_dim, self.max_nnz, self.workers,
                self.ws.data_ptr(), self.ws.numel()]
        if tune_key is None:
            st = self.lib.spm_batch_run(*args, s.cuda_stream)
            _lib.check(st, "spm_batch_run")
        else:
            st = self.lib.spm_batch_coo_to_csc_spmm(*args, tune_key.encode(), s.cuda_stream)
            _lib.check(st, "spm_batch_coo_to_csc_spmm")
        return o

    def run_single(self, out=None, stream=None, keep_plan: bool = True):
        """The same work as per-matrix calls of the four single-matrix entry points.  With
        keep_plan, each matrix's plan is also copied into the packed row_ptr / col_t / perm
        outputs (device copies outside the library, for comparison only)."""
        o = self.out if out is None else out
        s = stream if stream is not None else torch.cuda.current_stream(self.device)
        h = s.cuda_stream
        lib = self.lib
        k = self.k
        vt = _DT[self.val_dtype]
        xt = _DT[self.x_dtype]
        esz_v = self.val.element_size()
        esz_x = self.X.element_size()
        for b in range(self.B):
            nr, nc, nz = int(self.n_r[b]), int(self.n_c[b]), int(self.nnz[b])
            to, co = int(self.trip_off[b]), int(self.colptr_off[b])
            cp = o["col_ptr"].data_ptr() + 4 * co
            ri = o["row_idx"].data_ptr() + 4 * to
            vo = o["val_out"].data_ptr() + 4 * to
            st = lib.spm_coo_to_csc(nr, nc, nz, self.row.data_ptr() + 4 * to,
                                    self.col.data_ptr() + 4 * to,
                                    self.val.data_ptr() + esz_v * to, vt, cp, ri, vo, _lib.F32,
                                    o["info"].data_ptr() + 8 * b, self.asm_ws.data_ptr(),
                                    self.asm_ws.numel(), h)
            _lib.check(st, "spm_coo_to_csc[%d]" % b)
            st = lib.spm_csc_plan_build(nr, nc, nz, cp, ri, None, _lib.F32, self.plan.data_ptr(),
                                        self.plan.numel(), None, self.plan_info.data_ptr(),
                                        self.plan_ws.data_ptr(), self.plan_ws.numel(), h)
            _lib.check(st, "spm_csc_plan_build[%d]" % b)
            if keep_plan:
                rp, ct, pm = plan_arrays(self.plan, nr, nz)
                ro = int(self.rowptr_off[b])
                o["row_ptr"][ro: ro + nr + 1].copy_(rp)
                o["col_t"][to: to + nz].copy_(ct)
                o["perm"][to: to + nz].copy_(pm)
            xp = self.X.data_ptr() + esz_x * int(self.x_off[b])
            gp = self.G.data_ptr() + esz_x * int(self.g_off[b])
            st = lib.spm_csc_spmm(nr, nc, nz, k, self.plan.data_ptr(), vo, _lib.F32,
                                  _lib.ORDER_CSC, xp, k, xt,
                                  o["Y"].data_ptr() + 4 * int(self.g_off[b]), k, _lib.F32, h)
            _lib.check(st, "spm_csc_spmm[%d]" % b)
            st = lib.spm_csc_spmm_backward(nr, nc, nz, k, cp, ri, vo, _lib.F32, gp, k, xt, xp, k, xt,
                                           o["dX"].data_ptr() + 4 * int(self.x_off[b]), k,
                                           _lib.F32, o["dval"].data_ptr() + 4 * to, _lib.F32, h)
            _lib.check(st, "spm_csc_spmm_backward[%d]" % b)
        return o

    def matrix(self, out, b):
        """Host views of matrix b's results: (col_ptr, row_idx, values, Y, dX, dval, info)."""
        to, nz = int(self.trip_off[b]), int(self.nnz[b])
        co, nc, nr = int(self.colptr_off[b]), int(self.n_c[b]), int(self.n_r[b])
        k = self.k
        info = out["info"][2 * b: 2 * b + 2].cpu().numpy()
        n = int(info[0])
        return dict(col_ptr=out["col_ptr"][co: co + nc + 1].cpu().numpy(),
                    row_idx=out["row_idx"][to: to + n].cpu().numpy(),
                    values=out["val_out"][to: to + n].cpu().numpy(),
                    Y=out["Y"][int(self.g_off[b]): int(self.g_off[b]) + nr * k].cpu().numpy()
                    .reshape(nr, k),
                    dX=out["dX"][int(self.x_off[b]): int(self.x_off[b]) + nc * k].cpu().numpy()
                    .reshape(nc, k),
                    dval=out["dval"][to: to + n].cpu().numpy(), info=info, nnz_in=nz)
