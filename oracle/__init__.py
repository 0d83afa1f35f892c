"""Oracle for the sparse assembly + CSC SpMM path -- TEST INFRASTRUCTURE ONLY.

Plain CPU binary64 reference (``spm_oracle.cpp``) plus thin numpy wrappers.  Only ``tests/``,
``__graft_entry__.smoke()`` and the ``cpu_baseline`` leg of ``bench.py`` may import this package.
It shares no code with ``paper_1805_03380_amd`` and imports nothing from it.

Every wrapper widens its floating inputs to float64 first (exact for float32 and bfloat16), runs
the binary64 definition, and only then rounds once to the requested output precision with numpy's
round-to-nearest-even cast.

Paper: Sanderson & Curtin, "A User-Friendly Hybrid Sparse Matrix Class in C++", arXiv:1805.03380.
Sections cited in each function: 3.1 (CSC), 3.2 (COO), 3.3 (red-black tree, index encoding),
3 use case (iv) (dense x sparse products), Table 1 (speye, sum, X.t(), trace(A.t()*B)).
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "spm_oracle.cpp")
_LIB_PATH = os.path.join(_HERE, "liboracle.so")
_lib = None

# Status values (retyped here; the numbers match the public status enum by value only).
OK, EINVAL, EBOUNDS = 0, 1, 2


def build(force: bool = True) -> str:
    """Compile the oracle with g++ (-O2, no FMA contraction, no fast-math)."""
    global _lib
    if not force and os.path.exists(_LIB_PATH):
        return _LIB_PATH
    tmp = _LIB_PATH + ".tmp%d" % os.getpid()
    cmd = ["g++", "-std=c++17", "-O2", "-ffp-contract=off", "-fno-fast-math", "-fPIC", "-shared",
           _SRC, "-o", tmp]
    subprocess.run(cmd, check=True)
    os.replace(tmp, _LIB_PATH)
    _lib = None
    return _LIB_PATH


def _load():
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(_LIB_PATH) or os.path.getmtime(_LIB_PATH) < os.path.getmtime(_SRC):
        build()
    _lib = configure(ctypes.CDLL(_LIB_PATH))
    return _lib


def configure(lib):
    """Declare the argument types of an oracle library handle (also used for planted-mistake
    copies built by the test suite)."""
    p = ctypes.c_void_p
    i64 = ctypes.c_int64
    for name in ("oracle_coo_to_csc_rbt", "oracle_coo_to_csc_sort"):
        f = getattr(lib, name)
        f.argtypes = [i64, i64, i64, p, p, p, p, p, p, p]
        f.restype = ctypes.c_int
    lib.oracle_csc_insert.argtypes = [i64, i64, p, p, p, i64, p, p, p, p, p, p, p]
    lib.oracle_csc_insert.restype = ctypes.c_int
    lib.oracle_csc_transpose.argtypes = [i64, i64, p, p, p, p, p, p]
    lib.oracle_csc_transpose.restype = ctypes.c_int
    lib.oracle_trace_atb.argtypes = [i64, i64, p, p, p, p, p, p, p, p]
    lib.oracle_trace_atb.restype = ctypes.c_int
    lib.oracle_csc_add.argtypes = [i64, i64, p, p, p, p, p, p, p, p, p, p]
    lib.oracle_csc_add.restype = ctypes.c_int
    lib.oracle_triplet_grad.argtypes = [i64, i64, i64, i64, p, p, p, p, p, p]
    lib.oracle_triplet_grad.restype = None
    lib.oracle_spmm.argtypes = [i64, i64, i64, p, p, p, p, p, p, p]
    lib.oracle_spmm.restype = None
    lib.oracle_spmm_backward.argtypes = [i64, i64, i64, p, p, p, p, p, p, p, p, p]
    lib.oracle_spmm_backward.restype = None
    lib.oracle_column_sums.argtypes = [i64, p, p, p]
    lib.oracle_column_sums.restype = None
    return lib


def _ptr(a: np.ndarray):
    return ctypes.c_void_p(a.ctypes.data) if a.size else ctypes.c_void_p(0)


def widen(a) -> np.ndarray:
    """Exact widening to float64 (float32 / float64 / bfloat16-as-torch tensors)."""
    if hasattr(a, "detach"):  # a torch CPU tensor, e.g. bfloat16
        import torch
        return a.detach().to(torch.float64).cpu().numpy()
    return np.ascontiguousarray(np.asarray(a, dtype=np.float64))


class CSC:
    """CSC arrays of Section 3.1: col_ptr[n_cols+1], row_idx[N], values[N] (float64)."""

    def __init__(self, n_rows, n_cols, col_ptr, row_idx, values):
        self.n_rows, self.n_cols = int(n_rows), int(n_cols)
        self.col_ptr, self.row_idx, self.values = col_ptr, row_idx, values

    @property
    def nnz(self) -> int:
        return int(self.col_ptr[-1])

    def rounded(self, dtype) -> np.ndarray:
        """The stored values rounded once (round-to-nearest-even) to ``dtype``."""
        return self.values.astype(dtype)


def coo_to_csc(n_rows, n_cols, row, col, val, method: str = "sort"):
    """Assemble COO triplets (Section 3.2) into CSC (Section 3.1).

    Duplicates are summed left to right in input order in binary64; locations whose sum is 0.0
    are not stored; emission is column-major.  ``method`` picks the red-black-tree read
    ("rbt", Section 3.3) or the stable-sort read ("sort", Section 3.1 batch insertion).
    Returns (status, CSC or None).
    """
    lib = _load()
    row = np.ascontiguousarray(row, dtype=np.int32)
    col = np.ascontiguousarray(col, dtype=np.int32)
    v = widen(val)
    n = row.shape[0]
    assert col.shape[0] == n and v.shape[0] == n
    col_ptr = np.zeros(n_cols + 1, dtype=np.int32)
    row_idx = np.zeros(max(n, 1), dtype=np.int32)
    out = np.zeros(max(n, 1), dtype=np.float64)
    nnz = ctypes.c_int64(0)
    f = lib.oracle_coo_to_csc_rbt if method == "rbt" else lib.oracle_coo_to_csc_sort
    st = f(n_rows, n_cols, n, _ptr(row), _ptr(col), _ptr(v), _ptr(col_ptr), _ptr(row_idx),
           _ptr(out), ctypes.byref(nnz))
    if st != OK:
        return st, None
    m = nnz.value
    return OK, CSC(n_rows, n_cols, col_ptr, row_idx[:m].copy(), out[:m].copy())


def csc_insert(A: CSC, row, col, val):
    """Batch insertion of new triplets into the existing CSC A (Section 3.1: sort the new
    elements, then merge with the existing arrays), accumulating like X(r,c) += v (Fig. 1):
    at each location the existing value comes first, then the new values in input order, in
    binary64; zero sums are not stored.  Returns (status, CSC or None)."""
    lib = _load()
    row = np.ascontiguousarray(row, dtype=np.int32)
    col = np.ascontiguousarray(col, dtype=np.int32)
    v = widen(val)
    n = row.shape[0]
    assert col.shape[0] == n and v.shape[0] == n
    a_cp = np.ascontiguousarray(A.col_ptr, dtype=np.int32)
    a_ri = np.ascontiguousarray(A.row_idx, dtype=np.int32)
    a_v = np.ascontiguousarray(A.values, dtype=np.float64)
    cap = max(int(a_cp[-1]) + n, 1)
    col_ptr = np.zeros(A.n_cols + 1, dtype=np.int32)
    row_idx = np.zeros(cap, dtype=np.int32)
    out = np.zeros(cap, dtype=np.float64)
    nnz = ctypes.c_int64(0)
    st = lib.oracle_csc_insert(A.n_rows, A.n_cols, _ptr(a_cp), _ptr(a_ri), _ptr(a_v), n,
                               _ptr(row), _ptr(col), _ptr(v), _ptr(col_ptr), _ptr(row_idx),
                               _ptr(out), ctypes.byref(nnz))
    if st != OK:
        return st, None
    m = nnz.value
    return OK, CSC(A.n_rows, A.n_cols, col_ptr, row_idx[:m].copy(), out[:m].copy())


def csc_add(A: CSC, B: CSC):
    """A + B (both CSCs of one shape): per column, the sorted row lists merged; a row in both
    gives A's value plus B's in binary64; a 0.0 result is not stored.  Returns (status, CSC or
    None)."""
    lib = _load()
    assert (A.n_rows, A.n_cols) == (B.n_rows, B.n_cols)
    arrs = []
    for M in (A, B):
        arrs += [np.ascontiguousarray(M.col_ptr, dtype=np.int32),
                 np.ascontiguousarray(M.row_idx, dtype=np.int32),
                 np.ascontiguousarray(widen(M.values), dtype=np.float64)]
    cap = max(int(arrs[0][-1]) + int(arrs[3][-1]), 1)
    col_ptr = np.zeros(A.n_cols + 1, dtype=np.int32)
    row_idx = np.zeros(cap, dtype=np.int32)
    out = np.zeros(cap, dtype=np.float64)
    nnz = ctypes.c_int64(0)
    st = lib.oracle_csc_add(A.n_rows, A.n_cols, *(_ptr(a) for a in arrs), _ptr(col_ptr),
                            _ptr(row_idx), _ptr(out), ctypes.byref(nnz))
    if st != OK:
        return st, None
    m = nnz.value
    return OK, CSC(A.n_rows, A.n_cols, col_ptr, row_idx[:m].copy(), out[:m].copy())


def csc_transpose(A: CSC):
    """A^T as a CSC (X.t() of Table 1): element (r, c, v) of A becomes (c, r, v); each column
    of the result lists one row of A by increasing column.  Returns (status, CSC or None)."""
    lib = _load()
    a_cp = np.ascontiguousarray(A.col_ptr, dtype=np.int32)
    a_ri = np.ascontiguousarray(A.row_idx, dtype=np.int32)
    a_v = np.ascontiguousarray(A.values, dtype=np.float64)
    m = int(a_cp[-1])
    t_cp = np.zeros(A.n_rows + 1, dtype=np.int32)
    t_ri = np.zeros(max(m, 1), dtype=np.int32)
    t_v = np.zeros(max(m, 1), dtype=np.float64)
    st = lib.oracle_csc_transpose(A.n_rows, A.n_cols, _ptr(a_cp), _ptr(a_ri), _ptr(a_v),
                                  _ptr(t_cp), _ptr(t_ri), _ptr(t_v))
    if st != OK:
        return st, None
    return OK, CSC(A.n_cols, A.n_rows, t_cp, t_ri[:m].copy(), t_v[:m].copy())


def trace_atb(A: CSC, B: CSC):
    """trace(A^T B) without forming A^T or the product (Section 2, Table 1): the sum over
    locations stored in both A and B of A[i,j] * B[i,j], columns ascending and A's rows
    ascending within each, binary64 products added left to right.
    Returns (status, trace, hits) with hits = locations stored in both."""
    lib = _load()
    assert (A.n_rows, A.n_cols) == (B.n_rows, B.n_cols)
    arrs = []
    for M in (A, B):
        arrs += [np.ascontiguousarray(M.col_ptr, dtype=np.int32),
                 np.ascontiguousarray(M.row_idx, dtype=np.int32),
                 np.ascontiguousarray(widen(M.values), dtype=np.float64)]
    out = ctypes.c_double(0.0)
    hits = ctypes.c_int64(0)
    st = lib.oracle_trace_atb(A.n_rows, A.n_cols, *(_ptr(a) for a in arrs), ctypes.byref(out),
                              ctypes.byref(hits))
    if st != OK:
        return st, None, None
    return OK, out.value, hits.value


def triplet_grad(n_rows, n_cols, row, col, G, X):
    """dL/dv_t for every input triplet of an assembly followed by Y = A.X, with dL/dY = G:
    sum_j G[row_t, j] X[col_t, j] in binary64 (ascending j), also for triplets whose location
    summed to zero; 0 for a triplet outside the matrix.  Returns (dv, S), S = sum |G||X|."""
    lib = _load()
    row = np.ascontiguousarray(row, dtype=np.int32)
    col = np.ascontiguousarray(col, dtype=np.int32)
    Gd, Xd = widen(G), widen(X)
    if Gd.ndim == 1:
        Gd = Gd[:, None]
    if Xd.ndim == 1:
        Xd = Xd[:, None]
    Gd, Xd = np.ascontiguousarray(Gd), np.ascontiguousarray(Xd)
    k = Xd.shape[1]
    assert Gd.shape == (n_rows, k) and Xd.shape == (n_cols, k)
    n = row.shape[0]
    dv = np.zeros(max(n, 1), dtype=np.float64)
    S = np.zeros(max(n, 1), dtype=np.float64)
    lib.oracle_triplet_grad(n_rows, n_cols, n, k, _ptr(row), _ptr(col), _ptr(Gd), _ptr(Xd),
                            _ptr(dv), _ptr(S))
    return dv[:n].copy(), S[:n].copy()


def spmm(A: CSC, X, values=None):
    """Y = A.X in binary64 (Section 3 use case (iv)); returns (Y, S, M).

    S is the per-output sum of |terms| and M the per-row term count (error-bound inputs).
    ``values`` overrides A.values (e.g. values rounded to float32 and widened back).
    """
    lib = _load()
    Xd = widen(X)
    if Xd.ndim == 1:
        Xd = Xd[:, None]
    Xd = np.ascontiguousarray(Xd)
    k = Xd.shape[1]
    assert Xd.shape[0] == A.n_cols
    v = widen(A.values if values is None else values)
    Y = np.zeros((A.n_rows, k), dtype=np.float64)
    S = np.zeros((A.n_rows, k), dtype=np.float64)
    M = np.zeros(A.n_rows, dtype=np.int64)
    lib.oracle_spmm(A.n_rows, A.n_cols, k, _ptr(A.col_ptr), _ptr(A.row_idx), _ptr(v), _ptr(Xd),
                    _ptr(Y), _ptr(S), _ptr(M))
    return Y, S, M


def spmm_backward(A: CSC, G, X, values=None):
    """Adjoint of Y = A.X for L = sum(Y*G): returns (dX, dval, SdX, Sdv) in binary64."""
    lib = _load()
    Gd = widen(G)
    Xd = widen(X)
    if Gd.ndim == 1:
        Gd = Gd[:, None]
    if Xd.ndim == 1:
        Xd = Xd[:, None]
    Gd, Xd = np.ascontiguousarray(Gd), np.ascontiguousarray(Xd)
    k = Xd.shape[1]
    assert Gd.shape == (A.n_rows, k) and Xd.shape == (A.n_cols, k)
    v = widen(A.values if values is None else values)
    dX = np.zeros((A.n_cols, k), dtype=np.float64)
    SdX = np.zeros((A.n_cols, k), dtype=np.float64)
    dval = np.zeros(A.nnz, dtype=np.float64)
    Sdv = np.zeros(A.nnz, dtype=np.float64)
    lib.oracle_spmm_backward(A.n_rows, A.n_cols, k, _ptr(A.col_ptr), _ptr(A.row_idx), _ptr(v),
                             _ptr(Gd), _ptr(Xd), _ptr(dX), _ptr(dval), _ptr(SdX), _ptr(Sdv))
    return dX, dval, SdX, Sdv


def column_sums(A: CSC) -> np.ndarray:
    """sum(X, 0) of Table 1 through the CSC arrays, binary64, in CSC order."""
    lib = _load()
    out = np.zeros(A.n_cols, dtype=np.float64)
    lib.oracle_column_sums(A.n_cols, _ptr(A.col_ptr), _ptr(A.values), _ptr(out))
    return out


def gamma(m, u: float = 2.0 ** -53):
    """Higham's gamma_m = m u / (1 - m u): bound factor of a fixed-order sum of m terms."""
    m = np.asarray(m, dtype=np.float64)
    return m * u / (1.0 - m * u)


def check_csc_invariants(A: CSC) -> None:
    """Section 3.1 invariants plus the ones implied by ordered emission; raises AssertionError."""
    cp, ri = A.col_ptr, A.row_idx
    assert cp.shape == (A.n_cols + 1,)
    assert cp[0] == 0, "c[0] must be 0"
    assert cp[-1] == ri.shape[0] == A.values.shape[0], "c[n_cols] must equal N"
    assert np.all(np.diff(cp.astype(np.int64)) >= 0), "column offsets must be monotone"
    if ri.size:
        assert ri.min() >= 0 and ri.max() < A.n_rows, "row index out of range"
    if ri.size > 1:
        starts = np.zeros(ri.size, dtype=bool)
        s = cp[:-1]
        starts[s[s < ri.size]] = True  # positions where some column begins
        d = np.diff(ri.astype(np.int64))
        assert np.all(d[~starts[1:]] > 0), "rows must increase strictly within each column"
    assert not np.any(A.values == 0.0), "an exact zero was stored"
