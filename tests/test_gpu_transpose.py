"""GPU parity of the transpose X.t() of Table 1 (spm_csc_transpose) with the oracle's counting
transpose: structure and values bit-exact (values are moved, never changed), on random,
rectangular, empty and degenerate shapes; and of the row-vector product V.A of Fig. 1 built on
the adjoint's column walk."""
import numpy as np
import pytest
import torch

import oracle
from paper_1805_03380_amd import _lib, ops, synth
from gpu_util import DEV, assemble_gpu, assert_close, assert_csc_equal, dev

pytestmark = pytest.mark.gpu


def _oracle_csc(A_gpu):
    n = A_gpu.nnz
    return oracle.CSC(A_gpu.n_rows, A_gpu.n_cols, A_gpu.col_ptr.cpu().numpy(),
                      A_gpu.row_idx_buf[:n].cpu().numpy(),
                      oracle.widen(A_gpu.values_buf[:n].cpu()))


def _transpose_case(p, val_dtype=torch.float64):
    print("case %s %dx%d nnz_in=%d %s" % (p.name, p.n_rows, p.n_cols, p.nnz_in, val_dtype),
          flush=True)
    A = assemble_gpu(p, val_dtype=val_dtype)
    T = ops.csc_transpose(A)
    assert (T.n_rows, T.n_cols) == (A.n_cols, A.n_rows)
    st, R = oracle.csc_transpose(_oracle_csc(A))
    assert st == oracle.OK
    out_np = np.float64 if val_dtype == torch.float64 else np.float32
    assert_csc_equal(T, R, out_np)
    return A, T


@pytest.mark.parametrize("val_dtype", [torch.float64, torch.float32])
def test_transpose_random(val_dtype):
    p = synth.random_coo(91, 3000, 2000, 60_000, dup_frac=0.2, dist="normal")
    _transpose_case(p, val_dtype)


@pytest.mark.parametrize("shape", [(1, 50_000), (50_000, 1), (7, 40_000), (40_000, 7)])
def test_transpose_thin(shape):
    p = synth.random_coo(92, shape[0], shape[1], 30_000, dup_frac=0.3, dist="normal")
    _transpose_case(p)


def test_transpose_uniform_1e5():
    p = synth.uniform_1e5(seed=93, k=1)
    _transpose_case(p, torch.float32)


def test_transpose_twice_is_identity():
    p = synth.random_coo(94, 1200, 900, 25_000, dup_frac=0.1, dist="normal")
    A, T = _transpose_case(p)
    TT = ops.csc_transpose(T)
    assert torch.equal(TT.col_ptr, A.col_ptr)
    assert torch.equal(TT.row_idx, A.row_idx)
    assert torch.equal(TT.values.view(torch.int64), A.values.view(torch.int64))


@pytest.mark.parametrize("shape", [(5, 7), (0, 5), (5, 0), (1, 1)])
def test_transpose_empty(shape):
    p = synth.COOProblem("empty", shape[0], shape[1], np.zeros(0, np.int32),
                         np.zeros(0, np.int32), np.zeros(0))
    A, T = _transpose_case(p)
    assert T.nnz == 0 and T.col_ptr.numel() == shape[0] + 1


def test_transpose_spare_capacity():
    """A with capacity above nnz (duplicates folded): only the first nnz slots are read."""
    p = synth.random_coo(95, 800, 600, 20_000, dup_frac=0.5, dist="normal")
    A, T = _transpose_case(p)
    assert A.nnz_cap > A.nnz and T.nnz_cap == A.nnz_cap


def test_transpose_reports_malformed_csc():
    """A row index outside the matrix is a device-detected error (info[1] = SPM_EBOUNDS)."""
    p = synth.random_coo(96, 400, 300, 5000, dup_frac=0.0)
    A = assemble_gpu(p)
    A.row_idx_buf[A.nnz // 2] = 400
    with pytest.raises(IndexError):
        ops.csc_transpose(A)
    # a valid transpose afterwards is not affected
    A.row_idx_buf[A.nnz // 2] = 0
    ops.csc_transpose(A, sync=True)


def test_transpose_rejects_bad_arguments():
    lib = _lib.load()
    cp = torch.zeros(4, dtype=torch.int32, device=DEV)
    ri = torch.zeros(8, dtype=torch.int32, device=DEV)
    v = torch.zeros(8, dtype=torch.float64, device=DEV)
    t_cp = torch.zeros(6, dtype=torch.int32, device=DEV)
    info = torch.zeros(2, dtype=torch.int32, device=DEV)
    wb = _lib.ctypes.c_size_t(0)
    assert lib.spm_csc_transpose_workspace(5, 3, 8, _lib.ctypes.byref(wb)) == _lib.OK
    ws = torch.empty(wb.value, dtype=torch.uint8, device=DEV)
    args = [5, 3, 8, cp.data_ptr(), ri.data_ptr(), v.data_ptr(), _lib.F64, t_cp.data_ptr(),
            ri.data_ptr(), v.data_ptr(), info.data_ptr(), ws.data_ptr(), ws.numel(), None]
    bad = list(args)
    bad[6] = _lib.BF16
    assert lib.spm_csc_transpose(*bad) == _lib.EDTYPE
    bad = list(args)
    bad[12] = ws.numel() - 1
    assert lib.spm_csc_transpose(*bad) == _lib.EWORKSPACE
    bad = list(args)
    bad[7] = None
    assert lib.spm_csc_transpose(*bad) == _lib.EINVAL


@pytest.mark.parametrize("m", [1, 3, 16])
def test_rowvec_spmm(m):
    """W = V.A against the oracle's product of A^T with V^T: column i of A summed in
    increasing row order, within the binary64 error bound."""
    p = synth.random_coo(97, 2500, 1800, 40_000, dup_frac=0.1, dist="normal")
    A = assemble_gpu(p)
    rng = np.random.Generator(np.random.PCG64(98))
    V = rng.standard_normal((m, p.n_rows))
    W = ops.rowvec_spmm(dev(V[0] if m == 1 else V), A)
    st, T = oracle.csc_transpose(_oracle_csc(A))
    Y, S, M = oracle.spmm(T, V.T)
    got = W.reshape(1, -1) if m == 1 else W
    assert got.shape == (m, p.n_cols)
    assert_close(got.t(), Y, S, M, torch.float64, what="V.A")
