"""GPU parity of the sum of two CSCs (spm_csc_add) with the oracle's column merge: structure
and values bit-exact (a shared location is A's value plus B's in binary64, zero sums
dropped), and equal to inserting B's elements into A."""
import numpy as np
import pytest
import torch

import oracle
from paper_1805_03380_amd import _lib, ops, synth
from gpu_util import DEV, assemble_gpu, assert_csc_equal, dev

pytestmark = pytest.mark.gpu


def _host(A_gpu):
    n = A_gpu.nnz
    return oracle.CSC(A_gpu.n_rows, A_gpu.n_cols, A_gpu.col_ptr.cpu().numpy(),
                      A_gpu.row_idx_buf[:n].cpu().numpy(),
                      oracle.widen(A_gpu.values_buf[:n].cpu()))


def _add_case(A, B, out_np=np.float64, out_dtype=None):
    C = ops.csc_add(A, B, out_dtype=out_dtype)
    st, R = oracle.csc_add(_host(A), _host(B))
    assert st == oracle.OK
    assert_csc_equal(C, R, out_np)
    return C


@pytest.mark.parametrize("val_dtype", [torch.float64, torch.float32])
def test_add_random(val_dtype):
    pa = synth.random_coo(3100, 2500, 1800, 50_000, dup_frac=0.2, dist="normal")
    pb = synth.random_coo(3101, 2500, 1800, 40_000, dup_frac=0.2, dist="normal")
    print("case add %s" % val_dtype, flush=True)
    A, B = assemble_gpu(pa, val_dtype=val_dtype), assemble_gpu(pb, val_dtype=val_dtype)
    out_np = np.float64 if val_dtype == torch.float64 else np.float32
    C = _add_case(A, B, out_np)
    # the same as inserting B's elements (CSC order) into A
    b_col = torch.repeat_interleave(torch.arange(B.n_cols, device=DEV, dtype=torch.int32),
                                    torch.diff(B.col_ptr).long())
    I = ops.csc_insert(A, B.row_idx.contiguous(), b_col, B.values.contiguous())
    assert torch.equal(C.col_ptr, I.col_ptr) and torch.equal(C.row_idx, I.row_idx)
    assert torch.equal(C.values.view(torch.int32 if out_np == np.float32 else torch.int64),
                       I.values.view(torch.int32 if out_np == np.float32 else torch.int64))


def test_add_cancellation_and_empty():
    pa = synth.random_coo(3102, 600, 500, 8000, dup_frac=0.0, dist="normal")
    neg = synth.COOProblem("neg", pa.n_rows, pa.n_cols, pa.row, pa.col, -pa.val)
    A, N = assemble_gpu(pa), assemble_gpu(neg)
    C = _add_case(A, N)
    assert C.nnz == 0
    e = synth.COOProblem("empty", 600, 500, np.zeros(0, np.int32), np.zeros(0, np.int32),
                         np.zeros(0))
    E = assemble_gpu(e)
    C = _add_case(A, E)
    assert torch.equal(C.row_idx, A.row_idx)
    _add_case(E, A)
    _add_case(E, E)


def test_add_spare_capacity():
    """Both operands with capacity above their nnz (duplicates folded on assembly)."""
    pa = synth.random_coo(3103, 900, 700, 20_000, dup_frac=0.5, dist="normal")
    pb = synth.random_coo(3104, 900, 700, 20_000, dup_frac=0.5, dist="normal")
    A, B = assemble_gpu(pa), assemble_gpu(pb)
    assert A.nnz_cap > A.nnz and B.nnz_cap > B.nnz
    _add_case(A, B)


def test_add_uniform_1e5():
    p = synth.uniform_1e5(k=1)
    q = synth.random_coo(1006, p.n_rows, p.n_cols, 1_000_000, dup_frac=0.05, dtype=np.float32)
    print("case add uniform 1e5", flush=True)
    A, B = assemble_gpu(p), assemble_gpu(q)
    _add_case(A, B, np.float32)
    _add_case(A, B, np.float64, out_dtype=torch.float64)


def _csc_dev(n_rows, n_cols, col_ptr, row_idx, val):
    return ops.CSCMatrix(n_rows, n_cols, dev(np.array(col_ptr, np.int32)),
                         dev(np.array(row_idx, np.int32)), dev(np.array(val, np.float64)),
                         torch.zeros(2, dtype=torch.int32, device=DEV))


def test_add_reports_malformed_inputs():
    good = _csc_dev(4, 3, [0, 2, 3, 4], [0, 2, 1, 3], [1.0, 2.0, 3.0, 4.0])
    out_of_range = _csc_dev(4, 3, [0, 2, 3, 4], [0, 2, 1, 4], [1.0, 2.0, 3.0, 4.0])
    bad_offsets = _csc_dev(4, 3, [0, 3, 2, 4], [0, 2, 1, 3], [1.0, 2.0, 3.0, 4.0])
    for bad, exc in ((out_of_range, IndexError), (bad_offsets, ValueError)):
        with pytest.raises(exc):
            ops.csc_add(good, bad)
        with pytest.raises(exc):
            ops.csc_add(bad, good)
    C = ops.csc_add(good, good)
    assert C.values.cpu().tolist() == [2.0, 4.0, 6.0, 8.0]


def _with_capacity(A, cap):
    """The same CSC in buffers of a larger capacity (the extra slots hold garbage)."""
    ri = torch.full((cap,), 7, dtype=torch.int32, device=DEV)
    v = torch.full((cap,), 3.5, dtype=A.values_buf.dtype, device=DEV)
    ri[:A.nnz] = A.row_idx
    v[:A.nnz] = A.values
    return ops.CSCMatrix(A.n_rows, A.n_cols, A.col_ptr.clone(), ri, v, A.info)


def test_add_tile_order_by_ticket_and_by_index_agree():
    """Spare capacity of 10^6 per operand makes the merge grid larger than what fits on the
    device at once, so tiles number themselves by ticket; without it the workgroup index
    serves.  Both give the same bits."""
    pa = synth.random_coo(3109, 30_000, 20_000, 400_000, dup_frac=0.1, dist="normal")
    pb = synth.random_coo(3110, 30_000, 20_000, 300_000, dup_frac=0.1, dist="normal")
    A, B = assemble_gpu(pa), assemble_gpu(pb)
    C1 = _add_case(A, B)
    C2 = _add_case(_with_capacity(A, 1_000_000), _with_capacity(B, 1_000_000))
    assert torch.equal(C1.col_ptr, C2.col_ptr) and torch.equal(C1.row_idx, C2.row_idx)
    assert torch.equal(C1.values.view(torch.int64), C2.values.view(torch.int64))


def test_add_merge_and_insertion_paths_agree():
    """Short columns take the direct merge, long ones (by capacity) the insertion path: both
    give the same bits, and both match the oracle."""
    pa = synth.random_coo(3105, 4000, 3000, 60_000, dup_frac=0.1, dist="normal")
    pb = synth.random_coo(3106, 4000, 3000, 50_000, dup_frac=0.1, dist="normal")
    A, B = assemble_gpu(pa), assemble_gpu(pb)
    C1 = _add_case(A, B)  # average capacity per column well under 64: merge
    big = 70 * A.n_cols
    C2 = _add_case(_with_capacity(A, big), _with_capacity(B, big))  # insertion path
    assert torch.equal(C1.col_ptr, C2.col_ptr) and torch.equal(C1.row_idx, C2.row_idx)
    assert torch.equal(C1.values.view(torch.int64), C2.values.view(torch.int64))


def test_add_long_columns():
    pa = synth.random_coo(3107, 20_000, 60, 120_000, dup_frac=0.1, dist="normal")
    pb = synth.random_coo(3108, 20_000, 60, 100_000, dup_frac=0.1, dist="normal")
    _add_case(assemble_gpu(pa), assemble_gpu(pb))


@pytest.mark.parametrize("shape", [(0, 5), (1, 1), (7, 1), (1, 9)])
def test_add_degenerate_shapes(shape):
    n_rows, n_cols = shape
    n = 0 if n_rows == 0 else min(n_rows * n_cols, 5)
    pa = synth.random_coo(3109, n_rows, n_cols, n, dup_frac=0.0) if n else synth.COOProblem(
        "empty", n_rows, n_cols, np.zeros(0, np.int32), np.zeros(0, np.int32), np.zeros(0))
    pb = synth.random_coo(3110, n_rows, n_cols, n, dup_frac=0.0) if n else pa
    _add_case(assemble_gpu(pa), assemble_gpu(pb))


def test_add_overlapping_offsets_stay_in_bounds():
    """Offsets [0, cap, 0, cap, ...]: every even column passes its own checks and covers the
    whole capacity again, so the per-column counts total far more than the outputs hold.  The
    call must report SPM_EINVAL and write nothing past the capacity (a sentinel region right
    after it stays as it was)."""
    import ctypes
    n_rows, n_cols, a_cap = 16, 64, 8
    cp = np.array([0 if c % 2 == 0 else a_cap for c in range(n_cols + 1)], np.int32)
    a_cp, a_ri = dev(cp), dev(np.arange(a_cap, dtype=np.int32))
    a_v = dev(np.arange(1, a_cap + 1, dtype=np.float64))
    good = _csc_dev(n_rows, n_cols, [0] + [1] * 4 + [4] * (n_cols - 4), [0, 3, 5, 9],
                    [1.0, 2.0, 3.0, 4.0])
    b_cap = 4
    out_cap, spare = a_cap + b_cap, 4096
    lib = _lib.load()
    wb = ctypes.c_size_t(0)
    assert lib.spm_csc_add_workspace(n_rows, n_cols, a_cap, b_cap, ctypes.byref(wb)) == _lib.OK
    ws = torch.empty(max(wb.value, 256), dtype=torch.uint8, device=DEV)
    col_ptr = torch.empty(n_cols + 1, dtype=torch.int32, device=DEV)
    row_idx = torch.full((out_cap + spare,), -77, dtype=torch.int32, device=DEV)
    val_out = torch.full((out_cap + spare,), 1234.5, dtype=torch.float64, device=DEV)
    info = torch.zeros(2, dtype=torch.int32, device=DEV)
    for a_first in (True, False):
        A = (a_cp, a_ri, a_v, a_cap) if a_first else (good.col_ptr, good.row_idx_buf,
                                                      good.values_buf, b_cap)
        B = (good.col_ptr, good.row_idx_buf, good.values_buf, b_cap) if a_first else \
            (a_cp, a_ri, a_v, a_cap)
        st = lib.spm_csc_add(n_rows, n_cols, A[3], A[0].data_ptr(), A[1].data_ptr(),
                             A[2].data_ptr(), B[3], B[0].data_ptr(), B[1].data_ptr(),
                             B[2].data_ptr(), _lib.F64, col_ptr.data_ptr(), row_idx.data_ptr(),
                             val_out.data_ptr(), _lib.F64, info.data_ptr(), ws.data_ptr(),
                             ws.numel(), None)
        assert st == _lib.OK
        torch.cuda.synchronize()
        assert int(info[1]) == _lib.EINVAL
        assert torch.all(row_idx[out_cap:] == -77)
        assert torch.all(val_out[out_cap:] == 1234.5)


def test_add_hypersparse():
    """200,000 columns for a few thousand elements (tiles over many empty columns)."""
    pa = synth.random_coo(3111, 50_000, 200_000, 3000, dup_frac=0.0, dist="normal")
    pb = synth.random_coo(3112, 50_000, 200_000, 2500, dup_frac=0.0, dist="normal")
    _add_case(assemble_gpu(pa), assemble_gpu(pb))
