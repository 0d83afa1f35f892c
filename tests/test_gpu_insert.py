"""GPU parity of batch insertion into an existing CSC (spm_csc_insert) with the oracle: at a
location the existing value folds first, then the new values in input order; structure and
values bit-exact."""
import numpy as np
import pytest
import torch

import oracle
import pins
from paper_1805_03380_amd import ops, synth
from gpu_util import DEV, assemble_gpu, assert_csc_equal, dev

pytestmark = pytest.mark.gpu


def _oracle_csc(A_gpu):
    n = A_gpu.nnz
    return oracle.CSC(A_gpu.n_rows, A_gpu.n_cols, A_gpu.col_ptr.cpu().numpy(),
                      A_gpu.row_idx_buf[:n].cpu().numpy(),
                      oracle.widen(A_gpu.values_buf[:n].cpu()))


def _insert_case(p, q, dtype=np.float64, out_dtype=None):
    """A assembled on the GPU from p (capacity p.nnz_in, so some slots are unused), then q's
    triplets inserted; compared with the oracle's insertion into the same A."""
    print("case %s + %s %dx%d" % (p.name, q.name, p.n_rows, p.n_cols), flush=True)
    A = assemble_gpu(p, val_dtype=torch.float64 if dtype == np.float64 else torch.float32)
    B = ops.csc_insert(A, dev(q.row), dev(q.col), dev(q.val.astype(dtype)), out_dtype=out_dtype)
    st, R = oracle.csc_insert(_oracle_csc(A), q.row, q.col, q.val.astype(dtype))
    assert st == oracle.OK
    out_np = np.float64 if B.values_buf.dtype == torch.float64 else np.float32
    assert_csc_equal(B, R, out_np)
    return A, B, R


@pytest.mark.parametrize("dtype", [np.float64, np.float32])
def test_insert_random(dtype):
    p = synth.random_coo(81, 2000, 1500, 40_000, dup_frac=0.2, dist="normal")
    q = synth.random_coo(82, 2000, 1500, 15_000, dup_frac=0.2, dist="normal")
    _insert_case(p, q, dtype)


def test_insert_cancels_existing():
    """New triplets that cancel existing elements exactly, or sum to zero among themselves
    only after the existing value: those locations disappear."""
    rng = np.random.Generator(np.random.PCG64(83))
    p = synth.random_coo(84, 300, 200, 6000, dup_frac=0.0, dist="normal")
    st, A0 = oracle.coo_to_csc(p.n_rows, p.n_cols, p.row, p.col, p.val)
    a_col = np.repeat(np.arange(A0.n_cols), np.diff(A0.col_ptr))
    pick = rng.choice(A0.nnz, 2000, replace=False)
    row = A0.row_idx[pick].astype(np.int32)
    col = a_col[pick].astype(np.int32)
    val = -A0.values[pick]
    q = synth.COOProblem("cancel", p.n_rows, p.n_cols, row, col, val)
    A, B, R = _insert_case(p, q)
    assert B.nnz == A0.nnz - 2000


def test_insert_golden():
    g = pins.load_golden("insert_small.json")
    # A from its own triplets on the GPU (columns in CSC order give the same arrays)
    a_col = np.repeat(np.arange(g["n_cols"]), np.diff(g["a_col_ptr"])).astype(np.int32)
    p = synth.COOProblem("golden_a", g["n_rows"], g["n_cols"], np.array(g["a_row_idx"], np.int32),
                         a_col, np.array(g["a_val"], np.float64))
    q = synth.COOProblem("golden_t", g["n_rows"], g["n_cols"], np.array(g["row"], np.int32),
                         np.array(g["col"], np.int32), np.array(g["val"], np.float64))
    A, B, R = _insert_case(p, q)
    assert B.col_ptr.cpu().tolist() == g["expect_col_ptr"]
    assert B.row_idx.cpu().tolist() == g["expect_row_idx"]
    assert B.values.cpu().tolist() == g["expect_val"]


def test_insert_nothing_and_into_empty():
    p = synth.random_coo(85, 500, 400, 5000, dup_frac=0.1)
    empty = synth.COOProblem("none", 500, 400, np.zeros(0, np.int32), np.zeros(0, np.int32),
                             np.zeros(0))
    A, B, R = _insert_case(p, empty)
    assert torch.equal(A.col_ptr, B.col_ptr) and torch.equal(A.row_idx, B.row_idx)
    _insert_case(empty, p)


def test_insert_uniform_1e5():
    """10^5 new triplets into the 10^5 x 10^5 matrix assembled from 10^6 triplets."""
    p = synth.uniform_1e5(value_dtype=np.float32, k=0)
    q = synth.random_coo(86, p.n_rows, p.n_cols, 100_000, dup_frac=0.05)
    _insert_case(p, q, np.float32)


def test_insert_statuses():
    p = synth.random_coo(87, 100, 80, 900, dup_frac=0.1)
    A = assemble_gpu(p)
    row = np.array([3, 100, 5], np.int32)  # 100 is out of range
    col = np.array([1, 2, 79], np.int32)
    val = np.array([1.0, 2.0, 3.0])
    B = ops.csc_insert(A, dev(row), dev(col), dev(val), sync=False)
    torch.cuda.synchronize()
    assert int(B.info[1]) == oracle.EBOUNDS
    with pytest.raises(IndexError):
        B.sync()
    bad = ops.CSCMatrix(100, 80, A.col_ptr.clone(), A.row_idx_buf, A.values_buf, A.info)
    bad.col_ptr[5] = bad.col_ptr[4] - 1  # offsets not monotone
    with pytest.raises(ValueError):
        ops.csc_insert(bad, dev(row[:1]), dev(col[:1]), dev(val[:1]))
    with pytest.raises(ValueError):
        ops.csc_insert(A, dev(row[:1]), dev(col[:1]), dev(val[:1].astype(np.float32)))


def test_insert_long_runs_and_columns():
    """Work is cut by position in the merged sequence: a column longer than many threads'
    ranges, a location with 5,000 new values (one run across many ranges, folded by the thread
    owning its start, existing value first), new triplets in empty columns, all bit for bit."""
    rng = np.random.Generator(np.random.PCG64(88))
    n_rows, n_cols = 30_000, 500
    m = 40_000
    row = np.concatenate([rng.integers(0, n_rows, m), rng.permutation(n_rows)[:20_000]])
    col = np.concatenate([rng.integers(0, 400, m), np.full(20_000, 7)])  # column 7: 20k rows
    p = synth.COOProblem("long", n_rows, n_cols, row.astype(np.int32), col.astype(np.int32),
                         rng.standard_normal(row.size))
    r2 = np.concatenate([np.full(5000, 11), rng.integers(0, n_rows, 30_000),
                         rng.integers(0, n_rows, 3000)])
    c2 = np.concatenate([np.full(5000, 7), rng.integers(0, n_cols, 30_000),
                         rng.integers(450, n_cols, 3000)])  # columns 450.. hold no existing
    q = synth.COOProblem("runs", n_rows, n_cols, r2.astype(np.int32), c2.astype(np.int32),
                         rng.standard_normal(r2.size))
    _insert_case(p, q)
    _insert_case(p, q, np.float32)


@pytest.mark.parametrize("seed", range(6))
def test_insert_random_small_shapes(seed):
    """Small shapes around the per-thread range (8 merged positions): empty columns,
    single-column and single-row matrices, duplicates of existing locations."""
    rng = np.random.Generator(np.random.PCG64(890 + seed))
    n_rows, n_cols = [(1, 1), (1, 17), (19, 1), (5, 7), (40, 3), (3, 40)][seed]

    def iid(name, n):  # i.i.d. locations: duplicates as they fall
        return synth.COOProblem(name, n_rows, n_cols,
                                rng.integers(0, n_rows, n).astype(np.int32),
                                rng.integers(0, n_cols, n).astype(np.int32),
                                rng.choice([-1.0, 1.0, 0.5, 2.0], n))
    p = iid("small_a", int(rng.integers(0, 3 * n_rows * n_cols + 1)))
    q = iid("small_t", int(rng.integers(0, 4 * n_rows * n_cols + 1)))
    _insert_case(p, q)


def test_insert_existing_rows_out_of_order():
    """Existing rows that do not increase down a column are reported as SPM_EINVAL."""
    p = synth.random_coo(91, 60, 40, 900, dup_frac=0.0)
    A = assemble_gpu(p)
    ri = A.row_idx_buf.clone()
    cp = A.col_ptr.cpu().numpy()
    c = int(np.argmax(np.diff(cp) >= 2))
    a, b = int(cp[c]), int(cp[c] + 1)
    ri[a], ri[b] = A.row_idx_buf[b], A.row_idx_buf[a]  # swap two rows of one column
    bad = ops.CSCMatrix(60, 40, A.col_ptr, ri, A.values_buf, A.info)
    with pytest.raises(ValueError):
        ops.csc_insert(bad, dev(np.array([1], np.int32)), dev(np.array([2], np.int32)),
                       dev(np.array([1.0])))


def test_insert_hypersparse():
    """200,000 columns for a few thousand elements: every merge tile spans tens of thousands
    of mostly empty columns, and most columns start at the very end or share one start."""
    rng = np.random.Generator(np.random.PCG64(93))
    n_rows, n_cols = 50_000, 200_000

    def iid(name, n, lo=0, hi=n_cols):
        return synth.COOProblem(name, n_rows, n_cols,
                                rng.integers(0, n_rows, n).astype(np.int32),
                                rng.integers(lo, hi, n).astype(np.int32),
                                rng.standard_normal(n))
    p = iid("hyper_a", 3000)
    q = iid("hyper_t", 2500, 0, 150_000)  # the last 50,000 columns stay empty
    _insert_case(p, q)
    _insert_case(p, q, np.float32)
