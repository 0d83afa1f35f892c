"""Buckets above the usual in-LDS capacity (2048 elements): assembly, plan, the fused call
and batch insertion on inputs whose column (and row) buckets hold 2049..4096 elements (the
second level-2 launch, in LDS) and more than 4096 (the same launch, staged), bit for bit
against the oracle and against the two-call build."""
import numpy as np
import pytest
import torch

import oracle
from paper_1805_03380_amd import ops, synth
from gpu_util import assemble_gpu, assert_csc_equal, dev
from test_gpu_fused import _both, _check_plan_oracle

pytestmark = pytest.mark.gpu


def _heavy(seed, dtype=np.float64):
    """65,536 x 4,096 with 2e6 uniform triplets (2,048 column buckets of 2 columns, about 1,000
    elements; 2,048 row buckets of 32 rows, about 1,000, so both partitions take the second
    level-2 launch and the fused call still applies), plus heavy columns and rows: column 100
    +4,000 (its bucket above 4,096), columns 200, 201 +700 each and column 300 +1,200 (buckets
    between 2,048 and 4,096), row 7 with 3,500 distinct columns (its row bucket above 4,096)
    and row 1,000 with 1,800 (between).  Duplicates in the heavy columns."""
    rng = np.random.Generator(np.random.PCG64(seed))
    n_rows, n_cols, n = 65_536, 4096, 2_000_000
    rows = [rng.integers(0, n_rows, n)]
    cols = [rng.integers(0, n_cols, n)]
    for c, extra in ((100, 4000), (200, 700), (201, 700), (300, 1200)):
        rows.append(rng.integers(0, 3000, extra))  # repeats: folds inside the heavy columns
        cols.append(np.full(extra, c))
    for r, m in ((7, 3500), (1000, 1800)):
        rows.append(np.full(m, r))
        cols.append(rng.permutation(n_cols)[:m])
    row = np.concatenate(rows).astype(np.int32)
    col = np.concatenate(cols).astype(np.int32)
    perm = rng.permutation(row.size)
    row, col = row[perm], col[perm]
    val = rng.standard_normal(row.size)
    val[rng.choice(row.size, 5000, replace=False)] = 0.0
    return synth.COOProblem("heavy", n_rows, n_cols, row, col, val.astype(dtype))


def test_bucket_sizes_cover_both_big_paths():
    """The instance really has column buckets (2 columns) and row buckets (32 rows) in both
    ranges (checked on the host from the triplets)."""
    p = _heavy(6100)
    cb = np.bincount(p.col.astype(np.int64) >> 1)
    assert ((cb > 2048) & (cb <= 4096)).sum() >= 2 and (cb > 4096).sum() >= 1
    st, R = oracle.coo_to_csc(p.n_rows, p.n_cols, p.row, p.col, p.val)
    rb = np.bincount(R.row_idx.astype(np.int64) >> 5)
    assert ((rb > 2048) & (rb <= 4096)).sum() >= 1 and (rb > 4096).sum() >= 1


@pytest.mark.parametrize("dtype,out_dtype", [(np.float64, None), (np.float32, None),
                                             (np.float64, torch.float32)])
def test_big_buckets_assembly(dtype, out_dtype):
    p = _heavy(6101, dtype)
    print("case big buckets assembly %s" % np.dtype(dtype).name, flush=True)
    A = assemble_gpu(p, out_dtype=out_dtype)
    st, R = oracle.coo_to_csc(p.n_rows, p.n_cols, p.row, p.col, p.val)
    assert st == oracle.OK
    assert_csc_equal(A, R, A.values_buf.cpu().numpy().dtype)


@pytest.mark.parametrize("val_dtype", [torch.float64, torch.float32])
def test_big_buckets_fused_and_plan(val_dtype):
    p = _heavy(6102)
    B, vp, nnz, st = _both(p, val_dtype=val_dtype)
    assert st == 0
    q = synth.COOProblem(p.name, p.n_rows, p.n_cols, p.row, p.col,
                         p.val.astype(np.float32) if val_dtype == torch.float32 else p.val)
    _check_plan_oracle(B, q)


def test_big_buckets_insertion():
    p = _heavy(6103)
    A = assemble_gpu(p)
    rng = np.random.Generator(np.random.PCG64(6104))
    m = 300_000
    row = np.concatenate([rng.integers(0, p.n_rows, m - 3000),
                          rng.integers(0, 3000, 3000)]).astype(np.int32)
    col = np.concatenate([rng.integers(0, p.n_cols, m - 3000),
                          np.full(3000, 300)]).astype(np.int32)
    val = rng.standard_normal(m)
    print("case big buckets insertion", flush=True)
    I = ops.csc_insert(A, dev(row), dev(col), dev(val))
    n = A.nnz
    Ah = oracle.CSC(A.n_rows, A.n_cols, A.col_ptr.cpu().numpy(), A.row_idx_buf[:n].cpu().numpy(),
                    oracle.widen(A.values_buf[:n].cpu()))
    st, R = oracle.csc_insert(Ah, row, col, val)
    assert st == oracle.OK
    assert_csc_equal(I, R, np.float64)
