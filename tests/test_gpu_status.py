"""Device-reported statuses of assembly and plan.

Every call writes its own status word: nothing may carry over from an earlier call on the
same buffers, and a status buffer that starts as garbage must still end up exact.  For an
invalid CSC handed to the plan, an invalid shape (offsets not monotone, col_ptr[0] != 0,
more elements than the capacity) takes precedence over a row index out of range.
"""
import numpy as np
import pytest
import torch

import oracle
from paper_1805_03380_amd import ops, synth
from paper_1805_03380_amd.pipeline import Pipeline
from gpu_util import DEV

pytestmark = pytest.mark.gpu


def _csc(n_rows, n_cols, col_ptr, row_idx):
    d = DEV
    cp = torch.tensor(col_ptr, dtype=torch.int32, device=d)
    ri = torch.tensor(row_idx, dtype=torch.int32, device=d)
    v = torch.ones(len(row_idx), dtype=torch.float32, device=d)
    info = torch.tensor([len(row_idx), 0], dtype=torch.int32, device=d)
    return ops.CSCMatrix(n_rows, n_cols, cp, ri, v, info)


def test_plan_small_exact():
    # columns: 0 -> {2}, 1 -> {0, 1}, 2 -> {2}
    A = _csc(3, 3, [0, 1, 3, 4], [2, 0, 1, 2])
    plan = ops.build_plan(A)
    rp, ct, pm = ops.plan_arrays(plan, 3, 4)
    assert rp.cpu().tolist() == [0, 1, 2, 4]
    assert ct.cpu().tolist() == [1, 1, 0, 2]
    assert pm.cpu().tolist() == [1, 2, 0, 3]


def test_plan_row_out_of_range():
    with pytest.raises(IndexError):
        ops.build_plan(_csc(3, 3, [0, 1, 3, 4], [2, 0, 5, 2]))
    with pytest.raises(IndexError):
        ops.build_plan(_csc(3, 3, [0, 1, 3, 4], [2, -1, 1, 2]))


@pytest.mark.parametrize("col_ptr", [[0, 3, 1, 4], [1, 1, 3, 4], [0, 1, 3, 9]])
def test_plan_bad_shape(col_ptr):
    with pytest.raises(ValueError):
        ops.build_plan(_csc(3, 3, col_ptr, [2, 0, 1, 2]))


def test_plan_shape_takes_precedence():
    with pytest.raises(ValueError):
        ops.build_plan(_csc(3, 3, [0, 3, 1, 4], [2, 7, 1, 2]))


def test_plan_valid_after_invalid():
    with pytest.raises(IndexError):
        ops.build_plan(_csc(3, 3, [0, 1, 3, 4], [2, 0, 5, 2]))
    plan = ops.build_plan(_csc(3, 3, [0, 1, 3, 4], [2, 0, 1, 2]))
    rp, _, _ = ops.plan_arrays(plan, 3, 4)
    assert rp.cpu().tolist() == [0, 1, 2, 4]


def test_pipeline_status_not_stale():
    """Same Pipeline buffers: a call with an out-of-range triplet, then a valid call."""
    p = synth.random_coo(4242, 1000, 1000, 20_000, dup_frac=0.1)
    d = DEV
    pipe = Pipeline(p.n_rows, p.n_cols, p.nnz_in, 8, val_dtype=torch.float64,
                    x_dtype=torch.float64)
    X = torch.zeros(p.n_cols, 8, dtype=torch.float64, device=d)
    G = torch.zeros(p.n_rows, 8, dtype=torch.float64, device=d)
    bad_row = p.row.copy()
    bad_row[123] = p.n_rows
    pipe.step(torch.from_numpy(bad_row).to(d), torch.from_numpy(p.col).to(d),
              torch.from_numpy(p.val).to(d), X, G)
    _, st_a, st_p = pipe.status()
    assert st_a == oracle.EBOUNDS
    assert st_p == 0
    pipe.step(torch.from_numpy(p.row).to(d), torch.from_numpy(p.col).to(d),
              torch.from_numpy(p.val).to(d), X, G)
    nnz, st_a, st_p = pipe.status()
    assert (st_a, st_p) == (0, 0)
    st, R = oracle.coo_to_csc(p.n_rows, p.n_cols, p.row, p.col, p.val)
    assert st == oracle.OK
    assert nnz == R.nnz
    assert np.array_equal(pipe.col_ptr.cpu().numpy(), R.col_ptr)
    assert np.array_equal(pipe.row_idx[:nnz].cpu().numpy(), R.row_idx)
    assert np.array_equal(pipe.values[:nnz].cpu().numpy(), R.values)
