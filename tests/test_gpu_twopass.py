"""Level 1 in two passes (super-buckets, then buckets): inputs with more than 4096 coarse
buckets, for assembly, the plan build, the fused call and batch insertion, with binary64 and
binary32 values, bit for bit against the oracle and against the two-call build."""
import numpy as np
import pytest
import torch

import oracle
from paper_1805_03380_amd import ops, synth
from gpu_util import assemble_gpu, assert_csc_equal, dev
from test_gpu_fused import _both, _check_plan_oracle

pytestmark = pytest.mark.gpu


def _many(seed, dtype):
    """200,000 x 150,000 from 6e6 triplets (20 % duplicates, 1 % zeros): about 6,000 column
    buckets and 6,000 row buckets, both above the two-pass threshold."""
    return synth.random_coo(seed, 200_000, 150_000, 6_000_000, dup_frac=0.2, zero_frac=0.01,
                            dtype=dtype, dist="normal")


@pytest.mark.parametrize("dtype", [np.float64, np.float32])
def test_two_pass_assembly_and_plan(dtype):
    p = _many(6200, dtype)
    B, vp, nnz, st = _both(p)
    assert st == 0
    _check_plan_oracle(B, p)


def test_two_pass_binary64_to_binary32():
    p = _many(6201, np.float64)
    print("case two-pass f64 -> f32", flush=True)
    A = assemble_gpu(p, out_dtype=torch.float32)
    st, R = oracle.coo_to_csc(p.n_rows, p.n_cols, p.row, p.col, p.val)
    assert_csc_equal(A, R, np.float32)


def test_two_pass_insertion():
    p = _many(6202, np.float64)
    A = assemble_gpu(p)
    q = synth.random_coo(6203, p.n_rows, p.n_cols, 1_500_000, dup_frac=0.1, dist="normal")
    print("case two-pass insertion", flush=True)
    I = ops.csc_insert(A, dev(q.row), dev(q.col), dev(q.val))
    n = A.nnz
    Ah = oracle.CSC(A.n_rows, A.n_cols, A.col_ptr.cpu().numpy(), A.row_idx_buf[:n].cpu().numpy(),
                    oracle.widen(A.values_buf[:n].cpu()))
    st, R = oracle.csc_insert(Ah, q.row, q.col, q.val)
    assert st == oracle.OK
    assert_csc_equal(I, R, np.float64)
