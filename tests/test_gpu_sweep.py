"""A seeded sweep over small random shapes (tall, wide, single row or column, ragged chunk
tails, dense and nearly empty) for the operations around the hot path, each against the
oracle: insertion, the sum, the transpose, trace(A^T B) and the gradient per triplet."""
import numpy as np
import pytest
import torch

import oracle
from paper_1805_03380_amd import ops, synth
from gpu_util import DEV, assemble_gpu, assert_close, assert_csc_equal, dev

pytestmark = pytest.mark.gpu


def _host(A):
    n = A.nnz
    return oracle.CSC(A.n_rows, A.n_cols, A.col_ptr.cpu().numpy(), A.row_idx_buf[:n].cpu().numpy(),
                      oracle.widen(A.values_buf[:n].cpu()))


def _shapes():
    rng = np.random.Generator(np.random.PCG64(5000))
    out = []
    for i in range(24):
        kind = i % 6
        if kind == 0:
            n_rows, n_cols = int(rng.integers(1, 40)), int(rng.integers(1, 40))
        elif kind == 1:
            n_rows, n_cols = 1, int(rng.integers(1, 3000))
        elif kind == 2:
            n_rows, n_cols = int(rng.integers(1, 3000)), 1
        elif kind == 3:
            n_rows, n_cols = int(rng.integers(100, 5000)), int(rng.integers(10, 100))
        elif kind == 4:
            n_rows, n_cols = int(rng.integers(10, 100)), int(rng.integers(100, 5000))
        else:
            n_rows, n_cols = int(rng.integers(1000, 20000)), int(rng.integers(1000, 20000))
        cells = n_rows * n_cols
        density = float(rng.choice([0.001, 0.05, 0.5]))
        nnz = int(min(cells // 2, max(1, round(density * cells)), 200_000))
        out.append((i, n_rows, n_cols, nnz))
    return out


@pytest.mark.parametrize("case", _shapes(), ids=lambda c: "s%d_%dx%d" % (c[0], c[1], c[2]))
def test_sweep(case):
    i, n_rows, n_cols, nnz = case
    print("case sweep %d %dx%d nnz=%d" % case, flush=True)
    pa = synth.random_coo(5100 + i, n_rows, n_cols, nnz, dup_frac=0.2, dist="normal")
    pb = synth.random_coo(5200 + i, n_rows, n_cols, nnz, dup_frac=0.2, dist="normal")
    A, B = assemble_gpu(pa), assemble_gpu(pb)
    Ah, Bh = _host(A), _host(B)
    # insertion of B's triplets into A
    I = ops.csc_insert(A, dev(pb.row), dev(pb.col), dev(pb.val))
    st, R = oracle.csc_insert(Ah, pb.row, pb.col, pb.val)
    assert st == oracle.OK
    assert_csc_equal(I, R, np.float64)
    # the sum
    S = ops.csc_add(A, B)
    st, R = oracle.csc_add(Ah, Bh)
    assert st == oracle.OK
    assert_csc_equal(S, R, np.float64)
    # the transpose
    T = ops.csc_transpose(A)
    st, R = oracle.csc_transpose(Ah)
    assert st == oracle.OK
    assert_csc_equal(T, R, np.float64)
    # trace(A^T B)
    t, hits = ops.trace_atb(A, B)
    st, want, want_hits = oracle.trace_atb(Ah, Bh)
    assert st == oracle.OK and hits == want_hits
    Aa = oracle.CSC(Ah.n_rows, Ah.n_cols, Ah.col_ptr, Ah.row_idx, np.abs(Ah.values))
    Ba = oracle.CSC(Bh.n_rows, Bh.n_cols, Bh.col_ptr, Bh.row_idx, np.abs(Bh.values))
    _, s_abs, _ = oracle.trace_atb(Aa, Ba)
    assert abs(t - want) <= 2.0 * float(oracle.gamma(want_hits + 1)) * s_abs
    # the gradient per triplet, both forms
    k = 1 + i % 7 * 9
    rng = np.random.Generator(np.random.PCG64(5300 + i))
    G = rng.standard_normal((n_rows, k))
    X = rng.standard_normal((n_cols, k))
    Gd, Xd = dev(G), dev(X)
    dv = ops.triplet_grad(dev(pa.row), dev(pa.col), Gd, Xd, (n_rows, n_cols),
                          val_dtype=torch.float64)
    want, S_ = oracle.triplet_grad(n_rows, n_cols, pa.row, pa.col, G, X)
    assert_close(dv, want, S_, k, torch.float64, what="direct")
    _, dval = ops.spmm_backward(A, Gd, Xd, need_dX=False)
    dv2 = ops.triplet_grad_csc(dev(pa.row), dev(pa.col), A, dval, Gd, Xd)
    assert_close(dv2, want, S_, k, torch.float64, what="from dvalues")
