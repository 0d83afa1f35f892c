"""Differentiation through the hand-written adjoint (CscSpmm): gradcheck, central finite
differences in binary64, agreement with the oracle gradient, the adjoint identity, and the
full-size differentiation workload."""
import math

import numpy as np
import pytest
import torch

import oracle
from paper_1805_03380_amd import synth
from paper_1805_03380_amd.autograd import csc_spmm
from gpu_util import assemble_gpu, assert_close, dev

pytestmark = pytest.mark.gpu


def test_gradcheck_f64():
    p = synth.random_coo(501, 20, 15, 40, dup_frac=0.1, dist="normal", k=3)
    A = assemble_gpu(p)
    v = A.values.clone().requires_grad_(True)
    X = dev(p.X).requires_grad_(True)
    assert torch.autograd.gradcheck(lambda vv, xx: csc_spmm(A, vv, xx), (v, X), eps=1e-6,
                                    atol=1e-9, rtol=1e-7)


def test_central_fd_2000():
    """L = sum(A.X * G) is bilinear in (values, X): central differences with h = 2^-4 have
    no truncation error, so only the rounding of L remains."""
    p = synth.diff_fd()
    A = assemble_gpu(p)
    v = A.values.clone().requires_grad_(True)
    X = dev(p.X).requires_grad_(True)
    G = dev(p.G)
    L = (csc_spmm(A, v, X) * G).sum()
    L.backward()
    dv, dX = v.grad.detach(), X.grad.detach()
    h = 2.0 ** -4

    def loss(vv, xx):
        with torch.no_grad():
            return float((csc_spmm(A, vv, xx) * G).sum())

    rng = np.random.Generator(np.random.PCG64(77))
    v0, X0 = v.detach(), X.detach()
    for q in rng.choice(A.nnz, 16, replace=False):
        vp, vm = v0.clone(), v0.clone()
        vp[q] += h
        vm[q] -= h
        fd = (loss(vp, X0) - loss(vm, X0)) / (2 * h)
        assert abs(fd - float(dv[q])) <= 1e-8 * abs(float(dv[q])) + 1e-10
    for _ in range(16):
        c, j = int(rng.integers(p.n_cols)), int(rng.integers(p.k))
        Xp, Xm = X0.clone(), X0.clone()
        Xp[c, j] += h
        Xm[c, j] -= h
        fd = (loss(v0, Xp) - loss(v0, Xm)) / (2 * h)
        assert abs(fd - float(dX[c, j])) <= 1e-8 * abs(float(dX[c, j])) + 1e-10
    # and the oracle gradient
    st, R = oracle.coo_to_csc(p.n_rows, p.n_cols, p.row, p.col, p.val)
    dXr, dvr, SdX, Sdv = oracle.spmm_backward(R, p.G, p.X)
    assert_close(dX, dXr, SdX, np.diff(R.col_ptr), torch.float64, what="dX")
    assert_close(dv, dvr, Sdv, p.k, torch.float64, what="dval")
    # adjoint identity <A.X, G> = <X, A^T.G> = <values, dvalues>
    Y = csc_spmm(A, v0, X0)
    a = math.fsum((Y * G).double().flatten().cpu().tolist())
    b = math.fsum((X0 * dX).double().flatten().cpu().tolist())
    c = math.fsum((v0 * dv).double().cpu().tolist())
    scale = float((torch.abs(Y) * torch.abs(G)).sum()) + 1.0
    assert abs(a - b) <= 1e-12 * scale and abs(a - c) <= 1e-12 * scale


def test_diff_workload_full_f32():
    """200,000 x 200,000, 5,000,000 uniform triplets, k = 64, float32: Y, dX and dval against
    the oracle everywhere."""
    p = synth.diff_2e5()
    A = assemble_gpu(p)
    st, R = oracle.coo_to_csc(p.n_rows, p.n_cols, p.row, p.col, p.val)
    assert A.nnz == R.nnz
    assert np.array_equal(A.row_idx.cpu().numpy(), R.row_idx)
    v = A.values.clone().requires_grad_(True)
    X = dev(p.X).requires_grad_(True)
    G = dev(p.G)
    Y = csc_spmm(A, v, X)
    Y.backward(G)
    torch.cuda.synchronize()
    rv = A.values.double().cpu().numpy()
    Yr, S, M = oracle.spmm(R, p.X, values=rv)
    assert_close(Y, Yr, S, M, torch.float32, what="Y")
    dXr, dvr, SdX, Sdv = oracle.spmm_backward(R, p.G, p.X, values=rv)
    assert_close(X.grad, dXr, SdX, np.diff(R.col_ptr), torch.float32, what="dX")
    assert_close(v.grad, dvr, Sdv, p.k, torch.float32, what="dval")


def test_needs_input_grad_skips_outputs():
    p = synth.random_coo(502, 300, 200, 3000, dist="normal", k=8, dtype=np.float32)
    A = assemble_gpu(p)
    v = A.values.clone()
    X = dev(p.X).requires_grad_(True)
    (csc_spmm(A, v, X) * 2).sum().backward()
    assert X.grad is not None and v.grad is None
    v2 = A.values.clone().requires_grad_(True)
    X2 = dev(p.X)
    csc_spmm(A, v2, X2).sum().backward()
    assert v2.grad is not None


def test_gradcheck_f64_values_f32_x():
    """Binary64 values with a binary32 X: Y and so G are binary64, and the adjoint reads G as
    binary64 (no narrowing to X's type), so the dvalues pass gradcheck at binary64 tolerances."""
    p = synth.random_coo(503, 24, 18, 60, dup_frac=0.1, dist="normal", k=5)
    A = assemble_gpu(p)
    v = A.values.clone().requires_grad_(True)
    X = dev(p.X, torch.float32)
    assert v.dtype == torch.float64
    assert torch.autograd.gradcheck(lambda vv: csc_spmm(A, vv, X), (v,), eps=1e-6, atol=1e-9,
                                    rtol=1e-7)


def test_f64_values_f32_x_oracle_gradient():
    """The same mixed case against the oracle: a binary64 G, unrounded, gives binary64
    dvalues within 1e-12 relative plus the oracle's own a-priori slack."""
    p = synth.random_coo(504, 3000, 2500, 40_000, dup_frac=0.05, dist="normal", k=64)
    A = assemble_gpu(p)
    v = A.values.clone().requires_grad_(True)
    X = dev(p.X, torch.float32).requires_grad_(True)
    G = dev(p.G)
    assert G.dtype == torch.float64
    csc_spmm(A, v, X).backward(G)
    torch.cuda.synchronize()
    st, R = oracle.coo_to_csc(p.n_rows, p.n_cols, p.row, p.col, p.val)
    Xh = oracle.widen(X.detach().cpu())
    dXr, dvr, SdX, Sdv = oracle.spmm_backward(R, p.G, Xh)
    assert v.grad.dtype == torch.float64 and X.grad.dtype == torch.float32
    assert_close(v.grad, dvr, Sdv, p.k, torch.float64, what="dval")
    assert_close(X.grad, dXr, SdX, np.diff(R.col_ptr), torch.float32, what="dX")
