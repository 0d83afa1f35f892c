"""GPU parity of the plan (spm_csc_plan_build), the forward product (spm_csc_spmm) and the
fused adjoint (spm_csc_spmm_backward) against the oracle."""
import numpy as np
import pytest
import torch

import oracle
from paper_1805_03380_amd import ops, synth
from gpu_util import assemble_gpu, assert_close, dev

pytestmark = pytest.mark.gpu


def _ref(p):
    st, A = oracle.coo_to_csc(p.n_rows, p.n_cols, p.row, p.col, p.val)
    assert st == oracle.OK
    return A


def _check_plan(A_gpu, R):
    plan = A_gpu.plan()
    row_ptr, col_t, perm = ops.plan_arrays(plan, A_gpu.n_rows, A_gpu.nnz_cap)
    # reference CSR of the oracle's pattern: stable sort of the CSC slots by row
    cols = np.repeat(np.arange(R.n_cols), np.diff(R.col_ptr))
    order = np.lexsort((cols, R.row_idx))
    rp = np.zeros(R.n_rows + 1, np.int64)
    np.add.at(rp, R.row_idx + 1, 1)
    rp = np.cumsum(rp)
    assert np.array_equal(row_ptr.cpu().numpy(), rp)
    n = R.nnz
    assert np.array_equal(col_t[:n].cpu().numpy(), cols[order])
    assert np.array_equal(perm[:n].cpu().numpy(), order)


def _run(p, value_dtype, x_dtype, check_bitwise_f32=True, acc_f32=False, g_dtype=None):
    """g_dtype: G's own element type (default: X's); G is never converted to X's type."""
    R = _ref(p)
    A = assemble_gpu(p, val_dtype=None)
    vals = A.values_buf if value_dtype is None else A.values_buf.to(value_dtype)
    X = dev(p.X).to(x_dtype)
    Gm = dev(p.G).to(x_dtype if g_dtype is None else g_dtype)
    Y = ops.spmm(A, X, values=vals)
    dX, dval = ops.spmm_backward(A, Gm, X, values=vals)
    torch.cuda.synchronize()
    # oracle on exactly the operands the kernels saw (values rounded to their storage type)
    rv = oracle.widen(vals[: A.nnz].cpu())
    Xh, Gh = oracle.widen(X.cpu()), oracle.widen(Gm.cpu())
    Yr, S, M = oracle.spmm(R, Xh, values=rv)
    dXr, dvr, SdX, Sdv = oracle.spmm_backward(R, Gh, Xh, values=rv)
    out_t = Y.dtype
    # binary32 sums only when a dense operand of that call is bfloat16 and none of its
    # operands is binary64: the forward sees values and X, the adjoint values, G and X
    f64 = torch.float64
    fwd_f32 = acc_f32 and vals.dtype != f64 and X.dtype == torch.bfloat16
    bwd_f32 = acc_f32 and f64 not in (vals.dtype, Gm.dtype, X.dtype)
    assert_close(Y, Yr, S, M, out_t, fwd_f32, "Y")
    colcnt = np.diff(R.col_ptr)
    assert_close(dX, dXr, SdX, colcnt, dX.dtype, bwd_f32, "dX")
    assert_close(dval, dvr, Sdv, p.k, dval.dtype, bwd_f32, "dval")
    if check_bitwise_f32 and out_t == torch.float32 and not acc_f32 and \
            vals.dtype == torch.float32 and x_dtype == torch.float32 and \
            Gm.dtype == torch.float32:
        # binary32 operands, binary64 accumulation in the oracle's order: the products are
        # exact, so Y and dX round to exactly the oracle's values
        assert np.array_equal(Y.cpu().numpy(), Yr.astype(np.float32))
        assert np.array_equal(dX.cpu().numpy(), dXr.astype(np.float32))
    return A, R


def test_plan_matches_csr():
    p = synth.random_coo(3, 3000, 2000, 60_000, dup_frac=0.1, dist="normal")
    A = assemble_gpu(p)
    _check_plan(A, _ref(p))


def test_plan_giant_row():
    rng = np.random.Generator(np.random.PCG64(8))
    n = 30_000
    row = np.concatenate([np.full(12_000, 5), rng.integers(0, 100, n)]).astype(np.int32)
    col = np.concatenate([rng.permutation(20_000)[:12_000],
                          rng.integers(0, 20_000, n)]).astype(np.int32)
    p = synth.COOProblem("gr", 100, 20_000, row, col, rng.standard_normal(row.size))
    A = assemble_gpu(p)
    _check_plan(A, _ref(p))


def _plan_values_case(p, value_dtype, k):
    """Values carried to plan order by the plan build: exactly values[perm], and a forward
    product reading them (order="plan") bitwise equal to the CSC-order product."""
    A = assemble_gpu(p)
    vals = A.values_buf.to(value_dtype)
    vplan = torch.empty_like(vals)
    plan = ops.build_plan(A, values=vals, values_plan=vplan)
    _, _, perm = ops.plan_arrays(plan, A.n_rows, A.nnz_cap)
    n = A.nnz
    pm = perm[:n].long()
    assert torch.equal(vplan[:n], vals[pm])
    rng = np.random.Generator(np.random.PCG64(77))
    X = dev(rng.standard_normal((A.n_cols, k)), torch.float32)
    Y_csc = ops.spmm(A, X, values=vals, plan=plan)
    Y_plan = ops.spmm(A, X, values=vplan, plan=plan, order="plan")
    torch.cuda.synchronize()
    assert torch.equal(Y_csc, Y_plan)


@pytest.mark.parametrize("value_dtype", [torch.float32, torch.float64])
@pytest.mark.parametrize("k", [64, 5])
def test_plan_order_values(value_dtype, k):
    p = synth.random_coo(31, 3000, 2000, 60_000, dup_frac=0.1, dist="normal")
    _plan_values_case(p, value_dtype, k)


def test_plan_order_values_giant_row():
    """A row longer than one in-LDS bucket: its values are gathered on the staged path."""
    rng = np.random.Generator(np.random.PCG64(9))
    n = 30_000
    row = np.concatenate([np.full(12_000, 5), rng.integers(0, 100, n)]).astype(np.int32)
    col = np.concatenate([rng.permutation(20_000)[:12_000],
                          rng.integers(0, 20_000, n)]).astype(np.int32)
    p = synth.COOProblem("grv", 100, 20_000, row, col, rng.standard_normal(row.size))
    _plan_values_case(p, torch.float64, 64)


def test_plan_order_requires_values():
    p = synth.random_coo(32, 50, 40, 300)
    A = assemble_gpu(p)
    with pytest.raises(ValueError):
        ops.spmm(A, dev(np.ones((40, 4)), torch.float32), order="plan")


def test_tiny_spmv_f64():
    p = synth.tiny_spmv()
    A, R = _run(p, None, torch.float64)
    _check_plan(A, R)


@pytest.mark.parametrize("k", [1, 3, 4, 5, 16, 31, 64, 128, 300])
def test_widths_f32(k):
    p = synth.random_coo(40 + k, 700, 900, 20_000, dup_frac=0.1, dtype=np.float32, dist="normal",
                         k=k)
    _run(p, None, torch.float32)


@pytest.mark.parametrize("k", [2, 8, 64])
def test_widths_f64(k):
    p = synth.random_coo(60 + k, 500, 400, 8_000, dup_frac=0.1, dtype=np.float64, dist="normal",
                         k=k)
    _run(p, None, torch.float64)


def test_mixed_f64_values_f32_dense():
    """Binary64 values, binary32 X: Y is binary64, so G arrives in binary64 and is read as
    such; dvalues (binary64) meet the binary64 bound with the unrounded G."""
    p = synth.random_coo(71, 800, 800, 16_000, dup_frac=0.05, dtype=np.float64, k=64)
    p.X = p.X.astype(np.float32)
    _run(p, None, torch.float32, g_dtype=torch.float64)


@pytest.mark.parametrize("k", [5, 64, 128])
def test_g_f64_x_f32_values_f32(k):
    """Binary32 values and X with a binary64 G (a caller whose loss is in binary64)."""
    p = synth.random_coo(73 + k, 900, 700, 18_000, dup_frac=0.05, dtype=np.float32,
                         dist="normal", k=k)
    _run(p, None, torch.float32, g_dtype=torch.float64)


def test_g_f32_x_bf16():
    """A bfloat16 X gives a binary32 Y, so G arrives in binary32: read as binary32 (binary32
    accumulation, as for any bfloat16 operand)."""
    p = synth.random_coo(74, 1000, 1200, 30_000, dup_frac=0.1, dtype=np.float32, dist="normal",
                         k=32)
    _run(p, None, torch.bfloat16, acc_f32=True, g_dtype=torch.float32)


def test_g_f64_x_bf16_f64_accumulation():
    """A binary64 G with a bfloat16 X: binary64 takes part in the adjoint, so its sums run in
    binary64 (the forward, on binary32 values and a bfloat16 X, sums in binary32)."""
    p = synth.random_coo(75, 600, 500, 9_000, dup_frac=0.1, dtype=np.float32, dist="normal",
                         k=64)
    _run(p, None, torch.bfloat16, acc_f32=True, g_dtype=torch.float64)


def test_bf16_dense_f32_accumulation():
    p = synth.random_coo(72, 1000, 1200, 30_000, dup_frac=0.1, dtype=np.float32, dist="normal",
                         k=32)
    _run(p, None, torch.bfloat16, acc_f32=True)


def test_uniform_1e5_f32_k64():
    p = synth.uniform_1e5(value_dtype=np.float32, k=64)
    _run(p, None, torch.float32)


def test_uniform_1e5_f64_values():
    """The 1e5 workload with binary64 values: X binary32, G N(0,1) in the output type
    (binary64), unrounded; binary64 dvalues within 1e-12 relative plus the a-priori slack."""
    p = synth.uniform_1e5(value_dtype=np.float64, k=64)
    assert p.G.dtype == np.float64
    _run(p, None, torch.float32, g_dtype=torch.float64)


def test_deterministic_and_empty_rows():
    p = synth.random_coo(81, 5000, 300, 2000, dup_frac=0.0, dtype=np.float32, dist="normal",
                         k=64)
    A = assemble_gpu(p)
    X = dev(p.X)
    Y1 = ops.spmm(A, X)
    Y2 = ops.spmm(A, X)
    assert torch.equal(Y1, Y2)
    Gm = dev(p.G)
    a1, b1 = ops.spmm_backward(A, Gm, X)
    a2, b2 = ops.spmm_backward(A, Gm, X)
    assert torch.equal(a1, a2) and torch.equal(b1, b2)
    # rows with no stored element are exactly zero
    R = _ref(p)
    empty = np.setdiff1d(np.arange(p.n_rows), R.row_idx)
    assert empty.size > 0
    assert torch.all(Y1[torch.from_numpy(empty).to(Y1.device)] == 0)


def test_identity_gives_x_exactly():
    n, k = 4096, 64
    idx = np.arange(n, dtype=np.int32)
    p = synth.COOProblem("eye", n, n, idx, idx, np.ones(n, np.float32))
    A = assemble_gpu(p)
    torch.manual_seed(0)
    X = torch.randn(n, k, device="cuda:0")
    assert torch.equal(ops.spmm(A, X), X)
    dX, dval = ops.spmm_backward(A, X, X)
    assert torch.equal(dX, X)
