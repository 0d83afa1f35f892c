"""GPU parity of the gradient with respect to each input triplet (spm_coo_triplet_grad) with
the oracle: every triplet, duplicates and locations that summed to zero included, within the
a-priori bound of a k-term dot product; triplets outside the matrix get 0.  Also the
differentiable assembly + product (autograd.coo_spmm) against the oracle and gradcheck."""
import numpy as np
import pytest
import torch

import oracle
from paper_1805_03380_amd import _lib, autograd, ops, synth
from gpu_util import DEV, assert_close, dev

pytestmark = pytest.mark.gpu


def _case(p, G, X, val_dtype, x_dtype, out_dtype=None, what="", g_dtype=None):
    """g_dtype: G's own element type (default: X's)."""
    g_dtype = x_dtype if g_dtype is None else g_dtype
    print("case %s %dx%d nnz_in=%d k=%d x=%s g=%s" % (p.name, p.n_rows, p.n_cols, p.nnz_in,
                                                      X.shape[1], x_dtype, g_dtype), flush=True)
    Gd, Xd = dev(G, g_dtype), dev(X, x_dtype)
    dv = ops.triplet_grad(dev(p.row), dev(p.col), Gd, Xd, (p.n_rows, p.n_cols),
                          val_dtype=val_dtype, out_dtype=out_dtype)
    want, S = oracle.triplet_grad(p.n_rows, p.n_cols, p.row, p.col, Gd.cpu(), Xd.cpu())
    dense = (g_dtype, x_dtype)
    acc_f32 = torch.bfloat16 in dense and torch.float64 not in dense + (val_dtype,)
    assert_close(dv, want, S, X.shape[1], dv.dtype, acc_f32=acc_f32, what=what)
    return dv, want


def _with_specials(seed, n_rows, n_cols, nnz, k):
    """Random triplets with duplicates, an exactly cancelling pair and out-of-range entries."""
    p = synth.random_coo(seed, n_rows, n_cols, nnz, dup_frac=0.3, dist="normal")
    row, col, val = p.row.copy(), p.col.copy(), p.val.copy()
    row[:2], col[:2], val[:2] = 1, 2, (0.75, -0.75)
    keep = np.ones(len(row), bool)
    keep[2:] = ~((row[2:] == 1) & (col[2:] == 2))
    row, col, val = row[keep], col[keep], val[keep]
    row[5], col[7], row[9] = n_rows, n_cols, -1
    rng = np.random.Generator(np.random.PCG64(seed + 1))
    G = rng.standard_normal((n_rows, k))
    X = rng.standard_normal((n_cols, k))
    return synth.COOProblem("specials", n_rows, n_cols, row, col, val), G, X


@pytest.mark.parametrize("k", [1, 3, 16, 64, 100, 300])
def test_triplet_grad_random(k):
    p, G, X = _with_specials(2100 + k, 900, 700, 20_000, k)
    dv, want = _case(p, G, X, torch.float64, torch.float64, what="k=%d" % k)
    assert torch.all(dv[[5, 7, 9]] == 0)
    assert dv[0] == dv[1] and want[0] == want[1] and dv[0] != 0


@pytest.mark.parametrize("val_dtype,x_dtype,out_dtype", [
    (torch.float32, torch.float32, torch.float32), (torch.float32, torch.bfloat16, None),
    (torch.float64, torch.bfloat16, None), (torch.float32, torch.float32, torch.float64)])
def test_triplet_grad_dtypes(val_dtype, x_dtype, out_dtype):
    p, G, X = _with_specials(2200, 1200, 1000, 30_000, 32)
    _case(p, G, X, val_dtype, x_dtype, out_dtype, what=str(x_dtype))


@pytest.mark.parametrize("val_dtype,g_dtype,x_dtype", [
    (torch.float64, torch.float64, torch.float32), (torch.float32, torch.float64, torch.float32),
    (torch.float32, torch.float32, torch.bfloat16), (torch.float64, torch.float64,
                                                     torch.bfloat16)])
def test_triplet_grad_g_own_dtype(val_dtype, g_dtype, x_dtype):
    """G in an element type of its own (Y's type), read as such."""
    p, G, X = _with_specials(2250, 1100, 900, 25_000, 64)
    _case(p, G, X, val_dtype, x_dtype, torch.float64 if torch.float64 in (val_dtype, g_dtype)
          else None, what="g=%s x=%s" % (g_dtype, x_dtype), g_dtype=g_dtype)


def test_triplet_grad_uniform_1e5():
    p = synth.uniform_1e5()
    _case(p, p.G, p.X, torch.float32, torch.float32, what="uniform 1e5")


def test_triplet_grad_equals_dvalues_without_duplicates():
    """Each triplet of a duplicate-free, zero-free input owns one CSC slot: its gradient and
    the adjoint's dvalues there are the same dot product (both within the bound)."""
    p = synth.random_coo(2300, 3000, 2000, 40_000, dup_frac=0.0, dist="normal")
    p.val[:] = np.abs(p.val) + 1.0
    rng = np.random.Generator(np.random.PCG64(2301))
    G = rng.standard_normal((p.n_rows, 64))
    X = rng.standard_normal((p.n_cols, 64))
    A = ops.coo_to_csc(dev(p.row), dev(p.col), dev(p.val), (p.n_rows, p.n_cols))
    _, dval = ops.spmm_backward(A, dev(G), dev(X), need_dX=False)
    dv = ops.triplet_grad(dev(p.row), dev(p.col), dev(G), dev(X), (p.n_rows, p.n_cols),
                          val_dtype=torch.float64)
    # slot of every triplet from the CSC arrays
    cp = A.col_ptr.cpu().numpy()
    ri = A.row_idx.cpu().numpy()
    key = np.repeat(np.arange(p.n_cols, dtype=np.int64), np.diff(cp)) * p.n_rows + ri
    slot = np.searchsorted(key, p.col.astype(np.int64) * p.n_rows + p.row)
    assert np.array_equal(key[slot], p.col.astype(np.int64) * p.n_rows + p.row)
    _, S = oracle.triplet_grad(p.n_rows, p.n_cols, p.row, p.col, G, X)
    a, b = dv.cpu().numpy(), dval.cpu().numpy()[slot]
    assert np.all(np.abs(a - b) <= 4.0 * float(oracle.gamma(64)) * S)


def test_triplet_grad_empty_and_arguments():
    z = torch.zeros(0, dtype=torch.int32, device=DEV)
    G = torch.zeros(4, 8, dtype=torch.float64, device=DEV)
    X = torch.zeros(3, 8, dtype=torch.float64, device=DEV)
    assert ops.triplet_grad(z, z, G, X, (4, 3)).numel() == 0
    lib = _lib.load()
    r = torch.zeros(2, dtype=torch.int32, device=DEV)
    dv = torch.zeros(2, dtype=torch.float64, device=DEV)
    args = [4, 3, 2, 8, r.data_ptr(), r.data_ptr(), _lib.F64, G.data_ptr(), 8, _lib.F64,
            X.data_ptr(), 8, _lib.F64, dv.data_ptr(), _lib.F64, None]
    for i, val, want in ((3, 0, _lib.EINVAL), (8, 7, _lib.EINVAL), (11, 7, _lib.EINVAL),
                         (6, _lib.BF16, _lib.EDTYPE), (14, _lib.BF16, _lib.EDTYPE),
                         (12, 9, _lib.EDTYPE), (9, 9, _lib.EDTYPE), (4, None, _lib.EINVAL),
                         (13, None, _lib.EINVAL), (2, 2 ** 31, _lib.EOVERFLOW),
                         (0, -1, _lib.EINVAL)):
        bad = list(args)
        bad[i] = val
        assert lib.spm_coo_triplet_grad(*bad) == want, i


def test_coo_spmm_autograd():
    """Y = assemble(row, col, val).X: dval per triplet and dX against the oracle."""
    p, G, X = _with_specials(2400, 500, 400, 8000, 16)
    inside = (p.row >= 0) & (p.row < p.n_rows) & (p.col >= 0) & (p.col < p.n_cols)
    q = synth.COOProblem("inside", p.n_rows, p.n_cols, p.row[inside], p.col[inside],
                         p.val[inside])
    val = dev(q.val).requires_grad_(True)
    Xd = dev(X).requires_grad_(True)
    Y = autograd.coo_spmm(dev(q.row), dev(q.col), val, Xd, (q.n_rows, q.n_cols))
    Y.backward(dev(G))
    want_v, S = oracle.triplet_grad(q.n_rows, q.n_cols, q.row, q.col, G, X)
    assert_close(val.grad, want_v, S, 16, torch.float64, what="dval")
    st, A = oracle.coo_to_csc(q.n_rows, q.n_cols, q.row, q.col, q.val)
    dX, _, SdX, _ = oracle.spmm_backward(A, G, X)
    m = np.diff(A.col_ptr)
    assert_close(Xd.grad, dX, SdX, m, torch.float64, what="dX")


def test_coo_spmm_autograd_f64_values_f32_x():
    """Binary64 triplet values with a binary32 X: Y and G are binary64; the per-triplet
    gradients (binary64) come from the binary64 G, unrounded, within the binary64 bound."""
    p, G, X = _with_specials(2450, 600, 500, 9000, 32)
    inside = (p.row >= 0) & (p.row < p.n_rows) & (p.col >= 0) & (p.col < p.n_cols)
    q = synth.COOProblem("inside", p.n_rows, p.n_cols, p.row[inside], p.col[inside],
                         p.val[inside])
    val = dev(q.val).requires_grad_(True)
    Xd = dev(X, torch.float32).requires_grad_(True)
    Y = autograd.coo_spmm(dev(q.row), dev(q.col), val, Xd, (q.n_rows, q.n_cols))
    assert Y.dtype == torch.float64
    Y.backward(dev(G))
    Xh = oracle.widen(Xd.detach().cpu())
    want_v, S = oracle.triplet_grad(q.n_rows, q.n_cols, q.row, q.col, G, Xh)
    assert val.grad.dtype == torch.float64
    assert_close(val.grad, want_v, S, 32, torch.float64, what="dval")
    st, A = oracle.coo_to_csc(q.n_rows, q.n_cols, q.row, q.col, q.val)
    dX, _, SdX, _ = oracle.spmm_backward(A, G, Xh)
    assert_close(Xd.grad, dX, SdX, np.diff(A.col_ptr), torch.float32, what="dX")


def test_coo_spmm_gradcheck():
    rng = np.random.Generator(np.random.PCG64(2500))
    n_rows, n_cols, n, k = 12, 9, 40, 3
    row = rng.integers(0, n_rows, n).astype(np.int32)
    col = rng.integers(0, n_cols, n).astype(np.int32)
    val = dev(rng.standard_normal(n)).requires_grad_(True)
    X = dev(rng.standard_normal((n_cols, k))).requires_grad_(True)
    r, c = dev(row), dev(col)
    assert torch.autograd.gradcheck(
        lambda v, x: autograd.coo_spmm(r, c, v, x, (n_rows, n_cols)), (val, X),
        eps=1e-6, atol=1e-8, rtol=1e-6)


@pytest.mark.parametrize("k", [1, 16, 64, 100])
def test_triplet_grad_csc_reads_dvalues(k):
    """The dvalues form: a triplet whose location is stored gets the adjoint's dvalue there bit
    for bit; a dropped location gets the dot product of the direct form bit for bit; outside
    the matrix 0; all within the bound of the oracle."""
    p, G, X = _with_specials(2600 + k, 1500, 1100, 30_000, k)
    inside = (p.row >= 0) & (p.row < p.n_rows) & (p.col >= 0) & (p.col < p.n_cols)
    row, col = dev(p.row), dev(p.col)
    Gd, Xd = dev(G), dev(X)
    A = ops.coo_to_csc(row, col, dev(p.val), (p.n_rows, p.n_cols), sync=False)
    info = A.info.cpu()
    assert int(info[1]) == oracle.EBOUNDS  # the out-of-range triplets, skipped
    A._nnz = int(info[0])
    _, dval = ops.spmm_backward(A, Gd, Xd, need_dX=False)
    dv = ops.triplet_grad_csc(row, col, A, dval, Gd, Xd)
    direct = ops.triplet_grad(row, col, Gd, Xd, (p.n_rows, p.n_cols), val_dtype=torch.float64)
    cp = A.col_ptr.cpu().numpy()
    ri = A.row_idx.cpu().numpy()
    key = np.repeat(np.arange(p.n_cols, dtype=np.int64), np.diff(cp)) * p.n_rows + ri
    tkey = p.col.astype(np.int64) * p.n_rows + p.row
    slot = np.searchsorted(key, tkey)
    slot_c = np.minimum(slot, max(len(key) - 1, 0))
    stored = inside & (slot < len(key)) & (key[slot_c] == tkey)
    got = dv.cpu().numpy()
    assert np.array_equal(got[stored].view(np.int64), dval.cpu().numpy()[slot[stored]].view(np.int64))
    dropped = inside & ~stored
    assert dropped.sum() >= 2  # the cancelling pair
    assert np.array_equal(got[dropped].view(np.int64), direct.cpu().numpy()[dropped].view(np.int64))
    assert np.all(got[~inside] == 0)
    want, S = oracle.triplet_grad(p.n_rows, p.n_cols, p.row, p.col, G, X)
    assert_close(dv, want, S, k, torch.float64, what="csc form k=%d" % k)


def test_triplet_grad_csc_uniform_1e5():
    p = synth.uniform_1e5()
    row, col = dev(p.row), dev(p.col)
    Gd, Xd = dev(p.G), dev(p.X)
    A = ops.coo_to_csc(row, col, dev(p.val), (p.n_rows, p.n_cols))
    _, dval = ops.spmm_backward(A, Gd, Xd, need_dX=False, dval_dtype=torch.float64)
    dv = ops.triplet_grad_csc(row, col, A, dval, Gd, Xd)
    want, S = oracle.triplet_grad(p.n_rows, p.n_cols, p.row, p.col, p.G, p.X)
    assert_close(dv, want, S, 64, torch.float64, what="csc form uniform")
