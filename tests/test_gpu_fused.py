"""GPU parity of assembly and plan in one call (spm_coo_to_csc_plan).

Its outputs must equal, bit for bit, those of spm_coo_to_csc followed by spm_csc_plan_build
(with the values carried to plan order), on shapes that take the fused grouping and on
shapes that fall back to the two builds; the plan is also checked against the oracle's CSC
sorted by row, and the products of a pipeline step must not depend on which way the plan
was built.
"""
import numpy as np
import pytest
import torch

import oracle
from paper_1805_03380_amd import ops, synth
from paper_1805_03380_amd.pipeline import Pipeline
from gpu_util import DEV, assert_csc_equal, dev

pytestmark = pytest.mark.gpu


def _bits(t):
    t = t.contiguous()
    return t.view(torch.int32) if t.element_size() == 4 else t.view(torch.int64)


def _both(p, val_dtype=None, out_dtype=None, with_vplan=True):
    """Run the separate and the fused builds on the same triplets; assert they agree and
    return (fused CSC, fused plan-order values, nnz, assembly status)."""
    row, col = dev(p.row), dev(p.col)
    v = dev(p.val, val_dtype)
    shape = (p.n_rows, p.n_cols)
    print("case %s %dx%d nnz_in=%d val=%s out=%s" % (p.name, p.n_rows, p.n_cols, p.nnz_in,
                                                      v.dtype, out_dtype), flush=True)
    A = ops.coo_to_csc(row, col, v, shape, out_dtype=out_dtype, sync=False)
    vp_s = torch.empty_like(A.values_buf) if with_vplan else None
    plan_s = ops.build_plan(A, check=False, values=A.values_buf if with_vplan else None,
                            values_plan=vp_s)
    B, vp_f = ops.coo_to_csc_plan(row, col, v, shape, out_dtype=out_dtype,
                                  values_plan=with_vplan, sync=False)
    torch.cuda.synchronize()
    ia, ib = A.info.cpu().tolist(), B.info.cpu().tolist()
    assert ia == ib, (ia, ib)
    nnz, st = ib
    assert B.plan_info.cpu().tolist() == [nnz, 0]
    assert torch.equal(A.col_ptr, B.col_ptr)
    assert torch.equal(A.row_idx_buf[:nnz], B.row_idx_buf[:nnz])
    assert torch.equal(_bits(A.values_buf[:nnz]), _bits(B.values_buf[:nnz]))
    cap = p.nnz_in
    rs, cs, ps = ops.plan_arrays(plan_s, p.n_rows, cap)
    rf, cf, pf = ops.plan_arrays(B.plan(), p.n_rows, cap)
    assert torch.equal(rs, rf), "row_ptr differs"
    assert torch.equal(cs[:nnz], cf[:nnz]), "col_t differs"
    assert torch.equal(ps[:nnz], pf[:nnz]), "perm differs"
    if with_vplan:
        assert torch.equal(_bits(vp_s[:nnz]), _bits(vp_f[:nnz])), "plan-order values differ"
        assert torch.equal(_bits(vp_f[:nnz]), _bits(B.values_buf[:nnz][pf[:nnz].long()]))
    else:
        assert vp_f is None
    return B, vp_f, nnz, st


def _check_plan_oracle(B, p):
    st, R = oracle.coo_to_csc(p.n_rows, p.n_cols, p.row, p.col, p.val)
    assert st == oracle.OK
    assert_csc_equal(B, R, B.values_buf.cpu().numpy().dtype)
    row_ptr, col_t, perm = ops.plan_arrays(B.plan(), p.n_rows, p.nnz_in)
    cols = np.repeat(np.arange(R.n_cols), np.diff(R.col_ptr))
    order = np.lexsort((cols, R.row_idx))
    rp = np.zeros(R.n_rows + 1, np.int64)
    np.add.at(rp, R.row_idx + 1, 1)
    assert np.array_equal(row_ptr.cpu().numpy(), np.cumsum(rp))
    assert np.array_equal(col_t[:R.nnz].cpu().numpy(), cols[order])
    assert np.array_equal(perm[:R.nnz].cpu().numpy(), order)


@pytest.mark.parametrize("val_dtype,out_dtype", [
    (torch.float32, torch.float32), (torch.float64, torch.float64),
    (torch.float64, torch.float32), (torch.float32, torch.float64),
    (torch.bfloat16, torch.float32)])
def test_fused_random(val_dtype, out_dtype):
    p = synth.random_coo(41, 1000, 1200, 20_000, dup_frac=0.2, zero_frac=0.05, dist="normal")
    B, _, _, st = _both(p, val_dtype, out_dtype)
    assert st == 0
    if val_dtype == torch.float64:
        _check_plan_oracle(B, p)


def test_fused_uniform_1e5():
    """The full-size uniform workload (1e5 x 1e5, 1e6 triplets, binary32 values)."""
    p = synth.uniform_1e5(value_dtype=np.float32, k=0)
    B, _, nnz, st = _both(p)
    assert st == 0
    _check_plan_oracle(B, p)


def test_fused_without_plan_values():
    p = synth.random_coo(42, 3000, 500, 30_000, dup_frac=0.1)
    _both(p, torch.float64, torch.float64, with_vplan=False)


def test_fused_dense_row_and_column():
    """A row and a column longer than one in-LDS bucket: both groupings take their staged
    level-2 path for that bucket."""
    rng = np.random.Generator(np.random.PCG64(43))
    n = 30_000
    row = np.concatenate([np.full(12_000, 5), rng.permutation(20_000)[:10_000],
                          rng.integers(0, 20_000, n)]).astype(np.int32)
    col = np.concatenate([rng.permutation(20_000)[:12_000], np.full(10_000, 7),
                          rng.integers(0, 20_000, n)]).astype(np.int32)
    p = synth.COOProblem("dense_rc", 20_000, 20_000, row, col, rng.standard_normal(row.size))
    B, _, _, st = _both(p, torch.float64, torch.float64)
    assert st == 0
    _check_plan_oracle(B, p)


def test_fused_few_rows():
    """Few rows, long rows: row buckets hold many elements each."""
    rng = np.random.Generator(np.random.PCG64(44))
    n = 40_000
    row = rng.integers(0, 100, n).astype(np.int32)
    col = rng.integers(0, 20_000, n).astype(np.int32)
    p = synth.COOProblem("few_rows", 100, 20_000, row, col, rng.standard_normal(n))
    B, _, _, st = _both(p, torch.float64, torch.float32)
    assert st == 0


def test_fused_fallback_many_row_buckets():
    """More row buckets than the fused emit keeps cursors for: the two builds run in turn."""
    p = synth.random_coo(45, 300_000, 2000, 4_000_000, dup_frac=0.05)
    _, _, _, st = _both(p, torch.float32, torch.float32)
    assert st == 0


def test_fused_out_of_range_triplets():
    p = synth.random_coo(46, 800, 900, 10_000, dup_frac=0.1)
    row = p.row.copy()
    col = p.col.copy()
    row[17] = p.n_rows
    col[4000] = -3
    q = synth.COOProblem("oob", p.n_rows, p.n_cols, row, col, p.val)
    _, _, nnz, st = _both(q, torch.float64, torch.float64)
    assert st == oracle.EBOUNDS
    keep = ~(np.arange(q.nnz_in) == 17) & ~(np.arange(q.nnz_in) == 4000)
    st_o, R = oracle.coo_to_csc(q.n_rows, q.n_cols, row[keep], col[keep], q.val[keep])
    assert st_o == oracle.OK
    assert nnz == R.nnz


def test_fused_total_cancellation():
    """Every position sums to exactly zero: nnz_out = 0, an empty plan."""
    rng = np.random.Generator(np.random.PCG64(47))
    m = 5000
    lin = rng.choice(700 * 600, size=m, replace=False)  # distinct: each sum is v - v = 0
    r = (lin % 700).astype(np.int32)
    c = (lin // 700).astype(np.int32)
    v = rng.standard_normal(m)
    p = synth.COOProblem("cancel", 700, 600, np.concatenate([r, r]), np.concatenate([c, c]),
                         np.concatenate([v, -v]))
    B, _, nnz, st = _both(p, torch.float64, torch.float64)
    assert (nnz, st) == (0, 0)
    rp, _, _ = ops.plan_arrays(B.plan(), p.n_rows, p.nnz_in)
    assert int(rp.abs().sum()) == 0


@pytest.mark.parametrize("shape", [(5, 7), (1, 1), (5, 0), (0, 5)])
def test_fused_empty(shape):
    p = synth.COOProblem("empty", shape[0], shape[1], np.zeros(0, np.int32),
                         np.zeros(0, np.int32), np.zeros(0))
    _, _, nnz, st = _both(p, torch.float64, torch.float64)
    assert (nnz, st) == (0, 0)


def test_fused_single_row_and_column():
    rng = np.random.Generator(np.random.PCG64(48))
    for n_rows, n_cols in ((1, 5000), (5000, 1)):
        m = 8000
        p = synth.COOProblem("line", n_rows, n_cols,
                             rng.integers(0, n_rows, m).astype(np.int32),
                             rng.integers(0, n_cols, m).astype(np.int32), rng.standard_normal(m))
        B, _, _, st = _both(p, torch.float64, torch.float64)
        assert st == 0
        _check_plan_oracle(B, p)


@pytest.mark.parametrize("csc_dtype", [torch.float32, torch.float64])
def test_pipeline_fused_equals_separate(csc_dtype):
    """Two steps of the fused pipeline, each bitwise equal to the separate pipeline's step."""
    p = synth.random_coo(49, 5000, 4000, 100_000, dup_frac=0.1, k=64,
                         dtype=np.float32 if csc_dtype == torch.float32 else np.float64)
    d = DEV
    row, col, val = dev(p.row), dev(p.col), dev(p.val)
    X, G = dev(p.X), dev(p.G)
    pf = Pipeline(p.n_rows, p.n_cols, p.nnz_in, 64, val_dtype=val.dtype, x_dtype=X.dtype,
                  fused=True)
    ps = Pipeline(p.n_rows, p.n_cols, p.nnz_in, 64, val_dtype=val.dtype, x_dtype=X.dtype,
                  fused=False)
    ps.step(row, col, val, X, G)
    for it in range(2):
        pf.step(row, col, val, X, G)
        torch.cuda.synchronize(d)
        assert pf.status() == ps.status()
        nnz = pf.status()[0]
        assert torch.equal(pf.col_ptr, ps.col_ptr)
        assert torch.equal(pf.row_idx[:nnz], ps.row_idx[:nnz])
        for a, b in ((pf.values, ps.values), (pf.values_plan, ps.values_plan),
                     (pf.dval, ps.dval)):
            assert torch.equal(_bits(a[:nnz]), _bits(b[:nnz]))
        assert torch.equal(_bits(pf.Y), _bits(ps.Y))
        assert torch.equal(_bits(pf.dX), _bits(ps.dX))
