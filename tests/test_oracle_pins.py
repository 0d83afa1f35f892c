"""The oracle against what the paper and the mathematics fix (CPU only)."""
import numpy as np
import pytest
from hypothesis import given, settings, strategies as st

import oracle
import pins


@pytest.mark.parametrize("pin", pins.ALL_PINS, ids=lambda f: f.__name__)
def test_pin(pin):
    pin()


_special = st.sampled_from([0.0, -0.0, 1.0, -1.0, 0.5, -0.5, 1e300, -1e300, float("inf"),
                            float("-inf"), float("nan"), 5e-324])


@settings(max_examples=200, deadline=None)
@given(data=st.data())
def test_property_brute_force(data):
    """Random shapes 1..64, duplicates, +-0, cancelling pairs, NaN and Inf: both oracle reads
    equal the dense brute-force fold bit for bit."""
    n_rows = data.draw(st.integers(1, 64))
    n_cols = data.draw(st.integers(1, 64))
    nnz = data.draw(st.integers(0, 80))
    rows = data.draw(st.lists(st.integers(0, n_rows - 1), min_size=nnz, max_size=nnz))
    cols = data.draw(st.lists(st.integers(0, n_cols - 1), min_size=nnz, max_size=nnz))
    vals = data.draw(st.lists(st.one_of(_special, st.floats(-10, 10)), min_size=nnz, max_size=nnz))
    row = np.array(rows, np.int32)
    col = np.array(cols, np.int32)
    val = np.array(vals, np.float64)
    ecp, er, ev = pins.brute_force_csc(n_rows, n_cols, row, col, val)
    for method in ("sort", "rbt"):
        s, A = oracle.coo_to_csc(n_rows, n_cols, row, col, val, method=method)
        assert s == oracle.OK
        assert np.array_equal(A.col_ptr, ecp)
        assert np.array_equal(A.row_idx, er)
        assert pins.same_floats(A.values, ev)


@pytest.mark.parametrize("seed", [1, 2, 3])
def test_rbt_equals_sort_medium(seed):
    """The red-black-tree read and the stable-sort read agree bit for bit at 10^5 triplets."""
    from paper_1805_03380_amd import synth
    p = synth.random_coo(seed, 3000, 2000, 100_000, dup_frac=0.3, zero_frac=0.02, dist="normal")
    s1, A = oracle.coo_to_csc(p.n_rows, p.n_cols, p.row, p.col, p.val, method="sort")
    s2, B = oracle.coo_to_csc(p.n_rows, p.n_cols, p.row, p.col, p.val, method="rbt")
    assert s1 == s2 == oracle.OK
    assert np.array_equal(A.col_ptr, B.col_ptr)
    assert np.array_equal(A.row_idx, B.row_idx)
    assert pins.same_floats(A.values, B.values)
    oracle.check_csc_invariants(A)


def test_float32_fold_never_rounds_to_zero():
    """Reading for float32 output: fold in binary64, round once.  A non-zero binary64 sum of
    float32 values is a multiple of 2^-149, so its float32 rounding is never 0."""
    tiny = np.float32(2.0 ** -149)
    vals = np.array([np.float32(3 * 2.0 ** -149), np.float32(-2.0 ** -148)], np.float32)
    s, A = oracle.coo_to_csc(1, 1, np.zeros(2, np.int32), np.zeros(2, np.int32), vals)
    assert A.nnz == 1 and A.rounded(np.float32)[0] == tiny
    rng = np.random.Generator(np.random.PCG64(3))
    v = (rng.standard_normal(4000) * 2.0 ** rng.integers(-149, 100, 4000)).astype(np.float32)
    r = rng.integers(0, 5, 4000).astype(np.int32)
    s, A = oracle.coo_to_csc(5, 1, r, np.zeros(4000, np.int32), v)
    assert not np.any(A.rounded(np.float32) == 0)


@pytest.mark.parametrize("seed", [4, 5])
def test_insert_equals_concatenated_assembly(seed):
    """Insertion folds the existing value first, then the new ones in input order: the same as
    assembling the existing elements (in CSC order) followed by the new triplets."""
    from paper_1805_03380_amd import synth
    p = synth.random_coo(seed, 400, 300, 20_000, dup_frac=0.2, dist="normal")
    q = synth.random_coo(seed + 10, 400, 300, 8_000, dup_frac=0.2, dist="normal")
    s0, A = oracle.coo_to_csc(p.n_rows, p.n_cols, p.row, p.col, p.val)
    assert s0 == oracle.OK
    s1, R = oracle.csc_insert(A, q.row, q.col, q.val)
    a_col = np.repeat(np.arange(A.n_cols), np.diff(A.col_ptr)).astype(np.int32)
    s2, C = oracle.coo_to_csc(A.n_rows, A.n_cols, np.concatenate([A.row_idx, q.row]),
                              np.concatenate([a_col, q.col]), np.concatenate([A.values, q.val]))
    assert s1 == s2 == oracle.OK
    assert np.array_equal(R.col_ptr, C.col_ptr)
    assert np.array_equal(R.row_idx, C.row_idx)
    assert pins.same_floats(R.values, C.values)
