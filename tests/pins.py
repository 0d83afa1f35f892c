"""Checks that pin the oracle to something other than itself.

Each ``pin_*`` function raises AssertionError when the oracle disagrees with a definition,
closed form, invariant, brute force or hand-computed fixture.  They are run as ordinary tests
(test_oracle_pins.py) and against deliberately broken copies of the oracle
(test_oracle_mutants.py), to show that a plausible mistake in the oracle fails at least one.
"""
from __future__ import annotations

import json
import math
import os
from fractions import Fraction

import numpy as np

import oracle
from paper_1805_03380_amd import synth

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")


def load_golden(name):
    with open(os.path.join(GOLDEN, name)) as f:
        return json.load(f)


def brute_force_csc(n_rows, n_cols, row, col, val):
    """Dense brute force: D[r, c] += v in input order (Python floats are binary64), then every
    location whose total is not 0.0, in column-major order (Sections 3.1, 3.3)."""
    acc = {}
    for r, c, v in zip(row.tolist(), col.tolist(), np.asarray(val, dtype=np.float64).tolist()):
        acc[(c, r)] = acc.get((c, r), 0.0) + v
    items = sorted((key, s) for key, s in acc.items() if s != 0.0)
    col_ptr = np.zeros(n_cols + 1, dtype=np.int64)
    for (c, _r), _s in items:
        col_ptr[c + 1] += 1
    col_ptr = np.cumsum(col_ptr)
    rows = np.array([r for (_c, r), _s in items], dtype=np.int64)
    vals = np.array([s for _k, s in items], dtype=np.float64)
    return col_ptr, rows, vals


def same_floats(a, b) -> bool:
    """Bitwise equality of binary64 arrays, treating any NaN as equal to any NaN."""
    a = np.asarray(a, dtype=np.float64)
    b = np.asarray(b, dtype=np.float64)
    if a.shape != b.shape:
        return False
    na, nb = np.isnan(a), np.isnan(b)
    if not np.array_equal(na, nb):
        return False
    return bool(np.all(a.view(np.int64)[~na] == b.view(np.int64)[~nb]))


def dense_of(A: oracle.CSC) -> np.ndarray:
    D = np.zeros((A.n_rows, A.n_cols), dtype=np.float64)
    for c in range(A.n_cols):
        for p in range(A.col_ptr[c], A.col_ptr[c + 1]):
            D[A.row_idx[p], c] = A.values[p]
    return D


def csc_from_dense(D: np.ndarray) -> oracle.CSC:
    n_rows, n_cols = D.shape
    cols, rows, vals = [], [], []
    cp = [0]
    for c in range(n_cols):
        for r in range(n_rows):
            if D[r, c] != 0.0:
                rows.append(r)
                vals.append(D[r, c])
        cp.append(len(rows))
    return oracle.CSC(n_rows, n_cols, np.array(cp, np.int32), np.array(rows, np.int32),
                      np.array(vals, np.float64))


# ------------------------------------------------------------------------------ assembly pins

def pin_golden_assembly():
    for name in ("assembly_small.json", "fold_order.json"):
        g = load_golden(name)
        row = np.array(g["row"], np.int32)
        col = np.array(g["col"], np.int32)
        val = np.array(g["val"], np.float64)
        if "expect_val_hex" in g:
            expect = np.array([float.fromhex(h) for h in g["expect_val_hex"]])
        else:
            expect = np.array(g["expect_val"], np.float64)
        for method in ("sort", "rbt"):
            st, A = oracle.coo_to_csc(g["n_rows"], g["n_cols"], row, col, val, method=method)
            assert st == oracle.OK
            assert A.col_ptr.tolist() == g["expect_col_ptr"], (name, method)
            assert A.row_idx.tolist() == g["expect_row_idx"], (name, method)
            assert same_floats(A.values, expect), (name, method, A.values, expect)


def pin_brute_force(seeds=range(12)):
    """Both oracle reads equal dense brute force bit for bit on small random inputs with many
    duplicates, exact zeros and cancelling pairs."""
    for seed in seeds:
        rng = np.random.Generator(np.random.PCG64(5000 + seed))
        n_rows = int(rng.integers(1, 9))
        n_cols = int(rng.integers(1, 9))
        nnz = int(rng.integers(0, 60))
        row = rng.integers(0, n_rows, nnz).astype(np.int32)
        col = rng.integers(0, n_cols, nnz).astype(np.int32)
        val = rng.choice(np.array([-1.5, -1.0, -0.5, -0.0, 0.0, 0.25, 0.5, 1.0, 3.0]), nnz)
        val = val + rng.standard_normal(nnz) * (rng.random(nnz) < 0.3)
        ecp, er, ev = brute_force_csc(n_rows, n_cols, row, col, val)
        for method in ("sort", "rbt"):
            st, A = oracle.coo_to_csc(n_rows, n_cols, row, col, val, method=method)
            assert st == oracle.OK
            assert np.array_equal(A.col_ptr, ecp), (seed, method)
            assert np.array_equal(A.row_idx, er), (seed, method)
            assert same_floats(A.values, ev), (seed, method)


def pin_scipy_dyadic():
    """scipy.sparse COO->CSC with duplicates summed and zeros eliminated; dyadic values make
    every summation order exact, so structure and values must match exactly."""
    import scipy.sparse as sp
    for seed in range(4):
        rng = np.random.Generator(np.random.PCG64(7000 + seed))
        n_rows, n_cols, nnz = 300, 200, 4000
        row = rng.integers(0, n_rows, nnz).astype(np.int32)
        col = rng.integers(0, n_cols, nnz).astype(np.int32)
        val = rng.integers(-16, 17, nnz).astype(np.float64) / 8.0
        M = sp.coo_matrix((val, (row, col)), shape=(n_rows, n_cols)).tocsc()
        M.sum_duplicates()
        M.eliminate_zeros()
        M.sort_indices()
        st, A = oracle.coo_to_csc(n_rows, n_cols, row, col, val)
        assert st == oracle.OK
        assert np.array_equal(A.col_ptr, M.indptr)
        assert np.array_equal(A.row_idx, M.indices)
        assert np.array_equal(A.values, M.data)


def pin_invariants_and_totals():
    """Section 3.1 invariants on the 1000 x 1000 workload; the total of the stored values equals
    the total of the inputs up to the rounding of the per-location folds."""
    p = synth.tiny_spmv()
    st, A = oracle.coo_to_csc(p.n_rows, p.n_cols, p.row, p.col, p.val)
    assert st == oracle.OK
    oracle.check_csc_invariants(A)
    assert A.nnz <= p.nnz_in
    exact_in = math.fsum(p.val.tolist())
    exact_out = math.fsum(A.values.tolist())
    bound = 2.0 ** -52 * float(np.abs(p.val).sum())
    assert abs(exact_out - exact_in) <= bound
    # sum(X, 0) of Table 1: per-column totals equal brute-force per-column sums of the inputs
    cs = oracle.column_sums(A)
    ref = np.zeros(p.n_cols)
    np.add.at(ref, p.col, p.val)
    assert np.allclose(cs, ref, rtol=0, atol=1e-12)


def pin_index_encoding():
    """Section 3.3: index = row + column * n_rows; decoding with mod / floor-div is the inverse,
    and sorting by index is column-major order, the same order as the key (col << b) | row for
    any b with 2^b >= n_rows."""
    for n_rows, n_cols in ((1, 1), (3, 5), (7, 2), (16, 16), (17, 9)):
        rr, cc = np.meshgrid(np.arange(n_rows), np.arange(n_cols), indexing="ij")
        rr, cc = rr.ravel(), cc.ravel()
        idx = rr + cc * n_rows
        assert np.array_equal(idx % n_rows, rr) and np.array_equal(idx // n_rows, cc)
        b = max(1, int(math.ceil(math.log2(max(n_rows, 2)))))
        shift = (cc << b) | rr
        assert np.array_equal(np.argsort(idx, kind="stable"), np.argsort(shift, kind="stable"))
        lex = np.lexsort((rr, cc))
        assert np.array_equal(np.argsort(idx, kind="stable"), lex)
    # and the oracle emits in that order for a full dense pattern given in reverse order
    n_rows, n_cols = 5, 4
    rr, cc = np.meshgrid(np.arange(n_rows), np.arange(n_cols), indexing="ij")
    rr, cc = rr.ravel()[::-1].astype(np.int32), cc.ravel()[::-1].astype(np.int32)
    val = np.arange(1, rr.size + 1, dtype=np.float64)
    for method in ("sort", "rbt"):
        st, A = oracle.coo_to_csc(n_rows, n_cols, rr, cc, val, method=method)
        assert A.col_ptr.tolist() == [0, 5, 10, 15, 20]
        assert A.row_idx.tolist() == [0, 1, 2, 3, 4] * 4


def pin_special_cases():
    # empty input, zero columns, out-of-range rejection
    st, A = oracle.coo_to_csc(3, 4, np.zeros(0, np.int32), np.zeros(0, np.int32), np.zeros(0))
    assert st == oracle.OK and A.col_ptr.tolist() == [0] * 5 and A.nnz == 0
    st, A = oracle.coo_to_csc(3, 0, np.zeros(0, np.int32), np.zeros(0, np.int32), np.zeros(0))
    assert st == oracle.OK and A.col_ptr.tolist() == [0]
    for r, c in ((3, 0), (0, 4), (-1, 0), (0, -1)):
        st, _ = oracle.coo_to_csc(3, 4, np.array([0, r], np.int32), np.array([0, c], np.int32),
                                  np.array([1.0, 1.0]))
        assert st == oracle.EBOUNDS
    # every triplet on one location: one left fold in input order
    rng = np.random.Generator(np.random.PCG64(99))
    v = rng.standard_normal(1000)
    s = 0.0
    for x in v.tolist():
        s = s + x
    st, A = oracle.coo_to_csc(2, 2, np.ones(1000, np.int32), np.zeros(1000, np.int32), v)
    assert A.col_ptr.tolist() == [0, 1, 1] and A.row_idx.tolist() == [1]
    assert same_floats(A.values, [s])
    # NaN and Inf are stored; Inf + -Inf is NaN and stored; (a, -a, b) stores b
    st, A = oracle.coo_to_csc(4, 1, np.array([0, 1, 2, 2, 3, 3, 3], np.int32),
                              np.zeros(7, np.int32),
                              np.array([np.nan, np.inf, np.inf, -np.inf, 0.7, -0.7, 0.125]))
    assert A.row_idx.tolist() == [0, 1, 2, 3]
    assert np.isnan(A.values[0]) and A.values[1] == np.inf and np.isnan(A.values[2])
    assert A.values[3] == 0.125


# ---------------------------------------------------------------------------------- SpMM pins

def pin_golden_spmm():
    g = load_golden("assembly_small.json")
    st, A = oracle.coo_to_csc(g["n_rows"], g["n_cols"], np.array(g["row"], np.int32),
                              np.array(g["col"], np.int32), np.array(g["val"]))
    s = g["spmm"]
    Y, _S, M = oracle.spmm(A, np.array(s["X"]))
    assert np.array_equal(Y, np.array(s["expect_Y"]))
    assert M.tolist() == [1, 1, 1, 0]
    dX, dval, _a, _b = oracle.spmm_backward(A, np.array(s["G"]), np.array(s["X"]))
    assert np.array_equal(dX, np.array(s["expect_dX"]))
    assert np.array_equal(dval, np.array(s["expect_dval"]))


def pin_fraction_exact():
    """Exact rational arithmetic on tiny random inputs: every oracle output is within
    gamma_m * S of the exact value (m terms, S = sum of |terms|)."""
    for seed in range(5):
        rng = np.random.Generator(np.random.PCG64(8100 + seed))
        n_rows, n_cols, k = 7, 6, 3
        p = synth.random_coo(8100 + seed, n_rows, n_cols, 25, dup_frac=0.2, dist="normal")
        st, A = oracle.coo_to_csc(n_rows, n_cols, p.row, p.col, p.val)
        X = rng.standard_normal((n_cols, k))
        G = rng.standard_normal((n_rows, k))
        D = dense_of(A)
        Y, S, M = oracle.spmm(A, X)
        dX, dval, SdX, Sdv = oracle.spmm_backward(A, G, X)
        Fr = lambda x: Fraction(float(x))
        for r in range(n_rows):
            for j in range(k):
                exact = sum((Fr(D[r, c]) * Fr(X[c, j]) for c in range(n_cols)), Fraction(0))
                assert abs(Fraction(float(Y[r, j])) - exact) <= Fr(oracle.gamma(M[r]) * S[r, j])
        for c in range(n_cols):
            m = A.col_ptr[c + 1] - A.col_ptr[c]
            for j in range(k):
                exact = sum((Fr(D[r, c]) * Fr(G[r, j]) for r in range(n_rows)), Fraction(0))
                assert abs(Fraction(float(dX[c, j])) - exact) <= Fr(oracle.gamma(m) * SdX[c, j])
            for q in range(A.col_ptr[c], A.col_ptr[c + 1]):
                r = A.row_idx[q]
                exact = sum((Fr(G[r, j]) * Fr(X[c, j]) for j in range(k)), Fraction(0))
                assert abs(Fraction(float(dval[q])) - exact) <= Fr(oracle.gamma(k) * Sdv[q])


def pin_identity_and_permutation():
    """speye (Table 1) gives Y = X and dX = G exactly; a permutation matrix permutes rows
    exactly; one stored value per row is a single product, hence exact."""
    rng = np.random.Generator(np.random.PCG64(8200))
    n, k = 50, 5
    X = rng.standard_normal((n, k))
    G = rng.standard_normal((n, k))
    idx = np.arange(n, dtype=np.int32)
    st, I = oracle.coo_to_csc(n, n, idx, idx, np.ones(n))
    Y, _, _ = oracle.spmm(I, X)
    assert np.array_equal(Y, X)
    dX, dval, _, _ = oracle.spmm_backward(I, G, X)
    assert np.array_equal(dX, G)
    assert np.array_equal(dval, np.einsum("ij,ij->i", G, X)) or np.allclose(
        dval, (G * X).sum(1), rtol=1e-14, atol=0)
    perm = rng.permutation(n).astype(np.int32)
    st, P = oracle.coo_to_csc(n, n, perm, idx, np.ones(n))  # P[perm[c], c] = 1
    Y, _, _ = oracle.spmm(P, X)
    expect = np.zeros_like(X)
    expect[perm] = X
    assert np.array_equal(Y, expect)
    scale = rng.standard_normal(n)
    st, D = oracle.coo_to_csc(n, n, perm, idx, scale)
    Y, _, _ = oracle.spmm(D, X)
    expect = np.zeros_like(X)
    expect[perm] = scale[:, None] * X
    assert np.array_equal(Y, expect)
    # transposed operand mistake detector: non-symmetric 2x3 case by hand
    st, A = oracle.coo_to_csc(2, 3, np.array([0, 1], np.int32), np.array([2, 0], np.int32),
                              np.array([2.0, 5.0]))
    Y, _, _ = oracle.spmm(A, np.array([[1.0], [10.0], [100.0]]))
    assert Y.ravel().tolist() == [200.0, 5.0]


def pin_ones_closed_form():
    """All-ones n_rows x n_cols matrix times integer X: every output row is the column sum of X,
    exact in binary64 for small integers."""
    rng = np.random.Generator(np.random.PCG64(8300))
    n_rows, n_cols, k = 9, 13, 4
    rr, cc = np.meshgrid(np.arange(n_rows), np.arange(n_cols), indexing="ij")
    st, A = oracle.coo_to_csc(n_rows, n_cols, rr.ravel().astype(np.int32),
                              cc.ravel().astype(np.int32), np.ones(n_rows * n_cols))
    X = rng.integers(-50, 50, (n_cols, k)).astype(np.float64)
    Y, _, M = oracle.spmm(A, X)
    assert np.array_equal(Y, np.tile(X.sum(0), (n_rows, 1)))
    assert np.all(M == n_cols)
    G = rng.integers(-50, 50, (n_rows, k)).astype(np.float64)
    dX, dval, _, _ = oracle.spmm_backward(A, G, X)
    assert np.array_equal(dX, np.tile(G.sum(0), (n_cols, 1)))
    # dval at stored (r, c) is G[r] . X[c]
    expect = np.array([G[r] @ X[c] for c in range(n_cols) for r in range(n_rows)])
    assert np.array_equal(dval, expect)


def pin_dense_crosscheck():
    """numpy dense products on a 2000 x 2000 instance agree within the a-priori bound."""
    p = synth.diff_fd()
    st, A = oracle.coo_to_csc(p.n_rows, p.n_cols, p.row, p.col, p.val)
    D = np.zeros((p.n_rows, p.n_cols))
    D[A.row_idx, np.repeat(np.arange(p.n_cols), np.diff(A.col_ptr))] = A.values
    Y, S, M = oracle.spmm(A, p.X)
    Yd = D @ p.X
    assert np.all(np.abs(Y - Yd) <= 2 * oracle.gamma(p.n_cols) * (np.abs(D) @ np.abs(p.X)))
    dX, dval, SdX, Sdv = oracle.spmm_backward(A, p.G, p.X)
    dXd = D.T @ p.G
    assert np.all(np.abs(dX - dXd) <= 2 * oracle.gamma(p.n_rows) * (np.abs(D).T @ np.abs(p.G)))
    cols = np.repeat(np.arange(p.n_cols), np.diff(A.col_ptr))
    dvd = np.einsum("ij,ij->i", p.G[A.row_idx], p.X[cols])
    assert np.all(np.abs(dval - dvd) <= 2 * oracle.gamma(p.k) * Sdv)


def pin_adjoint_identity():
    """<A.X, G> = <X, A^T.G> = <values, dvalues> up to binary64 rounding."""
    p = synth.diff_fd()
    st, A = oracle.coo_to_csc(p.n_rows, p.n_cols, p.row, p.col, p.val)
    Y, S, _ = oracle.spmm(A, p.X)
    dX, dval, SdX, Sdv = oracle.spmm_backward(A, p.G, p.X)
    a = math.fsum((Y * p.G).ravel().tolist())
    b = math.fsum((p.X * dX).ravel().tolist())
    c = math.fsum((A.values * dval).tolist())
    scale = float((S * np.abs(p.G)).sum())
    tol = 4 * oracle.gamma(max(p.n_cols, p.k)) * scale
    assert abs(a - b) <= tol and abs(a - c) <= tol and abs(b - c) <= tol


def pin_central_fd(samples: int = 24):
    """Central differences of L = sum(A.X * G) in binary64.  L is bilinear in (values, X), so
    the difference quotient with h = 2^-4 has no truncation error; only the rounding of L
    remains (tolerance 1e-8 relative + 1e-10 absolute)."""
    p = synth.diff_fd()
    st, A = oracle.coo_to_csc(p.n_rows, p.n_cols, p.row, p.col, p.val)
    dX, dval, _, _ = oracle.spmm_backward(A, p.G, p.X)
    h = 2.0 ** -4

    def L(values, X):
        Y, _, _ = oracle.spmm(A, X, values=values)
        return math.fsum((Y * p.G).ravel().tolist())

    rng = np.random.Generator(np.random.PCG64(8400))
    for q in rng.choice(A.nnz, samples, replace=False):
        vp = A.values.copy()
        vp[q] += h
        vm = A.values.copy()
        vm[q] -= h
        fd = (L(vp, p.X) - L(vm, p.X)) / (2 * h)
        assert abs(fd - dval[q]) <= 1e-8 * abs(dval[q]) + 1e-10, (q, fd, dval[q])
    for _ in range(samples):
        c, j = int(rng.integers(p.n_cols)), int(rng.integers(p.k))
        Xp = p.X.copy()
        Xp[c, j] += h
        Xm = p.X.copy()
        Xm[c, j] -= h
        fd = (L(A.values, Xp) - L(A.values, Xm)) / (2 * h)
        assert abs(fd - dX[c, j]) <= 1e-8 * abs(dX[c, j]) + 1e-10, (c, j, fd, dX[c, j])


# ----------------------------------------------------------------------- batch insertion pins

def pin_golden_insert():
    """The hand-computed insertion of tests/golden/insert_small.json (existing value first)."""
    g = load_golden("insert_small.json")
    A = oracle.CSC(g["n_rows"], g["n_cols"], np.array(g["a_col_ptr"], np.int32),
                   np.array(g["a_row_idx"], np.int32), np.array(g["a_val"], np.float64))
    st, R = oracle.csc_insert(A, np.array(g["row"], np.int32), np.array(g["col"], np.int32),
                              np.array(g["val"], np.float64))
    assert st == oracle.OK
    assert R.col_ptr.tolist() == g["expect_col_ptr"]
    assert R.row_idx.tolist() == g["expect_row_idx"]
    assert same_floats(R.values, np.array(g["expect_val"], np.float64))


def pin_brute_force_insert(seeds=range(12)):
    """Dense brute force: start from the existing matrix, D[r, c] = D[r, c] + v for the new
    triplets in input order, store the non-zero entries column by column."""
    for seed in seeds:
        rng = np.random.Generator(np.random.PCG64(6000 + seed))
        n_rows = int(rng.integers(1, 9))
        n_cols = int(rng.integers(1, 9))
        D0 = rng.choice(np.array([-2.0, -1.0, 0.5, 1.5, 3.0]), (n_rows, n_cols))
        D0 = D0 * (rng.random((n_rows, n_cols)) < 0.5)
        D0 = D0 + rng.standard_normal((n_rows, n_cols)) * (D0 != 0) * (rng.random(D0.shape) < 0.3)
        A = csc_from_dense(D0)
        nnz = int(rng.integers(0, 40))
        row = rng.integers(0, n_rows, nnz).astype(np.int32)
        col = rng.integers(0, n_cols, nnz).astype(np.int32)
        val = rng.choice(np.array([-1.5, -1.0, -0.5, 0.25, 0.5, 1.0, 2.0]), nnz)
        cancel = rng.random(nnz) < 0.3  # some new values cancel the existing ones exactly
        val = np.where(cancel & (D0[row, col] != 0), -D0[row, col], val)
        D = D0.copy()
        for r, c, v in zip(row.tolist(), col.tolist(), val.tolist()):
            D[r, c] = D[r, c] + v
        E = csc_from_dense(D)
        st, R = oracle.csc_insert(A, row, col, val)
        assert st == oracle.OK
        assert np.array_equal(R.col_ptr, E.col_ptr), seed
        assert np.array_equal(R.row_idx, E.row_idx), seed
        assert same_floats(R.values, E.values), seed


def pin_insert_special_cases():
    """Nothing to insert leaves A as it is; inserting into an empty matrix is assembly; a
    new triplet out of range is rejected; a malformed existing CSC is rejected."""
    rng = np.random.Generator(np.random.PCG64(6100))
    D0 = rng.standard_normal((5, 4)) * (rng.random((5, 4)) < 0.5)
    A = csc_from_dense(D0)
    st, R = oracle.csc_insert(A, np.zeros(0, np.int32), np.zeros(0, np.int32), np.zeros(0))
    assert st == oracle.OK and np.array_equal(R.col_ptr, A.col_ptr)
    assert np.array_equal(R.row_idx, A.row_idx) and same_floats(R.values, A.values)
    E = oracle.CSC(5, 4, np.zeros(5, np.int32), np.zeros(0, np.int32), np.zeros(0))
    row = np.array([4, 0, 4, 2], np.int32)
    col = np.array([3, 0, 3, 1], np.int32)
    val = np.array([1.0, -2.0, 0.5, 3.0])
    st, R = oracle.csc_insert(E, row, col, val)
    ecp, er, ev = brute_force_csc(5, 4, row, col, val)
    assert st == oracle.OK and np.array_equal(R.col_ptr, ecp)
    assert np.array_equal(R.row_idx, er) and same_floats(R.values, ev)
    st, _ = oracle.csc_insert(A, np.array([5], np.int32), np.array([0], np.int32),
                              np.array([1.0]))
    assert st == oracle.EBOUNDS
    bad = oracle.CSC(5, 4, np.array([0, 2, 2, 2, 2], np.int32), np.array([3, 1], np.int32),
                     np.array([1.0, 2.0]))  # rows not increasing in column 0
    st, _ = oracle.csc_insert(bad, row, col, val)
    assert st == oracle.EINVAL


# ------------------------------------------------------------------------------ transpose pins

def pin_transpose_dense(seeds=range(10)):
    """The transpose equals the CSC of the transposed dense matrix (values moved bit for bit),
    transposing twice gives A back, and the identity is its own transpose."""
    for seed in seeds:
        rng = np.random.Generator(np.random.PCG64(6200 + seed))
        n_rows = int(rng.integers(1, 10))
        n_cols = int(rng.integers(1, 10))
        D = rng.standard_normal((n_rows, n_cols)) * (rng.random((n_rows, n_cols)) < 0.4)
        A = csc_from_dense(D)
        st, T = oracle.csc_transpose(A)
        assert st == oracle.OK
        E = csc_from_dense(D.T.copy())
        assert T.n_rows == n_cols and T.n_cols == n_rows
        assert np.array_equal(T.col_ptr, E.col_ptr), seed
        assert np.array_equal(T.row_idx, E.row_idx), seed
        assert same_floats(T.values, E.values), seed
        st, TT = oracle.csc_transpose(T)
        assert st == oracle.OK
        assert np.array_equal(TT.col_ptr, A.col_ptr) and np.array_equal(TT.row_idx, A.row_idx)
        assert same_floats(TT.values, A.values)
    eye = csc_from_dense(np.eye(7))
    st, T = oracle.csc_transpose(eye)
    assert st == oracle.OK and np.array_equal(T.col_ptr, eye.col_ptr)
    assert np.array_equal(T.row_idx, eye.row_idx)


# ------------------------------------------------------------------------------ sum A + B pins

def pin_add_dense(seeds=range(12)):
    """A + B equals the CSC of the dense sum (dyadic values: every sum exact), zeros dropped;
    A + B = B + A; A + (-A) is empty; A + empty = A."""
    for seed in seeds:
        rng = np.random.Generator(np.random.PCG64(6600 + seed))
        n_rows = int(rng.integers(1, 10))
        n_cols = int(rng.integers(1, 10))
        Da, Db = _trace_pair(rng, n_rows, n_cols, 0.5, _dyadic)
        # some exact cancellations
        Db = np.where(rng.random((n_rows, n_cols)) < 0.2, -Da, Db)
        A, B = csc_from_dense(Da), csc_from_dense(Db)
        st, R = oracle.csc_add(A, B)
        assert st == oracle.OK
        E = csc_from_dense(Da + Db)
        assert np.array_equal(R.col_ptr, E.col_ptr), seed
        assert np.array_equal(R.row_idx, E.row_idx), seed
        assert same_floats(R.values, E.values), seed
        st, R2 = oracle.csc_add(B, A)
        assert st == oracle.OK and np.array_equal(R2.row_idx, R.row_idx)
        assert same_floats(R2.values, R.values)
        st, Z = oracle.csc_add(A, csc_from_dense(-Da))
        assert st == oracle.OK and Z.nnz == 0 and np.all(Z.col_ptr == 0)
        st, S = oracle.csc_add(A, csc_from_dense(np.zeros_like(Da)))
        assert st == oracle.OK and np.array_equal(S.row_idx, A.row_idx)
        assert same_floats(S.values, A.values)
    bad = oracle.CSC(3, 2, np.array([0, 2, 2], np.int32), np.array([2, 0], np.int32),
                     np.array([1.0, 2.0]))
    st, _ = oracle.csc_add(bad, bad)
    assert st == oracle.EINVAL


def pin_add_is_insertion():
    """A + B equals the batch insertion of B's elements (as triplets, in CSC order) into A:
    at a shared location both fold A's value first."""
    rng = np.random.Generator(np.random.PCG64(6700))
    D1 = rng.standard_normal((30, 20)) * (rng.random((30, 20)) < 0.3)
    D2 = rng.standard_normal((30, 20)) * (rng.random((30, 20)) < 0.3)
    A, B = csc_from_dense(D1), csc_from_dense(D2)
    st, R = oracle.csc_add(A, B)
    b_col = np.repeat(np.arange(20), np.diff(B.col_ptr)).astype(np.int32)
    st2, I = oracle.csc_insert(A, B.row_idx, b_col, B.values)
    assert st == st2 == oracle.OK
    assert np.array_equal(R.col_ptr, I.col_ptr) and np.array_equal(R.row_idx, I.row_idx)
    assert same_floats(R.values, I.values)


# -------------------------------------------------------------------------- trace(A^T B) pins

def _trace_pair(rng, n_rows, n_cols, density, values):
    """Two independent random sparse matrices (dense form) of one shape."""
    out = []
    for _ in range(2):
        mask = rng.random((n_rows, n_cols)) < density
        out.append(np.where(mask, values(rng, (n_rows, n_cols)), 0.0))
    return out


def _dyadic(rng, shape):
    """Non-zero multiples of 1/4 in [-4, 4]: products and their sums are exact in binary64."""
    v = rng.integers(1, 17, size=shape) * rng.choice([-1, 1], size=shape)
    return v / 4.0


def pin_golden_trace():
    g = load_golden("trace_small.json")
    for case in g["cases"]:
        A = oracle.CSC(case["n_rows"], case["n_cols"], np.array(case["a_col_ptr"], np.int32),
                       np.array(case["a_row_idx"], np.int32), np.array(case["a_val"]))
        B = oracle.CSC(case["n_rows"], case["n_cols"], np.array(case["b_col_ptr"], np.int32),
                       np.array(case["b_row_idx"], np.int32), np.array(case["b_val"]))
        st, t, hits = oracle.trace_atb(A, B)
        assert st == oracle.OK
        assert same_floats([t], [case["expect_trace"]]), (case["name"], t)
        assert hits == case["expect_hits"], (case["name"], hits)


def pin_trace_dense(seeds=range(12)):
    """Brute force on small dense matrices: with dyadic values every product and sum is exact,
    so the trace equals numpy's trace of the dense A^T B exactly, and trace(A^T B) equals
    trace(B^T A); the matched count is the size of the pattern intersection.  With normal
    values the trace is within the a-priori bound of the exact (Fraction) sum."""
    for seed in seeds:
        rng = np.random.Generator(np.random.PCG64(6300 + seed))
        n_rows = int(rng.integers(1, 12))
        n_cols = int(rng.integers(1, 12))
        Da, Db = _trace_pair(rng, n_rows, n_cols, 0.5, _dyadic)
        A, B = csc_from_dense(Da), csc_from_dense(Db)
        st, t, hits = oracle.trace_atb(A, B)
        assert st == oracle.OK
        assert t == float(np.trace(Da.T @ Db)), seed
        assert hits == int(np.count_nonzero((Da != 0) & (Db != 0))), seed
        st, t2, hits2 = oracle.trace_atb(B, A)
        assert st == oracle.OK and t2 == t and hits2 == hits
        Na, Nb = _trace_pair(rng, n_rows, n_cols, 0.5, lambda r, sh: r.standard_normal(sh))
        st, t, hits = oracle.trace_atb(csc_from_dense(Na), csc_from_dense(Nb))
        assert st == oracle.OK
        exact = sum((Fraction(float(a)) * Fraction(float(b))
                     for a, b in zip(Na.ravel(), Nb.ravel()) if a != 0 and b != 0), Fraction(0))
        s_abs = float(np.sum(np.abs(Na * Nb)))
        assert abs(Fraction(t) - exact) <= Fraction(oracle.gamma(hits + 1) * s_abs), seed


def pin_trace_closed_forms():
    """trace(A^T A) is the squared Frobenius norm; trace(I^T B) (speye, Table 1) is the sum of
    B's diagonal; matrices with disjoint patterns give 0 with no match."""
    rng = np.random.Generator(np.random.PCG64(6400))
    D = np.where(rng.random((9, 6)) < 0.5, _dyadic(rng, (9, 6)), 0.0)
    A = csc_from_dense(D)
    st, t, hits = oracle.trace_atb(A, A)
    assert st == oracle.OK
    assert t == float(sum(Fraction(float(v)) ** 2 for v in D.ravel()))
    assert hits == int(np.count_nonzero(D))
    Db = np.where(rng.random((8, 8)) < 0.6, _dyadic(rng, (8, 8)), 0.0)
    st, t, hits = oracle.trace_atb(csc_from_dense(np.eye(8)), csc_from_dense(Db))
    assert st == oracle.OK
    assert t == float(sum(Fraction(float(Db[i, i])) for i in range(8)))
    assert hits == int(np.count_nonzero(np.diag(Db)))
    even = np.zeros((6, 5))
    odd = np.zeros((6, 5))
    even[0::2, :] = 1.5
    odd[1::2, :] = -2.0
    st, t, hits = oracle.trace_atb(csc_from_dense(even), csc_from_dense(odd))
    assert st == oracle.OK and t == 0.0 and hits == 0


def pin_trace_special_cases():
    """IEEE rules at matched locations only: an infinity of A facing a structural zero of B
    adds nothing, facing a stored 0.0 gives NaN; a NaN at a matched location propagates.
    Empty shapes give 0; an unsorted column is rejected."""
    A = oracle.CSC(3, 2, np.array([0, 2, 3], np.int32), np.array([0, 2, 1], np.int32),
                   np.array([np.inf, 2.0, 3.0]))
    B = oracle.CSC(3, 2, np.array([0, 1, 2], np.int32), np.array([2, 1], np.int32),
                   np.array([0.5, 4.0]))
    st, t, hits = oracle.trace_atb(A, B)
    assert st == oracle.OK and t == 13.0 and hits == 2
    Bz = oracle.CSC(3, 2, np.array([0, 1, 2], np.int32), np.array([0, 1], np.int32),
                    np.array([0.0, 4.0]))
    st, t, hits = oracle.trace_atb(A, Bz)
    assert st == oracle.OK and math.isnan(t) and hits == 2
    An = oracle.CSC(3, 2, np.array([0, 0, 1], np.int32), np.array([1], np.int32),
                    np.array([np.nan]))
    st, t, hits = oracle.trace_atb(An, B)
    assert st == oracle.OK and math.isnan(t) and hits == 1
    for shape in ((0, 4), (4, 0)):
        E = oracle.CSC(shape[0], shape[1], np.zeros(shape[1] + 1, np.int32),
                       np.zeros(0, np.int32), np.zeros(0))
        st, t, hits = oracle.trace_atb(E, E)
        assert st == oracle.OK and t == 0.0 and hits == 0
    bad = oracle.CSC(3, 2, np.array([0, 2, 3], np.int32), np.array([2, 0, 1], np.int32),
                     np.array([1.0, 2.0, 3.0]))
    st, _, _ = oracle.trace_atb(bad, B)
    assert st == oracle.EINVAL


# ----------------------------------------------------------------- triplet-level adjoint pins

def _small_triplets(seed, n_rows=7, n_cols=6, n_t=40, k=5):
    """Dyadic triplets with duplicates, an exactly cancelling pair, and dyadic G and X: every
    sum below is exact in binary64."""
    rng = np.random.Generator(np.random.PCG64(seed))
    row = rng.integers(0, n_rows, size=n_t).astype(np.int32)
    col = rng.integers(0, n_cols, size=n_t).astype(np.int32)
    val = _dyadic(rng, n_t)
    # a location whose two triplets cancel, so assembly drops it
    row[-2:], col[-2:] = 3, 4
    keep = ~((row[:-2] == 3) & (col[:-2] == 4))
    row = np.concatenate([row[:-2][keep], row[-2:]])
    col = np.concatenate([col[:-2][keep], col[-2:]])
    val = np.concatenate([val[:-2][keep], [1.25, -1.25]])
    G = _dyadic(rng, (n_rows, k))
    X = _dyadic(rng, (n_cols, k))
    return n_rows, n_cols, row, col, val, G, X


def pin_triplet_grad_fd():
    """Central differences of L = sum((assemble(v).X) * G) in each triplet's value: L is linear
    in v_t, the data are dyadic, so the quotient with h = 2^-4 is exact and must equal the
    gradient, for unique triplets, duplicates and both triplets of the cancelling pair."""
    n_rows, n_cols, row, col, val, G, X = _small_triplets(6500)
    dv, _ = oracle.triplet_grad(n_rows, n_cols, row, col, G, X)
    h = 2.0 ** -4

    def L(v):
        st, A = oracle.coo_to_csc(n_rows, n_cols, row, col, v)
        assert st == oracle.OK
        Y, _, _ = oracle.spmm(A, X)
        return float(sum(Fraction(float(y)) * Fraction(float(g))
                         for y, g in zip(Y.ravel(), G.ravel())))

    st, A0 = oracle.coo_to_csc(n_rows, n_cols, row, col, val)
    assert not np.any((A0.row_idx == 3) & (np.repeat(np.arange(n_cols), np.diff(A0.col_ptr)) == 4))
    for t in range(len(row)):
        vp, vm = val.copy(), val.copy()
        vp[t] += h
        vm[t] -= h
        fd = (L(vp) - L(vm)) / (2 * h)
        assert fd == dv[t], (t, fd, dv[t])


def pin_triplet_grad_matches_dvalues():
    """Without duplicates or zero sums every triplet has its own CSC slot, and its gradient is
    the adjoint's dvalues at that slot (the same binary64 sum in ascending j); a triplet
    outside the matrix has gradient 0; the gradient is within the a-priori bound of the exact
    (Fraction) dot product."""
    rng = np.random.Generator(np.random.PCG64(6501))
    n_rows, n_cols, k = 9, 8, 6
    pos = rng.choice(n_rows * n_cols, size=30, replace=False)
    row = (pos % n_rows).astype(np.int32)
    col = (pos // n_rows).astype(np.int32)
    val = rng.standard_normal(30) + 3.0
    G = rng.standard_normal((n_rows, k))
    X = rng.standard_normal((n_cols, k))
    st, A = oracle.coo_to_csc(n_rows, n_cols, row, col, val)
    assert st == oracle.OK and A.nnz == 30
    _, dval, _, _ = oracle.spmm_backward(A, G, X)
    dv, S = oracle.triplet_grad(n_rows, n_cols, row, col, G, X)
    a_col = np.repeat(np.arange(n_cols), np.diff(A.col_ptr))
    for t in range(30):
        slot = int(np.nonzero((A.row_idx == row[t]) & (a_col == col[t]))[0][0])
        assert same_floats([dv[t]], [dval[slot]]), t
        exact = sum((Fraction(float(G[row[t], j])) * Fraction(float(X[col[t], j]))
                     for j in range(k)), Fraction(0))
        assert abs(Fraction(float(dv[t])) - exact) <= Fraction(float(oracle.gamma(k) * S[t]))
    out = oracle.triplet_grad(n_rows, n_cols, np.array([n_rows, 0, -1], np.int32),
                              np.array([0, n_cols, 0], np.int32), G, X)[0]
    assert np.array_equal(out, np.zeros(3))


ASSEMBLY_PINS = [pin_golden_assembly, pin_brute_force, pin_scipy_dyadic, pin_invariants_and_totals,
                 pin_index_encoding, pin_special_cases, pin_golden_insert, pin_brute_force_insert,
                 pin_insert_special_cases, pin_transpose_dense]
SPMM_PINS = [pin_golden_spmm, pin_fraction_exact, pin_identity_and_permutation,
             pin_ones_closed_form, pin_dense_crosscheck, pin_adjoint_identity, pin_central_fd]
TRACE_PINS = [pin_golden_trace, pin_trace_dense, pin_trace_closed_forms, pin_trace_special_cases]
TRIPLET_GRAD_PINS = [pin_triplet_grad_fd, pin_triplet_grad_matches_dvalues]
ADD_PINS = [pin_add_dense, pin_add_is_insertion]
ALL_PINS = ASSEMBLY_PINS + SPMM_PINS + TRACE_PINS + TRIPLET_GRAD_PINS + ADD_PINS
