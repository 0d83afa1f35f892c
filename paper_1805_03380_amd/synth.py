"""Seeded synthetic inputs for the assembly + SpMM path.

This module only draws random numbers and lays them out; it holds none of the method's
arithmetic, so both the GPU path and the oracle consume exactly the same host arrays.  Every
generator uses numpy's PCG64 with a fixed seed and returns plain numpy arrays; ``digest`` gives
the SHA-256 of each array for run records.

The shapes follow the paper's workloads: random sparse matrices with a given density built by
unordered element insertion (Section 4: 10,000 x 10,000 at densities 0.01 % .. 10 %; Fig. 1:
1000 x 1000 at density 0.01 followed by a dense-vector product), scaled up to the sizes of the
workloads in the benchmark.

Position recipe shared by all generators: a set of distinct (row, col) locations is drawn
without replacement, duplicate triplets are drawn uniformly from that set, and the whole triplet
list is randomly permuted, so duplicates of one location are scattered through the input.
"""
from __future__ import annotations

import hashlib
import math
from dataclasses import dataclass, field

import numpy as np


@dataclass
class COOProblem:
    """One assembly + SpMM instance (all arrays on the host)."""
    name: str
    n_rows: int
    n_cols: int
    row: np.ndarray          # int32 [nnz_in]
    col: np.ndarray          # int32 [nnz_in]
    val: np.ndarray          # float64 / float32 [nnz_in]
    X: np.ndarray | None = None   # dense n_cols x k, row-major
    G: np.ndarray | None = None   # dense n_rows x k, row-major (dL/dY)
    meta: dict = field(default_factory=dict)

    @property
    def nnz_in(self) -> int:
        return int(self.row.shape[0])

    @property
    def k(self) -> int:
        return 0 if self.X is None else int(self.X.shape[1])


def digest(*arrays: np.ndarray) -> list[str]:
    """SHA-256 (hex, first 16 chars) of each array's bytes."""
    return [hashlib.sha256(np.ascontiguousarray(a).tobytes()).hexdigest()[:16] for a in arrays]


def _distinct_positions(rng: np.random.Generator, n_rows: int, n_cols: int, n_unique: int,
                        draw) -> np.ndarray:
    """``n_unique`` distinct linear locations col*n_rows+row, drawn by ``draw(rng, m)``."""
    total = n_rows * n_cols
    if n_unique > total:
        raise ValueError("more distinct locations requested than the matrix has")
    got = np.empty(0, dtype=np.int64)
    while got.size < n_unique:
        need = n_unique - got.size
        fresh = draw(rng, int(need * 1.05) + 16)
        got = np.union1d(got, fresh)
    # keep a uniformly random subset of exactly n_unique (union1d returns them sorted)
    keep = rng.choice(got.size, size=n_unique, replace=False)
    keep.sort()
    return got[keep]


def _uniform_draw(n_rows: int, n_cols: int):
    total = n_rows * n_cols

    def draw(rng, m):
        return rng.integers(0, total, size=m, dtype=np.int64)
    return draw


def _assemble_list(rng, positions: np.ndarray, n_dup: int, n_rows: int):
    """Distinct positions + n_dup duplicates drawn from them, randomly permuted -> (row, col)."""
    dup = positions[rng.integers(0, positions.size, size=n_dup)] if n_dup else positions[:0]
    allpos = np.concatenate([positions, dup])
    allpos = allpos[rng.permutation(allpos.size)]
    row = (allpos % n_rows).astype(np.int32)
    col = (allpos // n_rows).astype(np.int32)
    return row, col


def random_coo(seed: int, n_rows: int, n_cols: int, nnz_in: int, dup_frac: float = 0.1,
               zero_frac: float = 0.0, dtype=np.float64, dist: str = "uniform", k: int = 0,
               name: str = "random") -> COOProblem:
    """Generic seeded instance: uniform distinct positions, a fraction of duplicate triplets,
    a fraction of exact +0.0 values; values U[-1,1] ("uniform") or N(0,1) ("normal")."""
    rng = np.random.Generator(np.random.PCG64(seed))
    n_dup = int(round(nnz_in * dup_frac))
    n_unique = nnz_in - n_dup
    if n_unique == 0 and nnz_in > 0:
        n_unique, n_dup = 1, nnz_in - 1
    if nnz_in == 0:
        row = np.zeros(0, np.int32)
        col = np.zeros(0, np.int32)
    else:
        pos = _distinct_positions(rng, n_rows, n_cols, n_unique, _uniform_draw(n_rows, n_cols))
        row, col = _assemble_list(rng, pos, n_dup, n_rows)
    if dist == "uniform":
        val = rng.uniform(-1.0, 1.0, size=nnz_in)
    else:
        val = rng.standard_normal(size=nnz_in)
    n_zero = int(round(nnz_in * zero_frac))
    if n_zero:
        val[rng.choice(nnz_in, size=n_zero, replace=False)] = 0.0
    val = val.astype(dtype)
    X = G = None
    if k:
        X = rng.standard_normal(size=(n_cols, k)).astype(dtype)
        G = rng.standard_normal(size=(n_rows, k)).astype(dtype)
    return COOProblem(name, n_rows, n_cols, row, col, val, X, G,
                      meta=dict(seed=seed, dup_frac=dup_frac, zero_frac=zero_frac, dist=dist))


# ----------------------------------------------------------------------------------------------
# The five workloads.
# ----------------------------------------------------------------------------------------------

def tiny_spmv(seed: int = 1001) -> COOProblem:
    """1000 x 1000 from 10,000 triplets: 9,000 distinct uniform locations + 1,000 duplicates,
    100 values set to exactly +0.0, values U[-1,1] in float64; x and g of length 1000 U[-1,1]
    (the Fig. 1 scenario: density-0.01 random matrix times a dense vector)."""
    rng = np.random.Generator(np.random.PCG64(seed))
    n = 1000
    pos = _distinct_positions(rng, n, n, 9000, _uniform_draw(n, n))
    row, col = _assemble_list(rng, pos, 1000, n)
    val = rng.uniform(-1.0, 1.0, size=10000)
    val[rng.choice(10000, size=100, replace=False)] = 0.0
    x = rng.uniform(-1.0, 1.0, size=(n, 1))
    g = rng.uniform(-1.0, 1.0, size=(n, 1))
    return COOProblem("tiny_spmv_1000x1000_nnz1e4_f64_k1", n, n, row, col, val, x, g,
                      meta=dict(seed=seed))


def uniform_1e5(seed: int = 1002, value_dtype=np.float32, k: int = 64) -> COOProblem:
    """100,000 x 100,000 from 1,000,000 triplets (950,000 distinct uniform locations + 50,000
    duplicates), values U[-1,1] drawn in float64 then cast to ``value_dtype``; X is
    100,000 x k float32 N(0,1); G is N(0,1) in the output precision (float64 when the values
    are float64, else float32)."""
    rng = np.random.Generator(np.random.PCG64(seed))
    n = 100_000
    pos = _distinct_positions(rng, n, n, 950_000, _uniform_draw(n, n))
    row, col = _assemble_list(rng, pos, 50_000, n)
    val = rng.uniform(-1.0, 1.0, size=1_000_000).astype(value_dtype)
    X = rng.standard_normal(size=(n, k), dtype=np.float32)
    g_dtype = np.float64 if value_dtype == np.float64 else np.float32
    G = rng.standard_normal(size=(n, k)).astype(g_dtype)
    name = "uniform_1e5x1e5_nnz1e6_%s_k%d" % (np.dtype(value_dtype).name, k)
    return COOProblem(name, n, n, row, col, val, X, G, meta=dict(seed=seed))


def zipf_degrees(rng, n: int, exponent: float = 1.5, d_max: int = 335) -> np.ndarray:
    """n i.i.d. expected degrees from a discrete power law p(d) ~ d^-exponent on [1, d_max]."""
    d = np.arange(1, d_max + 1, dtype=np.float64)
    p = d ** (-exponent)
    p /= p.sum()
    return rng.choice(d_max, size=n, p=p).astype(np.float64) + 1.0


def powerlaw_1e6(seed: int = 1003, n: int = 1_000_000, n_unique: int = 14_000_000,
                 n_dup: int = 6_000_000, k: int = 128, d_max: int = 335,
                 with_dense: bool = True) -> COOProblem:
    """Chung-Lu power-law matrix: row and column expected degrees are i.i.d. Zipf(1.5) truncated
    to [1, d_max] (mean about 14 for d_max = 335); a location (r, c) is drawn with probability
    proportional to w_r * w_c.  n_unique distinct locations + n_dup duplicates (30 %), values
    N(0,1) float32, X n x k float32 N(0,1), G N(0,1)."""
    rng = np.random.Generator(np.random.PCG64(seed))
    wr = zipf_degrees(rng, n, 1.5, d_max)
    wc = zipf_degrees(rng, n, 1.5, d_max)
    cr = np.cumsum(wr)
    cr /= cr[-1]
    cc = np.cumsum(wc)
    cc /= cc[-1]

    def draw(rng_, m):
        r = np.minimum(np.searchsorted(cr, rng_.random(m), side="right"), n - 1)
        c = np.minimum(np.searchsorted(cc, rng_.random(m), side="right"), n - 1)
        return c.astype(np.int64) * n + r.astype(np.int64)

    pos = _distinct_positions(rng, n, n, n_unique, draw)
    row, col = _assemble_list(rng, pos, n_dup, n)
    val = rng.standard_normal(size=row.size, dtype=np.float32)
    X = G = None
    if with_dense:
        X = rng.standard_normal(size=(n, k), dtype=np.float32)
        G = rng.standard_normal(size=(n, k), dtype=np.float32)
    return COOProblem("powerlaw_1e6x1e6_nnz2e7_f32_k%d" % k, n, n, row, col, val, X, G,
                      meta=dict(seed=seed, d_max=d_max))


def diff_2e5(seed: int = 1004, n: int = 200_000, nnz_in: int = 5_000_000, k: int = 64,
             value_dtype=np.float32) -> COOProblem:
    """Differentiation workload: n x n from nnz_in i.i.d. uniform locations (natural
    collisions only), values N(0,1), X n x k N(0,1), G fixed N(0,1)."""
    rng = np.random.Generator(np.random.PCG64(seed))
    pos = rng.integers(0, n * n, size=nnz_in, dtype=np.int64)
    row = (pos % n).astype(np.int32)
    col = (pos // n).astype(np.int32)
    val = rng.standard_normal(size=nnz_in).astype(value_dtype)
    X = rng.standard_normal(size=(n, k)).astype(value_dtype)
    G = rng.standard_normal(size=(n, k)).astype(value_dtype)
    name = "diff_%dx%d_nnz%d_%s_k%d" % (n, n, nnz_in, np.dtype(value_dtype).name, k)
    return COOProblem(name, n, n, row, col, val, X, G, meta=dict(seed=seed))


def trace_pair(seed: int = 1007, n: int = 10_000, density: float = 0.001,
               value_dtype=np.float64) -> tuple[COOProblem, COOProblem]:
    """The trace(A^T B) workload of the paper's evaluation: two independent n x n matrices,
    each with round(density * n^2) distinct uniform locations (no duplicates) and values
    U[-1,1]; the paper uses 10,000 x 10,000 at densities 0.01 %, 0.1 %, 1 % and 10 %."""
    nnz = int(round(density * n * n))
    tag = "trace_%dx%d_d%g" % (n, n, density)
    a = random_coo(seed, n, n, nnz, dup_frac=0.0, dtype=value_dtype, name=tag + "_A")
    b = random_coo(seed + 1, n, n, nnz, dup_frac=0.0, dtype=value_dtype, name=tag + "_B")
    return a, b


def diff_fd(seed: int = 1014) -> COOProblem:
    """Finite-difference instance: 2,000 x 2,000, 20,000 i.i.d. uniform triplets, k = 16,
    everything float64 N(0,1)."""
    return diff_2e5(seed=seed, n=2000, nnz_in=20_000, k=16, value_dtype=np.float64)


@dataclass
class Batch:
    """A batch of independent square problems (host arrays, one COOProblem per matrix)."""
    problems: list
    seed: int

    @property
    def sizes(self) -> np.ndarray:
        return np.array([p.n_rows for p in self.problems], dtype=np.int64)


def batch_sizes(seed: int = 1005, count: int = 4096, lo: int = 64, hi: int = 8192) -> np.ndarray:
    """n_b = round(exp(U(ln lo, ln hi))) for each matrix (log-uniform sizes)."""
    rng = np.random.Generator(np.random.PCG64(seed))
    return np.rint(np.exp(rng.uniform(math.log(lo), math.log(hi), size=count))).astype(np.int64)


def batch_problems(seed: int = 1005, count: int = 4096, lo: int = 64, hi: int = 8192,
                   per_col: int = 16, dup_frac: float = 0.10, k: int = 32) -> Batch:
    """Batch workload: ``count`` square matrices with log-uniform n in [lo, hi], per_col*n
    triplets each (uniform distinct locations plus dup_frac duplicates), values N(0,1)
    float32, X_b and G_b n x k float32 N(0,1).  Matrix b draws from its own PCG64 stream
    spawned from SeedSequence(seed)."""
    sizes = batch_sizes(seed, count, lo, hi)
    children = np.random.SeedSequence(seed).spawn(count)
    probs = []
    for b, (n, ss) in enumerate(zip(sizes, children)):
        rng = np.random.Generator(np.random.PCG64(ss))
        n = int(n)
        nnz_in = per_col * n
        n_dup = int(round(nnz_in * dup_frac))
        pos = _distinct_positions(rng, n, n, nnz_in - n_dup, _uniform_draw(n, n))
        row, col = _assemble_list(rng, pos, n_dup, n)
        val = rng.standard_normal(size=nnz_in, dtype=np.float32)
        X = rng.standard_normal(size=(n, k), dtype=np.float32)
        G = rng.standard_normal(size=(n, k), dtype=np.float32)
        probs.append(COOProblem("batch[%d]" % b, n, n, row, col, val, X, G, meta=dict(b=b)))
    return Batch(probs, seed)
