"""GPU tests of the batched path (spm_batch_run): bitwise equal to the per-matrix
entry points, and per matrix equal to the oracle (assembly bit-exact, products within the
a-priori bound)."""
import numpy as np
import pytest
import torch

import oracle
from paper_1805_03380_amd import synth
from paper_1805_03380_amd.batch import PackedBatch
from gpu_util import assert_close

pytestmark = pytest.mark.gpu


def _small_batch(seed, count, lo, hi, per_col=16, k=32):
    return synth.batch_problems(seed=seed, count=count, lo=lo, hi=hi, per_col=per_col, k=k)


def _bitwise_equal(pb, o1, o2):
    info1 = o1["info"].cpu().numpy()
    info2 = o2["info"].cpu().numpy()
    assert np.array_equal(info1, info2)
    for key in ("col_ptr", "row_ptr", "Y", "dX"):
        assert torch.equal(o1[key].view(torch.int32), o2[key].view(torch.int32)), key
    for b in range(pb.B):
        to, n = int(pb.trip_off[b]), int(info1[2 * b])
        for key in ("row_idx", "val_out", "dval", "col_t", "perm"):
            a = o1[key][to:to + n].view(torch.int32)
            c = o2[key][to:to + n].view(torch.int32)
            assert torch.equal(a, c), (key, b)


def _oracle_check(pb, out, problems, b, acc_f32=False):
    p = problems[b]
    m = pb.matrix(out, b)
    assert m["info"][1] == 0
    vals = p.val
    if pb.val_dtype == torch.bfloat16:
        vals = oracle.widen(torch.from_numpy(p.val.astype(np.float32)).to(torch.bfloat16))
    st, R = oracle.coo_to_csc(p.n_rows, p.n_cols, p.row, p.col, vals)
    assert np.array_equal(m["col_ptr"], R.col_ptr)
    assert np.array_equal(m["row_idx"], R.row_idx)
    assert np.array_equal(m["values"], R.values.astype(np.float32))
    X = p.X.astype(np.float32)
    G = p.G.astype(np.float32)
    if pb.x_dtype == torch.bfloat16:
        X = oracle.widen(torch.from_numpy(X).to(torch.bfloat16))
        G = oracle.widen(torch.from_numpy(G).to(torch.bfloat16))
    rv = m["values"].astype(np.float64)
    Yr, S, M = oracle.spmm(R, X, values=rv)
    dXr, dvr, SdX, Sdv = oracle.spmm_backward(R, G, X, values=rv)
    assert_close(m["Y"], Yr, S, M, torch.float32, acc_f32, "Y[%d]" % b)
    assert_close(m["dX"], dXr, SdX, np.diff(R.col_ptr), torch.float32, acc_f32, "dX[%d]" % b)
    assert_close(m["dval"], dvr, Sdv, pb.k, torch.float32, acc_f32, "dval[%d]" % b)


@pytest.mark.parametrize("x_dtype", [torch.float32, torch.bfloat16])
def test_small_batch_equals_single_and_oracle(x_dtype):
    bt = _small_batch(2005, 96, 24, 600)
    pb = PackedBatch(bt.problems, val_dtype=x_dtype, x_dtype=x_dtype)
    o_b = pb.run_batched()
    o_s = pb.run_single(out=pb.new_outputs())
    torch.cuda.synchronize()
    _bitwise_equal(pb, o_b, o_s)
    for b in range(0, pb.B, 7):
        _oracle_check(pb, o_b, bt.problems, b, acc_f32=(x_dtype == torch.bfloat16))


@pytest.mark.parametrize("k,x_dtype", [(1, torch.float32), (5, torch.float32),
                                         (20, torch.float32), (64, torch.float32),
                                         (130, torch.float32), (20, torch.bfloat16)])
def test_other_k_general_products(k, x_dtype):
    """k other than 32: group widths 1 to 64 and the general product path (k not 4 lanes' worth
    per lane, pieces beyond one per lane, rows not 4-aligned), bitwise equal to the per-matrix
    calls and within the bound against the oracle."""
    bt = _small_batch(2010 + k, 40, 16, 700, k=k)
    pb = PackedBatch(bt.problems, val_dtype=x_dtype, x_dtype=x_dtype)
    o_b = pb.run_batched()
    o_s = pb.run_single(out=pb.new_outputs())
    torch.cuda.synchronize()
    _bitwise_equal(pb, o_b, o_s)
    for b in (0, 17, 39):
        _oracle_check(pb, o_b, bt.problems, b, acc_f32=(x_dtype == torch.bfloat16))


@pytest.mark.parametrize("val_dtype,x_dtype", [(torch.bfloat16, torch.float32),
                                               (torch.float32, torch.bfloat16)])
def test_mixed_value_and_dense_types(val_dtype, x_dtype):
    """Values and dense operands of different types (bfloat16 values with binary32 X and G,
    and the reverse): bitwise equal to the per-matrix calls, within the bound of the oracle."""
    bt = _small_batch(2020, 48, 24, 900)
    pb = PackedBatch(bt.problems, val_dtype=val_dtype, x_dtype=x_dtype)
    o_b = pb.run_batched()
    o_s = pb.run_single(out=pb.new_outputs())
    torch.cuda.synchronize()
    _bitwise_equal(pb, o_b, o_s)
    for b in (0, 23, 47):
        _oracle_check(pb, o_b, bt.problems, b, acc_f32=(x_dtype == torch.bfloat16))


def test_items_beyond_the_limits_are_refused_alone():
    """A call whose max_dim is below one matrix's rows: that matrix alone gets SPM_EINVAL and
    no output; every other matrix is assembled and multiplied as usual."""
    from paper_1805_03380_amd import _lib
    bt = _small_batch(2030, 12, 30, 400)
    big = synth.random_coo(2031, 1000, 900, 9000, dtype=np.float32, dist="normal", k=32)
    probs = bt.problems + [big]
    pb = PackedBatch(probs)
    assert pb.max_dim == 1000
    pb.max_dim = 999
    o = pb.run_batched(out=pb.new_outputs())
    torch.cuda.synchronize()
    info = o["info"].cpu().numpy().reshape(-1, 2)
    assert info[-1, 1] == _lib.EINVAL and info[-1, 0] == 0
    assert (info[:-1, 1] == 0).all()
    for b in (0, 5, 11):
        _oracle_check(pb, o, probs, b)


def test_large_dims_global_counters_and_giant_column():
    """One matrix larger than the LDS counter capacity, one with a column longer than an LDS
    sort chunk, one with an out-of-range triplet (its own status only), an empty one, and one
    whose row and input position do not fit the packed key (values gathered by position)."""
    rng = np.random.Generator(np.random.PCG64(31))
    probs = []
    n = 12_000
    probs.append(synth.random_coo(32, n, n, 50_000, dup_frac=0.1, dtype=np.float32,
                                  dist="normal", k=32))
    m = 3000
    row = rng.integers(0, m, 9000).astype(np.int32)
    col = np.where(rng.random(9000) < 0.8, 17, rng.integers(0, m, 9000)).astype(np.int32)
    g = synth.COOProblem("giant", m, m, row, col, rng.standard_normal(9000).astype(np.float32),
                         rng.standard_normal((m, 32)).astype(np.float32),
                         rng.standard_normal((m, 32)).astype(np.float32))
    probs.append(g)
    bad = synth.random_coo(33, 100, 100, 500, dtype=np.float32, dist="normal", k=32)
    bad.row = bad.row.copy()
    bad.row[10] = 100  # out of range
    probs.append(bad)
    probs.append(synth.random_coo(34, 50, 70, 0, dtype=np.float32, k=32))  # empty
    # row and input position need 16 + 17 bits: plain keys, values gathered by position
    probs.append(synth.random_coo(35, 65_536, 64, 70_000, dup_frac=0.1, dtype=np.float32,
                                  dist="normal", k=32))
    pb = PackedBatch(probs)
    o_b = pb.run_batched()
    o_s = pb.run_single(out=pb.new_outputs())
    torch.cuda.synchronize()
    info = o_b["info"].cpu().numpy().reshape(-1, 2)
    assert info[2, 1] == 2 and info[0, 1] == 0 and info[1, 1] == 0 and info[3, 1] == 0
    assert info[3, 0] == 0 and info[4, 1] == 0
    _bitwise_equal(pb, o_b, o_s)
    _oracle_check(pb, o_b, probs, 0)
    _oracle_check(pb, o_b, probs, 1)
    _oracle_check(pb, o_b, probs, 4)


def test_giant_row_in_the_plan():
    """A matrix with one row longer than an LDS sort chunk (5000 stored elements in row 5), so
    the per-row sort of the plan takes its global merge-sort path, beside ordinary ones."""
    rng = np.random.Generator(np.random.PCG64(36))
    n = 6000
    cols = rng.permutation(n)[:5000].astype(np.int32)
    row = np.concatenate([np.full(5000, 5, np.int32), rng.integers(0, n, 20_000).astype(np.int32)])
    col = np.concatenate([cols, rng.integers(0, n, 20_000).astype(np.int32)])
    perm = rng.permutation(row.size)
    g = synth.COOProblem("giant_row", n, n, row[perm], col[perm],
                         rng.standard_normal(row.size).astype(np.float32),
                         rng.standard_normal((n, 32)).astype(np.float32),
                         rng.standard_normal((n, 32)).astype(np.float32))
    probs = [g, synth.random_coo(37, 700, 500, 8000, dup_frac=0.1, dtype=np.float32,
                                 dist="normal", k=32)]
    pb = PackedBatch(probs)
    o_b = pb.run_batched()
    o_s = pb.run_single(out=pb.new_outputs())
    torch.cuda.synchronize()
    _bitwise_equal(pb, o_b, o_s)
    r0 = int(pb.rowptr_off[0])
    rp = o_b["row_ptr"][r0: r0 + n + 1].cpu().numpy()
    assert int(rp[6] - rp[5]) >= 5000
    _oracle_check(pb, o_b, probs, 0)
    _oracle_check(pb, o_b, probs, 1)


@pytest.fixture(scope="module")
def full_batch():
    return synth.batch_problems()


@pytest.mark.parametrize("dtype", [torch.float32, torch.bfloat16])
def test_full_batch_workload_bitwise_and_sampled_oracle(full_batch, dtype):
    """The 4096-matrix workload (n log-uniform in [64, 8192], 16 triplets per column, 10 %
    duplicates, k = 32), in float32 and in the bfloat16 variant (values, X and G rounded to
    bfloat16, binary32 accumulation): the batched entry point is bitwise equal to 4096
    per-matrix calls, and sampled matrices match the oracle."""
    bt = full_batch
    pb = PackedBatch(bt.problems, val_dtype=dtype, x_dtype=dtype)
    o_b = pb.run_batched()
    o_s = pb.run_single(out=pb.new_outputs())
    torch.cuda.synchronize()
    _bitwise_equal(pb, o_b, o_s)
    order = pb.order_host
    for b in [int(order[0]), int(order[-1]), 0, 1234, 4095]:
        _oracle_check(pb, o_b, bt.problems, b, acc_f32=(dtype == torch.bfloat16))
    if dtype == torch.float32:
        _all_structures_match_oracle(pb, o_b, bt.problems)


def _all_structures_match_oracle(pb, out, problems):
    """Every matrix of the batch: col_ptr, row_idx and the stored values bit for bit against
    the oracle (host threads; the oracle's C code runs without the interpreter lock)."""
    import os
    from concurrent.futures import ThreadPoolExecutor
    cp_all = out["col_ptr"].cpu().numpy()
    ri_all = out["row_idx"].cpu().numpy()
    vo_all = out["val_out"].cpu().numpy()
    info = out["info"].cpu().numpy().reshape(-1, 2)
    co = pb.colptr_off

    def one(b):
        p = problems[b]
        st, R = oracle.coo_to_csc(p.n_rows, p.n_cols, p.row, p.col, p.val)
        to = int(pb.trip_off[b])
        c0 = int(co[b])
        n = int(info[b, 0])
        ok = st == oracle.OK and info[b, 1] == 0 and n == R.nnz
        ok = ok and np.array_equal(cp_all[c0:c0 + p.n_cols + 1], R.col_ptr)
        ok = ok and np.array_equal(ri_all[to:to + n], R.row_idx)
        ok = ok and np.array_equal(vo_all[to:to + n], R.values.astype(np.float32))
        return b, ok

    workers = max(1, min(16, len(os.sched_getaffinity(0))))
    with ThreadPoolExecutor(max_workers=workers) as ex:
        bad = [b for b, ok in ex.map(one, range(pb.B)) if not ok]
    assert not bad, "matrices differing from the oracle: %s" % bad[:10]


def test_batch_with_named_tuning_equals_default():
    """spm_batch_coo_to_csc_spmm with a registered tune key: bitwise the same outputs as
    spm_batch_run under the process tuning (tuning never changes results)."""
    from paper_1805_03380_amd import _lib
    bt = _small_batch(2009, 300, 40, 3000)
    pb = PackedBatch(bt.problems)
    o_d = pb.run_batched(out=pb.new_outputs())
    _lib.register_tuning("test-batch-narrow", batch_wg_per_cu=1, batch_spmm_wg_per_cu=2)
    o_k = pb.run_batched(out=pb.new_outputs(), tune_key="test-batch-narrow")
    torch.cuda.synchronize()
    _bitwise_equal(pb, o_d, o_k)


def test_deterministic_rerun():
    bt = _small_batch(2006, 40, 64, 2000)
    pb = PackedBatch(bt.problems)
    o1 = pb.run_batched(out=pb.new_outputs())
    o2 = pb.run_batched(out=pb.new_outputs())
    torch.cuda.synchronize()
    _bitwise_equal(pb, o1, o2)


@pytest.mark.parametrize("k", [32, 5])
def test_flat_and_per_matrix_products_agree(k):
    """The products run flat over all rows / columns when the grouping workspace can hold the
    batch's row and column prefixes (16 bytes per matrix), else one workgroup per matrix.
    Many tiny matrices with one grouping workgroup per CU take the per-matrix form, the
    default tuning the flat one; both are bitwise equal to the per-matrix calls (k = 32: the
    full-width path; k = 5: the general one)."""
    from paper_1805_03380_amd import _lib
    bt = _small_batch(2008, 5000, 2, 6, per_col=2, k=k)
    pb = PackedBatch(bt.problems)
    o_s = pb.run_single(out=pb.new_outputs())
    torch.cuda.synchronize()
    cus = torch.cuda.get_device_properties(0).multi_processor_count
    max_nnz = max(p.nnz_in for p in bt.problems)
    max_dim = max(max(p.n_rows, p.n_cols) for p in bt.problems)
    stride = (16 * max_nnz + 4 * (max_dim + 1) + 255) // 256 * 256
    saved = _lib.get_tuning().as_dict()
    seen = set()
    try:
        for wpc in (1, 2):
            _lib.set_tuning(batch_wg_per_cu=wpc)
            w = min(cus * wpc, pb.B)
            seen.add(w * stride >= 16 * (pb.B + 1))
            pb2 = PackedBatch(bt.problems)
            o_b = pb2.run_batched(out=pb2.new_outputs())
            torch.cuda.synchronize()
            _bitwise_equal(pb2, o_b, o_s)
    finally:
        _lib.set_tuning(**saved)
    assert seen == {True, False}, "both product forms must be exercised"
