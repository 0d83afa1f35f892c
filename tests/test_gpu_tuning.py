"""Tuning never changes results: every spm_tuning choice gives bitwise the same CSC, plan,
plan-order values, forward and adjoint (single-matrix path, with assembly and plan in one
call or in two) and the same batched outputs."""
import numpy as np
import pytest
import torch

from paper_1805_03380_amd import _lib, synth
from paper_1805_03380_amd.batch import PackedBatch
from paper_1805_03380_amd.ops import plan_arrays
from paper_1805_03380_amd.pipeline import Pipeline

pytestmark = pytest.mark.gpu

TUNINGS = [
    dict(spmm_block=64, spmm_blocks_per_cu=8, part_bucket_target=512, part_max_tiles=64),
    dict(spmm_block=128, spmm_blocks_per_cu=1, part_bucket_target=1024, part_max_tiles=4096),
    dict(spmm_block=256, spmm_blocks_per_cu=64, part_bucket_target=256, part_max_tiles=256),
]


def _run(p, dev="cuda:0", fused=True):
    row = torch.from_numpy(p.row).to(dev)
    col = torch.from_numpy(p.col).to(dev)
    val = torch.from_numpy(p.val).to(dev)
    X = torch.from_numpy(p.X).to(dev)
    G = torch.from_numpy(p.G).to(dev)
    pipe = Pipeline(p.n_rows, p.n_cols, p.nnz_in, p.k, val_dtype=val.dtype, x_dtype=X.dtype,
                    fused=fused)
    pipe.step(row, col, val, X, G)
    torch.cuda.synchronize()
    nnz, sa, sp = pipe.status()
    assert sa == 0 and sp == 0
    rp, ct, pm = plan_arrays(pipe.plan, p.n_rows, p.nnz_in)
    return dict(col_ptr=pipe.col_ptr.clone(), row_idx=pipe.row_idx[:nnz].clone(),
                values=pipe.values[:nnz].clone(), row_ptr=rp.clone(), col_t=ct[:nnz].clone(),
                perm=pm[:nnz].clone(), values_plan=pipe.values_plan[:nnz].clone(),
                Y=pipe.Y.clone(), dX=pipe.dX.clone(), dval=pipe.dval[:nnz].clone())


def _same(a, b):
    for k in a:
        x, y = a[k], b[k]
        if x.dtype.is_floating_point:
            x, y = x.view(torch.int32 if x.element_size() == 4 else torch.int64), \
                y.view(torch.int32 if y.element_size() == 4 else torch.int64)
        assert torch.equal(x, y), k


@pytest.mark.parametrize("dims", [(50_000, 40_000, 400_000, 64), (3000, 200, 60_000, 32),
                                  (20_000, 20_000, 80_000, 16)])
def test_pipeline_invariant_under_tuning(dims):
    n_rows, n_cols, nnz, k = dims
    p = synth.random_coo(900 + k, n_rows, n_cols, nnz, dup_frac=0.2, dtype=np.float32,
                         dist="normal", k=k)
    ref = _run(p)
    _same(ref, _run(p, fused=False))  # assembly and plan as two calls
    saved = _lib.get_tuning().as_dict()
    try:
        for tu in TUNINGS:
            _lib.set_tuning(**tu)
            _same(ref, _run(p))
            _same(ref, _run(p, fused=False))
    finally:
        _lib.set_tuning(**saved)


def test_batch_invariant_under_workers():
    bt = synth.batch_problems(seed=2007, count=64, lo=64, hi=3000)
    pb = PackedBatch(bt.problems)
    ref = pb.run_batched(out=pb.new_outputs())
    torch.cuda.synchronize()
    saved = _lib.get_tuning().as_dict()
    try:
        for w, ws in ((1, 1), (4, 0), (2, 16)):
            _lib.set_tuning(batch_wg_per_cu=w, batch_spmm_wg_per_cu=ws)
            out = pb.run_batched(out=pb.new_outputs())
            torch.cuda.synchronize()
            for key in ("col_ptr", "Y", "dX", "info"):
                assert torch.equal(ref[key].view(torch.int32), out[key].view(torch.int32)), key
    finally:
        _lib.set_tuning(**saved)
