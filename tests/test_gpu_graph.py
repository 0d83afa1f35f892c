"""A whole step recorded into a HIP graph: every replay is bitwise equal to the eager step,
with the program's own eager work and synchronisations between the replays, and a replay
after refilling the input tensors equals the eager step on the new data."""
import numpy as np
import pytest
import torch

from paper_1805_03380_amd import synth
from paper_1805_03380_amd.ops import plan_arrays
from paper_1805_03380_amd.pipeline import Pipeline
from gpu_util import DEV, dev

pytestmark = pytest.mark.gpu

KEYS = ("col_ptr", "row_idx", "values", "values_plan", "row_ptr", "col_t", "perm", "Y", "dX",
        "dval", "info", "plan_info")


def _snap(pipe):
    """Everything a step writes (the first nnz entries of the capacity-sized arrays)."""
    torch.cuda.synchronize(DEV)
    nnz = int(pipe.info[0].item())
    rp, ct, pm = plan_arrays(pipe.plan, pipe.n_rows, pipe.nnz_in)
    out = dict(col_ptr=pipe.col_ptr, row_idx=pipe.row_idx[:nnz], values=pipe.values[:nnz],
               values_plan=pipe.values_plan[:nnz], row_ptr=rp, col_t=ct[:nnz], perm=pm[:nnz],
               Y=pipe.Y, dX=pipe.dX, dval=pipe.dval[:nnz], info=pipe.info,
               plan_info=pipe.plan_info)
    return {k: v.clone() for k, v in out.items()}


def _bits(t):
    return t.contiguous().view(torch.uint8)


def _equal(a, b):
    for k in KEYS:
        assert torch.equal(_bits(a[k]), _bits(b[k])), k


@pytest.mark.parametrize("fused", [True, False])
def test_graph_replays_equal_eager(fused):
    p = synth.random_coo(61, 20_000, 15_000, 300_000, dup_frac=0.1, dtype=np.float32, k=64)
    q = synth.random_coo(62, 20_000, 15_000, 300_000, dup_frac=0.1, dtype=np.float32, k=64)
    row, col, val, X, G = dev(p.row), dev(p.col), dev(p.val), dev(p.X), dev(p.G)
    ref_pipe = Pipeline(p.n_rows, p.n_cols, p.nnz_in, 64, fused=fused)
    ref_pipe.step(row, col, val, X, G)
    ref = _snap(ref_pipe)

    pipe = Pipeline(p.n_rows, p.n_cols, p.nnz_in, 64, fused=fused)
    g = pipe.capture(row, col, val, X, G)
    for i in range(3):
        # clobber the outputs, replay, compare; eager work of the program in between
        for k in ("Y", "dX", "dval", "col_ptr"):
            getattr(pipe, k).fill_(-1 - i)
        g.replay()
        torch.cuda.synchronize(DEV)
        _equal(ref, _snap(pipe))
        ref_pipe.step(row, col, val, X, G)
        _ = (X * 2.0).sum().item()
    # new data in the captured tensors
    row.copy_(dev(q.row))
    col.copy_(dev(q.col))
    val.copy_(dev(q.val))
    X.copy_(dev(q.X))
    G.copy_(dev(q.G))
    g.replay()
    ref_pipe.step(row, col, val, X, G)
    _equal(_snap(ref_pipe), _snap(pipe))
