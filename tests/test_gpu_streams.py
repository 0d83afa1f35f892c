"""Calls on different streams at once: every entry point keeps its state in the caller's
buffers and workspace (and in stream-ordered launches), so two pipelines driven concurrently
on two streams give bitwise what they give one after the other."""
import numpy as np
import pytest
import torch

from paper_1805_03380_amd import synth
from paper_1805_03380_amd.pipeline import Pipeline

pytestmark = pytest.mark.gpu


def _setup(p, dev):
    t = [torch.from_numpy(a).to(dev) for a in (p.row, p.col, p.val, p.X, p.G)]
    pipe = Pipeline(p.n_rows, p.n_cols, p.nnz_in, p.k, val_dtype=t[2].dtype, x_dtype=t[3].dtype)
    return pipe, t


def _outputs(pipe):
    return [x.clone() for x in (pipe.col_ptr, pipe.row_idx, pipe.values, pipe.Y, pipe.dX,
                                pipe.dval)]


def test_two_pipelines_on_two_streams():
    dev = torch.device("cuda:0")
    pa = synth.random_coo(2401, 20_000, 15_000, 300_000, dup_frac=0.1, dtype=np.float32,
                          dist="normal", k=64)
    pb = synth.random_coo(2402, 9_000, 30_000, 200_000, dup_frac=0.2, dtype=np.float32,
                          dist="normal", k=32)
    (A, ta), (B, tb) = _setup(pa, dev), _setup(pb, dev)
    A.step(*ta)
    B.step(*tb)
    torch.cuda.synchronize()
    ref_a, ref_b = _outputs(A), _outputs(B)
    s1, s2 = torch.cuda.Stream(device=dev), torch.cuda.Stream(device=dev)
    s1.wait_stream(torch.cuda.current_stream(dev))
    s2.wait_stream(torch.cuda.current_stream(dev))
    for _ in range(4):
        A.step(*ta, stream=s1)
        B.step(*tb, stream=s2)
    torch.cuda.synchronize()
    for got, want in zip(_outputs(A) + _outputs(B), ref_a + ref_b):
        assert torch.equal(got.view(torch.uint8), want.view(torch.uint8))
