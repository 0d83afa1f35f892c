"""The power-law workload at full size: 1,000,000 x 1,000,000 from 20,000,000 Chung-Lu
triplets (Zipf(1.5) expected degrees, 30 % duplicates), k = 128 -- assembly bit-exact against
the oracle, forward and adjoint against the oracle everywhere."""
import numpy as np
import pytest
import torch

import oracle
from paper_1805_03380_amd import synth
from paper_1805_03380_amd.pipeline import Pipeline
from gpu_util import assert_close

pytestmark = pytest.mark.gpu


def test_powerlaw_full():
    p = synth.powerlaw_1e6()
    dev = "cuda:0"
    pipe = Pipeline(p.n_rows, p.n_cols, p.nnz_in, p.k)
    X = torch.from_numpy(p.X).to(dev)
    G = torch.from_numpy(p.G).to(dev)
    pipe.step(torch.from_numpy(p.row).to(dev), torch.from_numpy(p.col).to(dev),
              torch.from_numpy(p.val).to(dev), X, G)
    torch.cuda.synchronize()
    nnz, sa, sp = pipe.status()
    assert sa == 0 and sp == 0
    st, R = oracle.coo_to_csc(p.n_rows, p.n_cols, p.row, p.col, p.val)
    assert nnz == R.nnz
    assert np.array_equal(pipe.col_ptr.cpu().numpy(), R.col_ptr)
    assert np.array_equal(pipe.row_idx[:nnz].cpu().numpy(), R.row_idx)
    vals = pipe.values[:nnz].cpu().numpy()
    assert np.array_equal(vals, R.values.astype(np.float32))
    rv = vals.astype(np.float64)
    Yr, S, M = oracle.spmm(R, p.X, values=rv)
    assert_close(pipe.Y, Yr, S, M, torch.float32, what="Y")
    del Yr, S
    dXr, dvr, SdX, Sdv = oracle.spmm_backward(R, p.G, p.X, values=rv)
    assert_close(pipe.dX, dXr, SdX, np.diff(R.col_ptr), torch.float32, what="dX")
    assert_close(pipe.dval[:nnz], dvr, Sdv, p.k, torch.float32, what="dval")
