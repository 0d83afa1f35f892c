"""Helpers shared by the GPU parity tests: move seeded host inputs to the device, run the HIP
path through the C ABI (via paper_1805_03380_amd.ops), and compare with the oracle."""
from __future__ import annotations

import numpy as np
import torch

import oracle
from paper_1805_03380_amd import ops

DEV = "cuda:0"


def dev(a, dtype=None):
    t = torch.from_numpy(np.ascontiguousarray(a))
    if dtype is not None:
        t = t.to(dtype)
    return t.to(DEV)


def assemble_gpu(p, out_dtype=None, val_dtype=None):
    v = dev(p.val, val_dtype)
    return ops.coo_to_csc(dev(p.row), dev(p.col), v, (p.n_rows, p.n_cols), out_dtype=out_dtype)


def assert_csc_equal(A_gpu, A_ref, out_np_dtype):
    """Structure bit-exact; values bit-exact against the oracle's binary64 fold rounded once."""
    cp = A_gpu.col_ptr.cpu().numpy()
    assert np.array_equal(cp, A_ref.col_ptr), "col_ptr differs"
    assert A_gpu.nnz == A_ref.nnz, (A_gpu.nnz, A_ref.nnz)
    ri = A_gpu.row_idx.cpu().numpy()
    assert np.array_equal(ri, A_ref.row_idx), "row_idx differs"
    got = A_gpu.values.cpu().numpy()
    want = A_ref.values.astype(out_np_dtype)
    assert got.dtype == want.dtype
    gn, wn = np.isnan(got), np.isnan(want)
    assert np.array_equal(gn, wn)
    assert np.array_equal(got[~gn].view(np.uint8), want[~wn].view(np.uint8)), \
        "values differ at %s" % np.nonzero(got[~gn] != want[~wn])[0][:10]


def rtol_for(dtype) -> float:
    return 1e-12 if dtype == torch.float64 else 1e-5


def assert_close(got, want, scale, m, out_dtype, acc_f32: bool = False, what: str = ""):
    """|got - want| <= rtol |want| + 2 gamma_m(u) * scale, per output (the oracle's own a-priori
    bound of a fixed-order sum, u = 2^-53, or 2^-24 when the kernel accumulates in binary32)."""
    got = got.detach().double().cpu().numpy() if hasattr(got, "detach") else np.asarray(got)
    got = np.asarray(got, dtype=np.float64).reshape(want.shape)
    m = np.broadcast_to(np.asarray(m, dtype=np.float64).reshape(
        (-1,) + (1,) * (want.ndim - 1)) if np.ndim(m) else m, want.shape)
    u = 2.0 ** -24 if acc_f32 else 2.0 ** -53
    tol = rtol_for(out_dtype) * np.abs(want) + 2.0 * oracle.gamma(m, u) * scale
    err = np.abs(got - want)
    bad = ~(err <= tol)
    if bad.any():
        i = np.argwhere(bad)[0]
        raise AssertionError("%s: %d outputs outside tolerance; first %s got %r want %r tol %r"
                             % (what, int(bad.sum()), tuple(i), got[tuple(i)], want[tuple(i)],
                                tol[tuple(i)]))
    return float(np.max(err / np.maximum(np.abs(want), 1e-300)))
