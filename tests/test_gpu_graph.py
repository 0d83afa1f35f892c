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


def test_graph_trace_and_triplet_grad():
    """trace(A^T B) and the gradient per input triplet recorded into one graph: every replay,
    with eager work between, equals the eager calls bit for bit (neither allocates, clears
    memory with a memset or synchronises)."""
    from paper_1805_03380_amd import _lib, ops
    p = synth.random_coo(4100, 3000, 2500, 60_000, dup_frac=0.2, dist="normal")
    q = synth.random_coo(4101, 3000, 2500, 60_000, dup_frac=0.2, dist="normal")
    A = ops.coo_to_csc(dev(p.row), dev(p.col), dev(p.val), (p.n_rows, p.n_cols))
    B = ops.coo_to_csc(dev(q.row), dev(q.col), dev(q.val), (q.n_rows, q.n_cols))
    rng = np.random.Generator(np.random.PCG64(4102))
    G = dev(rng.standard_normal((p.n_rows, 32)))
    X = dev(rng.standard_normal((p.n_cols, 32)))
    row, col = dev(p.row), dev(p.col)
    lib = _lib.load()
    wb = _lib.ctypes.c_size_t(0)
    assert lib.spm_csc_trace_atb_workspace(p.n_cols, _lib.ctypes.byref(wb)) == _lib.OK
    ws = torch.empty(max(wb.value, 256), dtype=torch.uint8, device=DEV)
    out = torch.empty(1, dtype=torch.float64, device=DEV)
    info = torch.empty(2, dtype=torch.int32, device=DEV)
    dv = torch.empty(p.nnz_in, dtype=torch.float64, device=DEV)

    def calls(stream):
        assert lib.spm_csc_trace_atb(
            A.n_rows, A.n_cols, A.nnz_cap, A.col_ptr.data_ptr(), A.row_idx_buf.data_ptr(),
            A.values_buf.data_ptr(), B.nnz_cap, B.col_ptr.data_ptr(), B.row_idx_buf.data_ptr(),
            B.values_buf.data_ptr(), _lib.F64, out.data_ptr(), info.data_ptr(), ws.data_ptr(),
            ws.numel(), stream) == _lib.OK
        assert lib.spm_coo_triplet_grad(
            p.n_rows, p.n_cols, p.nnz_in, 32, row.data_ptr(), col.data_ptr(), _lib.F64,
            G.data_ptr(), 32, _lib.F64, X.data_ptr(), 32, _lib.F64, dv.data_ptr(), _lib.F64,
            stream) == _lib.OK

    s = torch.cuda.Stream(device=DEV)
    with torch.cuda.stream(s):
        calls(s.cuda_stream)
    torch.cuda.synchronize(DEV)
    want = (out.clone(), info.clone(), dv.clone())
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g, stream=s):
        calls(s.cuda_stream)
    for i in range(3):
        out.fill_(float(i + 7))
        info.fill_(-1)
        dv.fill_(1.5)
        torch.cuda.synchronize(DEV)
        g.replay()
        torch.cuda.synchronize(DEV)
        assert torch.equal(_bits(out), _bits(want[0])), i
        assert torch.equal(info, want[1]), i
        assert torch.equal(_bits(dv), _bits(want[2])), i
