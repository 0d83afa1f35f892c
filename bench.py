#!/usr/bin/env python
"""Benchmark of the sparse hot path on one MI355X.

One step = one pass of the whole path over one batch of synthetic input already resident in
HBM: COO -> CSC assembly and plan in one call (spm_coo_to_csc_plan; with --separate,
spm_coo_to_csc then spm_csc_plan_build), forward Y = A.X (spm_csc_spmm) and adjoint dX,
dvalues (spm_csc_spmm_backward).

Headline workload (the largest single-GPU one): the power-law 1,000,000 x 1,000,000 matrix
from 20,000,000 triplets (14e6 distinct Chung-Lu locations with Zipf(1.5) expected row and
column degrees, 6e6 duplicates, float32 values N(0,1)), dense X and G 1,000,000 x 128 float32
N(0,1) (seed 1003).  --workload picks another one.

Prints ONE JSON line.  `value` is input triplets per second through the whole step, over K
eager steps on one stream with nothing recorded between them.  The per-phase breakdown comes
from a separate pass of K steps with HIP events between the phases; K replays of the step
recorded in a HIP graph are reported under "graph".  `roofline` covers the kernel that takes
the largest share of the step; `cpu_baseline` is the oracle timed on the host cores on a
bounded sample of the same workload.  `configs` holds the same step on the other workloads
(tiny, uniform float32 / float64, differentiation), each with its roofline fraction, and the
operations around the hot path are timed on the uniform workload's CSC.

    python bench.py [--gpus 1] [--steps 20] [--warmup 5] [--workload powerlaw] [--no-cpu]
                    [--no-side] [--no-batch] [--separate] [--no-graph] [--no-insert]
                    [--no-transpose] [--no-tgrad] [--no-trace] [--cold-steps 5]
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

HBM_PEAK_GBPS = 8000.0  # MI355X HBM3E, GB/s
HERE = os.path.dirname(os.path.abspath(__file__))

# workload -> (synth constructor name, keyword arguments, label)
WORKLOADS = {
    "powerlaw": ("powerlaw_1e6", {}, "powerlaw_1e6x1e6_nnz2e7_f32_k128"),
    "uniform": ("uniform_1e5", {"value_dtype": "float32"}, "uniform_1e5x1e5_nnz1e6_f32_k64"),
    "uniform_f64": ("uniform_1e5", {"value_dtype": "float64"},
                    "uniform_1e5x1e5_nnz1e6_f64_k64"),
    "diff": ("diff_2e5", {}, "diff_2e5x2e5_nnz5e6_f32_k64"),
    "tiny": ("tiny_spmv", {}, "tiny_1000x1000_nnz1e4_f64_k1"),
}
SIDE_ORDER = ("tiny", "uniform", "uniform_f64", "diff", "powerlaw")


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--workload", default="powerlaw", choices=sorted(WORKLOADS))
    ap.add_argument("--no-cpu", action="store_true", help="skip the oracle CPU baseline")
    ap.add_argument("--no-side", action="store_true",
                    help="skip the other workloads (and the operations timed on the uniform one)")
    ap.add_argument("--no-batch", action="store_true", help="skip batched vs per-matrix")
    ap.add_argument("--cpu-seconds", type=float, default=10.0)
    ap.add_argument("--cold-steps", type=int, default=5,
                    help="steps timed one by one after writing 1 GiB of scratch (cold caches)")
    ap.add_argument("--no-graph", action="store_true",
                    help="skip the K steps timed as replays of the step recorded in a HIP graph")
    ap.add_argument("--no-insert", action="store_true",
                    help="skip the batch-insertion measurement")
    ap.add_argument("--no-transpose", action="store_true",
                    help="skip the transpose and row-vector product measurement")
    ap.add_argument("--no-tgrad", action="store_true",
                    help="skip the per-triplet gradient measurement")
    ap.add_argument("--no-trace", action="store_true",
                    help="skip the trace(A^T B) measurement")
    ap.add_argument("--trace-densities", type=lambda t: [float(x) for x in t.split(",")],
                    default=[0.0001, 0.001, 0.01, 0.1],
                    help="densities of the trace(A^T B) workload (comma-separated)")
    ap.add_argument("--separate", action="store_true",
                    help="assembly and plan as two calls (default: spm_coo_to_csc_plan)")
    ap.add_argument("--copy-calib-mib", type=int, default=0,
                    help="only run a plain device copy of this many MiB (counter calibration)")
    ap.add_argument("--batch-only", choices=("float32", "bfloat16"), default=None,
                    help="only run the batched path of the 4096-matrix workload in this dtype, "
                         "--warmup then --steps calls (for profiling its kernels)")
    return ap.parse_args()


def batch_only(dtype_name, steps, warmup):
    """The batched entry point alone on the 4096-matrix workload: one JSON line with its
    average time per call."""
    import torch
    from paper_1805_03380_amd import autotune, synth
    from paper_1805_03380_amd.batch import PackedBatch
    autotune.apply(autotune.load_table(), autotune.batch_signature(dtype_name))
    dt = torch.bfloat16 if dtype_name == "bfloat16" else torch.float32
    pb = PackedBatch(synth.batch_problems().problems, val_dtype=dt, x_dtype=dt)
    for _ in range(max(1, warmup)):
        pb.run_batched()
    torch.cuda.synchronize()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(steps):
        pb.run_batched()
    e1.record()
    torch.cuda.synchronize()
    print(json.dumps({"workload": batch_workload_label(dtype_name), "steps": steps,
                      "batched_ms": e0.elapsed_time(e1) / max(1, steps)}), flush=True)


def make_problem(name):
    import numpy as np
    from paper_1805_03380_amd import synth
    ctor, kw, label = WORKLOADS[name]
    kw = dict(kw)
    if "value_dtype" in kw:
        kw["value_dtype"] = np.dtype(kw["value_dtype"]).type
    return getattr(synth, ctor)(**kw), label


def model_bytes(n_rows, n_cols, nnz_in, nnz, k, s_vin, s_v, s_x, s_y, s_dx, s_g=None):
    """Algorithmic (compulsory) HBM bytes of each call: every input read once, every output
    written once (the dense operands once per row, not once per nonzero).  The plan build
    also carries the values to plan order (read in CSC order, written in plan order), and
    the forward product reads row_ptr, col_t and those values."""
    s_g = s_y if s_g is None else s_g
    asm = nnz_in * (4 + 4 + s_vin) + nnz * (4 + s_v) + 4 * (n_cols + 1)
    plan = 4 * (n_cols + 1) + nnz * (4 + s_v) + 4 * (n_rows + 1) + nnz * (8 + s_v)
    fwd = 4 * (n_rows + 1) + nnz * (4 + s_v) + n_cols * k * s_x + n_rows * k * s_y
    bwd = (4 * (n_cols + 1) + nnz * (4 + s_v) + n_rows * k * s_g + n_cols * k * s_x
           + n_cols * k * s_dx + nnz * s_v)
    # one call: the plan's outputs only, its input is the assembly's own survivors
    asm_plan = asm + 4 * (n_rows + 1) + nnz * (8 + s_v)
    return dict(assemble=asm, plan=plan, assemble_plan=asm_plan, forward=fwd, backward=bwd)


def gather_bytes(nnz, k, s_x):
    """Dense-operand bytes when every nonzero re-reads its dense row (no reuse)."""
    return nnz * k * s_x


def _oracle_pass(p):
    import oracle
    st, A = oracle.coo_to_csc(p.n_rows, p.n_cols, p.row, p.col, p.val)
    oracle.spmm(A, p.X)
    oracle.spmm_backward(A, p.G, p.X)


def cpu_baseline(p, label, seconds):
    """The oracle as it stands (single thread, binary64) on the same workload: full
    assemble + forward + adjoint passes, at least one, until about `seconds` are spent."""
    t0 = time.perf_counter()
    reps = 0
    while True:
        _oracle_pass(p)
        reps += 1
        el = time.perf_counter() - t0
        if el >= seconds or reps >= 50:
            break
    return dict(value=p.nnz_in * reps / el, unit="nnz/s", cores=1, kind="oracle",
                sample="%d full pass(es) (assemble + forward + adjoint) of the %s workload "
                       "(%d triplets, k=%d), binary64 oracle, single thread, %.1f s"
                       % (reps, label, p.nnz_in, p.k, el))


def cpu_all_cores(p, label, seconds, threads):
    """The same oracle passes on all the host cores given: `threads` Python threads each run
    whole passes (the oracle's C code runs without the interpreter lock) on the shared
    read-only inputs, every thread at least one; the rate is the total over the threads."""
    import threading
    done = [0] * threads
    t0 = time.perf_counter()

    def work(i):
        while True:
            _oracle_pass(p)
            done[i] += 1
            if time.perf_counter() - t0 >= seconds:
                break

    ts = [threading.Thread(target=work, args=(i,)) for i in range(threads)]
    for t in ts:
        t.start()
    for t in ts:
        t.join()
    el = time.perf_counter() - t0
    reps = sum(done)
    return dict(value=p.nnz_in * reps / el, unit="nnz/s", cores=threads, kind="oracle",
                sample="%d full passes on %d threads (one independent pass per thread) of the "
                       "%s workload, binary64 oracle, %.1f s" % (reps, threads, label, el))


def batched_vs_single(bt, dtype_name="float32", reps_batched=5, reps_single=3):
    """The 4096-matrix workload: the batched entry point (one grouping launch, a prefix launch,
    two flat product launches) vs 4096 x 4 per-matrix calls of the same kernels; outputs
    compared bitwise.  dtype_name "bfloat16" is the variant with values, X and G in bfloat16
    and binary32 accumulation."""
    import torch
    from paper_1805_03380_amd.batch import PackedBatch
    from paper_1805_03380_amd import autotune
    autotune.apply(autotune.load_table(), autotune.batch_signature(dtype_name))
    dt = torch.bfloat16 if dtype_name == "bfloat16" else torch.float32
    t0 = time.perf_counter()
    pb = PackedBatch(bt.problems, val_dtype=dt, x_dtype=dt)
    gen_s = time.perf_counter() - t0
    o_single = pb.new_outputs()
    pb.run_batched()
    pb.run_single(out=o_single, keep_plan=False)
    torch.cuda.synchronize()

    def timed(fn, reps):
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        torch.cuda.synchronize()
        e0.record()
        for _ in range(reps):
            fn()
        e1.record()
        torch.cuda.synchronize()
        return e0.elapsed_time(e1) / reps

    ms_b = timed(lambda: pb.run_batched(), reps_batched)
    ms_s = timed(lambda: pb.run_single(out=o_single, keep_plan=False), reps_single)
    ob = pb.out
    same = bool(torch.equal(ob["info"], o_single["info"]))
    for key in ("col_ptr", "Y", "dX"):
        same = same and bool(torch.equal(ob[key].view(torch.int32), o_single[key].view(torch.int32)))
    info = ob["info"].cpu().numpy().reshape(-1, 2)
    mask = torch.zeros(ob["row_idx"].numel(), dtype=torch.bool, device=ob["row_idx"].device)
    offs = pb.trip_off
    for b in range(pb.B):
        mask[int(offs[b]): int(offs[b]) + int(info[b, 0])] = True
    for key in ("row_idx", "val_out", "dval"):
        same = same and bool(torch.equal(ob[key].view(torch.int32)[mask],
                                         o_single[key].view(torch.int32)[mask]))
    nnz_in = int(pb.trip_off[-1])
    nnz = int(info[:, 0].sum())
    # B_min of the batch: compulsory assembly bytes plus both products' B_min, every matrix
    sv = 2 if dt == torch.bfloat16 else 4
    sx = sv
    n_sum = int(sum(p.n_rows for p in bt.problems))
    k = int(bt.problems[0].X.shape[1])
    b_asm = nnz_in * (8 + sv) + nnz * (4 + 4) + 4 * (n_sum + len(bt.problems))
    b_plan = 4 * (n_sum + len(bt.problems)) + nnz * 8
    b_fwd = 4 * n_sum + nnz * 8 + n_sum * k * sx + n_sum * k * 4
    b_bwd = 4 * n_sum + nnz * 8 + 2 * n_sum * k * sx + n_sum * k * 4 + nnz * 4
    b_min = b_asm + b_plan + b_fwd + b_bwd
    return {"workload": batch_workload_label(dtype_name),
            "nnz_in": nnz_in, "nnz": nnz, "batched_ms": ms_b, "per_matrix_ms": ms_s,
            "speedup": ms_s / ms_b, "batched_nnz_per_s": nnz_in / (ms_b * 1e-3),
            "bitwise_equal": same, "pack_s": gen_s, "B_min_bytes": b_min,
            "B_min_GBps": b_min / (ms_b * 1e-3) / 1e9,
            "B_min_frac": b_min / (ms_b * 1e-3) / 1e9 / HBM_PEAK_GBPS}


def batch_workload_label(dtype_name):
    return ("4096 matrices, n log-uniform [64, 8192], 16 triplets/column, 10 percent "
            "duplicates, %s, k=32 (seed 1005)" % dtype_name)


def _traffic_record(label):
    path = os.path.join(HERE, "profiles", "traffic_%s.json" % label)
    if not os.path.exists(path):
        return None
    with open(path) as f:
        return json.load(f)


def _tuning_matches(tr, tuning, prefix):
    return all(tuning.get(k) == v for k, v in (tr.get("tuning") or {}).items()
               if k.startswith(prefix))


def stored_traffic(label, phase, tuning):
    """HBM bytes per launch of the SpMM kernel of `phase` on workload `label`, from the
    committed counter runs (profiles/traffic_<label>.json) -- None unless the kernel sources
    and the launch tuning are still the ones the counters were taken with."""
    from paper_1805_03380_amd import profiling
    tr = _traffic_record(label)
    if tr is None or tr.get("spmm_source_sha256") != profiling.spmm_source_hash():
        return None
    if not _tuning_matches(tr, tuning, "spmm_"):
        return None
    entry = tr.get(phase)
    return None if entry is None else float(entry["bytes_per_launch"])


def stored_step_traffic(label, tuning):
    """HBM bytes of the assembly-and-plan kernels of one step on workload `label`, from the
    same counter runs -- None unless their sources and the grouping tuning still match."""
    from paper_1805_03380_amd import profiling
    tr = _traffic_record(label)
    if tr is None or tr.get("partition_source_sha256") != profiling.partition_source_hash():
        return None
    if not _tuning_matches(tr, tuning, "part_"):
        return None
    entry = tr.get("assemble_plan")
    return None if entry is None else float(entry["bytes_per_step"])


def host_cpu():
    model = None
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    return {"model": model, "nproc": os.cpu_count()}


def rbt_context(problems):
    """The paper's own assembly (red-black tree, one insertion per triplet; the oracle's
    "rbt" read) timed once on each given workload: context for the bulk method, not a
    target."""
    import oracle
    out = {}
    for q, label in problems:
        t0 = time.perf_counter()
        st, _ = oracle.coo_to_csc(q.n_rows, q.n_cols, q.row, q.col, q.val, method="rbt")
        e = time.perf_counter() - t0
        out[label] = {"value": q.nnz_in / e, "unit": "nnz/s", "cores": 1, "seconds": e,
                      "status": int(st), "kind": "oracle (rbt)"}
    return out


def host_csc(A):
    """The device CSC's arrays on the host, as the oracle takes them."""
    import oracle
    n = A.nnz
    return oracle.CSC(A.n_rows, A.n_cols, A.col_ptr.cpu().numpy(),
                      A.row_idx_buf[:n].cpu().numpy(),
                      oracle.widen(A.values_buf[:n].cpu()))


def oracle_ms(fn):
    """One call of an oracle function on the host (single thread), in ms."""
    t0 = time.perf_counter()
    fn()
    return (time.perf_counter() - t0) * 1e3


def copy_calibration(mib):
    import torch
    n = mib * (1 << 20) // 4
    a = torch.ones(n, dtype=torch.float32, device="cuda:0")
    b = torch.empty_like(a)
    for _ in range(3):
        b.copy_(a)
    torch.cuda.synchronize()
    print(json.dumps({"copy_calibration_bytes": 4 * n, "dispatches": 3}), flush=True)


class Timer:
    """K calls of `run` between two HIP events on the launch stream; ms per call."""

    def __init__(self, stream, steps):
        self.stream, self.steps = stream, steps

    def __call__(self, run):
        import torch
        a = torch.cuda.Event(enable_timing=True)
        b = torch.cuda.Event(enable_timing=True)
        torch.cuda.synchronize()
        a.record(self.stream)
        run()
        b.record(self.stream)
        torch.cuda.synchronize()
        return a.elapsed_time(b) / self.steps


def measure_step(p, label, args, steps, warmup, graph, cold_steps, separate=False):
    """The whole step on workload p: K eager steps (the rate), K steps with phase events (the
    breakdown), optionally K graph replays and cold-cache steps; returns (record, state)."""
    import numpy as np
    import torch
    from paper_1805_03380_amd import autotune, _lib
    from paper_1805_03380_amd.pipeline import Pipeline

    dev = torch.device("cuda:0")
    row = torch.from_numpy(p.row).to(dev)
    col = torch.from_numpy(p.col).to(dev)
    val = torch.from_numpy(p.val).to(dev)
    X = torch.from_numpy(p.X).to(dev)
    G = torch.from_numpy(p.G).to(dev)  # in the output type, as a loss hands it over
    _lib.set_tuning(**DEFAULT_TUNING)
    vname = str(val.dtype).replace("torch.", "")
    sig = autotune.signature("pipeline", p.n_rows, p.n_cols, p.nnz_in, p.k, vname,
                             str(X.dtype).replace("torch.", ""))
    applied = autotune.apply(autotune.load_table(), sig)
    tuning_used = _lib.get_tuning().as_dict()
    pipe = Pipeline(p.n_rows, p.n_cols, p.nnz_in, p.k, val_dtype=val.dtype, x_dtype=X.dtype,
                    fused=not separate)
    if G.dtype != pipe.Y.dtype:
        raise RuntimeError("G must come in Y's element type (%s), got %s"
                           % (pipe.Y.dtype, G.dtype))
    phases = pipe.phases
    stream = torch.cuda.current_stream(dev)
    timed = Timer(stream, steps)

    for _ in range(warmup):
        pipe.step(row, col, val, X, G, stream)
    torch.cuda.synchronize()
    nnz, st_a, st_p = pipe.status()
    if st_a or st_p:
        raise RuntimeError("library reported status %d / %d" % (st_a, st_p))

    # phase breakdown: K steps with HIP events between the phases on the launch stream
    evs = [[torch.cuda.Event(enable_timing=True) for _ in range(len(phases) + 1)]
           for _ in range(steps)]

    def run_phases():
        for i in range(steps):
            pipe.step(row, col, val, X, G, stream, events=evs[i])
    ms_phased = timed(run_phases)
    phase_ms = {ph: float(np.mean([evs[i][j].elapsed_time(evs[i][j + 1])
                                   for i in range(steps)]))
                for j, ph in enumerate(phases)}
    step_ms = np.array([evs[i][0].elapsed_time(evs[i][-1]) for i in range(steps)])

    # K eager steps on one stream, nothing recorded in between
    def run_eager():
        for _ in range(steps):
            pipe.step(row, col, val, X, G, stream)
    ms_step = timed(run_eager)

    graph_rec = None
    if graph:
        g = pipe.capture(row, col, val, X, G)
        g.replay()

        def run_graph():
            for _ in range(steps):
                g.replay()
        g_ms = timed(run_graph)
        graph_rec = {"steps": steps, "ms_per_step": g_ms, "value": p.nnz_in / (g_ms * 1e-3)}
        del g

    # cold caches: 1 GiB written before each step evicts the 256 MB MALL and every L2
    cold = None
    if cold_steps > 0:
        flush = torch.empty(1 << 30, dtype=torch.uint8, device=dev)
        c_step, c_ph = [], []
        for i in range(cold_steps):
            flush.fill_(i & 0xFF)
            ev = [torch.cuda.Event(enable_timing=True) for _ in range(len(phases) + 1)]
            pipe.step(row, col, val, X, G, stream, events=ev)
            torch.cuda.synchronize()
            c_step.append(ev[0].elapsed_time(ev[-1]))
            c_ph.append([ev[j].elapsed_time(ev[j + 1]) for j in range(len(phases))])
        del flush
        c_step = np.array(c_step)
        cold = {"steps": cold_steps, "ms_per_step_median": float(np.median(c_step)),
                "value": p.nnz_in / (float(np.median(c_step)) * 1e-3),
                "phase_ms_median": {ph: float(np.median([c[j] for c in c_ph]))
                                    for j, ph in enumerate(phases)},
                "flush": "1 GiB device fill before each step"}

    s_vin = p.val.dtype.itemsize
    s_v = pipe.values.element_size()
    bytes_ = model_bytes(p.n_rows, p.n_cols, p.nnz_in, nnz, p.k, s_vin, s_v,
                         X.element_size(), pipe.Y.element_size(), pipe.dX.element_size(),
                         G.element_size())
    # the dominant single kernel: forward and adjoint are one kernel each (assembly and plan
    # are sequences of shorter kernels, each below either product in the kernel trace)
    dominant = max(("forward", "backward"), key=lambda ph: phase_ms[ph])
    kernel_name = dict(forward="k_spmm_fwd", backward="k_spmm_bwd")[dominant]
    ach = bytes_[dominant] / (phase_ms[dominant] * 1e-3) / 1e9
    spmm_ms = phase_ms["forward"] + phase_ms["backward"]
    spmm_gbps = (bytes_["forward"] + bytes_["backward"]) / (spmm_ms * 1e-3) / 1e9
    traffic = stored_traffic(label, dominant, tuning_used)
    spmm_measured = {}
    for ph in ("forward", "backward"):
        tb = stored_traffic(label, ph, tuning_used)
        gbps = None if tb is None else tb / (phase_ms[ph] * 1e-3) / 1e9
        sg = X.element_size() if ph == "forward" else G.element_size()
        spmm_measured[ph] = {"kernel_ms": phase_ms[ph], "bytes": tb, "GBps": gbps,
                             "frac": None if gbps is None else gbps / HBM_PEAK_GBPS,
                             "B_min_bytes": bytes_[ph],
                             "B_min_GBps": bytes_[ph] / (phase_ms[ph] * 1e-3) / 1e9,
                             "B_min_frac": bytes_[ph] / (phase_ms[ph] * 1e-3) / 1e9
                             / HBM_PEAK_GBPS,
                             "B_gat_GBps": (bytes_[ph] + gather_bytes(nnz, p.k, sg))
                             / (phase_ms[ph] * 1e-3) / 1e9}
    asm_t = phase_ms[phases[0]] * 1e-3
    asm_traffic = stored_step_traffic(label, tuning_used) if phases[0] == "assemble_plan" \
        else None
    asm_bytes = bytes_[phases[0]] if phases[0] == "assemble_plan" else bytes_["assemble"]
    rec = {
        "workload": label, "n_rows": p.n_rows, "n_cols": p.n_cols, "nnz_in": p.nnz_in,
        "nnz": nnz, "k": p.k, "seed": (p.meta or {}).get("seed"),
        "value_dtype": vname, "dense_dtype": str(X.dtype).replace("torch.", ""),
        "g_dtype": str(G.dtype).replace("torch.", ""),
        "steps": steps, "warmup": warmup,
        "ms_per_step": ms_step, "value": p.nnz_in / (ms_step * 1e-3),
        "ms_per_step_with_phase_events": ms_phased,
        "phase_ms": phase_ms,
        "step_ms_median": float(np.median(step_ms)),
        "step_ms_p10": float(np.percentile(step_ms, 10)),
        "step_ms_p90": float(np.percentile(step_ms, 90)),
        "cold": cold, "graph": graph_rec,
        "assembly_nnz_per_s": p.nnz_in / asm_t,
        "assembly_phase": phases[0],
        "assembly_compulsory_GBps": asm_bytes / asm_t / 1e9,
        "assembly_compulsory_frac": asm_bytes / asm_t / 1e9 / HBM_PEAK_GBPS,
        "assembly_measured": {"bytes": asm_traffic,
                              "GBps": None if asm_traffic is None else asm_traffic / asm_t / 1e9},
        "spmm_measured": spmm_measured,
        "spmm_fwd_bwd_GBps": spmm_gbps,
        "spmm_fwd_bwd_frac": spmm_gbps / HBM_PEAK_GBPS,
        "algorithmic_bytes": bytes_,
        "roofline": {"bound": "hbm", "kernel": kernel_name, "achieved": ach,
                     "peak": HBM_PEAK_GBPS, "unit": "GB/s", "frac": ach / HBM_PEAK_GBPS,
                     "traffic": traffic,
                     "traffic_GBps": None if traffic is None
                     else traffic / (phase_ms[dominant] * 1e-3) / 1e9,
                     "kernel_ms": phase_ms[dominant],
                     "algorithmic_bytes": bytes_[dominant],
                     "gather_model_GBps": (bytes_[dominant] + gather_bytes(nnz, p.k, 4))
                     / (phase_ms[dominant] * 1e-3) / 1e9},
        "tuning": tuning_used, "tuning_from_table": bool(applied),
    }
    state = dict(pipe=pipe, row=row, col=col, val=val, X=X, G=G, nnz=nnz, stream=stream,
                 timed=timed)
    return rec, state


def leg_tuning(sig):
    """The table's tuning for one side operation (signature `sig`), over the defaults; without
    an entry the tuning in effect stays.  Returns (previous tuning, applied or None, in effect)."""
    from paper_1805_03380_amd import _lib, autotune
    saved = _lib.get_tuning().as_dict()
    _lib.set_tuning(**DEFAULT_TUNING)
    applied = autotune.apply(autotune.load_table(), sig)
    if not applied:
        _lib.set_tuning(**saved)
    return saved, applied, _lib.get_tuning().as_dict()


def legs_on_csc(p, st, args):
    """Batch insertion, the sum A + B, the transpose and row-vector product, the gradient per
    input triplet and trace(A^T B), timed with the step's CSC (uniform workload)."""
    import numpy as np
    import torch
    from paper_1805_03380_amd import ops, synth, _lib
    pipe, row, col, val, X, G = (st[k] for k in ("pipe", "row", "col", "val", "X", "G"))
    nnz, stream, timed = st["nnz"], st["stream"], st["timed"]
    dev = X.device
    steps = timed.steps
    lib = _lib.load()
    out = {}

    if not args.no_insert:
        A = pipe.csc()
        q = synth.random_coo(1006, p.n_rows, p.n_cols, 100_000, dup_frac=0.05,
                             dtype=np.float64 if pipe.values.dtype == torch.float64
                             else np.float32)
        qr, qc, qv = (torch.from_numpy(a).to(dev) for a in (q.row, q.col, q.val))
        # the insertion's own tuned grouping parameters (for this leg only)
        from paper_1805_03380_amd import autotune
        saved_tuning, ins_tuned, ins_tuning = leg_tuning(autotune.insert_signature(
            p.n_rows, p.n_cols, q.nnz_in, str(qv.dtype).replace("torch.", "")))
        B = ops.csc_insert(A, qr, qc, qv)  # warm-up, and the workspace for the timed calls
        o = (B.col_ptr, B.row_idx_buf, B.values_buf, B.info)
        cap_a = A.nnz_cap

        def run_insert():
            for _ in range(steps):
                lib.spm_csc_insert(A.n_rows, A.n_cols, cap_a, A.col_ptr.data_ptr(),
                                   A.row_idx_buf.data_ptr(), A.values_buf.data_ptr(), q.nnz_in,
                                   qr.data_ptr(), qc.data_ptr(), qv.data_ptr(),
                                   ops._dtype_code(qv.dtype), o[0].data_ptr(),
                                   o[1].data_ptr(), o[2].data_ptr(),
                                   ops._dtype_code(o[2].dtype), o[3].data_ptr(),
                                   B._ws.data_ptr(), B._ws.numel(), stream.cuda_stream)
        i_ms = timed(run_insert)
        _lib.set_tuning(**saved_tuning)
        nnz_out, st_i = (int(x) for x in o[3].cpu())
        if st_i:
            raise RuntimeError("spm_csc_insert reported status %d" % st_i)
        sv = A.values_buf.element_size()
        i_bytes = (4 * (p.n_cols + 1) + nnz * (4 + sv) + q.nnz_in * (8 + sv)
                   + 4 * (p.n_cols + 1) + nnz_out * (4 + sv))
        cpu_ms = None
        if not args.no_cpu:
            import oracle
            Ah = host_csc(A)
            cpu_ms = oracle_ms(lambda: oracle.csc_insert(Ah, q.row, q.col, q.val))
        ins = {"cpu_oracle_ms": cpu_ms,
               "workload": "10^5 new triplets (5 percent duplicates, seed 1006) into the "
                           "assembled 1e5 x 1e5 CSC", "existing": nnz, "new": q.nnz_in,
               "nnz_out": nnz_out, "ms": i_ms,
               "tuning": {k: v for k, v in ins_tuning.items() if k.startswith("part_")},
               "tuning_from_table": bool(ins_tuned),
               "elements_per_s": (nnz + q.nnz_in) / (i_ms * 1e-3),
               "new_triplets_per_s": q.nnz_in / (i_ms * 1e-3),
               "compulsory_bytes": i_bytes,
               "compulsory_GBps": i_bytes / (i_ms * 1e-3) / 1e9}
        # the sum A + B with B the same 10^5 triplets assembled (spm_csc_add)
        Bq = ops.coo_to_csc(qr, qc, qv, (p.n_rows, p.n_cols))
        S = ops.csc_add(A, Bq)  # warm-up, and the buffers for the timed calls
        s_out = (S.col_ptr, S.row_idx_buf, S.values_buf, S.info)

        def run_add():
            for _ in range(steps):
                lib.spm_csc_add(A.n_rows, A.n_cols, cap_a, A.col_ptr.data_ptr(),
                                A.row_idx_buf.data_ptr(), A.values_buf.data_ptr(), Bq.nnz_cap,
                                Bq.col_ptr.data_ptr(), Bq.row_idx_buf.data_ptr(),
                                Bq.values_buf.data_ptr(), ops._dtype_code(qv.dtype),
                                s_out[0].data_ptr(), s_out[1].data_ptr(), s_out[2].data_ptr(),
                                ops._dtype_code(s_out[2].dtype), s_out[3].data_ptr(),
                                S._ws.data_ptr(), S._ws.numel(), stream.cuda_stream)
        a_ms = timed(run_add)
        nnz_s, st_s = (int(x) for x in s_out[3].cpu())
        if st_s:
            raise RuntimeError("spm_csc_add reported status %d" % st_s)
        nb = Bq.nnz
        a_bytes = (2 * 4 * (p.n_cols + 1) + (nnz + nb) * (4 + sv) + 4 * (p.n_cols + 1)
                   + nnz_s * (4 + sv))
        cpu_ms = None
        if not args.no_cpu:
            import oracle
            Ah, Bh = host_csc(A), host_csc(Bq)
            cpu_ms = oracle_ms(lambda: oracle.csc_add(Ah, Bh))
        ins["sum"] = {"workload": "A + B, A the assembled 1e5 x 1e5 CSC, B the same 10^5 "
                                  "triplets assembled", "nnz_a": nnz, "nnz_b": nb,
                      "nnz_out": nnz_s, "ms": a_ms, "cpu_oracle_ms": cpu_ms,
                      "elements_per_s": (nnz + nb) / (a_ms * 1e-3),
                      "compulsory_bytes": a_bytes,
                      "compulsory_GBps": a_bytes / (a_ms * 1e-3) / 1e9}
        out["insert"] = ins

    if not args.no_transpose:
        A = pipe.csc()
        from paper_1805_03380_amd import autotune
        saved_tuning, tr_tuned, tr_tuning = leg_tuning(autotune.transpose_signature(
            p.n_rows, p.n_cols, nnz, str(A.values_buf.dtype).replace("torch.", "")))
        T = ops.csc_transpose(A)  # warm-up, and the buffers for the timed calls
        t_info = T.info

        def run_transpose():
            for _ in range(steps):
                lib.spm_csc_transpose(A.n_rows, A.n_cols, A.nnz_cap, A.col_ptr.data_ptr(),
                                      A.row_idx_buf.data_ptr(), A.values_buf.data_ptr(),
                                      ops._dtype_code(A.values_buf.dtype), T.col_ptr.data_ptr(),
                                      T.row_idx_buf.data_ptr(), T.values_buf.data_ptr(),
                                      t_info.data_ptr(), T._ws.data_ptr(), T._ws.numel(),
                                      stream.cuda_stream)
        t_ms = timed(run_transpose)
        _lib.set_tuning(**saved_tuning)
        if int(t_info[1].item()):
            raise RuntimeError("spm_csc_transpose reported status %d" % int(t_info[1]))
        sv = A.values_buf.element_size()
        t_bytes = 4 * (p.n_cols + 1) + 4 * (p.n_rows + 1) + 2 * nnz * (4 + sv)
        V = torch.randn(p.n_rows, dtype=X.dtype, device=dev)
        ops.rowvec_spmm(V, A)

        def run_rowvec():
            with torch.cuda.stream(stream):
                for _ in range(steps):
                    ops.rowvec_spmm(V, A)
        r_ms = timed(run_rowvec)
        cpu_ms = None
        if not args.no_cpu:
            import oracle
            Ah = host_csc(A)
            cpu_ms = oracle_ms(lambda: oracle.csc_transpose(Ah))
        out["transpose"] = {"cpu_oracle_ms": cpu_ms,
                            "workload": "transpose of the assembled 1e5 x 1e5 CSC", "nnz": nnz,
                            "ms": t_ms, "elements_per_s": nnz / (t_ms * 1e-3),
                            "tuning": {k: v for k, v in tr_tuning.items()
                                       if k.startswith("part_")},
                            "tuning_from_table": bool(tr_tuned),
                            "compulsory_bytes": t_bytes,
                            "compulsory_GBps": t_bytes / (t_ms * 1e-3) / 1e9,
                            "rowvec_ms": r_ms, "rowvec_elements_per_s": nnz / (r_ms * 1e-3)}

    if not args.no_tgrad:
        tg_dv = torch.empty(p.nnz_in, dtype=torch.float32, device=dev)
        k_ = X.shape[1]
        vt_code = ops._dtype_code(val.dtype)
        g_code, x_code = ops._dtype_code(G.dtype), ops._dtype_code(X.dtype)

        def run_tgrad():
            for _ in range(steps):
                lib.spm_coo_triplet_grad(p.n_rows, p.n_cols, p.nnz_in, k_, row.data_ptr(),
                                         col.data_ptr(), vt_code, G.data_ptr(), G.stride(0),
                                         g_code, X.data_ptr(), X.stride(0), x_code,
                                         tg_dv.data_ptr(), _lib.F32, stream.cuda_stream)
        run_tgrad()
        tg_ms = timed(run_tgrad)
        xs = X.element_size()
        # compulsory: the triplet indices, every G and X row once, the gradients; the gather
        # model reads a G row and an X row per triplet
        tg_c = p.nnz_in * (8 + 4) + (p.n_rows + p.n_cols) * k_ * xs
        tg_g = p.nnz_in * (8 + 4 + 2 * k_ * xs)
        cpu_ms = None
        if not args.no_cpu:
            import oracle
            cpu_ms = oracle_ms(lambda: oracle.triplet_grad(p.n_rows, p.n_cols, p.row, p.col,
                                                           p.G, p.X))
        A_t = pipe.csc()
        dval_t = pipe.dval

        def run_tgrad_csc():
            for _ in range(steps):
                lib.spm_coo_triplet_grad_csc(p.n_rows, p.n_cols, p.nnz_in, k_, row.data_ptr(),
                                             col.data_ptr(), A_t.nnz_cap, A_t.col_ptr.data_ptr(),
                                             A_t.row_idx_buf.data_ptr(), dval_t.data_ptr(),
                                             ops._dtype_code(dval_t.dtype), vt_code,
                                             G.data_ptr(), G.stride(0), g_code, X.data_ptr(),
                                             X.stride(0), x_code, tg_dv.data_ptr(), _lib.F32,
                                             stream.cuda_stream)
        run_tgrad_csc()
        tgc_ms = timed(run_tgrad_csc)
        out["triplet_grad"] = {
            "cpu_oracle_ms": cpu_ms, "ms_from_dvalues": tgc_ms,
            "from_dvalues": "each triplet reads the adjoint's dvalue at its slot (the dot "
                            "product only where the location summed to zero)",
            "workload": "dL/dv for the %d input triplets of the step, k=%d" % (p.nnz_in, k_),
            "ms": tg_ms, "triplets_per_s": p.nnz_in / (tg_ms * 1e-3),
            "compulsory_bytes": tg_c, "compulsory_GBps": tg_c / (tg_ms * 1e-3) / 1e9,
            "gather_GBps": tg_g / (tg_ms * 1e-3) / 1e9}

    if not args.no_trace:
        from paper_1805_03380_amd import synth as _s
        trace = []
        for dens in args.trace_densities:
            qa, qb = _s.trace_pair(seed=1007, density=dens)
            TA, TB = (ops.coo_to_csc(*(torch.from_numpy(x).to(dev) for x in (q.row, q.col, q.val)),
                                     (q.n_rows, q.n_cols)) for q in (qa, qb))
            t_val, hits = ops.trace_atb(TA, TB)
            wb = _lib.ctypes.c_size_t(0)
            lib.spm_csc_trace_atb_workspace(TA.n_cols, _lib.ctypes.byref(wb))
            t_ws = torch.empty(max(wb.value, 256), dtype=torch.uint8, device=dev)
            t_out = torch.empty(1, dtype=torch.float64, device=dev)
            t_inf = torch.empty(2, dtype=torch.int32, device=dev)

            def run_trace():
                for _ in range(steps):
                    lib.spm_csc_trace_atb(TA.n_rows, TA.n_cols, TA.nnz_cap, TA.col_ptr.data_ptr(),
                                          TA.row_idx_buf.data_ptr(), TA.values_buf.data_ptr(),
                                          TB.nnz_cap, TB.col_ptr.data_ptr(),
                                          TB.row_idx_buf.data_ptr(), TB.values_buf.data_ptr(),
                                          _lib.F64, t_out.data_ptr(), t_inf.data_ptr(),
                                          t_ws.data_ptr(), t_ws.numel(), stream.cuda_stream)
            tr_ms = timed(run_trace)
            if int(t_inf[1].item()) or int(t_inf[0].item()) != hits:
                raise RuntimeError("spm_csc_trace_atb: status %d" % int(t_inf[1].item()))
            na, nb = TA.nnz, TB.nnz
            # compulsory: both offset arrays and both row-index arrays once, values where rows
            # match; the full-read model reads every value too
            c_bytes = 2 * 4 * (qa.n_cols + 1) + 4 * (na + nb) + 2 * 8 * hits
            f_bytes = 2 * 4 * (qa.n_cols + 1) + (4 + 8) * (na + nb)
            cpu_ms = None
            if not args.no_cpu:
                import oracle
                Ah, Bh = host_csc(TA), host_csc(TB)
                cpu_ms = oracle_ms(lambda: oracle.trace_atb(Ah, Bh))
            trace.append({"cpu_oracle_ms": cpu_ms,
                          "workload": "trace(A^T B), 10^4 x 10^4, density %g, float64 (seed 1007)"
                                      % dens, "nnz_a": na, "nnz_b": nb, "hits": hits,
                          "ms": tr_ms, "elements_per_s": (na + nb) / (tr_ms * 1e-3),
                          "compulsory_bytes": c_bytes,
                          "compulsory_GBps": c_bytes / (tr_ms * 1e-3) / 1e9,
                          "full_read_GBps": f_bytes / (tr_ms * 1e-3) / 1e9,
                          "frac_hbm_full_read": f_bytes / (tr_ms * 1e-3) / 1e9 / HBM_PEAK_GBPS})
            del TA, TB, t_ws
        out["trace_atb"] = trace
    return out


def side_summary(rec):
    """The compact record of a non-headline workload."""
    keep = ("workload", "n_rows", "n_cols", "nnz_in", "nnz", "k", "value_dtype", "dense_dtype",
            "g_dtype", "ms_per_step", "value", "phase_ms", "step_ms_median",
            "assembly_compulsory_frac", "spmm_fwd_bwd_frac", "spmm_measured", "roofline",
            "tuning_from_table")
    return {k: rec[k] for k in keep}


DEFAULT_TUNING = {}


def main():
    args = parse()
    if args.copy_calib_mib:
        copy_calibration(args.copy_calib_mib)
        return
    if args.batch_only:
        batch_only(args.batch_only, args.steps, args.warmup)
        return
    if args.gpus != 1:
        print("bench.py runs on one GPU only: it measures the single-GPU kernels "
              "(--gpus %d requested)" % args.gpus, file=sys.stderr)
        sys.exit(2)
    import torch
    from paper_1805_03380_amd import _lib
    DEFAULT_TUNING.update(_lib.get_tuning().as_dict())

    t0 = time.perf_counter()
    p, label = make_problem(args.workload)
    gen_s = time.perf_counter() - t0
    print("bench: %s generated in %.1f s" % (label, gen_s), file=sys.stderr, flush=True)
    head, head_state = measure_step(p, label, args, args.steps, args.warmup,
                                    graph=not args.no_graph, cold_steps=args.cold_steps,
                                    separate=args.separate)
    print("bench: %s %.3f ms per step" % (label, head["ms_per_step"]), file=sys.stderr,
          flush=True)
    head_dt = "f64" if head["value_dtype"] == "float64" else "f32"

    out = {
        "metric": "COO->CSC nnz/s; SpMM fwd+bwd HBM GB/s and % of roofline, batched vs single",
        "value": head["value"],
        "unit": "nnz/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": head["ms_per_step"],
        "timing": "eager library calls on one stream",
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": head_dt,
        "data": "synthetic",
        "config": {"workload": label, "n_rows": p.n_rows, "n_cols": p.n_cols,
                   "nnz_in": p.nnz_in, "nnz": head["nnz"], "k": p.k,
                   "seed": head["seed"], "value_dtype": head["value_dtype"],
                   "dense_dtype": head["dense_dtype"], "g_dtype": head["g_dtype"],
                   "accumulate": "binary64",
                   "step": "assemble+plan+forward+adjoint", "parallelism": "single GPU",
                   "generate_s": gen_s},
        "roofline": head["roofline"],
    }
    out["headline"] = head
    if args.workload == "uniform":  # the operations around the hot path use this CSC
        out.update(legs_on_csc(p, head_state, args))
    side_problems = []
    if not args.no_side:
        configs = {}
        for name in SIDE_ORDER:
            if name == args.workload:
                continue
            q, qlabel = make_problem(name)
            rec, st = measure_step(q, qlabel, args, args.steps, min(args.warmup, 3),
                                   graph=False, cold_steps=0, separate=args.separate)
            configs[qlabel] = side_summary(rec)
            print("bench: %s %.3f ms per step" % (qlabel, rec["ms_per_step"]), file=sys.stderr,
                  flush=True)
            if name == "uniform":
                out.update(legs_on_csc(q, st, args))
            if name in ("tiny", "uniform", "diff"):
                side_problems.append((q, qlabel))
            del st
            torch.cuda.empty_cache()
        out["configs"] = configs
    if not args.no_batch:
        from paper_1805_03380_amd import synth
        t0 = time.perf_counter()
        bt = synth.batch_problems()
        b_gen = time.perf_counter() - t0
        out["batched_vs_single"] = batched_vs_single(bt, "float32")
        out["batched_vs_single_bf16"] = batched_vs_single(bt, "bfloat16")
        out["batched_vs_single"]["generate_s"] = b_gen
        print("bench: batch %.2f ms" % out["batched_vs_single"]["batched_ms"], file=sys.stderr,
              flush=True)
    if not args.no_cpu:
        out["cpu_baseline"] = cpu_baseline(p, label, args.cpu_seconds)
        # every host core this process may use (the scheduler's set), at most 16
        n_thr = max(1, min(16, len(os.sched_getaffinity(0))))
        out["cpu_baseline_all_cores"] = cpu_all_cores(p, label, args.cpu_seconds, n_thr)
        out["cpu_baseline"]["host"] = host_cpu()
        if side_problems:
            out["cpu_rbt_context"] = rbt_context(side_problems)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
