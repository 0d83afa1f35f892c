"""Autotuner for the launch-shape parameters of libspm (spm_tuning).

Every parameter only decides how work is cut into workgroups -- never the order in which an
output is summed -- so any choice gives bitwise the same results; the tuner only measures
time.  It sweeps each group of parameters on a given problem with HIP-event timing, keeps the
fastest, and persists the choice in a JSON table keyed by device name, library version and a
problem signature (shape class, triplets, k, element types).

    python -m paper_1805_03380_amd.autotune            # tune the benchmark workloads
    table = autotune.load_table(); autotune.apply(table, signature)
"""
from __future__ import annotations

import itertools
import json
import math
import os
import time

from . import _lib

HERE = os.path.dirname(os.path.abspath(__file__))
DEFAULT_TABLE = os.path.join(HERE, "tuning", "mi355x.json")

SPMM_SPACE = {"spmm_block": [64, 128, 256], "spmm_blocks_per_cu": [8, 16, 32, 64]}
PART_SPACE = {"part_bucket_target": [512, 1024, 2048],
              "part_max_tiles": [64, 128, 256, 512, 1024]}
BATCH_SPACE = {"batch_wg_per_cu": [1, 2, 3, 4], "batch_spmm_wg_per_cu": [4, 8, 16]}


def table_path() -> str:
    return os.environ.get("SPM_TUNE_CACHE", DEFAULT_TABLE)


def signature(kind: str, n_rows: int, n_cols: int, nnz_in: int, k: int, val_dtype: str,
              x_dtype: str) -> str:
    """Problem class: sizes rounded to powers of two (tuned values carry over to neighbours)."""
    def p2(x):
        return 0 if x <= 0 else int(round(math.log2(x)))
    return "%s:r%d:c%d:n%d:k%d:%s:%s" % (kind, p2(n_rows), p2(n_cols), p2(nnz_in), k,
                                         val_dtype, x_dtype)


def device_key() -> str:
    """The device by architecture and compute-unit count (the marketing name that the runtime
    reports can differ between processes on one machine), plus the library version."""
    import torch
    lib = _lib.load()
    props = torch.cuda.get_device_properties(0)
    arch = getattr(props, "gcnArchName", "unknown").split(":")[0]
    return "%s:%dcu|%s" % (arch, props.multi_processor_count, lib.spm_version().decode())


def load_table(path: str | None = None) -> dict:
    path = path or table_path()
    if not os.path.exists(path):
        return {}
    with open(path) as f:
        return json.load(f)


def save_table(table: dict, path: str | None = None) -> str:
    path = path or table_path()
    os.makedirs(os.path.dirname(path), exist_ok=True)
    tmp = path + ".tmp"
    with open(tmp, "w") as f:
        json.dump(table, f, indent=1, sort_keys=True)
    os.replace(tmp, path)
    return path


def lookup(table: dict, sig: str, dev: str | None = None) -> dict | None:
    entry = table.get(dev or device_key(), {})
    return entry.get(sig, {}).get("tuning")


def apply(table: dict, sig: str, dev: str | None = None) -> dict | None:
    """Set the tuned values for `sig` if the table has them; returns what was applied."""
    tu = lookup(table, sig, dev)
    if tu:
        _lib.set_tuning(**tu)
    return tu


def _time(fn, reps: int, warm: int = 2) -> float:
    import torch
    for _ in range(warm):
        fn()
    torch.cuda.synchronize()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(reps):
        fn()
    e1.record()
    torch.cuda.synchronize()
    return e0.elapsed_time(e1) / reps


def _sweep(space: dict, run, reps: int) -> tuple[dict, float, list]:
    keys = list(space)
    best, best_ms, log = None, float("inf"), []
    saved = _lib.get_tuning().as_dict()
    try:
        for vals in itertools.product(*(space[k] for k in keys)):
            cand = dict(zip(keys, vals))
            _lib.set_tuning(**cand)
            ms = _time(run, reps)
            log.append((cand, ms))
            if ms < best_ms:
                best, best_ms = cand, ms
    finally:
        _lib.set_tuning(**saved)
    return best, best_ms, log


def tune_pipeline(p, reps: int = 10):
    """Tune the single-matrix path on problem p (a synth.COOProblem with X and G)."""
    import torch
    from .pipeline import Pipeline
    dev = torch.device("cuda:0")
    row = torch.from_numpy(p.row).to(dev)
    col = torch.from_numpy(p.col).to(dev)
    val = torch.from_numpy(p.val).to(dev)
    X = torch.from_numpy(p.X).to(dev)
    G = torch.from_numpy(p.G).to(dev)  # in Y's element type, as a loss hands it over
    result = {}

    def make():  # the workspace sizes follow the grouping parameters
        return Pipeline(p.n_rows, p.n_cols, p.nnz_in, p.k, val_dtype=val.dtype, x_dtype=X.dtype)

    pipe = make()
    pipe.step(row, col, val, X, G)
    torch.cuda.synchronize()

    def spmm_only():
        pipe.step_spmm(X, G)
    best_s, ms_s, log_s = _sweep(SPMM_SPACE, spmm_only, reps)
    result.update(best_s)

    # grouping: rebuild the pipeline per candidate (workspace sizes change), time assembly+plan
    keys = list(PART_SPACE)
    best_p, best_pms, log_p = None, float("inf"), []
    saved = _lib.get_tuning().as_dict()
    try:
        for vals in itertools.product(*(PART_SPACE[k] for k in keys)):
            cand = dict(zip(keys, vals))
            _lib.set_tuning(**cand)
            q = make()
            ms = _time(lambda: q.step_assemble_plan(row, col, val), reps)
            log_p.append((cand, ms))
            if ms < best_pms:
                best_p, best_pms = cand, ms
            del q
    finally:
        _lib.set_tuning(**saved)
    result.update(best_p)
    return result, {"spmm_ms": ms_s, "assemble_plan_ms": best_pms,
                    "spmm_log": log_s, "part_log": log_p}


def tune_batch(problems, dtype_name: str = "float32", reps: int = 3):
    """Tune the batched path on `problems` with values, X and G in dtype_name."""
    import torch
    from .batch import PackedBatch
    dt = torch.bfloat16 if dtype_name == "bfloat16" else torch.float32
    pb = PackedBatch(problems, val_dtype=dt, x_dtype=dt)
    best, ms, log = _sweep(BATCH_SPACE, lambda: pb.run_batched(), reps)
    return best, {"batch_ms": ms, "batch_log": log}


def batch_signature(dtype_name: str = "float32") -> str:
    """The 4096-matrix batch class (n up to 8192, up to 16 n triplets, k = 32)."""
    return signature("batch", 8192, 8192, 131072, 32, dtype_name, dtype_name)


BATCH_WORKLOADS = {"batch": "float32", "batch_bf16": "bfloat16"}


def insert_signature(n_rows: int, n_cols: int, nnz_new: int, dtype_name: str) -> str:
    """Batch insertion of nnz_new triplets into an n_rows x n_cols CSC (the grouping
    parameters sort the new triplets)."""
    return signature("insert", n_rows, n_cols, nnz_new, 0, dtype_name, dtype_name)


def transpose_signature(n_rows: int, n_cols: int, nnz: int, dtype_name: str) -> str:
    """Transpose of an n_rows x n_cols CSC holding nnz elements (the grouping parameters
    partition its elements by row)."""
    return signature("transpose", n_rows, n_cols, nnz, 0, dtype_name, dtype_name)


def tune_transpose(p, reps: int = 20):
    """Tune the grouping parameters of the transpose of p assembled."""
    import torch
    from . import ops
    dev = torch.device("cuda:0")
    A = ops.coo_to_csc(*(torch.from_numpy(a).to(dev) for a in (p.row, p.col, p.val)),
                       (p.n_rows, p.n_cols))
    ops.csc_transpose(A)
    best, ms, log = _sweep(PART_SPACE, lambda: ops.csc_transpose(A, sync=False), reps)
    return best, {"transpose_ms": ms, "transpose_log": log, "nnz": A.nnz}


def tune_insert(p, q, reps: int = 20):
    """Tune the grouping parameters of batch insertion of q's triplets into p assembled."""
    import torch
    from . import ops
    dev = torch.device("cuda:0")
    A = ops.coo_to_csc(*(torch.from_numpy(a).to(dev) for a in (p.row, p.col, p.val)),
                       (p.n_rows, p.n_cols))
    qr, qc, qv = (torch.from_numpy(a).to(dev) for a in (q.row, q.col, q.val))
    ops.csc_insert(A, qr, qc, qv)
    best, ms, log = _sweep(PART_SPACE, lambda: ops.csc_insert(A, qr, qc, qv, sync=False), reps)
    return best, {"insert_ms": ms, "insert_log": log}


# workload name -> (synth constructor, keyword arguments)
PIPELINE_WORKLOADS = {
    "tiny": ("tiny_spmv", {}),
    "uniform": ("uniform_1e5", {"value_dtype": "float32"}),
    "uniform_f64": ("uniform_1e5", {"value_dtype": "float64"}),
    "powerlaw": ("powerlaw_1e6", {}),
    "diff": ("diff_2e5", {}),
}


def pipeline_signature(p) -> str:
    return signature("pipeline", p.n_rows, p.n_cols, p.nnz_in, p.k, p.val.dtype.name,
                     p.X.dtype.name)


def main(argv=None):
    import argparse
    import numpy as np
    from . import synth
    ap = argparse.ArgumentParser()
    names = list(PIPELINE_WORKLOADS) + list(BATCH_WORKLOADS) + ["insert", "transpose"]
    ap.add_argument("--workloads", default=",".join(names),
                    help="comma-separated: %s" % ", ".join(names))
    args = ap.parse_args(argv)
    unknown = [n for n in args.workloads.split(",") if n not in names]
    if unknown:
        ap.error("unknown workloads: %s" % ", ".join(unknown))
    table = load_table()
    dev = device_key()
    entries = table.setdefault(dev, {})
    t0 = time.time()
    bt = None
    for name in args.workloads.split(","):
        if name == "insert":  # 10^5 new triplets into the uniform 1e5 x 1e5 CSC
            p = synth.uniform_1e5(value_dtype=np.float32, k=0)
            q = synth.random_coo(1006, p.n_rows, p.n_cols, 100_000, dup_frac=0.05,
                                 dtype=np.float32)
            ti, infoi = tune_insert(p, q)
            sigi = insert_signature(p.n_rows, p.n_cols, q.nnz_in, "float32")
            entries[sigi] = {"tuning": ti, "ms": {"insert": infoi["insert_ms"]}}
            print(sigi, ti, infoi["insert_ms"], flush=True)
            del p, q
            continue
        if name == "transpose":  # the uniform 1e5 x 1e5 CSC
            p = synth.uniform_1e5(value_dtype=np.float32, k=0)
            tt, infot = tune_transpose(p)
            sigt = transpose_signature(p.n_rows, p.n_cols, infot["nnz"], "float32")
            entries[sigt] = {"tuning": tt, "ms": {"transpose": infot["transpose_ms"]}}
            print(sigt, tt, infot["transpose_ms"], flush=True)
            del p
            continue
        if name in BATCH_WORKLOADS:
            if bt is None:
                bt = synth.batch_problems()
            tb, infob = tune_batch(bt.problems, BATCH_WORKLOADS[name])
            sigb = batch_signature(BATCH_WORKLOADS[name])
            entries[sigb] = {"tuning": tb, "ms": {"batch": infob["batch_ms"]}}
            print(sigb, tb, infob["batch_ms"], flush=True)
            continue
        ctor, kw = PIPELINE_WORKLOADS[name]
        kw = {k: (np.dtype(v).type if k == "value_dtype" else v) for k, v in kw.items()}
        p = getattr(synth, ctor)(**kw)
        tu, info = tune_pipeline(p)
        sig = pipeline_signature(p)
        entries[sig] = {"tuning": tu, "ms": {"spmm": info["spmm_ms"],
                                              "assemble_plan": info["assemble_plan_ms"]}}
        print(sig, tu, info["spmm_ms"], info["assemble_plan_ms"], flush=True)
        del p
    print("saved", save_table(table), "in %.1f s" % (time.time() - t0), flush=True)


if __name__ == "__main__":
    main()
