"""Host-side pieces of bench.py (no GPU): the exit for more than one GPU, the algorithmic
byte model, the workload labels that go into its JSON line, and the tuning of the side
operations."""
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

import bench  # noqa: E402


def test_batch_labels_format():
    for dt in ("float32", "bfloat16"):
        s = bench.batch_workload_label(dt)
        assert dt in s and "4096 matrices" in s and "seed 1005" in s


def test_model_bytes_uniform_f32():
    n, nnz_in, nnz, k = 100_000, 1_000_000, 950_000, 64
    b = bench.model_bytes(n, n, nnz_in, nnz, k, 4, 4, 4, 4, 4)
    assert b["assemble"] == nnz_in * 12 + nnz * 8 + 4 * (n + 1)
    # the fused call writes the plan's outputs but never re-reads the CSC it assembled
    assert b["assemble_plan"] == b["assemble"] + 4 * (n + 1) + nnz * 12
    assert b["plan"] == 4 * (n + 1) + nnz * 8 + 4 * (n + 1) + nnz * 12
    assert b["forward"] == 4 * (n + 1) + nnz * 8 + 2 * n * k * 4
    assert b["backward"] == 4 * (n + 1) + nnz * 8 + 3 * n * k * 4 + nnz * 4


def test_more_than_one_gpu_exits_with_message():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=300)
    assert r.returncode == 2
    assert "one GPU" in r.stderr


def test_model_bytes_g_in_its_own_type():
    """A binary64 G (binary64 values, binary32 X) is read at 8 bytes per element."""
    n, nnz_in, nnz, k = 1000, 5000, 4000, 16
    b4 = bench.model_bytes(n, n, nnz_in, nnz, k, 8, 8, 4, 8, 4)
    b8 = bench.model_bytes(n, n, nnz_in, nnz, k, 8, 8, 4, 8, 4, s_g=8)
    assert b4 == b8  # G defaults to Y's element size
    b_g4 = bench.model_bytes(n, n, nnz_in, nnz, k, 8, 8, 4, 8, 4, s_g=4)
    assert b8["backward"] - b_g4["backward"] == n * k * 4
    assert b8["forward"] == b_g4["forward"]


def test_workload_table():
    """Every workload names a generator that exists; the headline is the largest one."""
    from paper_1805_03380_amd import synth
    assert set(bench.SIDE_ORDER) == set(bench.WORKLOADS)
    for name, (ctor, kw, label) in bench.WORKLOADS.items():
        assert callable(getattr(synth, ctor)), name
        assert label and " " not in label
    p, label = bench.make_problem("tiny")
    assert label == bench.WORKLOADS["tiny"][2] and p.nnz_in == 10_000 and p.k == 1


def test_leg_tuning_applies_the_table_and_falls_back(monkeypatch):
    """bench.leg_tuning: a side operation with a table entry runs under it (over the defaults);
    one without keeps the tuning in effect; the caller gets the previous tuning back."""
    import json
    from paper_1805_03380_amd import _lib, autotune
    if not os.path.exists(_lib.LIB_PATH):
        from paper_1805_03380_amd import build
        build.build()
    _lib.load()
    with open(autotune.DEFAULT_TABLE) as f:
        table = json.load(f)
    dev = next(iter(table))
    monkeypatch.setattr(autotune, "device_key", lambda: dev)
    start = _lib.get_tuning().as_dict()
    monkeypatch.setattr(bench, "DEFAULT_TUNING", dict(start))
    sig = autotune.insert_signature(100_000, 100_000, 100_000, "float32")
    want = table[dev][sig]["tuning"]
    try:
        saved, applied, in_effect = bench.leg_tuning(sig)
        assert saved == start and applied == want
        assert all(in_effect[k] == v for k, v in want.items())
        _lib.set_tuning(**saved)
        saved2, applied2, in_effect2 = bench.leg_tuning("insert:r1:c1:n1:k0:float32:float32")
        assert applied2 is None and in_effect2 == saved2 == start
    finally:
        _lib.set_tuning(**start)
