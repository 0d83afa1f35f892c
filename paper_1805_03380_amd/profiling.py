"""Turn rocprofv3 CSV output into the short summaries kept under profiles/.

    python -m paper_1805_03380_amd.profiling stats --csv DIR/run_kernel_stats.csv \
        --command "rocprofv3 ..." --out profiles/<kernel>_<workload>.md
    python -m paper_1805_03380_amd.profiling traffic --fetch F.csv --write W.csv \
        --copy-fetch CF.csv --copy-write CW.csv --copy-bytes N --command "..." --out T.json

`traffic` converts the FETCH_SIZE / WRITE_SIZE counters (KiB per dispatch, bytes that leave
or enter the L2) of the two SpMM kernels into bytes per launch, each scaled by what the same
counter reads for a plain device copy of N bytes (the copy reads N and writes N bytes).  It
also totals the assembly-and-plan kernels of one step (their dispatches divided by the
number of steps, counted by the emit kernel's dispatches).  The result records hashes of the
kernel sources and the tuning it was taken with; bench.py uses each part only while they
still match.
"""
from __future__ import annotations

import argparse
import csv
import hashlib
import json
import os
from collections import defaultdict

HERE = os.path.dirname(os.path.abspath(__file__))
SPMM_SOURCES = ("csrc/spm_spmm.h", "csrc/spm_device.h")
SPMM_KERNELS = {"forward": "k_spmm_fwd", "backward": "k_spmm_bwd"}
PARTITION_SOURCES = ("csrc/spm_partition.h", "csrc/spm_assemble.h", "csrc/spm_device.h",
                     "csrc/spm_api.hip")
PARTITION_KERNELS = ("k_part_", "k_rows_scan", "k_small_scan", "k_expand_columns")
STEP_MARKER = "k_part_emit"


def _hash(sources) -> str:
    h = hashlib.sha256()
    for rel in sources:
        with open(os.path.join(HERE, rel), "rb") as f:
            h.update(f.read())
    return h.hexdigest()


def spmm_source_hash() -> str:
    """SHA-256 over the sources that define the SpMM kernels."""
    return _hash(SPMM_SOURCES)


def partition_source_hash() -> str:
    """SHA-256 over the sources that define the assembly and plan kernels and their launches."""
    return _hash(PARTITION_SOURCES)


def _counter_means(path: str) -> dict:
    """(kernel name, counter) -> mean value per dispatch."""
    acc = defaultdict(list)
    with open(path) as f:
        for r in csv.DictReader(f):
            acc[(r["Kernel_Name"], r["Counter_Name"])].append(float(r["Counter_Value"]))
    return {k: sum(v) / len(v) for k, v in acc.items()}


def _counter_sums(path: str) -> dict:
    """(kernel name, counter) -> (sum over dispatches, number of dispatches)."""
    acc = defaultdict(lambda: [0.0, 0])
    with open(path) as f:
        for r in csv.DictReader(f):
            a = acc[(r["Kernel_Name"], r["Counter_Name"])]
            a[0] += float(r["Counter_Value"])
            a[1] += 1
    return {k: tuple(v) for k, v in acc.items()}


def _step_bytes(sums: dict, counter: str, scale: float) -> tuple[float, dict]:
    """Bytes per step of the assembly-and-plan kernels, and per kernel."""
    steps = sum(n for (k, c), (_, n) in sums.items() if c == counter and STEP_MARKER in k)
    if steps == 0:
        raise KeyError("no %s dispatch with counter %s" % (STEP_MARKER, counter))
    per = {}
    for (k, c), (tot, _) in sums.items():
        if c == counter and any(t in k for t in PARTITION_KERNELS):
            name = k.split("(")[0].replace("void ", "")
            per[name] = per.get(name, 0.0) + tot * 1024.0 * scale / steps
    return sum(per.values()), per


def _pick(means: dict, needle: str, counter: str, exclude: str | None = None) -> float:
    hits = [(k, v) for k, v in means.items()
            if needle in k[0] and k[1] == counter and (exclude is None or exclude not in k[0])]
    if not hits:
        raise KeyError("no dispatch of %s with counter %s" % (needle, counter))
    # the busiest instantiation is the one the benchmark launches
    return max(hits, key=lambda kv: kv[1])[1]


def traffic(fetch_csv, write_csv, copy_fetch_csv, copy_write_csv, copy_bytes, command,
            tuning=None) -> dict:
    fm, wm = _counter_means(fetch_csv), _counter_means(write_csv)
    cf, cw = _counter_means(copy_fetch_csv), _counter_means(copy_write_csv)
    copy_fetch_kib = _pick(cf, "copyBuffer", "FETCH_SIZE")
    copy_write_kib = _pick(cw, "copyBuffer", "WRITE_SIZE")
    fscale = copy_bytes / (copy_fetch_kib * 1024.0)
    wscale = copy_bytes / (copy_write_kib * 1024.0)
    out = {
        "command": command,
        "spmm_source_sha256": spmm_source_hash(),
        "partition_source_sha256": partition_source_hash(),
        "tuning": tuning,
        "calibration": {"copy_bytes": copy_bytes, "fetch_kib": copy_fetch_kib,
                        "write_kib": copy_write_kib, "fetch_scale": fscale,
                        "write_scale": wscale},
    }
    for phase, name in SPMM_KERNELS.items():
        f_kib = _pick(fm, name, "FETCH_SIZE")
        w_kib = _pick(wm, name, "WRITE_SIZE")
        fb, wb = f_kib * 1024.0 * fscale, w_kib * 1024.0 * wscale
        out[phase] = {"kernel": name, "fetch_kib": f_kib, "write_kib": w_kib,
                      "fetch_bytes": fb, "write_bytes": wb, "bytes_per_launch": fb + wb}
    try:
        fsum, fper = _step_bytes(_counter_sums(fetch_csv), "FETCH_SIZE", fscale)
        wsum, wper = _step_bytes(_counter_sums(write_csv), "WRITE_SIZE", wscale)
        out["assemble_plan"] = {"fetch_bytes": fsum, "write_bytes": wsum,
                                "bytes_per_step": fsum + wsum,
                                "per_kernel": {k: {"fetch_bytes": fper.get(k, 0.0),
                                                   "write_bytes": wper.get(k, 0.0)}
                                               for k in sorted(set(fper) | set(wper))}}
    except KeyError:
        pass
    return out


def stats_table(stats_csv: str, top: int = 25) -> str:
    rows = list(csv.DictReader(open(stats_csv)))
    rows.sort(key=lambda r: -float(r["TotalDurationNs"]))
    lines = ["| kernel | calls | average us | min us | max us | % of GPU time |",
             "|---|---:|---:|---:|---:|---:|"]
    for r in rows[:top]:
        lines.append("| `%s` | %s | %.2f | %.2f | %.2f | %.2f |" % (
            r["Name"][:110], r["Calls"], float(r["AverageNs"]) / 1e3,
            float(r["MinNs"]) / 1e3, float(r["MaxNs"]) / 1e3, float(r["Percentage"])))
    return "\n".join(lines)


def main():
    ap = argparse.ArgumentParser()
    sub = ap.add_subparsers(dest="what", required=True)
    s = sub.add_parser("stats")
    s.add_argument("--csv", required=True)
    s.add_argument("--command", required=True)
    s.add_argument("--title", default="Kernel trace")
    s.add_argument("--note", default="")
    s.add_argument("--out", required=True)
    t = sub.add_parser("traffic")
    for a in ("--fetch", "--write", "--copy-fetch", "--copy-write", "--command", "--out"):
        t.add_argument(a, required=True)
    t.add_argument("--copy-bytes", type=int, required=True)
    t.add_argument("--tuning", default=None, help="JSON of the launch tuning in effect")
    a = ap.parse_args()
    if a.what == "stats":
        text = "# %s\n\nCommand:\n\n    %s\n\n%s\n\n%s\n" % (a.title, a.command, a.note,
                                                         stats_table(a.csv))
        with open(a.out, "w") as f:
            f.write(text)
    else:
        tu = json.loads(a.tuning) if a.tuning else None
        res = traffic(a.fetch, a.write, a.copy_fetch, a.copy_write, a.copy_bytes, a.command, tu)
        with open(a.out, "w") as f:
            json.dump(res, f, indent=1)
            f.write("\n")


if __name__ == "__main__":
    main()
