"""Turn rocprofv3 CSV output into the short summaries kept under profiles/.

    python -m paper_1805_03380_amd.profiling stats --csv DIR/run_kernel_stats.csv \
        --command "rocprofv3 ..." --out profiles/<kernel>_<workload>.md
    python -m paper_1805_03380_amd.profiling traffic --fetch F.csv --write W.csv \
        --copy-fetch CF.csv --copy-write CW.csv --copy-bytes N --command "..." --out T.json

`traffic` converts the FETCH_SIZE / WRITE_SIZE counters (KiB per dispatch, bytes that leave
or enter the L2) of the two SpMM kernels into bytes per launch, each scaled by what the same
counter reads for a plain device copy of N bytes (the copy reads N and writes N bytes).  The
result records a hash of the SpMM kernel sources and the launch tuning it was taken with;
bench.py uses it only while both still match.
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


def spmm_source_hash() -> str:
    """SHA-256 over the sources that define the SpMM kernels."""
    h = hashlib.sha256()
    for rel in SPMM_SOURCES:
        with open(os.path.join(HERE, rel), "rb") as f:
            h.update(f.read())
    return h.hexdigest()


def _counter_means(path: str) -> dict:
    """(kernel name, counter) -> mean value per dispatch."""
    acc = defaultdict(list)
    with open(path) as f:
        for r in csv.DictReader(f):
            acc[(r["Kernel_Name"], r["Counter_Name"])].append(float(r["Counter_Value"]))
    return {k: sum(v) / len(v) for k, v in acc.items()}


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
