"""Build libspm.so (gfx950) in-tree with hipcc.

    python -m paper_1805_03380_amd.build

Produces paper_1805_03380_amd/lib/libspm.so from csrc/spm_api.hip (the translation unit that
includes every kernel header of the assembly, plan, products and batch), csrc/spm_trace.hip
(trace(A^T B)), csrc/spm_tgrad.hip (the gradient per input triplet) and include/spm.h.
"""
from __future__ import annotations

import os
import shutil
import subprocess
import sys
from concurrent.futures import ThreadPoolExecutor

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
LIBDIR = os.path.join(HERE, "lib")
LIB = os.path.join(LIBDIR, "libspm.so")
ARCH = os.environ.get("SPM_OFFLOAD_ARCH", "gfx950")

HIPCC_FLAGS = [
    "--offload-arch=%s" % ARCH,
    "-O3",
    "-std=c++17",
    "-fPIC",
    # packed-FP32 instructions off: ordinary float code only
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-Wno-unused-result",
]


def hipcc() -> str:
    for cand in (os.environ.get("HIPCC"), shutil.which("hipcc"), "/opt/rocm/bin/hipcc"):
        if cand and os.path.exists(cand):
            return cand
    raise RuntimeError("hipcc not found")


def sources():
    return [os.path.join(CSRC, "spm_api.hip"), os.path.join(CSRC, "spm_trace.hip"),
            os.path.join(CSRC, "spm_tgrad.hip")]


def _run(cmd, verbose):
    if verbose:
        print(" ".join(cmd), flush=True)
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        sys.stderr.write(r.stdout + r.stderr)
        raise RuntimeError("hipcc failed: %s" % " ".join(cmd[-3:]))


def build(verbose: bool = False) -> str:
    """Each translation unit compiles to an object of its own (in parallel; no device code
    crosses units), then one link makes the shared library."""
    os.makedirs(LIBDIR, exist_ok=True)
    tag = "%d" % os.getpid()
    objs = [os.path.join(LIBDIR, os.path.basename(src) + ".%s.o" % tag) for src in sources()]
    inc = ["-I", os.path.join(ROOT, "include"), "-I", CSRC]
    cmds = [[hipcc()] + HIPCC_FLAGS + inc + ["-c", src, "-o", obj]
            for src, obj in zip(sources(), objs)]
    try:
        with ThreadPoolExecutor(max_workers=len(cmds)) as ex:
            for f in [ex.submit(_run, c, verbose) for c in cmds]:
                f.result()
        tmp = LIB + ".tmp%s" % tag
        _run([hipcc()] + HIPCC_FLAGS + ["-shared"] + objs + ["-o", tmp], verbose)
        os.replace(tmp, LIB)
    finally:
        for o in objs:
            if os.path.exists(o):
                os.remove(o)
    return LIB


if __name__ == "__main__":
    print(build(verbose=True))
