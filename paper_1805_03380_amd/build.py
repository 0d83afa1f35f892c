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
    "-shared",
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


def build(verbose: bool = False) -> str:
    os.makedirs(LIBDIR, exist_ok=True)
    tmp = LIB + ".tmp%d" % os.getpid()
    cmd = [hipcc()] + HIPCC_FLAGS + ["-I", os.path.join(ROOT, "include"), "-I", CSRC] + \
        sources() + ["-o", tmp]
    if verbose:
        print(" ".join(cmd), flush=True)
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        sys.stderr.write(r.stdout + r.stderr)
        raise RuntimeError("hipcc failed building libspm.so")
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose=True))
