"""Host code under AddressSanitizer and UndefinedBehaviorSanitizer (CPU only, no GPU):
  * the oracle, driven over seeded random and degenerate inputs of every function
    (tests/sanitize/oracle_driver.cpp, which also checks the invariants both assembly reads
    share);
  * the library's host side -- size queries and argument checks of every entry point -- in a
    build whose host code carries the sanitizers (tests/sanitize/abi_driver.cpp).
Any out-of-bounds access, use after free, signed overflow, invalid enumeration value or
misaligned access aborts the driver and fails the test."""
import os
import shutil
import subprocess
from concurrent.futures import ThreadPoolExecutor

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HERE = os.path.join(ROOT, "tests", "sanitize")
CSRC = os.path.join(ROOT, "paper_1805_03380_amd", "csrc")
INC = os.path.join(ROOT, "include")
# the sanitizers apply to host code only (each flag behind -Xarch_host on a hipcc line)
HOST_SAN = ["-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined",
            "-Xarch_host", "-fno-sanitize-recover=all"]
ENV = dict(os.environ, ASAN_OPTIONS="detect_leaks=0:abort_on_error=0",
           UBSAN_OPTIONS="print_stacktrace=1")


def _run(cmd, **kw):
    r = subprocess.run(cmd, capture_output=True, text=True, **kw)
    assert r.returncode == 0, "%s\n%s%s" % (" ".join(cmd), r.stdout[-4000:], r.stderr[-4000:])
    return r


def test_oracle_under_sanitizers(tmp_path):
    exe = str(tmp_path / "oracle_driver")
    _run(["g++", "-std=c++17", "-O1", "-g", "-ffp-contract=off", "-fsanitize=address,undefined",
          "-fno-sanitize-recover=all", os.path.join(ROOT, "oracle", "spm_oracle.cpp"),
          os.path.join(HERE, "oracle_driver.cpp"), "-o", exe])
    r = _run([exe], env=ENV, timeout=300)
    assert "clean" in r.stdout


def _hipcc():
    for cand in (os.environ.get("HIPCC"), shutil.which("hipcc"), "/opt/rocm/bin/hipcc"):
        if cand and os.path.exists(cand):
            return cand
    return None


@pytest.mark.skipif(_hipcc() is None, reason="hipcc not available")
def test_library_host_side_under_sanitizers(tmp_path):
    hipcc = _hipcc()
    common = ["--offload-arch=gfx950", "-O1", "-g", "-std=c++17", "-fPIC", "-Xclang",
              "-target-feature", "-Xclang", "-packed-fp32-ops", "-I", INC, "-I", CSRC] + HOST_SAN
    srcs = ["spm_api.hip", "spm_trace.hip", "spm_tgrad.hip"]
    objs = [str(tmp_path / (s + ".o")) for s in srcs]
    with ThreadPoolExecutor(max_workers=len(srcs)) as ex:
        for f in [ex.submit(_run, [hipcc] + common + ["-c", os.path.join(CSRC, s), "-o", o])
                  for s, o in zip(srcs, objs)]:
            f.result()
    lib = str(tmp_path / "libspm_san.so")
    _run([hipcc, "--offload-arch=gfx950", "-shared", "-fPIC"] + HOST_SAN[:4] + objs +
         ["-o", lib])
    exe = str(tmp_path / "abi_driver")
    _run([hipcc, "-O1", "-g", "-std=c++17", "-I", INC] + HOST_SAN[:4] +
         [os.path.join(HERE, "abi_driver.cpp"), "-L", str(tmp_path), "-lspm_san",
          "-Wl,-rpath," + str(tmp_path), "-o", exe])
    r = _run([exe], env=ENV, timeout=300)
    assert "clean" in r.stdout
