"""The C ABI without a GPU: the library loads, exports every function include/spm.h declares,
and rejects bad arguments on the host (before any HIP call)."""
import ctypes
import os
import re

import pytest

from paper_1805_03380_amd import _lib

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _lib_or_build():
    if not os.path.exists(_lib.LIB_PATH):
        from paper_1805_03380_amd import build
        build.build()
    return _lib.load()


def _declared():
    with open(os.path.join(ROOT, "include", "spm.h")) as f:
        text = f.read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(spm_[a-z0-9_]+)\s*\(", text)))


def test_exports_every_declared_symbol():
    lib = _lib_or_build()
    names = _declared()
    assert "spm_coo_to_csc" in names and "spm_csc_spmm_backward" in names
    missing = [n for n in names if not hasattr(lib, n)]
    assert not missing, missing
    assert set(names) == set(_lib.SIGNATURES), "binding and header disagree"


def test_status_strings_and_version():
    lib = _lib_or_build()
    assert lib.spm_status_string(0) == b"ok"
    assert lib.spm_status_string(2) == b"triplet index out of range"
    assert lib.spm_version().startswith(b"0.")


def test_workspace_sizes():
    lib = _lib_or_build()
    # the partition layout follows the tuning: sizes must be asked for with the same tuning
    # that runs the call
    ws = ctypes.c_size_t(0)
    assert lib.spm_coo_to_csc_workspace(10, 10, 100, ctypes.byref(ws)) == _lib.OK
    small = ws.value
    assert lib.spm_coo_to_csc_workspace(10, 10, 10_000, ctypes.byref(ws)) == _lib.OK
    assert ws.value > small and ws.value % 256 == 0
    assert lib.spm_coo_to_csc_workspace(-1, 10, 100, ctypes.byref(ws)) == _lib.EINVAL
    assert lib.spm_coo_to_csc_workspace(10, 2 ** 31, 100, ctypes.byref(ws)) == _lib.EOVERFLOW
    assert lib.spm_coo_to_csc_workspace(10, 10, 2 ** 31, ctypes.byref(ws)) == _lib.EOVERFLOW
    assert lib.spm_coo_to_csc_workspace(10, 10, 10, None) == _lib.EINVAL
    pb, wb = ctypes.c_size_t(0), ctypes.c_size_t(0)
    for shape in ((10, 10, 100), (100_000, 100_000, 1_000_000), (300_000, 2000, 4_000_000)):
        assert lib.spm_coo_to_csc_plan_size(*shape, ctypes.byref(pb), ctypes.byref(wb)) == _lib.OK
        assert lib.spm_coo_to_csc_workspace(*shape, ctypes.byref(ws)) == _lib.OK
        assert wb.value >= ws.value and wb.value % 256 == 0
        plan_b, plan_w = ctypes.c_size_t(0), ctypes.c_size_t(0)
        assert lib.spm_csc_plan_size(*shape, ctypes.byref(plan_b), ctypes.byref(plan_w)) == _lib.OK
        assert pb.value == plan_b.value
    assert lib.spm_coo_to_csc_plan_size(10, 10, 10, None, ctypes.byref(wb)) == _lib.EINVAL
    pb, wb = ctypes.c_size_t(0), ctypes.c_size_t(0)
    assert lib.spm_csc_plan_size(100, 50, 1000, ctypes.byref(pb), ctypes.byref(wb)) == _lib.OK
    assert pb.value >= 4 * (101 + 2000) and wb.value >= 16 * 1000


def test_host_validation_rejects_before_launch():
    lib = _lib_or_build()
    fake = 0x1000  # never dereferenced: every call below fails validation first
    ws = ctypes.c_void_p(0x100000)
    args = dict(n_rows=4, n_cols=4, nnz=8)

    def c2c(n_rows=4, n_cols=4, nnz=8, row=fake, col=fake, val=fake, vt=_lib.F64, cp=fake,
            ri=fake, vo=fake, ot=_lib.F64, info=fake, w=ws, wsb=1 << 30):
        return lib.spm_coo_to_csc(n_rows, n_cols, nnz, row, col, val, vt, cp, ri, vo, ot, info,
                                  w, wsb, None)

    assert c2c(n_rows=-1) == _lib.EINVAL
    assert c2c(nnz=2 ** 31) == _lib.EOVERFLOW
    assert c2c(vt=7) == _lib.EDTYPE
    assert c2c(ot=_lib.BF16) == _lib.EDTYPE
    assert c2c(row=None) == _lib.EINVAL
    assert c2c(info=None) == _lib.EINVAL
    assert c2c(w=ctypes.c_void_p(0x100010)) == _lib.EINVAL  # not 256-byte aligned
    assert c2c(wsb=16) == _lib.EWORKSPACE
    # spmm / backward argument checks
    csc = _lib.ORDER_CSC
    assert lib.spm_csc_spmm(4, 4, 8, 0, fake, fake, _lib.F32, csc, fake, 4, _lib.F32, fake, 4,
                            _lib.F32, None) == _lib.EINVAL
    assert lib.spm_csc_spmm(4, 4, 8, 8, fake, fake, _lib.F32, csc, fake, 4, _lib.F32, fake, 8,
                            _lib.F32, None) == _lib.EINVAL  # ldx < k
    assert lib.spm_csc_spmm(4, 4, 8, 4, fake, fake, _lib.BF16, csc, fake, 4, _lib.F32, fake, 4,
                            _lib.F32, None) == _lib.EDTYPE
    assert lib.spm_csc_spmm(4, 4, 8, 4, fake, fake, _lib.F32, 7, fake, 4, _lib.F32, fake, 4,
                            _lib.F32, None) == _lib.EINVAL  # unknown value order
    assert lib.spm_csc_spmm_backward(4, 4, 8, 4, None, fake, fake, _lib.F32, fake, 4, _lib.F32,
                                     fake, 4, _lib.F32, fake, 4, _lib.F32, fake, _lib.F32,
                                     None) == _lib.EINVAL

    def bw(gt=_lib.F64, xt=_lib.F32, dxt=_lib.F32, dvt=_lib.F64, ldg=4):
        return lib.spm_csc_spmm_backward(4, 4, 8, 4, None, fake, fake, _lib.F64, fake, ldg, gt,
                                         fake, 4, xt, fake, 4, dxt, fake, dvt, None)

    # G's element type is checked on its own (a NULL col_ptr is reported only after it)
    assert bw(gt=7) == _lib.EDTYPE
    assert bw(gt=_lib.F64, xt=_lib.F32) == _lib.EINVAL
    assert bw(gt=_lib.BF16, xt=_lib.F64) == _lib.EINVAL
    assert bw(ldg=3) == _lib.EINVAL
    assert lib.spm_csc_plan_build(4, 4, 8, fake, fake, None, _lib.F32, fake, 16, None, fake, ws,
                                  1 << 30, None) == _lib.EWORKSPACE
    assert lib.spm_csc_plan_build(4, 4, 8, fake, fake, fake, _lib.F32, fake, 1 << 20, None,
                                  fake, ws, 1 << 30, None) == _lib.EINVAL  # val without val_plan
    assert lib.spm_csc_plan_build(4, 4, 8, fake, fake, fake, _lib.BF16, fake, 1 << 20, fake,
                                  fake, ws, 1 << 30, None) == _lib.EDTYPE
    # assembly + plan in one call

    def c2cp(n_rows=4, n_cols=4, nnz=8, vt=_lib.F64, ot=_lib.F64, plan=fake, pb=1 << 20,
             vplan=fake, pinfo=fake, w=ws, wsb=1 << 30):
        return lib.spm_coo_to_csc_plan(n_rows, n_cols, nnz, fake, fake, fake, vt, fake, fake,
                                       fake, ot, fake, plan, pb, vplan, pinfo, w, wsb, None)

    assert c2cp(n_cols=-2) == _lib.EINVAL
    assert c2cp(n_rows=2 ** 31) == _lib.EOVERFLOW
    assert c2cp(vt=9) == _lib.EDTYPE
    assert c2cp(ot=_lib.BF16) == _lib.EDTYPE
    assert c2cp(plan=None) == _lib.EINVAL
    assert c2cp(pinfo=None) == _lib.EINVAL
    assert c2cp(plan=ctypes.c_void_p(0x1010)) == _lib.EINVAL  # not 256-byte aligned
    assert c2cp(pb=16) == _lib.EWORKSPACE
    assert c2cp(wsb=16) == _lib.EWORKSPACE
    # batch insertion

    def ins(n_rows=4, n_cols=4, cap=8, nt=3, vt=_lib.F64, ot=_lib.F64, acp=fake, cp=fake,
            info=fake, w=ws, wsb=1 << 30):
        return lib.spm_csc_insert(n_rows, n_cols, cap, acp, fake, fake, nt, fake, fake, fake, vt,
                                  cp, fake, fake, ot, info, w, wsb, None)

    assert ins(cap=-1) == _lib.EINVAL
    assert ins(nt=2 ** 31) == _lib.EOVERFLOW
    assert ins(cap=2 ** 30, nt=2 ** 30) == _lib.EOVERFLOW
    assert ins(vt=_lib.BF16) == _lib.EDTYPE
    assert ins(ot=_lib.BF16) == _lib.EDTYPE
    assert ins(acp=None) == _lib.EINVAL
    assert ins(info=None) == _lib.EINVAL
    assert ins(n_cols=0) == _lib.EINVAL  # no columns: nothing for the partition to group
    assert ins(wsb=16) == _lib.EWORKSPACE
    # transpose

    def tr(n_rows=4, n_cols=4, cap=8, vt=_lib.F64, cp=fake, tcp=fake, tri=fake, info=fake, w=ws,
           wsb=1 << 30):
        return lib.spm_csc_transpose(n_rows, n_cols, cap, cp, fake, fake, vt, tcp, tri, fake,
                                     info, w, wsb, None)

    wb = ctypes.c_size_t(0)
    assert lib.spm_csc_transpose_workspace(4, 4, 8, ctypes.byref(wb)) == _lib.OK and wb.value
    assert lib.spm_csc_transpose_workspace(4, -1, 8, ctypes.byref(wb)) == _lib.EINVAL
    assert tr(cap=-1) == _lib.EINVAL
    assert tr(n_rows=2 ** 31) == _lib.EOVERFLOW
    assert tr(vt=_lib.BF16) == _lib.EDTYPE
    assert tr(cp=None) == _lib.EINVAL
    assert tr(tcp=None) == _lib.EINVAL
    assert tr(tri=None) == _lib.EINVAL
    assert tr(info=None) == _lib.EINVAL
    assert tr(w=ctypes.c_void_p(0x1010)) == _lib.EINVAL
    assert tr(wsb=16) == _lib.EWORKSPACE
    # trace(A^T B)

    def ta(n_rows=4, n_cols=4, ca=8, cb=8, vt=_lib.F64, acp=fake, bcp=fake, ari=fake, out=fake,
           info=fake, w=ws, wsb=1 << 30):
        return lib.spm_csc_trace_atb(n_rows, n_cols, ca, acp, ari, fake, cb, bcp, fake, fake, vt,
                                     out, info, w, wsb, None)

    assert lib.spm_csc_trace_atb_workspace(4, ctypes.byref(wb)) == _lib.OK and wb.value >= 256
    assert lib.spm_csc_trace_atb_workspace(-1, ctypes.byref(wb)) == _lib.EINVAL
    assert lib.spm_csc_trace_atb_workspace(2 ** 31, ctypes.byref(wb)) == _lib.EOVERFLOW
    assert ta(ca=-1) == _lib.EINVAL
    assert ta(n_rows=2 ** 31) == _lib.EOVERFLOW
    assert ta(cb=2 ** 31) == _lib.EOVERFLOW
    assert ta(vt=_lib.BF16) == _lib.EDTYPE
    assert ta(acp=None) == _lib.EINVAL
    assert ta(bcp=None) == _lib.EINVAL
    assert ta(ari=None) == _lib.EINVAL
    assert ta(out=None) == _lib.EINVAL
    assert ta(info=None) == _lib.EINVAL
    assert ta(w=ctypes.c_void_p(0x1010)) == _lib.EINVAL
    assert ta(wsb=16) == _lib.EWORKSPACE
    # the allocation-free assembly + plan: sizes whose workspace exceeds the fixed scratch
    # array are rejected on the host, before anything touches the device
    assert lib.spm_coo_to_csc_plan_noalloc(200_000, 200_000, 5_000_000, fake, fake, fake,
                                           _lib.F32, fake, fake, fake, _lib.F32, fake, fake,
                                           1 << 30, None, fake, None) == _lib.EWORKSPACE
    assert lib.spm_coo_to_csc_plan_noalloc(-1, 4, 4, fake, fake, fake, _lib.F32, fake, fake,
                                           fake, _lib.F32, fake, fake, 1 << 30, None, fake,
                                           None) == _lib.EINVAL
    # more columns than one launch of 16-lane groups covers (2^32 lanes): rejected on the host
    assert ta(n_cols=2 ** 28 + 16, wsb=1 << 40) == _lib.EOVERFLOW
    # sum of two CSCs

    def ad(n_rows=4, n_cols=4, ca=8, cb=8, vt=_lib.F64, ot=_lib.F64, acp=fake, bcp=fake,
           info=fake, w=ws, wsb=1 << 30):
        return lib.spm_csc_add(n_rows, n_cols, ca, acp, fake, fake, cb, bcp, fake, fake, vt,
                               fake, fake, fake, ot, info, w, wsb, None)

    assert lib.spm_csc_add_workspace(4, 4, 8, 8, ctypes.byref(wb)) == _lib.OK and wb.value
    assert ad(ca=-1) == _lib.EINVAL
    assert ad(cb=2 ** 31) == _lib.EOVERFLOW
    assert ad(ca=2 ** 30, cb=2 ** 30) == _lib.EOVERFLOW
    assert ad(vt=_lib.BF16) == _lib.EDTYPE
    assert ad(ot=_lib.BF16) == _lib.EDTYPE
    assert ad(acp=None) == _lib.EINVAL
    assert ad(bcp=None) == _lib.EINVAL
    assert ad(info=None) == _lib.EINVAL
    assert ad(n_cols=0) == _lib.EINVAL
    assert ad(wsb=16) == _lib.EWORKSPACE
    # gradient per input triplet

    def tg(n_rows=4, n_cols=4, n=8, k=4, row=fake, vt=_lib.F32, ldg=4, gt=_lib.F32, ldx=4,
           xt=_lib.F32, dv=fake, dvt=_lib.F32):
        return lib.spm_coo_triplet_grad(n_rows, n_cols, n, k, row, fake, vt, fake, ldg, gt, fake,
                                        ldx, xt, dv, dvt, None)

    assert tg(n=0) == _lib.OK  # nothing to do, nothing enqueued
    assert tg(k=0) == _lib.EINVAL
    assert tg(ldg=3) == _lib.EINVAL
    assert tg(ldx=3) == _lib.EINVAL
    assert tg(n=-1) == _lib.EINVAL
    assert tg(n=2 ** 31) == _lib.EOVERFLOW
    assert tg(vt=_lib.BF16) == _lib.EDTYPE
    assert tg(xt=7) == _lib.EDTYPE
    assert tg(gt=7) == _lib.EDTYPE
    assert tg(dvt=_lib.BF16) == _lib.EDTYPE
    assert tg(row=None) == _lib.EINVAL
    assert tg(dv=None) == _lib.EINVAL

    def tgc(n=8, cap=8, cp=fake, ri=fake, dvt=_lib.F64, k=4, gt=_lib.F64):
        return lib.spm_coo_triplet_grad_csc(4, 4, n, k, fake, fake, cap, cp, ri, fake, dvt,
                                            _lib.F32, fake, 4, gt, fake, 4, _lib.F32, fake,
                                            _lib.F32, None)

    assert tgc(n=0) == _lib.OK
    assert tgc(k=0) == _lib.EINVAL
    assert tgc(cap=-1) == _lib.EINVAL
    assert tgc(cp=None) == _lib.EINVAL
    assert tgc(ri=None) == _lib.EINVAL
    assert tgc(dvt=_lib.BF16) == _lib.EDTYPE
    assert tgc(gt=9) == _lib.EDTYPE


def test_tuning_roundtrip():
    lib = _lib_or_build()
    t = _lib.Tuning()
    assert lib.spm_tuning_get(ctypes.byref(t)) == _lib.OK
    saved = _lib.Tuning.from_buffer_copy(t)
    bad = _lib.Tuning.from_buffer_copy(t)
    bad.spmm_block = 100
    assert lib.spm_tuning_set(ctypes.byref(bad)) == _lib.EINVAL
    bad = _lib.Tuning.from_buffer_copy(t)
    bad.part_bucket_target = 1000  # not a power of two
    assert lib.spm_tuning_set(ctypes.byref(bad)) == _lib.EINVAL
    bad = _lib.Tuning.from_buffer_copy(t)
    bad.batch_spmm_wg_per_cu = 33
    assert lib.spm_tuning_set(ctypes.byref(bad)) == _lib.EINVAL
    bad = _lib.Tuning.from_buffer_copy(t)
    bad.trace_group_width = 8
    assert lib.spm_tuning_set(ctypes.byref(bad)) == _lib.EINVAL
    bad = _lib.Tuning.from_buffer_copy(t)
    bad.part_max_tiles = 8192
    assert lib.spm_tuning_set(ctypes.byref(bad)) == _lib.EINVAL
    good = _lib.Tuning.from_buffer_copy(t)
    good.spmm_block = 128
    good.part_bucket_target = 1024
    assert lib.spm_tuning_set(ctypes.byref(good)) == _lib.OK
    chk = _lib.Tuning()
    lib.spm_tuning_get(ctypes.byref(chk))
    assert chk.spmm_block == 128 and chk.part_bucket_target == 1024
    assert lib.spm_tuning_set(ctypes.byref(saved)) == _lib.OK


def test_named_tunings_per_thread():
    """A named tuning selected by one thread is that thread's alone; NULL goes back to the
    process values; unknown keys and invalid values are refused."""
    import threading
    lib = _lib_or_build()
    base = _lib.get_tuning().as_dict()
    _lib.register_tuning("narrow", spmm_block=64, spmm_blocks_per_cu=4)
    _lib.register_tuning("wide", spmm_block=256, spmm_blocks_per_cu=64)
    seen = {}

    def worker(key):
        _lib.select_tuning(key)
        seen[key] = _lib.get_tuning().as_dict()
        _lib.select_tuning(None)
        seen[key + "/after"] = _lib.get_tuning().as_dict()

    ts = [threading.Thread(target=worker, args=(k,)) for k in ("narrow", "wide")]
    for t in ts:
        t.start()
    for t in ts:
        t.join()
    assert seen["narrow"]["spmm_block"] == 64 and seen["narrow"]["spmm_blocks_per_cu"] == 4
    assert seen["wide"]["spmm_block"] == 256 and seen["wide"]["spmm_blocks_per_cu"] == 64
    assert seen["narrow/after"] == base and seen["wide/after"] == base
    assert _lib.get_tuning().as_dict() == base  # this thread never selected one
    assert lib.spm_tuning_select(b"no such key") == _lib.EINVAL
    bad = _lib.Tuning.from_buffer_copy(_lib.get_tuning())
    bad.spmm_block = 100
    assert lib.spm_tuning_register(b"bad", ctypes.byref(bad)) == _lib.EINVAL
    assert lib.spm_tuning_register(None, ctypes.byref(bad)) == _lib.EINVAL


def test_plan_bytes_alias_and_batch_key_checks():
    lib = _lib_or_build()
    pb, wb, pb2 = ctypes.c_size_t(0), ctypes.c_size_t(0), ctypes.c_size_t(0)
    for shape in ((10, 10, 100), (100_000, 100_000, 1_000_000)):
        assert lib.spm_csc_plan_size(*shape, ctypes.byref(pb), ctypes.byref(wb)) == _lib.OK
        assert lib.spm_csc_plan_bytes(*shape, ctypes.byref(pb2)) == _lib.OK
        assert pb.value == pb2.value
    assert lib.spm_csc_plan_bytes(-1, 1, 1, ctypes.byref(pb2)) == _lib.EINVAL
    fake = 0x1000
    args = [4, 32] + [fake] * 5 + [_lib.F32, fake, fake, _lib.F32] + [fake] * 10 + \
        [64, 1024, 0, 0x100000, 1 << 30]
    # an unknown key is refused before anything is enqueued
    assert lib.spm_batch_coo_to_csc_spmm(*args, b"never registered", None) == _lib.EINVAL


def test_roctx_ranges_are_optional():
    """With SPM_ROCTX=1 the compute entry points push and pop a roctx range (roctx found by
    dlopen); rejected calls still return their status, with or without the variable.  Each
    setting runs in a process of its own (the lookup happens once per process)."""
    import subprocess
    import sys
    _lib_or_build()
    code = ("import ctypes, sys; sys.path.insert(0, %r); "
            "from paper_1805_03380_amd import _lib; lib = _lib.load(); f = 0x1000; "
            "st = [lib.spm_coo_to_csc(-1, 4, 8, f, f, f, _lib.F64, f, f, f, _lib.F64, f, "
            "ctypes.c_void_p(0x100000), 1 << 30, None) for _ in range(3)]; "
            "st.append(lib.spm_csc_spmm(4, 4, 8, 0, f, f, _lib.F32, _lib.ORDER_CSC, f, 4, "
            "_lib.F32, f, 4, _lib.F32, None)); "
            "print(st)") % ROOT
    for value in ("1", "0", ""):
        env = dict(os.environ, SPM_ROCTX=value)
        out = subprocess.run([sys.executable, "-c", code], env=env, capture_output=True,
                             text=True, timeout=120)
        assert out.returncode == 0, out.stderr
        assert out.stdout.strip() == str([_lib.EINVAL] * 4), (value, out.stdout)
