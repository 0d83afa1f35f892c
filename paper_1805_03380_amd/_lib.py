"""ctypes binding of libspm.so (the C ABI in include/spm.h).

Argument marshalling only: every step of the path runs in the library's HIP kernels.  There
is no fallback -- if the library is missing the first call raises.
"""
from __future__ import annotations

import ctypes
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "lib", "libspm.so")

# spm_status
OK, EINVAL, EBOUNDS, EOVERFLOW, EWORKSPACE, EDTYPE, EHIP = range(7)
# spm_dtype
F64, F32, BF16 = 0, 1, 2
# spm_val_order
ORDER_CSC, ORDER_PLAN = 0, 1
# SPM_NOALLOC_SCRATCH_BYTES
NOALLOC_SCRATCH_BYTES = 64 << 20

_lib = None

c_i64 = ctypes.c_int64
c_i32 = ctypes.c_int32
c_p = ctypes.c_void_p
c_size_p = ctypes.POINTER(ctypes.c_size_t)


class BatchItem(ctypes.Structure):
    """spm_batch_item."""
    _fields_ = [("n_rows", ctypes.c_int32), ("n_cols", ctypes.c_int32),
                ("nnz_in", ctypes.c_int32), ("reserved", ctypes.c_int32),
                ("trip_off", ctypes.c_int64), ("colptr_off", ctypes.c_int64),
                ("rowptr_off", ctypes.c_int64), ("x_off", ctypes.c_int64),
                ("g_off", ctypes.c_int64)]


class Tuning(ctypes.Structure):
    """spm_tuning."""
    _fields_ = [("spmm_block", ctypes.c_int32), ("spmm_blocks_per_cu", ctypes.c_int32),
                ("batch_wg_per_cu", ctypes.c_int32), ("part_bucket_target", ctypes.c_int32),
                ("part_max_tiles", ctypes.c_int32), ("batch_spmm_wg_per_cu", ctypes.c_int32),
                ("trace_group_width", ctypes.c_int32), ("reserved", ctypes.c_int32)]

    FIELDS = ("spmm_block", "spmm_blocks_per_cu", "batch_wg_per_cu", "part_bucket_target",
              "part_max_tiles", "batch_spmm_wg_per_cu", "trace_group_width")

    def as_dict(self):
        return {f: int(getattr(self, f)) for f in self.FIELDS}


def get_tuning() -> Tuning:
    t = Tuning()
    check(load().spm_tuning_get(ctypes.byref(t)), "spm_tuning_get")
    return t


def set_tuning(**kw) -> Tuning:
    """Update some tuning fields (spm_tuning_set); returns the previous values."""
    old = get_tuning()
    t = Tuning.from_buffer_copy(old)
    for k, v in kw.items():
        if k not in Tuning.FIELDS:
            raise KeyError(k)
        setattr(t, k, int(v))
    check(load().spm_tuning_set(ctypes.byref(t)), "spm_tuning_set")
    return old


def register_tuning(key: str, **kw) -> None:
    """Store a named tuning (spm_tuning_register): the current values with `kw` changed."""
    t = Tuning.from_buffer_copy(get_tuning())
    for k, v in kw.items():
        if k not in Tuning.FIELDS:
            raise KeyError(k)
        setattr(t, k, int(v))
    check(load().spm_tuning_register(key.encode(), ctypes.byref(t)), "spm_tuning_register")


def select_tuning(key: str | None) -> None:
    """Make a named tuning the calling thread's (spm_tuning_select); None: process values."""
    check(load().spm_tuning_select(None if key is None else key.encode()), "spm_tuning_select")


# name -> (restype, argtypes)
SIGNATURES = {
    "spm_status_string": (ctypes.c_char_p, [ctypes.c_int]),
    "spm_version": (ctypes.c_char_p, []),
    "spm_coo_to_csc_workspace": (ctypes.c_int, [c_i64, c_i64, c_i64, c_size_p]),
    "spm_coo_to_csc": (ctypes.c_int, [c_i64, c_i64, c_i64, c_p, c_p, c_p, ctypes.c_int, c_p, c_p,
                                      c_p, ctypes.c_int, c_p, c_p, ctypes.c_size_t, c_p]),
    "spm_csc_plan_size": (ctypes.c_int, [c_i64, c_i64, c_i64, c_size_p, c_size_p]),
    "spm_csc_plan_build": (ctypes.c_int, [c_i64, c_i64, c_i64, c_p, c_p, c_p, ctypes.c_int, c_p,
                                          ctypes.c_size_t, c_p, c_p, c_p, ctypes.c_size_t,
                                          c_p]),
    "spm_coo_to_csc_plan_size": (ctypes.c_int, [c_i64, c_i64, c_i64, c_size_p, c_size_p]),
    "spm_coo_to_csc_plan": (ctypes.c_int, [c_i64, c_i64, c_i64, c_p, c_p, c_p, ctypes.c_int,
                                           c_p, c_p, c_p, ctypes.c_int, c_p, c_p,
                                           ctypes.c_size_t, c_p, c_p, c_p, ctypes.c_size_t,
                                           c_p]),
    "spm_coo_to_csc_plan_noalloc": (ctypes.c_int, [c_i64, c_i64, c_i64, c_p, c_p, c_p,
                                                   ctypes.c_int, c_p, c_p, c_p, ctypes.c_int,
                                                   c_p, c_p, ctypes.c_size_t, c_p, c_p, c_p]),
    "spm_csc_transpose_workspace": (ctypes.c_int, [c_i64, c_i64, c_i64, c_size_p]),
    "spm_csc_transpose": (ctypes.c_int, [c_i64, c_i64, c_i64, c_p, c_p, c_p, ctypes.c_int, c_p,
                                         c_p, c_p, c_p, c_p, ctypes.c_size_t, c_p]),
    "spm_csc_trace_atb_workspace": (ctypes.c_int, [c_i64, c_size_p]),
    "spm_csc_trace_atb": (ctypes.c_int, [c_i64, c_i64, c_i64, c_p, c_p, c_p, c_i64, c_p, c_p, c_p,
                                         ctypes.c_int, c_p, c_p, c_p, ctypes.c_size_t, c_p]),
    "spm_coo_triplet_grad": (ctypes.c_int, [c_i64, c_i64, c_i64, c_i64, c_p, c_p, ctypes.c_int,
                                            c_p, c_i64, ctypes.c_int, c_p, c_i64, ctypes.c_int,
                                            c_p, ctypes.c_int, c_p]),
    "spm_csc_add_workspace": (ctypes.c_int, [c_i64, c_i64, c_i64, c_i64, c_size_p]),
    "spm_csc_add": (ctypes.c_int, [c_i64, c_i64, c_i64, c_p, c_p, c_p, c_i64, c_p, c_p, c_p,
                                   ctypes.c_int, c_p, c_p, c_p, ctypes.c_int, c_p, c_p,
                                   ctypes.c_size_t, c_p]),
    "spm_coo_triplet_grad_csc": (ctypes.c_int, [c_i64, c_i64, c_i64, c_i64, c_p, c_p, c_i64,
                                                c_p, c_p, c_p, ctypes.c_int, ctypes.c_int, c_p,
                                                c_i64, ctypes.c_int, c_p, c_i64, ctypes.c_int,
                                                c_p, ctypes.c_int, c_p]),
    "spm_csc_insert_workspace": (ctypes.c_int, [c_i64, c_i64, c_i64, c_i64, c_size_p]),
    "spm_csc_insert": (ctypes.c_int, [c_i64, c_i64, c_i64, c_p, c_p, c_p, c_i64, c_p, c_p, c_p,
                                      ctypes.c_int, c_p, c_p, c_p, ctypes.c_int, c_p, c_p,
                                      ctypes.c_size_t, c_p]),
    "spm_csc_spmm": (ctypes.c_int, [c_i64, c_i64, c_i64, c_i64, c_p, c_p, ctypes.c_int,
                                    ctypes.c_int, c_p, c_i64, ctypes.c_int, c_p, c_i64,
                                    ctypes.c_int, c_p]),
    "spm_csc_spmm_backward": (ctypes.c_int, [c_i64, c_i64, c_i64, c_i64, c_p, c_p, c_p,
                                             ctypes.c_int, c_p, c_i64, ctypes.c_int, c_p, c_i64,
                                             ctypes.c_int, c_p, c_i64, ctypes.c_int, c_p,
                                             ctypes.c_int, c_p]),
    "spm_batch_workspace": (ctypes.c_int, [c_i64, c_i64, c_i32, c_size_p]),
    "spm_batch_schedule": (ctypes.c_int, [c_p, c_i32, c_i64, c_p]),
    "spm_batch_run": (ctypes.c_int, [c_i32, c_i64, c_p, c_p, c_p, c_p, c_p, ctypes.c_int, c_p,
                                     c_p, ctypes.c_int, c_p, c_p, c_p, c_p, c_p, c_p, c_p, c_p,
                                     c_p, c_p, c_i64, c_i64, c_i32, c_p, ctypes.c_size_t, c_p]),
    "spm_batch_coo_to_csc_spmm": (ctypes.c_int, [c_i32, c_i64, c_p, c_p, c_p, c_p, c_p,
                                                 ctypes.c_int, c_p, c_p, ctypes.c_int, c_p, c_p,
                                                 c_p, c_p, c_p, c_p, c_p, c_p, c_p, c_p, c_i64,
                                                 c_i64, c_i32, c_p, ctypes.c_size_t,
                                                 ctypes.c_char_p, c_p]),
    "spm_csc_plan_bytes": (ctypes.c_int, [c_i64, c_i64, c_i64, c_size_p]),
    "spm_tuning_get": (ctypes.c_int, [ctypes.POINTER(Tuning)]),
    "spm_tuning_set": (ctypes.c_int, [ctypes.POINTER(Tuning)]),
    "spm_tuning_register": (ctypes.c_int, [ctypes.c_char_p, ctypes.POINTER(Tuning)]),
    "spm_tuning_select": (ctypes.c_int, [ctypes.c_char_p]),
}


class SpmError(RuntimeError):
    def __init__(self, status: int, where: str):
        self.status = status
        super().__init__("%s: %s (status %d)" % (where, status_string(status), status))


def load():
    """Load libspm.so (raises if it has not been built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError("libspm.so is not built (%s); run `python -m paper_1805_03380_amd.build`"
                           % LIB_PATH)
    lib = ctypes.CDLL(LIB_PATH)
    for name, (res, args) in SIGNATURES.items():
        f = getattr(lib, name)
        f.restype = res
        f.argtypes = args
    _lib = lib
    return lib


def status_string(status: int) -> str:
    return load().spm_status_string(int(status)).decode()


def check(status: int, where: str) -> None:
    if status == OK:
        return
    if status == EBOUNDS:
        raise IndexError(SpmError(status, where))
    if status in (EINVAL, EDTYPE, EWORKSPACE):
        raise ValueError(SpmError(status, where))
    if status == EOVERFLOW:
        raise OverflowError(SpmError(status, where))
    raise SpmError(status, where)
