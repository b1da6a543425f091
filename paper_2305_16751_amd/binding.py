"""ctypes declarations of the C-ABI in include/dom_agg.h.

Argument marshalling only: every step of the computation runs in the HIP
kernels of libdom_agg.so.  Loading fails loudly when the library has not been
built; there is no fallback.
"""
from __future__ import annotations

import ctypes
import os

_PKG = os.path.dirname(os.path.abspath(__file__))
LIB_NAME = "libdom_agg.so"

# dom_agg_status
OK, EINVAL, ENAN, ENOMEM, ETOOBIG, EUNSUPPORTED, ENODEV, EHIP = range(8)
STATUS_NAMES = {OK: "OK", EINVAL: "EINVAL", ENAN: "ENAN", ENOMEM: "ENOMEM", ETOOBIG: "ETOOBIG",
                EUNSUPPORTED: "EUNSUPPORTED", ENODEV: "ENODEV", EHIP: "EHIP"}
# dom_agg_op
SUM, MAX, COUNT = 0, 1, 2
OPS = {"sum": SUM, "max": MAX, "count": COUNT}
# dom_agg_dtype
I32, I64, F32, F64 = 0, 1, 2, 3
# plan flags
KEEP, RECOMPUTE, GRAPH, NO_TUNE, BASIC = 0, 2, 4, 8, 16


def LE(axis: int) -> int:
    """DOM_AGG_LE(axis): <= instead of < on that axis."""
    return 0x100 << axis

# exported functions, in the order include/dom_agg.h declares them
EXPORTS = (
    "dom_agg_set_allocator",
    "dom_agg_plan",
    "dom_agg_forward",
    "dom_agg_forward_records",
    "dom_agg_backward",
    "dom_agg_run",
    "dom_agg_run_static",
    "dom_agg_plan_get_info",
    "dom_agg_plan_destroy",
    "dom_agg_status_string",
    "dom_agg_last_error",
    "dom_agg_timing_enable",
    "dom_agg_timing_read",
)


class DomAggError(RuntimeError):
    def __init__(self, status: int, message: str):
        super().__init__(f"{STATUS_NAMES.get(status, status)}: {message}")
        self.status = status
        self.message = message


class PlanInfo(ctypes.Structure):
    _fields_ = [
        ("n_inst", ctypes.c_int64),
        ("n_data", ctypes.c_int64),
        ("n_query", ctypes.c_int64),
        ("records", ctypes.c_int64),
        ("data_records", ctypes.c_int64),
        ("m", ctypes.c_int32),
        ("key_bits", ctypes.c_int32),
        ("L", ctypes.c_int32 * 4),
        ("sort_passes", ctypes.c_int32),
        ("digit_bits", ctypes.c_int32),
        ("sort_tile", ctypes.c_int32),
        ("scan_tile", ctypes.c_int32),
        ("regroup_slots", ctypes.c_int32),
        ("sort_classes", ctypes.c_int32),
        ("sort_class_records", ctypes.c_int64 * 4),
        ("workspace_bytes", ctypes.c_size_t),
        ("le_mask", ctypes.c_uint32),
        ("basic", ctypes.c_int32),
        ("graph_captures", ctypes.c_int64),
        ("record_bytes", ctypes.c_int32),
    ]

    def as_dict(self) -> dict:
        d = {f: getattr(self, f) for f, _ in self._fields_ if f not in ("L", "sort_class_records")}
        d["L"] = [self.L[i] for i in range(self.m if self.basic else max(self.m - 1, 0))]
        d["sort_class_records"] = [self.sort_class_records[i] for i in range(self.sort_classes)]
        return d


ALLOC_FN = ctypes.CFUNCTYPE(ctypes.c_void_p, ctypes.c_size_t, ctypes.c_void_p, ctypes.c_void_p)
RELEASE_FN = ctypes.CFUNCTYPE(None, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p)

_lib = None


def lib_path() -> str:
    return os.path.join(_PKG, LIB_NAME)


def load(path: str | None = None):
    """Loads libdom_agg.so (built in-tree by paper_2305_16751_amd.build)."""
    global _lib
    if _lib is not None and path is None:
        return _lib
    p = path or lib_path()
    if not os.path.exists(p):
        raise RuntimeError(
            f"{p} is missing: the HIP library has not been built "
            "(run `python -m paper_2305_16751_amd.build` or __graft_entry__.build())")
    lib = ctypes.CDLL(p)
    P, I, I64, U32 = ctypes.c_void_p, ctypes.c_int, ctypes.c_int64, ctypes.c_uint32
    lib.dom_agg_set_allocator.argtypes = [ALLOC_FN, RELEASE_FN, P]
    lib.dom_agg_set_allocator.restype = I
    lib.dom_agg_plan.argtypes = [ctypes.POINTER(P), I, I, P, P, I64, P, P, U32, P]
    lib.dom_agg_plan.restype = I
    lib.dom_agg_forward.argtypes = [P, I, I, P, P, P]
    lib.dom_agg_forward.restype = I
    lib.dom_agg_forward_records.argtypes = [P, I, I, P, P, P, P]
    lib.dom_agg_forward_records.restype = I
    lib.dom_agg_backward.argtypes = [P, I, P, P, P]
    lib.dom_agg_backward.restype = I
    lib.dom_agg_run.argtypes = [I, I, P, P, I64, P, P, I, I, P, P, U32, P]
    lib.dom_agg_run.restype = I
    lib.dom_agg_run_static.argtypes = [I, I, P, P, I64, P, P, I, I, P, P, U32, P]
    lib.dom_agg_run_static.restype = I
    lib.dom_agg_plan_get_info.argtypes = [P, ctypes.POINTER(PlanInfo)]
    lib.dom_agg_plan_get_info.restype = I
    lib.dom_agg_plan_destroy.argtypes = [P]
    lib.dom_agg_plan_destroy.restype = None
    lib.dom_agg_status_string.argtypes = [I]
    lib.dom_agg_status_string.restype = ctypes.c_char_p
    lib.dom_agg_last_error.argtypes = []
    lib.dom_agg_last_error.restype = ctypes.c_char_p
    lib.dom_agg_timing_enable.argtypes = [I]
    lib.dom_agg_timing_enable.restype = I
    lib.dom_agg_timing_read.argtypes = [ctypes.POINTER(ctypes.c_char_p), ctypes.POINTER(ctypes.c_double),
                                        ctypes.POINTER(ctypes.c_int64), I]
    lib.dom_agg_timing_read.restype = I
    if path is None:
        _lib = lib
    return lib


def check(status: int):
    if status != OK:
        msg = load().dom_agg_last_error()
        raise DomAggError(status, msg.decode() if msg else "")


def timing_enable(enable: bool = True):
    check(load().dom_agg_timing_enable(1 if enable else 0))


def timing_read(cap: int = 64) -> dict:
    """{kernel name: (total ms, launches)} since timing was enabled."""
    lib = load()
    names = (ctypes.c_char_p * cap)()
    ms = (ctypes.c_double * cap)()
    cnt = (ctypes.c_int64 * cap)()
    k = lib.dom_agg_timing_read(names, ms, cnt, cap)
    if k < 0:
        raise DomAggError(EHIP, "timing read failed")
    return {names[i].decode(): (ms[i], cnt[i]) for i in range(min(k, cap))}
