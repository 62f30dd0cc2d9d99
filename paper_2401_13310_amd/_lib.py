"""ctypes declarations of the C ABI in ``include/hist.h``.

Argument marshalling only: every step of histogram filling runs in the HIP
kernels of ``libhist.so``.  The library is loaded from this directory; if it
has not been built yet it is built with hipcc first, and any failure to build
or load raises -- there is no fallback path.
"""
from __future__ import annotations

import ctypes
import os
import threading

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libhist.so")

HIST_OK, HIST_EINVAL, HIST_ENOMEM, HIST_EDEVICE, HIST_ECAPTURE, HIST_ENOTSUP = range(6)
HIST_F64, HIST_F32 = 0, 1
HIST_F_ACC_F32C = 1 << 0
HIST_F_LEARNED = 1 << 1
HIST_F_NO_ALLOC = 1 << 2
HIST_HOST_PINNED = 1 << 0
(HIST_PROBE_READ, HIST_PROBE_LDS_U32, HIST_PROBE_LDS_F64, HIST_PROBE_GLOBAL_U64,
 HIST_PROBE_GLOBAL_F64) = range(5)
HIST_STRAT_AUTO, HIST_STRAT_LDS, HIST_STRAT_GLOBAL, HIST_STRAT_TILED, HIST_STRAT_PART = range(5)
HIST_SEARCH_BINARY, HIST_SEARCH_LEARNED = 0, 1
ACC_NAMES = {0: "u32", 1: "u16", 2: "f64", 3: "f32c"}
STRAT_NAMES = {0: "auto", 1: "lds", 2: "global", 3: "tiled", 4: "part"}


class HistAxis(ctypes.Structure):
    _fields_ = [("nbins", ctypes.c_int32), ("xmin", ctypes.c_double),
                ("xmax", ctypes.c_double), ("edges", ctypes.POINTER(ctypes.c_double))]


class HistFillDesc(ctypes.Structure):
    _fields_ = [("coords", ctypes.c_void_p * 3), ("weights", ctypes.c_void_p),
                ("n", ctypes.c_int64), ("dtype", ctypes.c_int)]


class HistOp(ctypes.Structure):
    _fields_ = [("op", ctypes.c_int32), ("col", ctypes.c_int32), ("value", ctypes.c_double)]


class HistExpr(ctypes.Structure):
    _fields_ = [("ops", ctypes.POINTER(HistOp)), ("nops", ctypes.c_int32)]


class HistDefine(ctypes.Structure):
    _fields_ = [("filter", HistExpr), ("coord", HistExpr * 3), ("weight", HistExpr)]


_lock = threading.Lock()
_lib = None

_H = ctypes.c_void_p
_P = ctypes.c_void_p
_st = ctypes.c_int

PROTOTYPES = {
    "hist_create": (_st, [ctypes.c_int, ctypes.POINTER(HistAxis), ctypes.c_uint32,
                          ctypes.POINTER(_H)]),
    "hist_destroy": (_st, [_H]),
    "hist_fill": (_st, [_H, ctypes.POINTER(_P), _P, ctypes.c_int64, ctypes.c_int, _P]),
    "hist_fill_static": (_st, [_H, ctypes.POINTER(_P), _P, ctypes.c_int64, ctypes.c_int, _P]),
    "hist_static_scratch_bytes": (ctypes.c_int64, []),
    "hist_fill_host": (_st, [_H, ctypes.POINTER(_P), _P, ctypes.c_int64, ctypes.c_int,
                             ctypes.c_int64, ctypes.c_uint32, _P]),
    "hist_findbin": (_st, [_H, ctypes.POINTER(_P), ctypes.c_int64, ctypes.c_int, _P, _P]),
    "hist_reserve": (_st, [_H, ctypes.c_int64, ctypes.c_int, ctypes.c_int, _P]),
    "hist_stats": (_st, [_H, ctypes.POINTER(ctypes.c_double), ctypes.c_int,
                         ctypes.POINTER(ctypes.c_int), _P]),
    "hist_read": (_st, [_H, ctypes.POINTER(ctypes.c_double), ctypes.POINTER(ctypes.c_double),
                        ctypes.POINTER(ctypes.c_int64), _P]),
    "hist_reset": (_st, [_H, _P]),
    "hist_train_index": (_st, [_H, ctypes.c_int, _P]),
    "hist_set_search": (_st, [_H, ctypes.c_int, ctypes.c_int]),
    "hist_index_info": (_st, [_H, ctypes.c_int, ctypes.POINTER(ctypes.c_int),
                              ctypes.POINTER(ctypes.c_int), ctypes.POINTER(ctypes.c_double),
                              ctypes.POINTER(ctypes.c_double)]),
    "hist_set_strategy": (_st, [_H, ctypes.c_int, ctypes.c_int, ctypes.c_int]),
    "hist_set_window": (_st, [_H, ctypes.c_int64, ctypes.c_int]),
    "hist_tune": (_st, [_H, ctypes.POINTER(_P), _P, ctypes.c_int64, ctypes.c_int, _P]),
    "hist_plan_info": (_st, [_H, ctypes.c_int64, ctypes.c_int, ctypes.c_int,
                             ctypes.POINTER(ctypes.c_int), ctypes.POINTER(ctypes.c_int),
                             ctypes.POINTER(ctypes.c_int), ctypes.POINTER(ctypes.c_int64),
                             ctypes.POINTER(ctypes.c_int64), ctypes.POINTER(ctypes.c_int)]),
    "hist_set_threads": (_st, [_H, ctypes.c_int]),
    "hist_set_shape": (_st, [_H, ctypes.c_int, ctypes.c_int]),
    "hist_plan_shape": (_st, [_H, ctypes.c_int64, ctypes.c_int, ctypes.c_int,
                              ctypes.POINTER(ctypes.c_int), ctypes.POINTER(ctypes.c_int),
                              ctypes.POINTER(ctypes.c_int)]),
    "hist_timing": (_st, [_H, ctypes.c_int]),
    "hist_timing_read": (_st, [_H, ctypes.POINTER(ctypes.c_double), ctypes.POINTER(ctypes.c_double),
                               ctypes.POINTER(ctypes.c_int64)]),
    "hist_batch_create": (_st, [ctypes.c_int, ctypes.POINTER(_H), ctypes.POINTER(HistFillDesc),
                                ctypes.POINTER(_H), _P]),
    "hist_batch_launch": (_st, [_H, _P]),
    "hist_batch_launch_eager": (_st, [_H, _P]),
    "hist_batch_destroy": (_st, [_H]),
    "hist_multi_create": (_st, [ctypes.c_int, ctypes.POINTER(_H), ctypes.POINTER(HistDefine),
                                ctypes.c_int, ctypes.c_int, ctypes.POINTER(_H)]),
    "hist_multi_fill": (_st, [_H, ctypes.POINTER(_P), ctypes.c_int64, _P]),
    "hist_multi_info": (_st, [_H, ctypes.c_int, ctypes.POINTER(ctypes.c_int),
                              ctypes.POINTER(ctypes.c_int), ctypes.POINTER(ctypes.c_int)]),
    "hist_multi_destroy": (_st, [_H]),
    "hist_probe": (_st, [ctypes.c_int, _P, ctypes.c_int64, ctypes.c_int, _P,
                         ctypes.POINTER(ctypes.c_double), ctypes.POINTER(ctypes.c_double)]),
    "hist_nbins_total": (ctypes.c_int64, [_H]),
    "hist_nstats": (ctypes.c_int, [_H]),
    "hist_strerror": (ctypes.c_char_p, [ctypes.c_int]),
    "hist_last_error": (ctypes.c_char_p, []),
    "hist_version": (ctypes.c_char_p, []),
}


def load():
    """The loaded ``libhist.so`` (built first if it is missing)."""
    global _lib
    with _lock:
        if _lib is None:
            if not os.path.exists(LIB_PATH):
                from . import build as _build
                _build.build()
            lib = ctypes.CDLL(LIB_PATH)
            for name, (res, args) in PROTOTYPES.items():
                fn = getattr(lib, name)
                fn.restype = res
                fn.argtypes = args
            _lib = lib
    return _lib


class HistError(RuntimeError):
    def __init__(self, status: int, where: str):
        lib = load()
        msg = lib.hist_last_error().decode(errors="replace")
        super().__init__("%s failed: %s (%s)" % (where, lib.hist_strerror(status).decode(), msg))
        self.status = status


def check(status: int, where: str) -> None:
    if status != HIST_OK:
        raise HistError(status, where)
