"""MI355X (gfx950) histogram filling: find bin, weighted increment and
statistics sums of arXiv:2401.13310 Sec. 3.1, in hand-written HIP kernels
behind the C ABI of ``include/hist.h``.

This module is a thin binding with the C function names (``hist_create``,
``hist_fill``, ...) plus a small ``Hist`` convenience class.  PyTorch supplies
device memory and streams; every step of the fill runs in ``libhist.so``.
"""
from __future__ import annotations

import ctypes

import numpy as np

from ._lib import (ACC_NAMES, HIST_F32, HIST_F64, HIST_F_ACC_F32C, HIST_F_LEARNED, HIST_F_NO_ALLOC,
                   HIST_HOST_PINNED, HIST_SEARCH_BINARY, HIST_SEARCH_LEARNED, HIST_STRAT_AUTO, HIST_STRAT_GLOBAL,
                   HIST_STRAT_LDS, HIST_STRAT_PART, HIST_STRAT_TILED, STRAT_NAMES, HistAxis, HistError,
                   HistDefine, HistExpr, HistFillDesc, HistOp, check, load)
from .expr import OPS, parse

__all__ = [
    "Hist", "HistError", "hist_create", "hist_destroy", "hist_fill", "hist_fill_static", "hist_static_scratch_bytes", "hist_fill_host", "hist_probe", "hist_findbin",
    "hist_reserve",
    "hist_stats", "hist_read", "hist_reset", "hist_train_index", "hist_set_search",
    "hist_index_info", "hist_set_strategy", "hist_set_window", "hist_tune", "hist_plan_info",
    "hist_timing", "hist_timing_read", "hist_set_threads", "hist_set_shape", "hist_plan_shape",
    "hist_batch_create", "hist_batch_launch", "hist_batch_launch_eager", "hist_batch_destroy",
    "hist_multi_create", "hist_multi_fill", "hist_multi_info", "hist_multi_destroy", "Multi",
    "OPS", "parse",
    "HIST_F64", "HIST_F32", "HIST_F_ACC_F32C", "HIST_F_LEARNED", "HIST_F_NO_ALLOC", "HIST_HOST_PINNED",
    "HIST_STRAT_AUTO",
    "HIST_STRAT_LDS", "HIST_STRAT_GLOBAL", "HIST_STRAT_TILED", "HIST_STRAT_PART", "HIST_SEARCH_BINARY",
    "HIST_SEARCH_LEARNED", "Batch",
]


def _stream_ptr(stream) -> int:
    import torch
    if stream is None:
        stream = torch.cuda.current_stream()
    return int(stream.cuda_stream) if hasattr(stream, "cuda_stream") else int(stream)


def _axes_struct(axes):
    arr = (HistAxis * len(axes))()
    keep = []
    for i, ax in enumerate(axes):
        arr[i].nbins = int(ax["nbins"])
        if ax.get("edges") is not None:
            e = np.ascontiguousarray(np.asarray(ax["edges"], dtype=np.float64))
            keep.append(e)
            arr[i].edges = e.ctypes.data_as(ctypes.POINTER(ctypes.c_double))
            arr[i].xmin = 0.0
            arr[i].xmax = 0.0
        else:
            arr[i].xmin = float(ax["xmin"])
            arr[i].xmax = float(ax["xmax"])
            arr[i].edges = None
    return arr, keep


def _col_ptrs(cols):
    arr = (ctypes.c_void_p * 3)()
    for i, c in enumerate(cols):
        arr[i] = c
    return arr


# ---- the C functions, same names ------------------------------------------

def hist_create(axes, flags: int = 0) -> ctypes.c_void_p:
    arr, _keep = _axes_struct(axes)
    h = ctypes.c_void_p()
    check(load().hist_create(len(axes), arr, flags, ctypes.byref(h)), "hist_create")
    return h


def hist_destroy(h) -> None:
    check(load().hist_destroy(h), "hist_destroy")


def hist_fill(h, coord_ptrs, weight_ptr, n: int, dtype: int, stream: int) -> None:
    check(load().hist_fill(h, _col_ptrs(coord_ptrs), weight_ptr, n, dtype, stream), "hist_fill")


def hist_fill_static(h, coord_ptrs, weight_ptr, n: int, dtype: int, stream: int) -> None:
    check(load().hist_fill_static(h, _col_ptrs(coord_ptrs), weight_ptr, n, dtype, stream),
          "hist_fill_static")


def hist_probe(kind: int, buf_ptr, nbytes: int, reps: int, stream: int) -> dict:
    rate, ms = ctypes.c_double(), ctypes.c_double()
    check(load().hist_probe(kind, buf_ptr, nbytes, reps, stream, ctypes.byref(rate), ctypes.byref(ms)),
          "hist_probe")
    return {"rate": rate.value, "ms": ms.value}


def hist_static_scratch_bytes() -> int:
    return int(load().hist_static_scratch_bytes())


def hist_fill_host(h, coord_ptrs, weight_ptr, n: int, dtype: int, chunk: int, flags: int,
                   stream: int) -> None:
    check(load().hist_fill_host(h, _col_ptrs(coord_ptrs), weight_ptr, n, dtype, chunk, flags, stream),
          "hist_fill_host")


def hist_findbin(h, coord_ptrs, n: int, dtype: int, bins_ptr: int, stream: int) -> None:
    check(load().hist_findbin(h, _col_ptrs(coord_ptrs), n, dtype, bins_ptr, stream),
          "hist_findbin")


def hist_reserve(h, n_max: int, dtype: int, weighted: bool, stream: int) -> None:
    check(load().hist_reserve(h, n_max, dtype, int(bool(weighted)), stream), "hist_reserve")


def hist_stats(h, stream: int) -> np.ndarray:
    lib = load()
    out = np.zeros(11, dtype=np.float64)
    cnt = ctypes.c_int(0)
    check(lib.hist_stats(h, out.ctypes.data_as(ctypes.POINTER(ctypes.c_double)), 11,
                         ctypes.byref(cnt), stream), "hist_stats")
    return out[:cnt.value].copy()


def hist_read(h, stream: int):
    lib = load()
    T = lib.hist_nbins_total(h)
    sumw = np.empty(T, dtype=np.float64)
    sumw2 = np.empty(T, dtype=np.float64)
    entries = ctypes.c_int64(0)
    check(lib.hist_read(h, sumw.ctypes.data_as(ctypes.POINTER(ctypes.c_double)),
                        sumw2.ctypes.data_as(ctypes.POINTER(ctypes.c_double)),
                        ctypes.byref(entries), stream), "hist_read")
    return sumw, sumw2, int(entries.value)


def hist_reset(h, stream: int) -> None:
    check(load().hist_reset(h, stream), "hist_reset")


def hist_train_index(h, axis: int, stream: int) -> None:
    check(load().hist_train_index(h, axis, stream), "hist_train_index")


def hist_set_search(h, axis: int, mode: int) -> None:
    check(load().hist_set_search(h, axis, mode), "hist_set_search")


def hist_index_info(h, axis: int) -> dict:
    seg, feat = ctypes.c_int(), ctypes.c_int()
    mean_w, max_w = ctypes.c_double(), ctypes.c_double()
    check(load().hist_index_info(h, axis, ctypes.byref(seg), ctypes.byref(feat),
                                 ctypes.byref(mean_w), ctypes.byref(max_w)), "hist_index_info")
    return {"segments": seg.value, "feature": ["key", "linear"][feat.value],
            "mean_window": mean_w.value, "max_window": max_w.value}


def hist_set_strategy(h, strategy: int, blocks: int = 0, subhists: int = 0) -> None:
    check(load().hist_set_strategy(h, strategy, blocks, subhists), "hist_set_strategy")


def hist_set_window(h, window_lo: int = -1, merge: int = -1) -> None:
    check(load().hist_set_window(h, window_lo, merge), "hist_set_window")


def hist_tune(h, coord_ptrs, weight_ptr, n: int, dtype: int, stream: int) -> None:
    check(load().hist_tune(h, _col_ptrs(coord_ptrs), weight_ptr, n, dtype, stream), "hist_tune")


def hist_plan_info(h, n: int, dtype: int, weighted: bool) -> dict:
    s, b, c, acc = ctypes.c_int(), ctypes.c_int(), ctypes.c_int(), ctypes.c_int()
    lo, ln = ctypes.c_int64(), ctypes.c_int64()
    check(load().hist_plan_info(h, n, dtype, int(bool(weighted)), ctypes.byref(s),
                                ctypes.byref(b), ctypes.byref(c), ctypes.byref(lo),
                                ctypes.byref(ln), ctypes.byref(acc)), "hist_plan_info")
    return {"strategy": STRAT_NAMES[s.value], "blocks": b.value, "copies": c.value,
            "window_lo": lo.value, "window_len": ln.value, "accumulator": ACC_NAMES[acc.value]}


def hist_set_threads(h, threads: int) -> None:
    check(load().hist_set_threads(h, threads), "hist_set_threads")


def hist_set_shape(h, unroll: int = 0, stats_ept: int = 0) -> None:
    check(load().hist_set_shape(h, unroll, stats_ept), "hist_set_shape")


def hist_plan_shape(h, n: int, dtype: int, weighted: bool) -> dict:
    u, e, t = ctypes.c_int(), ctypes.c_int(), ctypes.c_int()
    check(load().hist_plan_shape(h, n, dtype, int(bool(weighted)), ctypes.byref(u), ctypes.byref(e),
                                 ctypes.byref(t)), "hist_plan_shape")
    return {"unroll": u.value, "stats_ept": e.value, "threads": t.value}


def hist_timing(h, enable: bool) -> None:
    check(load().hist_timing(h, int(bool(enable))), "hist_timing")


def hist_timing_read(h):
    f, m, n = ctypes.c_double(), ctypes.c_double(), ctypes.c_int64()
    check(load().hist_timing_read(h, ctypes.byref(f), ctypes.byref(m), ctypes.byref(n)),
          "hist_timing_read")
    return {"fill_ms": f.value, "merge_ms": m.value, "launches": n.value}


def hist_batch_create(handles, descs, stream: int):
    k = len(handles)
    harr = (ctypes.c_void_p * k)(*[h.value if isinstance(h, ctypes.c_void_p) else h
                                  for h in handles])
    darr = (HistFillDesc * k)(*descs)
    b = ctypes.c_void_p()
    check(load().hist_batch_create(k, harr, darr, ctypes.byref(b), stream), "hist_batch_create")
    return b


def hist_batch_launch(b, stream: int) -> None:
    check(load().hist_batch_launch(b, stream), "hist_batch_launch")


def hist_batch_launch_eager(b, stream: int) -> None:
    check(load().hist_batch_launch_eager(b, stream), "hist_batch_launch_eager")


def hist_batch_destroy(b) -> None:
    check(load().hist_batch_destroy(b), "hist_batch_destroy")


def _expr_struct(ops, keep):
    e = HistExpr()
    if not ops:
        e.ops = None
        e.nops = 0
        return e
    arr = (HistOp * len(ops))()
    for i, (op, col, value) in enumerate(ops):
        arr[i].op = int(op)
        arr[i].col = int(col)
        arr[i].value = float(value)
    keep.append(arr)
    e.ops = ctypes.cast(arr, ctypes.POINTER(HistOp))
    e.nops = len(ops)
    return e


def _define_structs(defs, keep):
    arr = (HistDefine * len(defs))()
    for i, d in enumerate(defs):
        d = d or {}
        arr[i].filter = _expr_struct(d.get("filter"), keep)
        coords = d.get("coords") or []
        for a in range(3):
            arr[i].coord[a] = _expr_struct(coords[a] if a < len(coords) else None, keep)
        arr[i].weight = _expr_struct(d.get("weight"), keep)
    return arr


def hist_multi_create(handles, defs, ncols: int, dtype: int):
    """defs: None, or one dict per handle with optional "filter", "coords"
    (list per axis) and "weight", each a list of (op, col, value)."""
    k = len(handles)
    harr = (ctypes.c_void_p * k)(*[h.value if isinstance(h, ctypes.c_void_p) else h
                                  for h in handles])
    keep = []
    darr = None if defs is None else _define_structs(defs, keep)
    m = ctypes.c_void_p()
    check(load().hist_multi_create(k, harr, darr, ncols, dtype, ctypes.byref(m)),
          "hist_multi_create")
    return m


def hist_multi_fill(m, col_ptrs, n: int, stream: int) -> None:
    arr = (ctypes.c_void_p * max(1, len(col_ptrs)))(*col_ptrs)
    check(load().hist_multi_fill(m, arr, n, stream), "hist_multi_fill")


def hist_multi_info(m, member: int) -> dict:
    in_lds, copies, lds = ctypes.c_int(), ctypes.c_int(), ctypes.c_int()
    check(load().hist_multi_info(m, member, ctypes.byref(in_lds), ctypes.byref(copies),
                                 ctypes.byref(lds)), "hist_multi_info")
    return {"in_lds": bool(in_lds.value), "copies": copies.value, "lds_bytes": lds.value}


def hist_multi_destroy(m) -> None:
    check(load().hist_multi_destroy(m), "hist_multi_destroy")


# ---- convenience wrapper over torch tensors ---------------------------------

def _check_cols(coords, weights):
    import torch
    cols = list(coords)
    if not cols:
        raise ValueError("need at least one coordinate column")
    dt = cols[0].dtype
    if dt not in (torch.float64, torch.float32):
        raise TypeError("coordinates must be float64 or float32")
    n = cols[0].numel()
    for c in cols + ([weights] if weights is not None else []):
        if not c.is_cuda:
            raise ValueError("tensors must live on the GPU")
        if c.dtype != dt:
            raise TypeError("coordinates and weights must share one dtype")
        if not c.is_contiguous() or c.dim() != 1 or c.numel() != n:
            raise ValueError("columns must be contiguous 1-D tensors of equal length")
    return cols, n, (HIST_F32 if dt == torch.float32 else HIST_F64)


class Hist:
    """A GPU histogram (owns its device state through the C handle)."""

    def __init__(self, axes, flags: int = 0):
        self.axes = [dict(a) for a in axes]
        self.dims = len(axes)
        self.flags = flags
        self._h = hist_create(axes, flags)
        self.nbins_total = load().hist_nbins_total(self._h)
        self.nstats = load().hist_nstats(self._h)

    @property
    def handle(self):
        return self._h

    def close(self):
        if getattr(self, "_h", None) is not None and self._h.value:
            hist_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def fill(self, coords, weights=None, stream=None):
        cols, n, dt = _check_cols(coords, weights)
        if len(cols) != self.dims:
            raise ValueError("need %d coordinate columns" % self.dims)
        hist_fill(self._h, [c.data_ptr() for c in cols],
                  None if weights is None else weights.data_ptr(), n, dt, _stream_ptr(stream))

    def fill_host(self, coords, weights=None, chunk: int = 0, pinned: bool = False, stream=None):
        """Fill from host columns (numpy arrays or CPU tensors, one dtype,
        contiguous); pinned=True for page-locked tensors (pin_memory)."""
        import torch
        cols = [torch.as_tensor(c) for c in coords]
        if len(cols) != self.dims:
            raise ValueError("need %d coordinate columns" % self.dims)
        w = None if weights is None else torch.as_tensor(weights)
        dt = cols[0].dtype
        if dt not in (torch.float64, torch.float32):
            raise TypeError("coordinates must be float64 or float32")
        n = cols[0].numel()
        for c in cols + ([w] if w is not None else []):
            if c.is_cuda:
                raise ValueError("fill_host takes host columns")
            if c.dtype != dt or not c.is_contiguous() or c.dim() != 1 or c.numel() != n:
                raise ValueError("columns must be contiguous 1-D arrays of one dtype and length")
            if pinned and not c.is_pinned():
                raise ValueError("pinned=True needs page-locked tensors")
        hist_fill_host(self._h, [c.data_ptr() for c in cols], None if w is None else w.data_ptr(), n,
                       HIST_F32 if dt == torch.float32 else HIST_F64, chunk,
                       HIST_HOST_PINNED if pinned else 0, _stream_ptr(stream))

    def reserve(self, n_max: int, dtype: int = HIST_F64, weighted: bool = False, stream=None):
        hist_reserve(self._h, n_max, dtype, weighted, _stream_ptr(stream))

    def findbin(self, coords, stream=None):
        import torch
        cols, n, dt = _check_cols(coords, None)
        out = torch.empty(n, dtype=torch.int32, device=cols[0].device)
        hist_findbin(self._h, [c.data_ptr() for c in cols], n, dt, out.data_ptr(),
                     _stream_ptr(stream))
        return out

    def stats(self, stream=None) -> np.ndarray:
        return hist_stats(self._h, _stream_ptr(stream))

    def read(self, stream=None):
        """(sumw, sumw2, entries) as host arrays."""
        return hist_read(self._h, _stream_ptr(stream))

    def reset(self, stream=None):
        hist_reset(self._h, _stream_ptr(stream))

    def train_index(self, axis: int = 0, stream=None):
        hist_train_index(self._h, axis, _stream_ptr(stream))

    def set_search(self, axis: int, learned: bool):
        hist_set_search(self._h, axis, HIST_SEARCH_LEARNED if learned else HIST_SEARCH_BINARY)

    def index_info(self, axis: int = 0) -> dict:
        return hist_index_info(self._h, axis)

    def set_strategy(self, strategy: int, blocks: int = 0, subhists: int = 0):
        hist_set_strategy(self._h, strategy, blocks, subhists)

    def set_window(self, window_lo: int = -1, merge: int = -1):
        hist_set_window(self._h, window_lo, merge)

    def tune(self, coords, weights=None, stream=None):
        cols, n, dt = _check_cols(coords, weights)
        hist_tune(self._h, [c.data_ptr() for c in cols],
                  None if weights is None else weights.data_ptr(), n, dt, _stream_ptr(stream))

    def plan_info(self, n: int, dtype: int = HIST_F64, weighted: bool = False) -> dict:
        return hist_plan_info(self._h, n, dtype, weighted)

    def set_threads(self, threads: int):
        hist_set_threads(self._h, threads)

    def set_shape(self, unroll: int = 0, stats_ept: int = 0):
        hist_set_shape(self._h, unroll, stats_ept)

    def plan_shape(self, n: int, dtype: int = HIST_F64, weighted: bool = False) -> dict:
        return hist_plan_shape(self._h, n, dtype, weighted)

    def timing(self, enable: bool = True):
        hist_timing(self._h, enable)

    def timing_read(self) -> dict:
        return hist_timing_read(self._h)


class Multi:
    """One pass over shared columns filling several histograms, each with an
    optional filter, computed coordinates and weight (hist_define).  defs
    entries may give programs as infix strings over `columns` names."""

    def __init__(self, hists, defs=None, columns=("c0",), dtype: int = HIST_F64):
        self.columns = list(columns)
        self.hists = list(hists)
        prog = None
        if defs is not None:
            prog = []
            for d in defs:
                d = dict(d or {})
                out = {}
                for key in ("filter", "weight"):
                    if d.get(key) is not None:
                        out[key] = self._ops(d[key])
                if d.get("coords") is not None:
                    out["coords"] = [None if c is None else self._ops(c) for c in d["coords"]]
                prog.append(out)
        self.dtype = dtype
        self._m = hist_multi_create([h.handle for h in self.hists], prog, len(self.columns), dtype)

    def _ops(self, e):
        return parse(e, self.columns) if isinstance(e, str) else list(e)

    def fill(self, cols, stream=None):
        cols = list(cols)
        if len(cols) != len(self.columns):
            raise ValueError("need %d columns" % len(self.columns))
        import torch
        n = cols[0].numel()
        want = torch.float32 if self.dtype == HIST_F32 else torch.float64
        for c in cols:
            if not c.is_cuda or not c.is_contiguous() or c.dim() != 1 or c.numel() != n:
                raise ValueError("columns must be contiguous 1-D GPU tensors of equal length")
            if c.dtype != want:
                raise TypeError("the plan was made for %s columns" % want)
        hist_multi_fill(self._m, [c.data_ptr() for c in cols], n, _stream_ptr(stream))

    def info(self, member: int) -> dict:
        return hist_multi_info(self._m, member)

    def close(self):
        if getattr(self, "_m", None) is not None and self._m.value:
            hist_multi_destroy(self._m)
            self._m = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Batch:
    """Many histograms filled by one persistent launch replayed from a HIP graph."""

    def __init__(self, hists, coords_list, weights_list, stream=None):
        descs = []
        self.hists = list(hists)   # every launch writes their sums: they live as long as the batch
        self._keep = []
        for h, coords, w in zip(hists, coords_list, weights_list):
            cols, n, dt = _check_cols(coords, w)
            d = HistFillDesc()
            for i, c in enumerate(cols):
                d.coords[i] = c.data_ptr()
            d.weights = None if w is None else w.data_ptr()
            d.n = n
            d.dtype = dt
            descs.append(d)
            self._keep.append((cols, w))
        self._b = hist_batch_create([h.handle for h in hists], descs, _stream_ptr(stream))

    def launch(self, stream=None, graph: bool = True):
        if graph:
            hist_batch_launch(self._b, _stream_ptr(stream))
        else:
            hist_batch_launch_eager(self._b, _stream_ptr(stream))

    def close(self):
        if getattr(self, "_b", None) is not None and self._b.value:
            hist_batch_destroy(self._b)
            self._b = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
