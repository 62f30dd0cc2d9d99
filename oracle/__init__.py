"""Plain CPU oracle for histogram filling -- TEST INFRASTRUCTURE ONLY.

Only ``tests/``, ``__graft_entry__.smoke()`` and the CPU-baseline leg of
``bench.py`` may import this package.  The GPU library never imports, links or
calls it, and it imports nothing from the GPU library.

The arithmetic lives in ``hist_oracle.c`` (plain sequential C, binary64,
``-ffp-contract=off``); this module builds it with gcc when no build is
present and exposes it through ctypes.  Each function follows arXiv:2401.13310
Sec. 3.1 (find bin, increment, statistics), Sec. 3.2 (statistics as
transform-reduce sums) and Sec. 3.3 (sums accumulate across bulks); the
readings of the paper's gaps are documented at the top of ``hist_oracle.c``.

Parity status per function (what pins each one, see ``tests/test_oracle_*``):
  bin_uniform      -- dyadic exact cases, midpoints, monotonicity, brute force
  bin_variable     -- brute-force count, numpy.searchsorted(side='right')
  global_bin       -- closed-form round trip over every bin of small axes
  Oracle.fill/read -- math.fsum of per-event terms, invariants, closed forms,
                      accumulation A+B == A||B
"""
from __future__ import annotations

import ctypes
import os
import subprocess
import threading

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "hist_oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")
_lock = threading.Lock()
_lib = None

MAX_DIMS = 3


def build(force: bool = False) -> str:
    """Compile ``liboracle.so`` with gcc (plain -O2, no FP contraction)."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp%d" % os.getpid()
        cmd = ["gcc", "-O2", "-std=c99", "-ffp-contract=off", "-fno-fast-math",
               "-fPIC", "-shared", "-o", tmp, _SRC, "-lm"]
        subprocess.run(cmd, check=True)
        os.replace(tmp, _LIB)
    return _LIB


class _Axis(ctypes.Structure):
    _fields_ = [("nbins", ctypes.c_int32), ("xmin", ctypes.c_double),
                ("xmax", ctypes.c_double), ("edges", ctypes.POINTER(ctypes.c_double))]


def _bind(lib):
    dp = ctypes.POINTER(ctypes.c_double)
    lib.oracle_bin_uniform.restype = ctypes.c_int32
    lib.oracle_bin_uniform.argtypes = [ctypes.c_double, ctypes.c_int32,
                                       ctypes.c_double, ctypes.c_double]
    lib.oracle_bin_variable.restype = ctypes.c_int32
    lib.oracle_bin_variable.argtypes = [ctypes.c_double, ctypes.c_int32, dp]
    lib.oracle_bin_variable_count.restype = ctypes.c_int32
    lib.oracle_bin_variable_count.argtypes = [ctypes.c_double, ctypes.c_int32, dp]
    lib.oracle_global_bin.restype = ctypes.c_int64
    lib.oracle_global_bin.argtypes = [ctypes.c_int, ctypes.POINTER(_Axis),
                                      ctypes.POINTER(ctypes.c_int32)]
    lib.oracle_findbin.restype = None
    lib.oracle_findbin.argtypes = [ctypes.c_int, ctypes.POINTER(_Axis),
                                   ctypes.POINTER(dp), ctypes.c_int64,
                                   ctypes.POINTER(ctypes.c_int32)]
    lib.oracle_nstats.restype = ctypes.c_int
    lib.oracle_nstats.argtypes = [ctypes.c_int]
    lib.oracle_hist_create.restype = ctypes.c_void_p
    lib.oracle_hist_create.argtypes = [ctypes.c_int, ctypes.POINTER(_Axis)]
    lib.oracle_hist_destroy.restype = None
    lib.oracle_hist_destroy.argtypes = [ctypes.c_void_p]
    lib.oracle_hist_nbins_total.restype = ctypes.c_int64
    lib.oracle_hist_nbins_total.argtypes = [ctypes.c_void_p]
    lib.oracle_hist_fill.restype = None
    lib.oracle_hist_fill.argtypes = [ctypes.c_void_p, ctypes.POINTER(dp), dp,
                                     ctypes.c_int64]
    lib.oracle_hist_read.restype = None
    lib.oracle_hist_read.argtypes = [ctypes.c_void_p, dp, dp, dp,
                                     ctypes.POINTER(ctypes.c_int64)]
    lib.oracle_stats_abs.restype = None
    lib.oracle_stats_abs.argtypes = [ctypes.c_int, ctypes.POINTER(_Axis),
                                     ctypes.POINTER(dp), dp, ctypes.c_int64, dp]
    return lib


def _load():
    global _lib
    with _lock:
        if _lib is None:
            _lib = _bind(ctypes.CDLL(build()))
    return _lib


_override = threading.local()


def _active():
    """The library in use: a test may swap in another build of the same
    source (see ``use_library``); everything else uses ``liboracle.so``."""
    lib = getattr(_override, "lib", None)
    return lib if lib is not None else _load()


class use_library:
    """Context manager that routes this module's calls to the shared library
    at ``path`` (another build of ``hist_oracle.c``) on the current thread."""

    def __init__(self, path: str):
        self._lib = _bind(ctypes.CDLL(path))

    def __enter__(self):
        self._prev = getattr(_override, "lib", None)
        _override.lib = self._lib
        return self

    def __exit__(self, *exc):
        _override.lib = self._prev
        return False


def _dptr(a: np.ndarray):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def _f64(a) -> np.ndarray:
    """Contiguous binary64 copy-or-view; float32 widens exactly."""
    return np.ascontiguousarray(np.asarray(a), dtype=np.float64)


class _Axes:
    """Keeps the ctypes axis array and the edge buffers it points to alive."""

    def __init__(self, axes):
        if not 1 <= len(axes) <= MAX_DIMS:
            raise ValueError("dims must be 1..3")
        self.dims = len(axes)
        self.arr = (_Axis * self.dims)()
        self._keep = []
        self.nbins = []
        for i, ax in enumerate(axes):
            nb = int(ax["nbins"])
            self.nbins.append(nb)
            self.arr[i].nbins = nb
            if ax.get("edges") is not None:
                e = _f64(ax["edges"])
                if e.shape != (nb + 1,):
                    raise ValueError("edges must hold nbins+1 values")
                self._keep.append(e)
                self.arr[i].edges = _dptr(e)
                self.arr[i].xmin = float(e[0])
                self.arr[i].xmax = float(e[-1])
            else:
                self.arr[i].xmin = float(ax["xmin"])
                self.arr[i].xmax = float(ax["xmax"])
                self.arr[i].edges = None


def _coord_ptrs(coords, dims):
    cols = [_f64(c) for c in coords]
    if len(cols) != dims:
        raise ValueError("need one coordinate column per axis")
    n = cols[0].shape[0]
    for c in cols:
        if c.shape != (n,):
            raise ValueError("coordinate columns must be 1-D and of equal length")
    arr = (ctypes.POINTER(ctypes.c_double) * max(dims, 1))()
    for i, c in enumerate(cols):
        arr[i] = _dptr(c)
    return cols, arr, n


def nstats(dims: int) -> int:
    return _active().oracle_nstats(dims)


def bin_uniform(x: float, nbins: int, xmin: float, xmax: float) -> int:
    return _active().oracle_bin_uniform(float(x), int(nbins), float(xmin), float(xmax))


def bin_variable(x: float, edges) -> int:
    e = _f64(edges)
    return _active().oracle_bin_variable(float(x), e.shape[0] - 1, _dptr(e))


def bin_variable_count(x: float, edges) -> int:
    e = _f64(edges)
    return _active().oracle_bin_variable_count(float(x), e.shape[0] - 1, _dptr(e))


def global_bin(axes, bins) -> int:
    ax = _Axes(axes)
    b = (ctypes.c_int32 * MAX_DIMS)(*([int(v) for v in bins] + [0] * (MAX_DIMS - len(bins))))
    return _active().oracle_global_bin(ax.dims, ax.arr, b)


def findbin(axes, coords) -> np.ndarray:
    """Global bin (int32) of every event."""
    ax = _Axes(axes)
    cols, arr, n = _coord_ptrs(coords, ax.dims)
    out = np.empty(n, dtype=np.int32)
    _active().oracle_findbin(ax.dims, ax.arr, arr, n,
                           out.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)))
    return out


def stats_abs(axes, coords, weights=None) -> np.ndarray:
    """Sum of |per-event term| of every statistic (tolerance scale)."""
    ax = _Axes(axes)
    cols, arr, n = _coord_ptrs(coords, ax.dims)
    w = None if weights is None else _f64(weights)
    out = np.zeros(nstats(ax.dims), dtype=np.float64)
    _active().oracle_stats_abs(ax.dims, ax.arr, arr, None if w is None else _dptr(w), n,
                             _dptr(out))
    return out


class Oracle:
    """Sequential histogram: create, fill (accumulating), read.

    ``axes`` is a list of dicts: ``{"nbins": n, "xmin": a, "xmax": b}`` for a
    fixed-width axis or ``{"nbins": n, "edges": array}`` for a variable one.
    """

    def __init__(self, axes):
        self._axes = _Axes(axes)
        self.dims = self._axes.dims
        self.nbins = list(self._axes.nbins)
        self._lib = _active()
        h = self._lib.oracle_hist_create(self.dims, self._axes.arr)
        if not h:
            raise ValueError("oracle_hist_create rejected the axes")
        self._h = ctypes.c_void_p(h)
        self.nbins_total = self._lib.oracle_hist_nbins_total(self._h)
        self.nstats = nstats(self.dims)

    def __del__(self):
        h = getattr(self, "_h", None)
        if h is not None:
            self._lib.oracle_hist_destroy(h)
            self._h = None

    def fill(self, coords, weights=None) -> None:
        cols, arr, n = _coord_ptrs(coords, self.dims)
        w = None
        if weights is not None:
            w = _f64(weights)
            if w.shape != (n,):
                raise ValueError("weights must match the coordinate length")
        self._lib.oracle_hist_fill(self._h, arr, None if w is None else _dptr(w), n)

    def read(self):
        """Returns (sumw, sumw2, stats, entries)."""
        T = self.nbins_total
        sumw = np.empty(T, dtype=np.float64)
        sumw2 = np.empty(T, dtype=np.float64)
        stats = np.empty(self.nstats, dtype=np.float64)
        entries = ctypes.c_int64(0)
        self._lib.oracle_hist_read(self._h, _dptr(sumw), _dptr(sumw2), _dptr(stats),
                                 ctypes.byref(entries))
        return sumw, sumw2, stats, int(entries.value)
