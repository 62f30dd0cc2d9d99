"""The C-ABI library loads, exports every symbol include/hist.h declares, and
rejects bad arguments before touching a GPU (no compute calls here)."""
import ctypes
import os
import re

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_symbols():
    text = open(os.path.join(ROOT, "include", "hist.h")).read()
    return sorted(set(re.findall(r"HIST_API\s+[\w\s\*]*?\b(hist_\w+)\s*\(", text)))


@pytest.fixture(scope="module")
def lib():
    from paper_2401_13310_amd import _lib
    return _lib.load()


def test_header_declares_the_core_calls():
    names = declared_symbols()
    for core in ["hist_create", "hist_destroy", "hist_fill", "hist_stats", "hist_read",
                 "hist_reset", "hist_findbin", "hist_train_index", "hist_tune",
                 "hist_batch_create", "hist_batch_launch"]:
        assert core in names


def test_library_exports_every_declared_symbol(lib):
    for name in declared_symbols():
        assert hasattr(lib, name), name


def test_binding_prototypes_cover_the_header():
    from paper_2401_13310_amd import _lib
    assert set(declared_symbols()) == set(_lib.PROTOTYPES)


def test_strerror_and_version(lib):
    assert lib.hist_strerror(0) == b"ok"
    assert lib.hist_strerror(1) == b"invalid argument"
    assert lib.hist_version().startswith(b"histgpu")
    assert lib.hist_last_error() is not None


def _axis(nbins, lo=0.0, hi=1.0, edges=None):
    from paper_2401_13310_amd._lib import HistAxis
    a = HistAxis()
    a.nbins = nbins
    a.xmin, a.xmax = lo, hi
    keep = None
    if edges is not None:
        keep = np.ascontiguousarray(edges, dtype=np.float64)
        a.edges = keep.ctypes.data_as(ctypes.POINTER(ctypes.c_double))
    return a, keep


@pytest.mark.parametrize("case", ["dims0", "dims4", "nbins0", "lo_ge_hi", "nan_range",
                                  "edges_not_increasing", "edges_nan", "too_many_bins",
                                  "null_out", "bad_flags"])
def test_create_rejects_bad_arguments(lib, case):
    from paper_2401_13310_amd._lib import HIST_EINVAL, HistAxis
    dims, flags = 1, 0
    axes = (HistAxis * 3)()
    keep = []
    a, k = _axis(10)
    axes[0] = a
    if case == "dims0":
        dims = 0
    elif case == "dims4":
        dims = 4
    elif case == "nbins0":
        axes[0].nbins = 0
    elif case == "lo_ge_hi":
        axes[0].xmin, axes[0].xmax = 1.0, 1.0
    elif case == "nan_range":
        axes[0].xmin = float("nan")
    elif case == "edges_not_increasing":
        a, k = _axis(3, edges=[0.0, 1.0, 1.0, 2.0])
        axes[0] = a
        keep.append(k)
    elif case == "edges_nan":
        a, k = _axis(2, edges=[0.0, float("nan"), 2.0])
        axes[0] = a
        keep.append(k)
    elif case == "too_many_bins":
        dims = 3
        for i in range(3):
            axes[i].nbins = 2000
            axes[i].xmin, axes[i].xmax = 0.0, 1.0
    elif case == "bad_flags":
        flags = 1 << 7
    h = ctypes.c_void_p()
    out = None if case == "null_out" else ctypes.byref(h)
    st = lib.hist_create(dims, axes, flags, out)
    assert st == HIST_EINVAL
    assert not h.value
    assert len(lib.hist_last_error()) > 0


def test_calls_on_null_handle_are_einval(lib):
    from paper_2401_13310_amd._lib import HIST_EINVAL
    assert lib.hist_fill(None, None, None, 10, 0, None) == HIST_EINVAL
    assert lib.hist_findbin(None, None, 10, 0, None, None) == HIST_EINVAL
    assert lib.hist_stats(None, None, 0, None, None) == HIST_EINVAL
    assert lib.hist_read(None, None, None, None, None) == HIST_EINVAL
    assert lib.hist_reset(None, None) == HIST_EINVAL
    assert lib.hist_train_index(None, 0, None) == HIST_EINVAL
    assert lib.hist_tune(None, None, None, 1, 0, None) == HIST_EINVAL
    assert lib.hist_set_strategy(None, 0, 0, 0) == HIST_EINVAL
    assert lib.hist_destroy(None) == 0
    assert lib.hist_nbins_total(None) == -1
    assert lib.hist_nstats(None) == -1


def test_binding_has_every_c_name():
    import paper_2401_13310_amd as pkg
    for name in declared_symbols():
        if name in ("hist_nbins_total", "hist_nstats", "hist_strerror", "hist_last_error",
                    "hist_version"):
            continue
        assert hasattr(pkg, name), name
