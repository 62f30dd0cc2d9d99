"""hist_fill_static (the fill for callers that cannot allocate) against
hist_fill through the C ABI: two calls in a row on one handle, the second
with fewer events, for every scratch use (staged merge, tiled and partitioned
bin arrays) and for plans without scratch.  Counts must be identical and
weighted sums within 1e-12; the handle was created with HIST_F_NO_ALLOC and
never reserved, so the static fill cannot have used the handle's scratch."""
import ctypes

import numpy as np
import pytest

import oracle
import synth
from tests.gpu_helpers import assert_bins_equal, assert_stats_close, assert_sums_close, dev

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def hg():
    import torch
    assert torch.cuda.is_available(), "GPU tests need an MI355X"
    import paper_2401_13310_amd as pkg
    return pkg


def _ptrs(cols):
    arr = (ctypes.c_void_p * 3)()
    for i, c in enumerate(cols):
        arr[i] = c.data_ptr()
    return arr


def _run(hg, axes, coords, w, sizes, strategy=None, learned=False, blocks=0):
    import torch
    lib = hg._lib.load()
    stream = torch.cuda.current_stream().cuda_stream
    a = hg.Hist(axes, hg.HIST_F_NO_ALLOC)
    b = hg.Hist(axes)
    for h in (a, b):
        if learned:
            h.train_index(0)
        if strategy is not None:
            h.set_strategy(strategy, blocks, 0)
    tc = [dev(c) for c in coords]
    tw = None if w is None else dev(w)
    for n in sizes:
        cols = [c[:n] for c in tc]
        wp = None if tw is None else tw[:n].data_ptr()
        print("static fill n=%d strategy=%s" % (n, strategy), flush=True)
        st = lib.hist_fill_static(a.handle, _ptrs(cols), wp, n, hg.HIST_F64, stream)
        assert st == 0, lib.hist_last_error().decode()
        b.fill(cols, None if tw is None else tw[:n])
    sa, sa2, ea = a.read()
    sb, sb2, eb = b.read()
    assert ea == eb == sum(sizes)
    if w is None:
        assert_bins_equal(sa, sb, "counts")
    else:
        assert_sums_close(sa, sb, what="sumw")
        assert_sums_close(sa2, sb2, what="sumw2")
    oc = [np.concatenate([c[:n] for n in sizes]) for c in coords]
    ow = None if w is None else np.concatenate([w[:n] for n in sizes])
    assert_stats_close(a.stats(), b.stats(), oracle.stats_abs(axes, oc, ow))
    return a


def test_static_staged_merge(hg):
    """The benchmark's plan: a u16 LDS window merged through staging slots."""
    wl = synth.variable_1d(3_000_001)
    a = _run(hg, wl["axes"], wl["coords"], None, [3_000_001, 1_234_567], learned=True)
    assert a.plan_info(3_000_001)["strategy"] == "lds"


def test_static_partitioned_chunks(hg):
    """A 3D histogram larger than LDS: the partitioned passes run in chunks
    that fit the static region (more chunks than hist_fill takes)."""
    wl = synth.corr_3d(9_000_011)
    _run(hg, wl["axes"], wl["coords"], None, [9_000_011, 4_500_003],
         strategy=hg.HIST_STRAT_PART)


def test_static_partitioned_weighted(hg):
    rng = np.random.default_rng(91)
    axes = [{"nbins": 250_000, "xmin": -4.0, "xmax": 4.0}]
    n = 6_000_007
    x = rng.normal(0, 1.3, n)
    w = rng.lognormal(0.0, 1.0, n)
    _run(hg, axes, [x], w, [n, 2_000_001], strategy=hg.HIST_STRAT_PART)


def test_static_tiled(hg):
    rng = np.random.default_rng(92)
    axes = [{"nbins": 60_000, "xmin": -4.0, "xmax": 4.0}]
    n = 17_000_003
    x = rng.normal(0, 1.0, n)
    _run(hg, axes, [x], None, [n, 5_000_001], strategy=hg.HIST_STRAT_TILED)


def test_static_small_weighted_no_scratch(hg):
    wl = synth.plain_1d(1_000_000)
    _run(hg, wl["axes"], wl["coords"], wl["weights"], [1_000_000, 99_991])


def test_static_rejects_oversized_staging(hg):
    """Staging slots beyond the static region: HIST_ENOMEM, nothing filled."""
    import torch
    lib = hg._lib.load()
    wl = synth.variable_1d(8_400_000)
    h = hg.Hist(wl["axes"], hg.HIST_F_NO_ALLOC)
    # 4096 slots of one byte per bin of a window of more than 16384 bins
    h.set_strategy(hg.HIST_STRAT_LDS, 4096, 0)
    h.set_window(0, 1)
    x = dev(wl["coords"][0])
    st = lib.hist_fill_static(h.handle, _ptrs([x]), None, x.numel(), hg.HIST_F64,
                              torch.cuda.current_stream().cuda_stream)
    assert st == hg._lib.HIST_ENOMEM
    assert b"exceed" in lib.hist_last_error()
    assert h.read()[2] == 0
    assert lib.hist_static_scratch_bytes() == 64 << 20
