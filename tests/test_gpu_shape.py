"""GPU parity of the launch-shape variants (events per thread, statistics
fused or in separate reduction kernels) and of the autotuner's refinement:
every shape must give the oracle's counts bit for bit and its statistics
within the tolerance."""
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


def _workloads():
    rng = np.random.default_rng(61)
    n = 1_000_003
    x = rng.normal(0, 1.2, n)
    w = rng.uniform(0.5, 1.5, n)
    return {
        "fixed_unit": ([{"nbins": 100, "xmin": -5.0, "xmax": 5.0}], [x], None, False),
        "fixed_weighted": ([{"nbins": 100, "xmin": -5.0, "xmax": 5.0}], [x], w, False),
        "learned_u16": None,   # built from the variable-bin recipe below
        "staged_edges": ([{"nbins": 999, "edges": np.sort(rng.uniform(-4, 4, 1000))}], [x], None,
                         False),
    }


def _check(hg, axes, coords, w, learned, unroll, stats_ept):
    h = hg.Hist(axes)
    if learned:
        h.train_index(0)
    h.set_shape(unroll, stats_ept)
    shape = h.plan_shape(len(coords[0]), weighted=w is not None)
    print("shape unroll=%d stats_ept=%d -> %r" % (unroll, stats_ept, shape), flush=True)
    h.fill([dev(c) for c in coords], None if w is None else dev(w))
    sumw, sumw2, entries = h.read()
    o = oracle.Oracle(axes)
    o.fill(coords, w)
    osw, osw2, ost, oent = o.read()
    assert entries == oent
    if w is None:
        assert_bins_equal(sumw, osw, "counts")
    else:
        assert_sums_close(sumw, osw, what="sumw")
        assert_sums_close(sumw2, osw2, what="sumw2")
    assert_stats_close(h.stats(), ost, oracle.stats_abs(axes, coords, w))
    return shape


@pytest.mark.parametrize("kind", ["fixed_unit", "fixed_weighted", "learned_u16", "staged_edges"])
@pytest.mark.parametrize("unroll", [1, 2, 4, 8])
def test_events_per_thread_variants(hg, kind, unroll):
    if kind == "learned_u16":
        wl = synth.variable_1d(2_000_003)
        axes, coords, w, learned = wl["axes"], wl["coords"], None, True
    else:
        axes, coords, w, learned = _workloads()[kind]
    shape = _check(hg, axes, coords, w, learned, unroll, 0)
    assert shape["unroll"] == unroll and shape["stats_ept"] == 0


@pytest.mark.parametrize("kind", ["fixed_unit", "fixed_weighted", "learned_u16"])
@pytest.mark.parametrize("ept", [1, 4, 16])
def test_separate_statistics_kernels(hg, kind, ept):
    if kind == "learned_u16":
        wl = synth.variable_1d(1_500_001)
        axes, coords, w, learned = wl["axes"], wl["coords"], None, True
    else:
        axes, coords, w, learned = _workloads()[kind]
    shape = _check(hg, axes, coords, w, learned, 0, ept)
    assert shape["stats_ept"] == ept


def test_unsupported_shape_keeps_the_heuristic(hg):
    rng = np.random.default_rng(62)
    axes = [{"nbins": 40, "xmin": -3.0, "xmax": 3.0}, {"nbins": 30, "xmin": -3.0, "xmax": 3.0}]
    coords = [rng.normal(0, 1, 300_001), rng.normal(0, 1, 300_001)]
    h = hg.Hist(axes)
    h.set_shape(2, 4)
    assert h.plan_shape(300_001)["stats_ept"] == 0
    _check(hg, axes, coords, None, False, 2, 4)
    with pytest.raises(hg.HistError):
        h.set_shape(3, 0)
    with pytest.raises(hg.HistError):
        h.set_shape(0, 2)


def test_tuner_refines_copies_and_unroll(hg):
    """The tuner's refinement picks some copies and events per thread; the
    tuned fill still matches the oracle, and a batch member of the tuned
    shape follows the tuned strategy."""
    import torch
    wl = synth.plain_1d(2_000_000)
    axes, coords, w = wl["axes"], wl["coords"], wl["weights"]
    h = hg.Hist(axes)
    tc = [dev(c) for c in coords]
    tw = dev(w)
    h.tune(tc, tw)
    info = h.plan_info(len(coords[0]), weighted=True)
    shape = h.plan_shape(len(coords[0]), weighted=True)
    print("tuned plan %r shape %r" % (info, shape), flush=True)
    assert 1 <= info["copies"] <= 64 and shape["unroll"] in (1, 2, 4, 8)
    h.fill(tc, tw)
    sumw, sumw2, entries = h.read()
    o = oracle.Oracle(axes)
    o.fill(coords, w)
    osw, osw2, ost, oent = o.read()
    assert entries == oent
    assert_sums_close(sumw, osw, what="sumw")
    assert_stats_close(h.stats(), ost, oracle.stats_abs(axes, coords, w))
    # a batch of members of the tuned shape
    hs = [hg.Hist(axes) for _ in range(3)]
    b = hg.Batch(hs, [tc] * 3, [tw] * 3)
    b.launch()
    torch.cuda.synchronize()
    for m in hs:
        s, _, e = m.read()
        assert e == oent
        assert_sums_close(s, osw, what="batch member sumw")
