"""GPU parity of the learned one-axis kernel (one binary64 axis with a trained
index and more edges than LDS holds, unit weights, 16-bit window): the
benchmark workload, inputs that put nearly every event on or next to an edge
(so most intervals hold two bins and are decided by an edge read), a window
narrower than the histogram, axes whose range crosses zero (key feature of
signed values), evenly spaced edges (linear feature), and edges so unevenly
spread that some segment's interval holds three or more bins (the variant that
searches those)."""
import numpy as np
import pytest

import oracle
import synth
from tests.gpu_helpers import assert_bins_equal, assert_stats_close, dev

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def hg():
    import torch
    assert torch.cuda.is_available(), "GPU tests need an MI355X"
    import paper_2401_13310_amd as pkg
    return pkg


def _fill(hg, axes, x, window_lo=None, fills=1):
    h = hg.Hist(axes)
    h.train_index(0)
    if window_lo is not None:
        h.set_window(window_lo, -1)
    plan = h.plan_info(len(x))
    print("learned fill: %d bins, %d events, plan %r, index %r"
          % (axes[0]["nbins"], len(x), plan, h.index_info(0)), flush=True)
    t = dev(x)
    for _ in range(fills):
        h.fill([t])
    sumw, sumw2, entries = h.read()
    o = oracle.Oracle(axes)
    xs = np.concatenate([x] * fills)
    o.fill([xs])
    osw, _, ost, oent = o.read()
    assert entries == oent
    assert_bins_equal(sumw, osw, "counts")
    assert_bins_equal(sumw2, osw, "counts (sumw2)")
    assert_stats_close(h.stats(), ost, oracle.stats_abs(axes, [xs], None))
    return plan


def test_learned_benchmark_workload(hg):
    wl = synth.variable_1d(4_000_037)
    plan = _fill(hg, wl["axes"], wl["coords"][0], fills=2)
    assert plan["accumulator"] == "u16" and plan["strategy"] == "lds"


def test_learned_events_on_edges(hg):
    e = synth.log_edges()
    rng = np.random.default_rng(51)
    up = np.nextafter(e, np.inf)
    down = np.nextafter(e, -np.inf)
    x = np.concatenate([e, up, down, e, [0.0, -0.0, np.nan, np.inf, -np.inf, 1e-320, 1e300, -5.0]])
    x = np.tile(x, 4)
    rng.shuffle(x)
    _fill(hg, [{"nbins": len(e) - 1, "edges": e}], x)


def test_learned_window_narrower_than_histogram(hg):
    wl = synth.variable_1d(3_000_001)
    # a window starting well inside the axis: low bins and flow bins spill
    _fill(hg, wl["axes"], wl["coords"][0], window_lo=20_000)


def test_learned_signed_axis(hg):
    rng = np.random.default_rng(52)
    e = np.unique(np.concatenate([-np.logspace(-2, 2, 40000)[::-1], np.logspace(-2, 2, 40000)]))
    x = np.concatenate([rng.standard_normal(2_000_000) * 3.0, e[::7], -e[::11]])
    _fill(hg, [{"nbins": len(e) - 1, "edges": e}], x)


def test_learned_evenly_spaced_edges(hg):
    rng = np.random.default_rng(53)
    e = np.linspace(-5.0, 5.0, 90001)
    x = np.concatenate([rng.normal(0.0, 1.5, 2_000_000), e[::3]])
    _fill(hg, [{"nbins": len(e) - 1, "edges": e}], x)


def test_learned_wide_intervals(hg):
    rng = np.random.default_rng(54)
    # a dense cluster of edges inside an otherwise sparse axis: the segment
    # holding the cluster cannot be fitted to within two bins
    e = np.unique(np.concatenate([np.linspace(1.0, 1000.0, 60000),
                                  rng.uniform(7.0, 7.0 + 1e-6, 40000)]))
    axes = [{"nbins": len(e) - 1, "edges": e}]
    h = hg.Hist(axes)
    h.train_index(0)
    assert h.index_info(0)["max_window"] >= 2.0
    x = np.concatenate([rng.uniform(0.5, 1100.0, 1_500_000), rng.uniform(7.0, 7.0 + 1e-6, 500_000),
                        e[::5]])
    rng.shuffle(x)
    plan = _fill(hg, axes, x)
    assert plan["accumulator"] == "u16" and plan["strategy"] == "lds"
