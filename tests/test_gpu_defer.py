"""GPU parity of deferred merges (HIST_F_DEFER_MERGE): the learned one-axis
fill's staged merge done by the next such fill, or by hist_read / hist_flush.
Every sequence below must give the oracle's counts bit for bit: several fills
then one read, reads between fills, a reset with a merge pending, a change of
strategy, fills on two streams, tuning, host-resident fills, and graph capture
(refused while a merge is pending, fine after a flush)."""
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


@pytest.fixture(scope="module")
def wl():
    return synth.variable_1d(2_500_001, seed=71)


def _hist(hg, wl):
    h = hg.Hist(wl["axes"], hg.HIST_F_DEFER_MERGE)
    h.train_index(0)
    plan = h.plan_info(len(wl["coords"][0]))
    assert plan["accumulator"] == "u16" and plan["strategy"] == "lds", plan
    return h


def _check(hg, h, wl, fills):
    sumw, sumw2, entries = h.read()
    xs = np.concatenate([wl["coords"][0]] * fills) if fills else np.zeros(0)
    o = oracle.Oracle(wl["axes"])
    if fills:
        o.fill([xs])
    osw, _, ost, oent = o.read()
    assert entries == oent
    assert_bins_equal(sumw, osw, "counts")
    assert_bins_equal(sumw2, osw, "counts (sumw2)")
    if fills:
        assert_stats_close(h.stats(), ost, oracle.stats_abs(wl["axes"], [xs], None))


def test_several_fills_one_read(hg, wl):
    h = _hist(hg, wl)
    x = dev(wl["coords"][0])
    for _ in range(4):
        h.fill([x])
    _check(hg, h, wl, 4)


def test_reads_between_fills(hg, wl):
    h = _hist(hg, wl)
    x = dev(wl["coords"][0])
    h.fill([x])
    _check(hg, h, wl, 1)
    h.fill([x])
    h.fill([x])
    _check(hg, h, wl, 3)
    h.flush()
    h.flush()   # nothing pending: no effect
    _check(hg, h, wl, 3)


def test_reset_drops_the_pending_merge(hg, wl):
    h = _hist(hg, wl)
    x = dev(wl["coords"][0])
    h.fill([x])
    h.fill([x])
    h.reset()
    _check(hg, h, wl, 0)
    h.fill([x])
    _check(hg, h, wl, 1)


def test_other_strategy_after_deferred_fill(hg, wl):
    h = _hist(hg, wl)
    x = dev(wl["coords"][0])
    h.fill([x])
    h.set_strategy(hg.HIST_STRAT_GLOBAL)
    h.fill([x])
    h.set_strategy(hg.HIST_STRAT_AUTO)
    h.fill([x])
    _check(hg, h, wl, 3)


def test_fills_on_two_streams(hg, wl):
    import torch
    h = _hist(hg, wl)
    x = dev(wl["coords"][0])
    torch.cuda.synchronize()
    s1, s2 = torch.cuda.Stream(), torch.cuda.Stream()
    h.fill([x], stream=s1)
    h.fill([x], stream=s2)
    h.fill([x], stream=s1)
    s1.synchronize()
    s2.synchronize()
    _check(hg, h, wl, 3)


def test_tune_keeps_contents(hg, wl):
    h = _hist(hg, wl)
    x = dev(wl["coords"][0])
    h.fill([x])
    h.tune([x[:1_000_000]])
    h.fill([x])
    _check(hg, h, wl, 2)


def test_host_fills(hg, wl):
    h = _hist(hg, wl)
    h.fill_host([wl["coords"][0]])
    h.fill([dev(wl["coords"][0])])
    h.fill_host([wl["coords"][0]])
    _check(hg, h, wl, 3)


def test_capture_needs_a_flush(hg, wl):
    import torch
    h = _hist(hg, wl)
    x = dev(wl["coords"][0])
    h.fill([x])
    torch.cuda.synchronize()
    stream = torch.cuda.Stream()
    graph = torch.cuda.CUDAGraph()
    status = {}
    with torch.cuda.graph(graph, stream=stream, capture_error_mode="thread_local"):
        try:
            h.fill([x])
            status["fill"] = 0
        except hg.HistError as e:
            status["fill"] = e.status
    assert status == {"fill": hg._lib.HIST_ECAPTURE}
    h.flush()
    torch.cuda.synchronize()
    graph = torch.cuda.CUDAGraph()
    with torch.cuda.graph(graph, stream=stream, capture_error_mode="thread_local"):
        h.fill([x])
    for _ in range(2):
        graph.replay()
        torch.cuda.synchronize()
    _check(hg, h, wl, 3)
