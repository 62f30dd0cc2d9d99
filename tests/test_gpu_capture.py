"""Stream capture and the scratch contract of hist_fill, through the C ABI.

- hist_read and hist_stats refuse to run while the stream is capturing
  (HIST_ECAPTURE) and leave the handle as it was;
- a hist_fill captured into a HIP graph (after hist_reserve) fills once per
  replay: every replay, with eager work and synchronizations in between, is
  checked against the oracle filled the same number of times (Sec. 3.3: sums
  accumulate across bulks), and the entry count, kept on the device, grows
  by n per replay;
- a handle created with HIST_F_NO_ALLOC refuses to grow its scratch
  (HIST_ENOMEM, histogram untouched) until hist_reserve has sized it, and
  refuses fills larger than the reservation.
"""
import numpy as np
import pytest

import oracle
import synth
from tests.gpu_helpers import assert_bins_equal, assert_sums_close, dev

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def hg():
    import torch
    assert torch.cuda.is_available(), "GPU tests need an MI355X"
    import paper_2401_13310_amd as pkg
    return pkg


def _cases(hg):
    """(name, workload, strategy, window merge, learned): plans with and
    without scratch -- an LDS window merged through staging slots, the
    partitioned strategy, a small LDS histogram with weights."""
    return {
        "lds_weighted": (synth.plain_1d(200_003), None, None, False),
        "staged_merge_learned": (synth.variable_1d(1_000_003), hg.HIST_STRAT_LDS, 1, True),
        "partitioned_3d": (synth.corr_3d(600_001), hg.HIST_STRAT_PART, None, False),
        "tiled_3d": (synth.corr_3d(300_007), hg.HIST_STRAT_TILED, None, False),
    }


def _make(hg, wl, strategy, merge, learned, flags=0):
    h = hg.Hist(wl["axes"], flags)
    if learned:
        for a, ax in enumerate(wl["axes"]):
            if ax.get("edges") is not None:
                h.train_index(a)
    if strategy is not None:
        h.set_strategy(strategy)
    if merge is not None:
        h.set_window(-1, merge)
    return h


def _check(h, o, unit):
    sumw, sumw2, entries = h.read()
    osw, osw2, ost, oent = o.read()
    assert entries == oent
    if unit:
        assert_bins_equal(sumw, osw, "counts")
        assert_bins_equal(sumw2, osw2, "counts (sumw2)")
    else:
        assert_sums_close(sumw, osw, what="sumw")
        assert_sums_close(sumw2, osw2, what="sumw2")


def test_read_and_stats_refuse_capture(hg):
    import torch
    wl = synth.plain_1d(10_000)
    x, w = dev(wl["coords"][0]), dev(wl["weights"])
    h = hg.Hist(wl["axes"])
    h.fill([x], w)
    torch.cuda.synchronize()
    before = h.read()
    stream = torch.cuda.Stream()
    graph = torch.cuda.CUDAGraph()
    status = {}
    with torch.cuda.graph(graph, stream=stream, capture_error_mode="thread_local"):
        for name, call in (("read", h.read), ("stats", h.stats)):
            try:
                call()
                status[name] = 0
            except hg.HistError as e:
                status[name] = e.status
    assert status == {"read": hg._lib.HIST_ECAPTURE, "stats": hg._lib.HIST_ECAPTURE}
    after = h.read()
    assert np.array_equal(before[0], after[0]) and before[2] == after[2]


@pytest.mark.parametrize("case", ["lds_weighted", "staged_merge_learned", "partitioned_3d",
                                  "tiled_3d"])
def test_captured_fill_replays(hg, case):
    import torch
    wl, strategy, merge, learned = _cases(hg)[case]
    cols = [dev(c) for c in wl["coords"]]
    w = None if wl["weights"] is None else dev(wl["weights"])
    n = cols[0].numel()
    # an eager fill of the same plan first: its kernels are set up outside capture
    eager = _make(hg, wl, strategy, merge, learned)
    eager.fill(cols, w)
    o = oracle.Oracle(wl["axes"])
    o.fill(wl["coords"], wl["weights"])
    _check(eager, o, w is None)

    h = _make(hg, wl, strategy, merge, learned)
    h.reserve(n, hg.HIST_F64, w is not None)
    torch.cuda.synchronize()
    stream = torch.cuda.Stream()
    graph = torch.cuda.CUDAGraph()
    with torch.cuda.graph(graph, stream=stream, capture_error_mode="thread_local"):
        h.fill(cols, w)
    # capture records the fill without running it
    assert h.read()[2] == 0
    o = oracle.Oracle(wl["axes"])
    junk = torch.zeros(1 << 20, dtype=torch.float64, device="cuda")
    for r in range(1, 4):
        graph.replay()
        torch.cuda.synchronize()
        junk.add_(cols[0][:1 << 20] if n >= 1 << 20 else 1.0)   # eager work between replays
        torch.cuda.synchronize()
        o.fill(wl["coords"], wl["weights"])
        _check(h, o, w is None)
        assert h.read()[2] == r * n


def test_no_alloc_handle_needs_reserve(hg):
    import torch
    wl = synth.corr_3d(400_003)
    cols = [dev(c) for c in wl["coords"]]
    n = cols[0].numel()
    h = hg.Hist(wl["axes"], hg.HIST_F_NO_ALLOC)
    h.set_strategy(hg.HIST_STRAT_PART)
    with pytest.raises(hg.HistError) as e:
        h.fill(cols)
    assert e.value.status == hg._lib.HIST_ENOMEM
    sumw, _, entries = h.read()
    assert entries == 0 and not sumw.any()
    h.reserve(n, hg.HIST_F64, False)
    h.fill(cols)
    o = oracle.Oracle(wl["axes"])
    o.fill(wl["coords"])
    _check(h, o, True)
    # a fill larger than the reservation needs more scratch: refused, nothing added
    big = [torch.cat([c, c]) for c in cols]
    with pytest.raises(hg.HistError) as e:
        h.fill(big)
    assert e.value.status == hg._lib.HIST_ENOMEM
    _check(h, o, True)
