"""Batched filling: one persistent launch over many uneven histograms, replayed
from a HIP graph, against the oracle member by member."""
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


def make_members(n_scale, k=64, bins_scale=1.0, seed=3):
    return synth.batched_64(seed=seed, k=k, n_scale=n_scale, bins_scale=bins_scale)


def oracle_for(m, times=1):
    o = oracle.Oracle(m["axes"])
    for _ in range(times):
        o.fill(m["coords"], m["weights"])
    return o.read()


def check_member(h, m, times=1):
    sumw, sumw2, entries = h.read()
    osw, osw2, ost, oent = oracle_for(m, times)
    assert entries == oent
    if m["weights"] is None:
        assert_bins_equal(sumw, osw)
    else:
        assert_sums_close(sumw, osw)
        assert_sums_close(sumw2, osw2)
    scale = times * oracle.stats_abs(m["axes"], m["coords"], m["weights"])
    assert_stats_close(h.stats(), ost, scale)


def build(hg, members, learned=False, dtypes=None):
    import torch
    hists, cols, ws = [], [], []
    for i, m in enumerate(members):
        h = hg.Hist(m["axes"])
        if learned:
            for a, ax in enumerate(m["axes"]):
                if ax.get("edges") is not None:
                    h.train_index(a)
        dt = None if dtypes is None else dtypes[i]
        hists.append(h)
        cols.append([dev(c, dt) for c in m["coords"]])
        ws.append(None if m["weights"] is None else dev(m["weights"], dt))
    return hists, cols, ws


def test_batch_graph_matches_oracle(hg):
    members = make_members(2e-3)
    hists, cols, ws = build(hg, members)
    b = hg.Batch(hists, cols, ws)
    b.launch()
    for h, m in zip(hists, members):
        check_member(h, m)


def test_batch_replays_accumulate_and_match_eager(hg):
    import torch
    members = make_members(1e-3, k=16, seed=11)
    hists, cols, ws = build(hg, members, learned=True)
    b = hg.Batch(hists, cols, ws)
    eh, ecols, ews = build(hg, members, learned=True)
    eb = hg.Batch(eh, ecols, ews)
    for rep in range(3):
        b.launch(graph=True)
        torch.cuda.synchronize()
        # eager work on the same stream between replays
        scratch = torch.ones(1 << 20, device="cuda").sum()
        eb.launch(graph=False)
        torch.cuda.synchronize()
        assert float(scratch) == float(1 << 20)
        for h, e, m in zip(hists, eh, members):
            g = h.read()
            r = e.read()
            assert g[2] == r[2] == (rep + 1) * len(m["coords"][0])
            assert_sums_close(g[0], r[0])
            assert_sums_close(g[1], r[1])
    for h, m in zip(hists, members):
        check_member(h, m, times=3)


def test_batch_equals_individual_fills(hg):
    members = make_members(1e-3, k=24, seed=5)
    hists, cols, ws = build(hg, members)
    hg.Batch(hists, cols, ws).launch()
    single, scols, sws = build(hg, members)
    for h, c, w in zip(single, scols, sws):
        h.fill(c, w)
    for a, s in zip(hists, single):
        ra, rs = a.read(), s.read()
        assert ra[2] == rs[2]
        assert_sums_close(ra[0], rs[0])
        assert_sums_close(ra[1], rs[1])


def test_batch_mixed_dtypes_unit_weights_and_empty(hg):
    import torch
    rng = np.random.default_rng(99)
    members = [
        {"axes": [{"nbins": 50, "xmin": -3.0, "xmax": 3.0}],
         "coords": [rng.normal(0, 1, 40_000)], "weights": None},
        {"axes": [{"nbins": 20, "xmin": 0.0, "xmax": 1.0}, {"nbins": 7, "edges": np.array([0, .1, .2, .4, .5, .6, .9, 1.0])}],
         "coords": [rng.uniform(-0.05, 1.05, 30_000), rng.uniform(-0.05, 1.05, 30_000)],
         "weights": rng.uniform(0, 2, 30_000)},
        {"axes": [{"nbins": 300_000, "xmin": -4.0, "xmax": 4.0}],
         "coords": [rng.normal(0, 1, 50_000)], "weights": rng.uniform(0, 2, 50_000)},
        {"axes": [{"nbins": 10, "xmin": 0.0, "xmax": 1.0}], "coords": [np.zeros(0)], "weights": None},
        {"axes": [{"nbins": 100, "xmin": -4.0, "xmax": 4.0}] * 3,
         "coords": [rng.normal(0, 1, 20_000) for _ in range(3)], "weights": None},
    ]
    dtypes = [torch.float32, None, None, None, torch.float32]
    hists, cols, ws = build(hg, members, dtypes=dtypes)
    hg.Batch(hists, cols, ws).launch()
    for i, (h, m) in enumerate(zip(hists, members)):
        if dtypes[i] is torch.float32:
            m = dict(m)
            m["coords"] = [c.astype(np.float32).astype(np.float64) for c in m["coords"]]
            if m["weights"] is not None:
                m["weights"] = m["weights"].astype(np.float32).astype(np.float64)
        check_member(h, m)


def test_batch_partitioned_members(hg):
    """Members far larger than LDS with many events go through the count /
    scan / scatter / accumulate passes; replays add up."""
    import torch
    rng = np.random.default_rng(123)
    e = np.sort(rng.uniform(0.0, 10.0, 100_001))
    members = [
        {"axes": [{"nbins": 300_000, "xmin": -4.0, "xmax": 4.0}],
         "coords": [rng.normal(0, 1, 400_003)], "weights": rng.uniform(0, 2, 400_003)},
        {"axes": [{"nbins": 100_000, "edges": e}],
         "coords": [rng.exponential(2.0, 300_001)], "weights": None},
        {"axes": [{"nbins": 100, "xmin": -4.0, "xmax": 4.0}] * 3,
         "coords": [rng.normal(0, 1, 200_000) for _ in range(3)], "weights": None},
        {"axes": [{"nbins": 1000, "xmin": 0.0, "xmax": 1.0}, {"nbins": 500, "xmin": 0.0, "xmax": 1.0}],
         "coords": [rng.uniform(-0.1, 1.1, 70_000), rng.uniform(-0.1, 1.1, 70_000)],
         "weights": rng.uniform(0, 2, 70_000)},
        {"axes": [{"nbins": 50, "xmin": -3.0, "xmax": 3.0}],
         "coords": [rng.normal(0, 1, 100_000)], "weights": None},
    ]
    dtypes = [None, None, torch.float32, torch.float32, None]
    hists, cols, ws = build(hg, members, learned=True, dtypes=dtypes)
    b = hg.Batch(hists, cols, ws)
    b.launch(graph=True)
    b.launch(graph=True)
    torch.cuda.synchronize()
    for i, (h, m) in enumerate(zip(hists, members)):
        if dtypes[i] is torch.float32:
            m = dict(m)
            m["coords"] = [c.astype(np.float32).astype(np.float64) for c in m["coords"]]
            if m["weights"] is not None:
                m["weights"] = m["weights"].astype(np.float32).astype(np.float64)
        check_member(h, m, times=2)


def test_batch_rejects_bad_arguments(hg):
    h = hg.Hist([{"nbins": 10, "xmin": 0.0, "xmax": 1.0}])
    x = dev(np.zeros(10))
    with pytest.raises(hg.HistError):
        hg.Batch([h, h], [[x], [x]], [None, None])


def test_batch_holds_its_histograms(hg):
    """A batch keeps its histograms alive (the caller may drop them), and the
    library refuses to destroy a handle while a live batch holds it."""
    import gc
    import torch
    members = make_members(2e-3, k=6, seed=5)

    def batch_only():
        hists, cols, ws = build(hg, members)
        return hg.Batch(hists, cols, ws)

    b = batch_only()
    gc.collect()
    b.launch()
    torch.cuda.synchronize()
    for h, m in zip(b.hists, members):
        check_member(h, m)
    lib = hg._lib.load()
    assert lib.hist_destroy(b.hists[0].handle) == hg._lib.HIST_EINVAL
    assert b"live batch" in lib.hist_last_error()
    hists = b.hists
    b.close()
    for h in hists:
        h.close()                          # released with the batch
