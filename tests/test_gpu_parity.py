"""GPU parity: the HIP path through the C ABI against the CPU oracle, on the
same seeded inputs.  Bin indices and unit-weight counts must be identical;
binary64 weighted sums within 1e-12 (see gpu_helpers)."""
import math

import numpy as np
import pytest

import oracle
import synth
from tests.gpu_helpers import (assert_bins_equal, assert_stats_close, assert_sums_close, dev,
                               max_rel_err)
from tests.test_golden import axis_from_json, load as load_golden, unhex

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def hg():
    import torch
    assert torch.cuda.is_available(), "GPU tests need an MI355X"
    import paper_2401_13310_amd as pkg
    return pkg


def gpu_findbin(hg, axes, cols, learned=False, dtype=None):
    import torch
    h = hg.Hist(axes)
    if learned:
        for a, ax in enumerate(axes):
            if ax.get("edges") is not None:
                h.train_index(a)
    tcols = [dev(c, dtype) for c in cols]
    out = h.findbin(tcols).cpu().numpy()
    torch.cuda.synchronize()
    return out, h


def _assert(cond, msg):
    if not cond:
        raise AssertionError(msg)


def fill_and_compare(hg, axes, coords, w, strategy=None, flags=0, learned=False, dtype=None,
                     window=None, blocks=0, copies=0, check_sums=True):
    import torch
    h = hg.Hist(axes, flags)
    if learned:
        for a, ax in enumerate(axes):
            if ax.get("edges") is not None:
                h.train_index(a)
    if strategy is not None:
        h.set_strategy(strategy, blocks, copies)
    if window is not None:
        h.set_window(*window)
    tc = [dev(c, dtype) for c in coords]
    tw = None if w is None else dev(w, dtype)
    h.fill(tc, tw)
    sumw, sumw2, entries = h.read()
    st = h.stats()
    o = oracle.Oracle(axes)
    oc = [np.asarray(c.astype(np.float64) if dtype is None else
                     torch.tensor(c).to(dtype).double().numpy()) for c in coords]
    ow = None if w is None else (w.astype(np.float64) if dtype is None else
                                 torch.tensor(w).to(dtype).double().numpy())
    o.fill(oc, ow)
    osw, osw2, ost, oent = o.read()
    scale = oracle.stats_abs(axes, oc, ow)
    # every check runs and every failure is reported together, so that a
    # failure tells lost events (bins low, totals and statistics short) from
    # mis-binned ones (as much gained as lost, statistics intact)
    failures = []

    def collect(check, *args, **kw):
        try:
            check(*args, **kw)
        except AssertionError as e:
            failures.append(str(e))

    collect(lambda: _assert(entries == oent, "entries %d want %d" % (entries, oent)))
    if w is None:
        collect(assert_bins_equal, sumw, osw, "unit-weight counts")
        collect(assert_bins_equal, sumw2, osw2, "unit-weight counts (sumw2)")
    elif check_sums:
        collect(assert_sums_close, sumw, osw, what="sumw")
        collect(assert_sums_close, sumw2, osw2, what="sumw2")
    if check_sums:
        collect(assert_stats_close, st, ost, scale)
    if failures:
        raise AssertionError("; ".join(failures) + "; stats got %r want %r" % (list(st), list(ost)))
    torch.cuda.synchronize()
    return h, (sumw, sumw2, st, entries), (osw, osw2, ost, oent)


# ------------------------------------------------------------------ find bin --

def test_findbin_golden_special_values(hg):
    g = load_golden("findbin_special_values.json")
    for case in g["cases"]:
        ax = axis_from_json(case["axis"])
        x = unhex(case["x"])
        got, _ = gpu_findbin(hg, [ax], [x])
        assert_bins_equal(got, case["bins"], "golden bins")
        if ax.get("edges") is not None:
            got, _ = gpu_findbin(hg, [ax], [x], learned=True)
            assert_bins_equal(got, case["bins"], "golden bins (learned)")


@pytest.mark.parametrize("nb,lo,hi", [(100, -5.0, 5.0), (10_000, 0.0, 100.0), (1000, 0.0, 1.0),
                                      (97, -3.7, 11.1), (1, -1.0, 1.0), (3, 0.1, 0.7)])
def test_findbin_uniform_adversarial(hg, nb, lo, hi):
    rng = np.random.default_rng(nb)
    x = np.concatenate([synth.special_values((nb, lo, hi), count_near=4),
                        rng.uniform(lo - 1, hi + 1, 300_001)])
    ax = [{"nbins": nb, "xmin": lo, "xmax": hi}]
    got, _ = gpu_findbin(hg, ax, [x])
    assert_bins_equal(got, oracle.findbin(ax, [x]))


def _edge_sets():
    rng = np.random.default_rng(7)
    return {
        "log_1e5": synth.log_edges(100_000),
        "sorted_uniform_1e6": synth._sorted_edges(rng, 1_000_000, 0.0, 1.0),
        "sorted_normal_5000": np.unique(np.sort(rng.normal(0, 1, 5001))),
        "one_bin": np.array([-1.0, 2.0]),
        "two_bins_signed": np.array([-2.0, 0.0, 3.0]),
        "wide_range": np.concatenate([-np.logspace(300, -300, 400), np.logspace(-300, 300, 401)]),
        "paper_1000": np.linspace(0.0, 1.0, 1001),
        "clustered": np.unique(np.concatenate([np.linspace(0, 1, 200),
                                               1 + np.logspace(-12, -1, 3000)])),
    }


@pytest.mark.parametrize("name", list(_edge_sets()))
def test_findbin_variable_bsearch_and_learned(hg, name):
    e = _edge_sets()[name]
    nb = e.size - 1
    ax = [{"nbins": nb, "edges": e}]
    rng = np.random.default_rng(nb)
    span = e[-1] - e[0]
    x = np.concatenate([synth.special_values(e, count_near=2),
                        rng.uniform(e[0] - 0.05 * span, e[-1] + 0.05 * span, 200_000)
                        if np.isfinite(span) else rng.normal(0, 1e3, 200_000),
                        rng.choice(e, 50_000) * (1 + rng.normal(0, 1e-9, 50_000))])
    want = oracle.findbin(ax, [x])
    got_b, _ = gpu_findbin(hg, ax, [x], learned=False)
    assert_bins_equal(got_b, want, "bsearch bins")
    got_l, h = gpu_findbin(hg, ax, [x], learned=True)
    assert_bins_equal(got_l, want, "learned bins")
    info = h.index_info(0)
    assert info["segments"] >= 1


def test_findbin_learned_variable_1d_workload(hg):
    wl = synth.variable_1d(4_000_000)
    ax = wl["axes"]
    want = oracle.findbin(ax, wl["coords"])
    got, h = gpu_findbin(hg, ax, wl["coords"], learned=True)
    assert_bins_equal(got, want)
    info = h.index_info(0)
    assert info["feature"] == "key"
    assert info["mean_window"] < 2.0


def test_findbin_3d_and_float32(hg):
    wl = synth.corr_3d(500_000)
    got, _ = gpu_findbin(hg, wl["axes"], wl["coords"])
    assert_bins_equal(got, oracle.findbin(wl["axes"], wl["coords"]))
    import torch
    x32 = [c.astype(np.float32) for c in wl["coords"]]
    got32, _ = gpu_findbin(hg, wl["axes"], x32)
    assert_bins_equal(got32, oracle.findbin(wl["axes"], [c.astype(np.float64) for c in x32]))


# ---------------------------------------------- edges staged in LDS (fills) --
# Variable axes of at most 4096 edges (32 KB of edges per histogram) are
# copied to LDS and searched there; fills whose variable axes are all staged
# run a kernel that reads edges from LDS only.  These cases pin the staged
# searches (learned and binary) against the oracle, at the size limit and
# past it, and a histogram whose edge budget stages only some of its axes.

def _staged_sets():
    rng = np.random.default_rng(11)
    sets = {k: v for k, v in _edge_sets().items() if v.size <= 4096}
    sets["at_limit_4096_edges"] = synth._sorted_edges(rng, 4095, -3.0, 3.0)
    sets["past_limit_4097_edges"] = synth._sorted_edges(rng, 4096, -3.0, 3.0)
    return sets


@pytest.mark.parametrize("learned", [False, True])
@pytest.mark.parametrize("name", list(_staged_sets()))
def test_fill_staged_edges_1d(hg, name, learned):
    e = _staged_sets()[name]
    ax = [{"nbins": e.size - 1, "edges": e}]
    rng = np.random.default_rng(e.size)
    span = e[-1] - e[0]
    n = 300_001
    x = (rng.uniform(e[0] - 0.05 * span, e[-1] + 0.05 * span, n) if np.isfinite(span)
         else rng.normal(0, 1e3, n))
    x[:1000] = rng.choice(e, 1000)   # exact edges: the lower edge belongs to the bin
    # coordinates near 1e300 overflow the x^2 statistic (inf on both sides,
    # or NaN where the oracle's sum order meets inf - inf): bins only there
    finite = bool(np.all(np.abs(x) < 1e150))
    fill_and_compare(hg, ax, [x], None, learned=learned, check_sums=finite)
    w = rng.uniform(0.0, 2.0, n)
    h, got, want = fill_and_compare(hg, ax, [x], w, learned=learned, check_sums=finite)
    if not finite:
        assert_sums_close(got[0], want[0], what="sumw")


@pytest.mark.parametrize("learned", [False, True])
def test_fill_staged_edges_3d(hg, learned):
    rng = np.random.default_rng(12)
    axes = [{"nbins": 30, "edges": synth._sorted_edges(rng, 30, -4.0, 4.0)},
            {"nbins": 17, "xmin": -3.0, "xmax": 3.0},
            {"nbins": 45, "edges": synth._sorted_edges(rng, 45, -4.0, 4.0)}]
    n = 400_003
    coords = [rng.normal(0, 1, n) for _ in range(3)]
    fill_and_compare(hg, axes, coords, None, learned=learned)
    fill_and_compare(hg, axes, coords, rng.uniform(0.0, 2.0, n), learned=learned)


def test_fill_edges_partly_staged(hg):
    # 2 x 2101 edges: the first axis fits the 32 KB budget, the second is
    # searched in HBM, so the fill mixes both kinds of search
    rng = np.random.default_rng(13)
    axes = [{"nbins": 2100, "edges": synth._sorted_edges(rng, 2100, -4.0, 4.0)} for _ in range(2)]
    n = 200_001
    coords = [rng.normal(0, 1, n) for _ in range(2)]
    for learned in (False, True):
        fill_and_compare(hg, axes, coords, None, learned=learned, strategy=hg.HIST_STRAT_GLOBAL)


# ---------------------------------------------------------------------- fill --

def test_fill_plain_1d_full_size(hg):
    wl = synth.plain_1d()
    fill_and_compare(hg, wl["axes"], wl["coords"], wl["weights"])


@pytest.mark.parametrize("copies", [1, 7, 64])
def test_fill_plain_1d_lds_copies(hg, copies):
    wl = synth.plain_1d(300_001)
    fill_and_compare(hg, wl["axes"], wl["coords"], wl["weights"],
                     strategy=hg.HIST_STRAT_LDS, copies=copies)


@pytest.mark.parametrize("strategy", ["lds", "global"])
@pytest.mark.parametrize("learned", [False, True])
def test_fill_variable_1d(hg, strategy, learned):
    wl = synth.variable_1d(3_000_017)
    s = {"lds": hg.HIST_STRAT_LDS, "global": hg.HIST_STRAT_GLOBAL}[strategy]
    fill_and_compare(hg, wl["axes"], wl["coords"], None, strategy=s, learned=learned)


@pytest.mark.parametrize("merge", [0, 1])
def test_fill_variable_1d_window_merges(hg, merge):
    wl = synth.variable_1d(2_000_003)
    fill_and_compare(hg, wl["axes"], wl["coords"], None, strategy=hg.HIST_STRAT_LDS,
                     learned=True, window=(20_000, merge))


@pytest.mark.parametrize("strategy", ["lds", "global", "tiled", "part"])
def test_fill_corr_3d(hg, strategy):
    wl = synth.corr_3d(2_000_000)
    s = {"lds": hg.HIST_STRAT_LDS, "global": hg.HIST_STRAT_GLOBAL,
         "tiled": hg.HIST_STRAT_TILED, "part": hg.HIST_STRAT_PART}[strategy]
    fill_and_compare(hg, wl["axes"], wl["coords"], None, strategy=s)


@pytest.mark.parametrize("strategy", ["auto", "lds", "global", "tiled", "part"])
def test_fill_weighted_2d_mixed_axes(hg, strategy):
    rng = np.random.default_rng(21)
    e = np.sort(rng.uniform(-3, 3, 301))
    axes = [{"nbins": 300, "edges": e}, {"nbins": 80, "xmin": -2.5, "xmax": 2.5}]
    n = 1_000_003
    coords = [rng.normal(0, 1, n), rng.normal(0, 1, n)]
    w = rng.uniform(0.0, 2.0, n)
    s = {"auto": None, "lds": hg.HIST_STRAT_LDS, "global": hg.HIST_STRAT_GLOBAL,
         "tiled": hg.HIST_STRAT_TILED, "part": hg.HIST_STRAT_PART}[strategy]
    fill_and_compare(hg, axes, coords, w, strategy=s, learned=True)


# The partitioned strategy: a learned variable axis of 1e5 bins (ragged last
# bucket), FP32 weighted input, a 3D histogram whose event count spans two
# partition chunks (2^25 events each), and few events over many buckets.
def test_fill_part_variable_learned(hg):
    wl = synth.variable_1d(3_000_017)
    fill_and_compare(hg, wl["axes"], wl["coords"], None, strategy=hg.HIST_STRAT_PART,
                     learned=True)


def test_fill_part_weighted_f32(hg):
    import torch
    rng = np.random.default_rng(41)
    axes = [{"nbins": 250_000, "xmin": -4.0, "xmax": 4.0}]
    n = 2_000_001
    x = rng.normal(0, 1.3, n)
    w = rng.lognormal(0.0, 1.0, n)
    fill_and_compare(hg, axes, [x], w, strategy=hg.HIST_STRAT_PART, dtype=torch.float32)


def test_fill_part_two_chunks(hg):
    rng = np.random.default_rng(42)
    axes = [{"nbins": 60, "xmin": -3.0, "xmax": 3.0}, {"nbins": 70, "xmin": -3.0, "xmax": 3.0},
            {"nbins": 80, "xmin": -3.0, "xmax": 3.0}]
    n = (1 << 25) + 4099
    coords = [rng.normal(0, 1, n) for _ in range(3)]
    fill_and_compare(hg, axes, coords, None, strategy=hg.HIST_STRAT_PART)


def test_fill_scratch_regrowth_across_strategies(hg):
    """One handle alternates the partitioned and tiled strategies with growing
    and shrinking fills, so their scratch buffers are reallocated in between;
    every fill adds to the same histogram."""
    import torch
    rng = np.random.default_rng(44)
    axes = [{"nbins": 400, "xmin": -3.0, "xmax": 3.0}, {"nbins": 500, "xmin": -3.0, "xmax": 3.0}]
    h = hg.Hist(axes)
    o = oracle.Oracle(axes)
    for strat, n in [(hg.HIST_STRAT_PART, 300_000), (hg.HIST_STRAT_TILED, 900_000),
                     (hg.HIST_STRAT_PART, 200_000), (hg.HIST_STRAT_PART, 1_200_000),
                     (hg.HIST_STRAT_TILED, 100_000)]:
        coords = [rng.normal(0, 1, n), rng.normal(0, 1, n)]
        h.set_strategy(strat, 0, 0)
        h.fill([dev(c) for c in coords], None)
        o.fill(coords, None)
    sumw, _, entries = h.read()
    osw, _, _, oent = o.read()
    assert entries == oent
    assert_bins_equal(sumw, osw, "counts after regrowth")
    torch.cuda.synchronize()


def test_fill_part_sparse(hg):
    rng = np.random.default_rng(43)
    axes = [{"nbins": 1_000_000, "xmin": 0.0, "xmax": 1.0}]
    x = rng.uniform(-0.1, 1.1, 777)
    w = rng.uniform(0.0, 2.0, 777)
    fill_and_compare(hg, axes, [x], w, strategy=hg.HIST_STRAT_PART)


def test_fill_weighted_signed_weights(hg):
    rng = np.random.default_rng(22)
    axes = [{"nbins": 50, "xmin": -1.0, "xmax": 1.0}]
    n = 500_000
    x = rng.uniform(-1.2, 1.2, n)
    w = rng.normal(0.0, 1.0, n)
    h, got, want = fill_and_compare(hg, axes, [x], w, check_sums=False)
    # signed weights cancel: compare against the sum of |w| per bin
    ab = oracle.Oracle(axes)
    ab.fill([x], np.abs(w))
    scale = ab.read()[0]
    assert np.all(np.abs(got[0] - want[0]) <= 1e-12 * np.maximum(np.abs(want[0]), scale))
    assert_sums_close(got[1], want[1], what="sumw2")


def test_fill_u16_counters_never_overflow(hg):
    """Every event in one bin of a histogram held in 16-bit LDS counters:
    each workgroup sees far more than 65535 increments of that counter."""
    import torch
    nb = 60_000
    axes = [{"nbins": nb, "xmin": 0.0, "xmax": float(nb)}]
    n = 3_000_000
    x = np.full(n, 12_345.5)
    h = hg.Hist(axes)
    plan = h.plan_info(n)
    assert plan["accumulator"] == "u16"
    h.set_strategy(hg.HIST_STRAT_LDS, 8, 0)   # 8 workgroups: 375k events each
    h.fill([dev(x)])
    sumw, _, entries = h.read()
    assert sumw[12_346] == n and entries == n
    assert sumw.sum() == n


@pytest.mark.parametrize("learned", [False, True])
def test_fill_u16_staged_merge_saturation(hg, learned):
    """16-bit LDS counters merged through 8-bit staging slots: bins with more
    than 255 (and more than 65535) events in a workgroup stage 255 and add the
    rest directly; counts must stay exact either way."""
    rng = np.random.default_rng(31)
    n = 2_000_003
    if learned:
        axes = [{"nbins": 99_999, "edges": synth.log_edges(100_000)}]
        x = rng.exponential(1.0, n)
        x[: n // 3] = 0.5              # one bin, ~42k events per workgroup
        x[n // 3: n // 3 + 40_000] = 2.0
        x[-300:] = 1e-5                # underflow
    else:
        nb = 60_000
        axes = [{"nbins": nb, "xmin": 0.0, "xmax": float(nb)}]
        x = rng.uniform(-10.0, nb + 10.0, n)
        x[: n // 3] = 12_345.5
        x[n // 3: n // 3 + 40_000] = 17.25
        x[n // 3 + 40_000: n // 3 + 45_000] = 59_999.0   # the window's last bin
    rng.shuffle(x)
    h = hg.Hist(axes)
    if learned:
        h.train_index(0)
    assert h.plan_info(n)["accumulator"] == "u16"
    h.set_strategy(hg.HIST_STRAT_LDS, 16, 0)
    h.set_window(-1, 1)                 # staged merge
    assert h.plan_info(n)["strategy"] == "lds"
    h.timing(True)
    for _ in range(2):
        h.fill([dev(x)])
    sumw, sumw2, entries = h.read()
    assert h.timing_read()["merge_ms"] > 0.0      # the staged merge ran
    o = oracle.Oracle(axes)
    o.fill([np.concatenate([x, x])])
    osw, _, _, oent = o.read()
    assert entries == oent
    assert_bins_equal(sumw, osw, "counts")
    assert_bins_equal(sumw2, osw, "counts (sumw2)")


def test_fill_precision_f32_compensated(hg):
    import torch
    axes = synth.precision_axes()
    xs, ws = [], []
    for x, w in synth.precision_slices(n=3 * (1 << 20), slice_len=1 << 20):
        xs.append(x)
        ws.append(w)
    h32 = hg.Hist(axes, hg.HIST_F_ACC_F32C)
    assert h32.plan_info(1 << 20, hg.HIST_F32, True)["accumulator"] == "f32c"
    h64 = hg.Hist(axes)
    o = oracle.Oracle(axes)
    for x, w in zip(xs, ws):
        h32.fill([dev(x)], dev(w))
        h64.fill([dev(x.astype(np.float64))], dev(w.astype(np.float64)))
        o.fill([x.astype(np.float64)], w.astype(np.float64))
    osw, osw2, ost, oent = o.read()
    s32, s32_2, e32 = h32.read()
    s64, s64_2, e64 = h64.read()
    assert e32 == e64 == oent
    # all-FP64 path on the widened data: the 1e-12 rule
    assert_sums_close(s64, osw)
    assert_sums_close(s64_2, osw2)
    # compensated FP32 LDS accumulation: error stated, bounded far below FP32 rounding
    assert max_rel_err(s32, osw) < 1e-9
    assert max_rel_err(s32_2, osw2) < 1e-9
    xw = [np.concatenate(xs).astype(np.float64)]
    scale = oracle.stats_abs(axes, xw, np.concatenate(ws).astype(np.float64))
    assert_stats_close(h32.stats(), ost, scale)
    assert_stats_close(h64.stats(), ost, scale)


def test_golden_fill_small_2d(hg):
    g = load_golden("fill_small_2d.json")
    axes = [axis_from_json(a) for a in g["axes"]]
    h = hg.Hist(axes)
    h.fill([dev(unhex(g["x"])), dev(unhex(g["y"]))], dev(unhex(g["w"])))
    sumw, sumw2, entries = h.read()
    assert entries == g["entries"]
    assert_sums_close(sumw, unhex(g["sumw"]))
    assert_sums_close(sumw2, unhex(g["sumw2"]))
    assert_stats_close(h.stats(), unhex(g["stats"]), np.abs(unhex(g["stats"])) + 1.0)


# ------------------------------------------------------------ semantics ------

def test_accumulate_across_fills(hg):
    """Sec. 3.3: fill(A); fill(B) gives the sums of fill(A||B)."""
    wl = synth.plain_1d(400_000)
    x, w = wl["coords"][0], wl["weights"]
    a = hg.Hist(wl["axes"])
    a.fill([dev(x)], dev(w))
    b = hg.Hist(wl["axes"])
    b.fill([dev(x[:123_457])], dev(w[:123_457]))
    b.fill([dev(x[123_457:])], dev(w[123_457:]))
    ra, rb = a.read(), b.read()
    assert ra[2] == rb[2] == x.size
    assert_sums_close(ra[0], rb[0])
    sa, sb = a.stats(), b.stats()
    scale = oracle.stats_abs(wl["axes"], [x], w)
    assert_stats_close(sa, sb, scale)


def test_input_reuse_after_fill_is_stream_ordered(hg):
    """Sec. 3.3's race: overwriting the input after an asynchronous fill on the
    same stream must not change what the fill counted."""
    import torch
    axes = [{"nbins": 10, "xmin": 0.0, "xmax": 10.0}]
    x = dev(np.full(1_000_000, 2.5))
    h = hg.Hist(axes)
    s = torch.cuda.Stream()
    with torch.cuda.stream(s):
        h.fill([x], stream=s)
        x.fill_(7.5)   # same stream: runs after the fill
    s.synchronize()
    sumw = h.read(stream=s)[0]
    assert sumw[3] == 1_000_000 and sumw[8] == 0
    # second stream ordered by an event
    s2 = torch.cuda.Stream()
    h2 = hg.Hist(axes)
    y = dev(np.full(500_000, 4.5))
    with torch.cuda.stream(s2):
        h2.fill([y], stream=s2)
        ev = torch.cuda.Event()
        ev.record(s2)
    s.wait_event(ev)
    with torch.cuda.stream(s):
        y.fill_(9.5)
    torch.cuda.synchronize()
    assert h2.read()[0][5] == 500_000


@pytest.mark.parametrize("n", [0, 1, 2, 63, 64, 65, 1023, 1025, 8191, 8193, 99_991])
def test_empty_and_ragged_sizes(hg, n):
    rng = np.random.default_rng(n)
    axes = [{"nbins": 7, "xmin": -1.0, "xmax": 1.0}, {"nbins": 5, "edges": np.array([-1, -.5, 0, .2, .9, 1.0])}]
    coords = [rng.uniform(-1.1, 1.1, n), rng.uniform(-1.1, 1.1, n)]
    w = rng.uniform(0.1, 1.0, n)
    fill_and_compare(hg, axes, coords, w)
    fill_and_compare(hg, axes, coords, None, learned=True)


def test_reset_and_flow_excluded_from_stats(hg):
    axes = [{"nbins": 4, "xmin": 0.0, "xmax": 4.0}]
    x = np.array([-1.0, 0.5, 1.5, 3.99, 4.0, np.nan, np.inf, -np.inf])
    h = hg.Hist(axes)
    h.fill([dev(x)])
    sumw, _, entries = h.read()
    assert sumw.tolist() == [2.0, 1.0, 1.0, 0.0, 1.0, 3.0]
    assert entries == 8
    st = h.stats()
    assert st[0] == 3.0 and st[2] == 0.5 + 1.5 + 3.99
    h.reset()
    sumw, _, entries = h.read()
    assert not sumw.any() and entries == 0 and not h.stats().any()


def test_tune_keeps_contents_and_agrees(hg):
    wl = synth.variable_1d(1_000_000)
    h = hg.Hist(wl["axes"])
    h.train_index(0)
    x = dev(wl["coords"][0])
    h.fill([x])
    before = h.read()
    h.tune([x])
    after = h.read()
    assert_bins_equal(before[0], after[0])
    assert before[2] == after[2]
    h.fill([x])
    o = oracle.Oracle(wl["axes"])
    o.fill(wl["coords"])
    o.fill(wl["coords"])
    assert_bins_equal(h.read()[0], o.read()[0])
