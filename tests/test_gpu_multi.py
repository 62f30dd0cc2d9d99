"""GPU parity of the one-pass fill of several histograms with filters and
computed columns (hist_multi_*): every member against the oracle fill of the
events its filter keeps, with coordinates and weights from the oracle's own
evaluation of the member's programs (oracle/expr.py)."""
import ctypes
import math

import numpy as np
import pytest

import oracle
from oracle import expr as E
from tests.gpu_helpers import assert_bins_equal, assert_stats_close, assert_sums_close, dev

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def hg():
    import torch
    assert torch.cuda.is_available(), "GPU tests need an MI355X"
    import paper_2401_13310_amd as pkg
    return pkg


def _member_ops(hg, cols, d):
    out = {}
    for key in ("filter", "weight"):
        if d.get(key) is not None:
            out[key] = hg.parse(d[key], cols) if isinstance(d[key], str) else d[key]
    if d.get("coords") is not None:
        out["coords"] = [None if c is None else (hg.parse(c, cols) if isinstance(c, str) else c)
                         for c in d["coords"]]
    return out


def _compare(h, axes, define_ops, columns):
    coords, w = E.apply_define(define_ops, columns, len(axes))
    o = oracle.Oracle(axes)
    o.fill(coords, w)
    osw, osw2, ost, oent = o.read()
    sumw, sumw2, entries = h.read()
    assert entries == oent, "entries %d want %d" % (entries, oent)
    if w is None:
        assert_bins_equal(sumw, osw, "counts")
    else:
        assert_sums_close(sumw, osw, what="sumw")
        assert_sums_close(sumw2, osw2, what="sumw2")
    assert_stats_close(h.stats(), ost, oracle.stats_abs(axes, coords, w))


def _run(hg, names, columns, members, dtype=None, fills=1):
    import torch
    hists = [hg.Hist(m["axes"]) for m in members]
    defs = [_member_ops(hg, names, m.get("define") or {}) for m in members]
    tdt = torch.float64 if dtype is None else dtype
    plan = hg.Multi(hists, defs, names, hg.HIST_F32 if tdt == torch.float32 else hg.HIST_F64)
    tcols = [dev(c, tdt) for c in columns]
    for _ in range(fills):
        print("multi fill: %d members, %d columns, n=%d" % (len(members), len(names), len(columns[0])),
              flush=True)
        plan.fill(tcols)
    torch.cuda.synchronize()
    ocols = [t.double().cpu().numpy() for t in tcols]
    for h, m, d in zip(hists, members, defs):
        if fills == 1:
            _compare(h, m["axes"], d, ocols)
        else:
            _compare(h, m["axes"], d, [np.concatenate([c] * fills) for c in ocols])
    return plan, hists


def _columns(n, seed, k=3):
    rng = np.random.default_rng(seed)
    z = rng.standard_normal((3, n))
    return [z[0], 0.5 * z[0] + z[1], z[2] * 2.0 + 0.3][:k]


def test_projections_filters_and_defines(hg):
    names = ["x", "y", "z"]
    cols = _columns(1_000_003, 81)
    edges = np.sort(np.random.default_rng(82).uniform(-3, 3, 41))
    members = [
        {"axes": [{"nbins": 100, "xmin": -4.0, "xmax": 4.0}]},                       # x
        {"axes": [{"nbins": 40, "edges": edges}], "define": {"coords": ["y"]}},     # y
        {"axes": [{"nbins": 60, "xmin": -3.0, "xmax": 3.0},
                  {"nbins": 40, "xmin": -3.0, "xmax": 3.0}]},                       # x:y
        {"axes": [{"nbins": 200, "xmin": 0.0, "xmax": 8.0}],
         "define": {"filter": "z > 0 && abs(x) < 2.5", "coords": ["sqrt(x*x + y*y + z*z)"]}},
        {"axes": [{"nbins": 50, "xmin": -5.0, "xmax": 5.0}],
         "define": {"coords": ["x - y"], "weight": "select(x > 0, 2.0, 0.5) * (1 + z*z)"}},
        {"axes": [{"nbins": 30, "xmin": -1.0, "xmax": 1.0}, {"nbins": 30, "xmin": 0.0, "xmax": 1.0},
                  {"nbins": 20, "xmin": -4.0, "xmax": 4.0}],
         "define": {"filter": "x*x + y*y > 0.01",
                    "coords": ["x / sqrt(x*x + y*y)", "abs(y) / sqrt(x*x + y*y)", "z"]}},
    ]
    plan, _ = _run(hg, names, cols, members)
    assert all(plan.info(i)["in_lds"] for i in range(len(members)))


def test_default_defines_equal_separate_fills(hg):
    """No programs: each member reads columns 0..d-1; counts equal a plain
    hist_fill of the same columns, bit for bit."""
    import torch
    names = ["x", "y"]
    cols = _columns(777_777, 83, 2)
    axes = [[{"nbins": 80, "xmin": -3.0, "xmax": 3.0}],
            [{"nbins": 80, "xmin": -3.0, "xmax": 3.0}, {"nbins": 25, "xmin": -3.0, "xmax": 3.0}]]
    hists = [hg.Hist(a) for a in axes]
    plan = hg.Multi(hists, None, names)
    t = [dev(c) for c in cols]
    plan.fill(t)
    for h, a in zip(hists, axes):
        ref = hg.Hist(a)
        ref.fill(t[:len(a)])
        s, _, e = h.read()
        rs, _, re_ = ref.read()
        assert e == re_ == len(cols[0])
        assert_bins_equal(s, rs, "counts")
        assert_stats_close(h.stats(), ref.stats(), oracle.stats_abs(a, cols[:len(a)], None))
    torch.cuda.synchronize()


def test_member_larger_than_lds_uses_global_atomics(hg):
    names = ["x", "y"]
    cols = _columns(500_001, 84, 2)
    members = [
        {"axes": [{"nbins": 1000, "xmin": -4.0, "xmax": 4.0}, {"nbins": 1000, "xmin": -4.0, "xmax": 4.0}],
         "define": {"weight": "1 + x*x"}},
        {"axes": [{"nbins": 2000, "xmin": -4.0, "xmax": 4.0}], "define": {"coords": ["y"]}},
    ]
    plan, _ = _run(hg, names, cols, members)
    assert not plan.info(0)["in_lds"] and plan.info(1)["in_lds"]


def test_fp32_columns_and_accumulation_across_passes(hg):
    import torch
    names = ["x", "w"]
    rng = np.random.default_rng(85)
    n = 300_007
    cols = [rng.gamma(2.0, 10.0, n), rng.lognormal(0.0, 1.0, n)]
    members = [
        {"axes": [{"nbins": 1000, "xmin": 0.0, "xmax": 100.0}], "define": {"weight": "w"}},
        {"axes": [{"nbins": 64, "edges": np.linspace(0.0, 64.0, 65) ** 1.1}],
         "define": {"filter": "w > 0.5", "coords": ["x / w"]}},
    ]
    _run(hg, names, cols, members, dtype=torch.float32, fills=2)


def test_defined_coordinates_round_like_the_oracle(hg):
    """Coordinates landing exactly on edges: x/3*3, sqrt(x*x) and (x+y)-y on
    integers and thirds, with edges at those values; a single rounding
    difference moves an event to the neighbouring bin."""
    names = ["a", "b"]
    k = np.arange(-600, 601, dtype=np.float64)
    a = np.concatenate([k / 3.0, k, k * 0.1])
    b = np.concatenate([np.full(k.size, 3.0), np.full(k.size, 1e16), np.full(k.size, 0.7)])
    edges = np.unique(np.concatenate([k / 3.0, k * 0.1]))
    edges = edges[(edges >= -200) & (edges <= 200)]
    members = [
        {"axes": [{"nbins": len(edges) - 1, "edges": edges}], "define": {"coords": ["a / b * b"]}},
        {"axes": [{"nbins": len(edges) - 1, "edges": edges}], "define": {"coords": ["sqrt(a*a)"]}},
        {"axes": [{"nbins": len(edges) - 1, "edges": edges}], "define": {"coords": ["(a + b) - b"]}},
        {"axes": [{"nbins": 400, "xmin": -200.0, "xmax": 200.0}], "define": {"coords": ["min(a, b) - max(a, -b)"]}},
    ]
    _run(hg, names, [a, b], members)


def test_multi_fill_replays_from_a_graph(hg):
    import torch
    names = ["x", "y"]
    cols = _columns(400_000, 86, 2)
    axes = [{"nbins": 120, "xmin": -4.0, "xmax": 4.0}]
    defs = [{"filter": "y > -0.5", "coords": ["x + y"]}]
    h = hg.Hist(axes)
    plan = hg.Multi([h], defs, names)
    t = [dev(c) for c in cols]
    s = torch.cuda.Stream()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.stream(s):
        plan.fill(t, stream=s)          # first run outside capture
        torch.cuda.synchronize()
        with torch.cuda.graph(g, stream=s):
            plan.fill(t, stream=s)
    for r in range(3):
        g.replay()
        torch.cuda.synchronize()
        x = torch.zeros(1000, device="cuda")
        x += 1.0                         # eager work between replays
    ops = {"filter": hg.parse(defs[0]["filter"], names), "coords": [hg.parse("x + y", names)]}
    _compare(h, axes, ops, [np.concatenate([c] * 4) for c in cols])


def test_invalid_programs_are_rejected(hg):
    h = hg.Hist([{"nbins": 10, "xmin": 0.0, "xmax": 1.0}])
    bad = [
        [(E.ADD, 0, 0.0)],                                     # stack underflow
        [(E.COL, 0, 0.0), (E.COL, 0, 0.0)],                    # leaves two values
        [(E.COL, 5, 0.0)],                                     # column out of range
        [(99, 0, 0.0)],                                        # unknown operation
        [(E.CONST, 0, 1.0)] * 7 + [(E.ADD, 0, 0.0)] * 6,       # deeper than 6
    ]
    for ops in bad:
        with pytest.raises(hg.HistError):
            hg.Multi([h], [{"coords": [ops]}], ["x", "y"])
    with pytest.raises(hg.HistError):
        hg.Multi([h, h], None, ["x"])                          # repeated handle


def test_multi_holds_its_histograms(hg):
    """hist_destroy refuses a handle a live multi-fill set holds."""
    h = hg.Hist([{"nbins": 10, "xmin": 0.0, "xmax": 1.0}])
    plan = hg.Multi([h], None, ["x"])
    lib = hg._lib.load()
    assert lib.hist_destroy(h.handle) == hg._lib.HIST_EINVAL
    plan.close()
    h.close()
