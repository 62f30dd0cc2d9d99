"""The oracle still reproduces its stored fixtures (regression guard on the
oracle itself); the GPU tests reuse the same fixtures."""
import json
import os

import numpy as np

import oracle

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")


def load(name):
    with open(os.path.join(GOLDEN, name)) as f:
        return json.load(f)


def unhex(v):
    return np.array([float.fromhex(s) for s in v], dtype=np.float64)


def axis_from_json(a):
    if "edges" in a:
        return {"nbins": a["nbins"], "edges": unhex(a["edges"])}
    return dict(a)


def test_findbin_special_values_fixture():
    g = load("findbin_special_values.json")
    for case in g["cases"]:
        ax = axis_from_json(case["axis"])
        got = oracle.findbin([ax], [unhex(case["x"])])
        assert got.tolist() == case["bins"]


def test_fill_small_2d_fixture():
    g = load("fill_small_2d.json")
    o = oracle.Oracle([axis_from_json(a) for a in g["axes"]])
    o.fill([unhex(g["x"]), unhex(g["y"])], unhex(g["w"]))
    sumw, sumw2, stats, entries = o.read()
    assert entries == g["entries"]
    np.testing.assert_array_equal(sumw, unhex(g["sumw"]))
    np.testing.assert_array_equal(sumw2, unhex(g["sumw2"]))
    np.testing.assert_array_equal(stats, unhex(g["stats"]))
