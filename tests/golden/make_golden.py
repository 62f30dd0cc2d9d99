"""Writes the stored expected values under tests/golden/ by calling only the
CPU oracle (``oracle/``).  Run from the repository root:

    python tests/golden/make_golden.py

Each fixture stores its inputs as float.hex strings (bit exact, NaN and inf
included) and the oracle's outputs.
"""
import json
import os
import sys

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import oracle  # noqa: E402
import synth  # noqa: E402

HERE = os.path.dirname(os.path.abspath(__file__))


def _hex(a):
    return [float(v).hex() for v in np.asarray(a, dtype=np.float64)]


def findbin_special_values():
    """Find-bin of adversarial coordinates (every edge and its two floating
    point neighbours each side, +-inf, NaN, +-0, denormals, +-max) on a fixed
    axis and a variable axis; Sec. 3.1 step (1), lower-edge inclusive."""
    out = {"citation": "arXiv:2401.13310 Sec. 3.1, find-bin step with underflow/overflow bins",
           "cases": []}
    fixed = {"nbins": 100, "xmin": -5.0, "xmax": 5.0}
    xs = synth.special_values((100, -5.0, 5.0))
    out["cases"].append({"axis": fixed, "x": _hex(xs),
                         "bins": oracle.findbin([fixed], [xs]).tolist()})
    e = synth.log_edges(101)
    var = {"nbins": 100, "edges": _hex(e)}
    xs = synth.special_values(e)
    out["cases"].append({"axis": var, "x": _hex(xs),
                         "bins": oracle.findbin([{"nbins": 100, "edges": e}], [xs]).tolist()})
    return out


def fill_small_2d():
    """A weighted 2D fill of 64 events (mixed fixed/variable axes) with flow
    and NaN coordinates: bin sums, sums of squares, statistics, entries;
    Sec. 3.1 steps (1)-(3)."""
    rng = np.random.default_rng(2024)
    axes = [{"nbins": 4, "xmin": -1.0, "xmax": 1.0},
            {"nbins": 3, "edges": np.array([-1.0, -0.25, 0.5, 1.0])}]
    x = np.concatenate([rng.uniform(-1.2, 1.2, 60), [np.nan, 1.0, -1.0, np.inf]])
    y = np.concatenate([rng.uniform(-1.2, 1.2, 60), [0.0, 0.5, -np.inf, -0.25]])
    w = rng.uniform(0.25, 2.0, 64)
    o = oracle.Oracle(axes)
    o.fill([x, y], w)
    sumw, sumw2, stats, entries = o.read()
    return {"citation": "arXiv:2401.13310 Sec. 3.1 steps (1)-(3), Sec. 3.2 statistics",
            "axes": [axes[0], {"nbins": 3, "edges": _hex(axes[1]["edges"])}],
            "x": _hex(x), "y": _hex(y), "w": _hex(w),
            "sumw": _hex(sumw), "sumw2": _hex(sumw2), "stats": _hex(stats),
            "entries": entries}


def main():
    for name, fn in [("findbin_special_values.json", findbin_special_values),
                     ("fill_small_2d.json", fill_small_2d)]:
        with open(os.path.join(HERE, name), "w") as f:
            json.dump(fn(), f, indent=1)
            f.write("\n")


if __name__ == "__main__":
    main()
