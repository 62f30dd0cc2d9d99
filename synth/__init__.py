"""Seeded synthetic event streams shared by the oracle-side tests and the GPU side.

This module only draws random numbers with numpy's PCG64 (``default_rng``) in a
fixed order; it holds none of the histogramming arithmetic, so both sides of
every parity check receive bit-identical host arrays from it.

The paper (arXiv:2401.13310, Sec. 4.2) measures synthetic single-column
RNTuple datasets of uniform [0, 1] doubles; those files are not available, so
these generators stand in for them with the workload shapes below.  Every
generator takes the event count as an argument so tests can run the same
recipe at small sizes.

Workloads (names used across the repository):
  plain_1d     100 fixed bins on [-5, 5), x ~ N(0,1), w ~ U[0.5,1.5), FP64, seed 0
  variable_1d  1e5 log-spaced edges on [1e-3, 1e3] (99,999 bins), x ~ Exp(1),
               unit weights, FP64, seed 1
  corr_3d      100^3 fixed bins on [-4,4)^3, correlated Gaussian (rho = 0.5),
               unit weights, FP64, seed 2
  batched_64   64 histograms, dims 1..3, log-uniform bins per axis and event
               counts, fixed or variable axes, N(0,1) or U, w ~ U[0,2), seed 3
  precision    1e4 fixed bins on [0, 100), x ~ Gamma(2, 10), w ~ LogNormal(0, 2),
               FP32, streamed in 2^24-event slices, seed 4
  paper_1d     the paper's own benchmark shape (Sec. 4.2): 1000 bins on [0, 1]
               given as an edge array, x ~ U[0, 1], FP64
"""
from __future__ import annotations

import math

import numpy as np

PLAIN_1D_N = 1_000_000
VARIABLE_1D_N = 50_000_000
CORR_3D_N = 20_000_000
PRECISION_N = 200_000_000
PRECISION_SLICE = 1 << 24


def _rng(seed: int) -> np.random.Generator:
    return np.random.default_rng(seed)


def plain_1d(n: int = PLAIN_1D_N, seed: int = 0) -> dict:
    rng = _rng(seed)
    x = rng.normal(0.0, 1.0, n)
    w = rng.uniform(0.5, 1.5, n)
    return {"name": "plain_1d", "axes": [{"nbins": 100, "xmin": -5.0, "xmax": 5.0}],
            "coords": [x], "weights": w}


def log_edges(nedges: int = 100_000, lo_exp: float = -3.0, hi_exp: float = 3.0) -> np.ndarray:
    """10**linspace(lo_exp, hi_exp, nedges): the variable_1d edge array."""
    return 10.0 ** np.linspace(lo_exp, hi_exp, nedges)


def variable_1d(n: int = VARIABLE_1D_N, seed: int = 1, nedges: int = 100_000) -> dict:
    rng = _rng(seed)
    edges = log_edges(nedges)
    x = rng.exponential(1.0, n)
    return {"name": "variable_1d", "axes": [{"nbins": nedges - 1, "edges": edges}],
            "coords": [x], "weights": None}


def corr_3d(n: int = CORR_3D_N, seed: int = 2, rho: float = 0.5, nbins: int = 100) -> dict:
    rng = _rng(seed)
    cov = np.full((3, 3), rho) + (1.0 - rho) * np.eye(3)
    L = np.linalg.cholesky(cov)
    z = rng.standard_normal((3, n))
    X = L @ z
    ax = {"nbins": nbins, "xmin": -4.0, "xmax": 4.0}
    return {"name": "corr_3d", "axes": [dict(ax), dict(ax), dict(ax)],
            "coords": [np.ascontiguousarray(X[0]), np.ascontiguousarray(X[1]),
                       np.ascontiguousarray(X[2])], "weights": None}


def _sorted_edges(rng, nbins: int, lo: float, hi: float) -> np.ndarray:
    """Strictly increasing edges: both endpoints plus nbins-1 sorted U(lo, hi) draws."""
    while True:
        inner = np.sort(rng.uniform(lo, hi, nbins - 1))
        e = np.concatenate([[lo], inner, [hi]])
        if np.all(np.diff(e) > 0):
            return e


def batched_64(seed: int = 3, k: int = 64, n_scale: float = 1.0, bins_scale: float = 1.0,
               n_min: float = 1e4, n_max: float = 1e7) -> list:
    """Members of the batched workload.

    Per member: d ~ U{1,2,3}; per axis nbins = round(exp(U(ln 10, ln 10**(6/d))))
    (the per-axis cap 10**(6/d) keeps every member at <= ~1e6 bins); fixed or
    variable axes 50/50 (variable = both endpoints plus sorted uniform draws);
    x ~ N(0,1) on [-4, 4) or U on [0, 1) 50/50, uniform draws widened by 5%
    each side so the flow bins are hit; n = round(exp(U(ln n_min, ln n_max)));
    w ~ U[0, 2).  ``n_scale`` / ``bins_scale`` shrink the workload for tests.
    """
    rng = _rng(seed)
    plans = []
    for _ in range(k):                     # every member's shape first ...
        d = int(rng.integers(1, 4))
        normal = bool(rng.integers(0, 2))
        lo, hi = (-4.0, 4.0) if normal else (0.0, 1.0)
        axes = []
        for _a in range(d):
            cap = 10.0 ** (6.0 / d)
            nb = int(round(math.exp(rng.uniform(math.log(10.0), math.log(cap)))))
            nb = max(1, int(round(nb * bins_scale)))
            if bool(rng.integers(0, 2)):
                axes.append({"nbins": nb, "edges": _sorted_edges(rng, nb, lo, hi)})
            else:
                axes.append({"nbins": nb, "xmin": lo, "xmax": hi})
        n = int(round(math.exp(rng.uniform(math.log(n_min), math.log(n_max)))))
        plans.append((d, normal, lo, hi, axes, max(0, int(round(n * n_scale)))))
    members = []
    for d, normal, lo, hi, axes, n in plans:   # ... then the event data
        if normal:
            coords = [rng.normal(0.0, 1.0, n) for _a in range(d)]
        else:
            wd = 0.05 * (hi - lo)
            coords = [rng.uniform(lo - wd, hi + wd, n) for _a in range(d)]
        w = rng.uniform(0.0, 2.0, n)
        members.append({"axes": axes, "coords": coords, "weights": w})
    return members


def precision_axes() -> list:
    return [{"nbins": 10_000, "xmin": 0.0, "xmax": 100.0}]


def precision_slices(n: int = PRECISION_N, seed: int = 4, slice_len: int = PRECISION_SLICE):
    """Yields (x, w) float32 slices of the precision workload, drawn in order
    from one generator: x ~ Gamma(shape 2, scale 10), w ~ LogNormal(0, 2)."""
    rng = _rng(seed)
    done = 0
    while done < n:
        m = min(slice_len, n - done)
        x = rng.gamma(2.0, 10.0, m).astype(np.float32)
        w = rng.lognormal(0.0, 2.0, m).astype(np.float32)
        yield x, w
        done += m


def paper_1d(n: int, seed: int = 5, nbins: int = 1000) -> dict:
    rng = _rng(seed)
    edges = np.linspace(0.0, 1.0, nbins + 1)
    x = rng.uniform(0.0, 1.0, n)
    return {"name": "paper_1d", "axes": [{"nbins": nbins, "edges": edges}],
            "coords": [x], "weights": None}


def special_values(edges_or_range, count_near: int = 2) -> np.ndarray:
    """Adversarial coordinates: every edge, its floating-point neighbours, the
    range ends, +-inf, NaN, +-0 and a denormal.  ``edges_or_range`` is an edge
    array or a (nbins, xmin, xmax) tuple (the fixed-width edges are then the
    exact multiples xmin + i*(xmax-xmin)/nbins, rounded once)."""
    if isinstance(edges_or_range, tuple):
        nb, lo, hi = edges_or_range
        e = lo + (hi - lo) * (np.arange(nb + 1, dtype=np.float64) / nb)
        e[-1] = hi
    else:
        e = np.asarray(edges_or_range, dtype=np.float64)
    vals = [e]
    up = e.copy()
    dn = e.copy()
    for _ in range(count_near):
        up = np.nextafter(up, np.inf)
        dn = np.nextafter(dn, -np.inf)
        vals += [up, dn]
    vals.append(np.array([np.inf, -np.inf, np.nan, 0.0, -0.0, 5e-324, -5e-324,
                          np.finfo(np.float64).max, -np.finfo(np.float64).max]))
    return np.concatenate(vals)
