"""Pins of the CPU oracle against facts the paper and mathematics fix.

None of these checks retypes the oracle's code: they use brute force written
independently here, numpy's own search, exact rational arithmetic
(``fractions.Fraction``), ``math.fsum`` (exactly rounded sums), closed forms
and invariants.  Paper references are to arXiv:2401.13310.
"""
import math
from fractions import Fraction

import numpy as np
import pytest

import oracle
import synth


# ---------------------------------------------------------------- find bin ----

def brute_variable(x, edges):
    """Sec. 3.1 variable bins, lower-edge inclusive: walk the edges."""
    if math.isnan(x):
        return len(edges)          # every !(x < e) holds
    b = 0
    for e in edges:
        if x >= e:
            b += 1
        else:
            break
    return b


def exact_uniform_floor(x, nbins, lo, hi):
    """floor(nbins*(x-lo)/(hi-lo)) in exact rational arithmetic."""
    q = Fraction(nbins) * (Fraction(x) - Fraction(lo)) / (Fraction(hi) - Fraction(lo))
    return math.floor(q), q


def test_variable_matches_bruteforce_tiny():
    rng = np.random.default_rng(11)
    for nb in [1, 2, 3, 7, 16]:
        e = np.sort(rng.uniform(-2, 2, nb + 1))
        xs = np.concatenate([synth.special_values(e), rng.uniform(-3, 3, 200)])
        for x in xs:
            assert oracle.bin_variable(x, e) == brute_variable(float(x), e), (nb, x)
            assert oracle.bin_variable_count(x, e) == brute_variable(float(x), e), (nb, x)


def test_variable_matches_searchsorted_right():
    e = synth.log_edges(100_000)
    rng = np.random.default_rng(12)
    x = np.concatenate([synth.special_values(e)[:-9], rng.exponential(1.0, 200_000)])
    x = x[~np.isnan(x)]
    got = oracle.findbin([{"nbins": e.size - 1, "edges": e}], [x])
    want = np.searchsorted(e, x, side="right")
    assert np.array_equal(got, want.astype(np.int32))


def test_variable_special_cases():
    e = np.array([0.0, 1.0, 2.5, 4.0])
    n = 3
    assert oracle.bin_variable(0.0, e) == 1                           # x = e_0 -> first bin
    assert oracle.bin_variable(4.0, e) == n + 1                       # x = e_n -> overflow
    for i in range(n + 1):
        assert oracle.bin_variable(e[i], e) == i + 1                  # lower edge inclusive
        assert oracle.bin_variable(np.nextafter(e[i], -np.inf), e) == i
    assert oracle.bin_variable(-np.inf, e) == 0
    assert oracle.bin_variable(np.inf, e) == n + 1
    assert oracle.bin_variable(np.nan, e) == n + 1
    assert oracle.bin_variable(-0.0, e) == 1                           # -0 == e_0


def test_uniform_dyadic_exact():
    # min = 0, max = nbins: every integer x is a bin's lower edge -> bin x+1
    for nb in [1, 5, 100, 1000]:
        for x in range(nb):
            assert oracle.bin_uniform(float(x), nb, 0.0, float(nb)) == x + 1
        assert oracle.bin_uniform(float(nb), nb, 0.0, float(nb)) == nb + 1
    # [0, 1) with 2^k bins: j / 2^k is exact
    for k in [0, 3, 10]:
        nb = 1 << k
        for j in range(nb):
            assert oracle.bin_uniform(j / nb, nb, 0.0, 1.0) == j + 1
            assert oracle.bin_uniform(np.nextafter(j / nb, -np.inf), nb, 0.0, 1.0) == max(j, 0)


def test_uniform_midpoints_and_flow():
    for nb, lo, hi in [(100, -5.0, 5.0), (10_000, 0.0, 100.0), (37, -1.3, 2.9)]:
        width = (hi - lo) / nb
        for j in range(nb):
            assert oracle.bin_uniform(lo + (j + 0.5) * width, nb, lo, hi) == j + 1
        assert oracle.bin_uniform(np.nextafter(lo, -np.inf), nb, lo, hi) == 0
        assert oracle.bin_uniform(lo, nb, lo, hi) == 1
        assert oracle.bin_uniform(hi, nb, lo, hi) == nb + 1
        assert oracle.bin_uniform(np.nextafter(hi, -np.inf), nb, lo, hi) == nb
        assert oracle.bin_uniform(np.nan, nb, lo, hi) == nb + 1
        assert oracle.bin_uniform(np.inf, nb, lo, hi) == nb + 1
        assert oracle.bin_uniform(-np.inf, nb, lo, hi) == 0


def test_uniform_against_exact_rational():
    """The binary64 formula is within one bin of the exact real formula, and
    equal to it whenever the exact quotient is not within 1e-9 of an integer."""
    rng = np.random.default_rng(13)
    cases = [(100, -5.0, 5.0), (1000, 0.0, 1.0), (10_000, 0.0, 100.0), (97, -3.7, 11.1)]
    for nb, lo, hi in cases:
        xs = np.concatenate([synth.special_values((nb, lo, hi))[:-9],
                             rng.uniform(lo, hi, 3000)])
        for x in xs:
            x = float(x)
            b = oracle.bin_uniform(x, nb, lo, hi)
            if x < lo:
                assert b == 0
                continue
            if x >= hi:
                assert b == nb + 1
                continue
            f, q = exact_uniform_floor(x, nb, lo, hi)
            exact_bin = min(1 + f, nb)
            assert abs(b - exact_bin) <= 1, (x, b, exact_bin)
            frac = q - f
            if Fraction(1, 10**9) < frac < 1 - Fraction(1, 10**9):
                assert b == exact_bin, (x, b, exact_bin)


def test_uniform_monotone():
    rng = np.random.default_rng(14)
    for nb, lo, hi in [(100, -5.0, 5.0), (1000, 0.0, 1.0), (100, -4.0, 4.0)]:
        x = np.sort(rng.uniform(lo - 1, hi + 1, 100_000))
        b = oracle.findbin([{"nbins": nb, "xmin": lo, "xmax": hi}], [x])
        assert np.all(np.diff(b) >= 0)


def test_global_bin_round_trip():
    axes = [{"nbins": 3, "xmin": 0, "xmax": 1}, {"nbins": 2, "xmin": 0, "xmax": 1},
            {"nbins": 4, "edges": np.array([0, 1, 2, 3, 4.0])}]
    n = [a["nbins"] + 2 for a in axes]
    seen = set()
    for b2 in range(n[2]):
        for b1 in range(n[1]):
            for b0 in range(n[0]):
                g = oracle.global_bin(axes, [b0, b1, b2])
                assert g % n[0] == b0
                assert (g // n[0]) % n[1] == b1
                assert g // (n[0] * n[1]) == b2
                seen.add(g)
    assert seen == set(range(n[0] * n[1] * n[2]))
    assert oracle.global_bin(axes[:1], [2]) == 2
    assert oracle.global_bin(axes[:2], [1, 3]) == 1 + 5 * 3


# --------------------------------------------------------------- fill / stats --

def brute_fill(axes, coords, w):
    """Pure-Python Sec. 3.1 steps (1)-(3), exact sums via math.fsum."""
    d = len(axes)
    n = len(coords[0])
    sizes = [a["nbins"] + 2 for a in axes]
    T = int(np.prod(sizes))
    terms_w = [[] for _ in range(T)]
    terms_w2 = [[] for _ in range(T)]
    nst = 2 + 2 * d + d * (d - 1) // 2
    st = [[] for _ in range(nst)]
    for i in range(n):
        x = [float(coords[a][i]) for a in range(d)]
        wi = 1.0 if w is None else float(w[i])
        bs = []
        for a, ax in enumerate(axes):
            if ax.get("edges") is not None:
                bs.append(brute_variable(x[a], ax["edges"]))
            else:
                xv, lo, hi, nb = x[a], ax["xmin"], ax["xmax"], ax["nbins"]
                if xv < lo:
                    bs.append(0)
                elif not xv < hi:
                    bs.append(nb + 1)
                else:
                    bs.append(min(nb, 1 + int(nb * (xv - lo) / (hi - lo))))
        g, mul = 0, 1
        for a in range(d):
            g += bs[a] * mul
            mul *= sizes[a]
        terms_w[g].append(wi)
        terms_w2[g].append(wi * wi)
        if all(1 <= bs[a] <= axes[a]["nbins"] for a in range(d)):
            k = 0
            st[k].append(wi); k += 1
            st[k].append(wi * wi); k += 1
            for a in range(d):
                st[k].append(wi * x[a]); k += 1
                st[k].append(wi * x[a] * x[a]); k += 1
                for c in range(a):
                    st[k].append(wi * x[c] * x[a]); k += 1
    return (np.array([math.fsum(t) for t in terms_w]),
            np.array([math.fsum(t) for t in terms_w2]),
            np.array([math.fsum(t) for t in st]), n)


def _tiny_cases():
    rng = np.random.default_rng(15)
    e = np.sort(rng.uniform(-1, 1, 6))
    axes1 = [{"nbins": 5, "edges": e}]
    axes2 = [{"nbins": 4, "xmin": -1.0, "xmax": 1.0}, {"nbins": 3, "edges": np.array([-1, -0.2, 0.3, 1.0])}]
    axes3 = [{"nbins": 3, "xmin": -1.0, "xmax": 1.0}, {"nbins": 2, "xmin": -0.5, "xmax": 0.7},
             {"nbins": 4, "edges": np.array([-1, -0.5, 0, 0.5, 1.0])}]
    out = []
    for axes in (axes1, axes2, axes3):
        d = len(axes)
        n = 700
        coords = [np.concatenate([rng.uniform(-1.3, 1.3, n - 4), [np.nan, np.inf, -np.inf, 0.0]])
                  for _ in range(d)]
        w = rng.uniform(-0.5, 2.0, n)
        out.append((axes, coords, w))
        out.append((axes, coords, None))
    return out


@pytest.mark.parametrize("case", range(6))
def test_fill_matches_bruteforce_fsum(case):
    axes, coords, w = _tiny_cases()[case]
    o = oracle.Oracle(axes)
    o.fill(coords, w)
    sumw, sumw2, stats, entries = o.read()
    bw, bw2, bst, bn = brute_fill(axes, coords, w)
    assert entries == bn
    # the oracle's compensated sums are within a few ulps of the exactly rounded value
    np.testing.assert_allclose(sumw, bw, rtol=1e-15, atol=1e-15)
    np.testing.assert_allclose(sumw2, bw2, rtol=1e-15, atol=1e-15)
    np.testing.assert_allclose(stats, bst, rtol=1e-14, atol=1e-14)


def test_fill_invariants_plain_1d():
    wl = synth.plain_1d(200_000)
    o = oracle.Oracle(wl["axes"])
    o.fill(wl["coords"], wl["weights"])
    sumw, sumw2, stats, entries = o.read()
    w = wl["weights"]
    x = wl["coords"][0]
    assert entries == x.size
    assert math.isclose(math.fsum(sumw), math.fsum(w), rel_tol=1e-14)
    assert math.isclose(math.fsum(sumw2), math.fsum(w * w), rel_tol=1e-14)
    inside = (x >= -5.0) & (x < 5.0)
    assert math.isclose(stats[0], math.fsum(w[inside]), rel_tol=1e-15)
    assert math.isclose(stats[0], math.fsum(sumw[1:-1]), rel_tol=1e-14)
    assert math.isclose(stats[2], math.fsum(w[inside] * x[inside]), rel_tol=1e-13,
                        abs_tol=1e-12 * math.fsum(np.abs(w * x)))
    assert math.isclose(stats[3], math.fsum((w * x * x)[inside]), rel_tol=1e-14)


def test_unit_weights_integer_counts():
    wl = synth.variable_1d(300_000)
    o = oracle.Oracle(wl["axes"])
    o.fill(wl["coords"])
    sumw, sumw2, stats, entries = o.read()
    assert np.array_equal(sumw, sumw2)
    assert np.all(sumw == np.round(sumw))
    assert sumw.sum() == 300_000 == entries
    b = np.searchsorted(wl["axes"][0]["edges"], wl["coords"][0], side="right")
    assert np.array_equal(sumw, np.bincount(b, minlength=sumw.size).astype(np.float64))
    assert stats[0] == float(np.count_nonzero((b >= 1) & (b <= 99_999)))


def test_midpoint_closed_form():
    """k events on every bin's midpoint: exactly k per interior bin, none in
    flow, and Sum x = k * sum of midpoints (an arithmetic series)."""
    nb, lo, hi, k = 64, 0.0, 16.0, 3       # width 0.25: midpoints exact in binary64
    mids = lo + (np.arange(nb) + 0.5) * 0.25
    x = np.tile(mids, k)
    o = oracle.Oracle([{"nbins": nb, "xmin": lo, "xmax": hi}])
    o.fill([x])
    sumw, sumw2, stats, entries = o.read()
    assert sumw[0] == 0 and sumw[-1] == 0
    assert np.all(sumw[1:-1] == k)
    assert stats[0] == k * nb and stats[1] == k * nb
    # sum of midpoints (j + 1/2)/4 for j = 0..63 = (64*63/2 + 32)/4 = 512
    assert stats[2] == k * 512.0
    # sum of squares: sum_j ((2j+1)/8)^2 = (1/64) * sum_{m odd < 128} m^2 = 64*(4*64^2-1)/3/64
    assert stats[3] == k * (nb * (4 * nb * nb - 1) / 3) / 64.0


def test_uniform_statistical_occupancy():
    nb = 100
    n = 500_000
    x = np.random.default_rng(16).uniform(0.0, 1.0, n)
    o = oracle.Oracle([{"nbins": nb, "xmin": 0.0, "xmax": 1.0}])
    o.fill([x])
    sumw = o.read()[0]
    mu = n / nb
    assert np.all(np.abs(sumw[1:-1] - mu) < 5 * math.sqrt(mu))
    assert sumw[0] == 0 and sumw[-1] == 0


def test_accumulate_across_fills():
    """Sec. 3.3: the sums of a bulk add to those of earlier bulks."""
    axes, coords, w = _tiny_cases()[2]
    a = oracle.Oracle(axes)
    a.fill(coords, w)
    half = len(coords[0]) // 2
    b = oracle.Oracle(axes)
    b.fill([c[:half] for c in coords], w[:half])
    b.fill([c[half:] for c in coords], w[half:])
    ra, rb = a.read(), b.read()
    for u, v in zip(ra[:3], rb[:3]):
        np.testing.assert_allclose(u, v, rtol=1e-15, atol=1e-15)
    assert ra[3] == rb[3]


def test_stats_layout_3d_cross_terms():
    """Each statistic slot holds the named moment: build events that are all
    inside and check every slot against fsum of the intended product."""
    rng = np.random.default_rng(17)
    axes = [{"nbins": 10, "xmin": -1.0, "xmax": 1.0}] * 3
    x, y, z = (rng.uniform(-0.9, 0.9, 5000) for _ in range(3))
    w = rng.uniform(0.1, 2.0, 5000)
    o = oracle.Oracle(axes)
    o.fill([x, y, z], w)
    st = o.read()[2]
    want = [w, w * w, w * x, w * x * x, w * y, w * y * y, w * x * y,
            w * z, w * z * z, w * x * z, w * y * z]
    for k, t in enumerate(want):
        assert math.isclose(st[k], math.fsum(t), rel_tol=1e-13, abs_tol=1e-12), k


def test_float32_inputs_widen_exactly():
    x32 = np.random.default_rng(18).gamma(2.0, 10.0, 10_000).astype(np.float32)
    axes = synth.precision_axes()
    b32 = oracle.findbin(axes, [x32])
    b64 = oracle.findbin(axes, [x32.astype(np.float64)])
    assert np.array_equal(b32, b64)
