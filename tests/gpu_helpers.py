"""Helpers shared by the GPU parity tests: device upload, tolerance checks.

Tolerance (weighted binary64 sums): the GPU adds the same per-event terms as
the oracle in a different order.  Bin sums of non-negative weights must agree
to 1e-12 relative; statistics that can cancel are held to 1e-12 of
max(|value|, sum of |terms|).  Bin indices and unit-weight counts must be
identical.
"""
import math

import numpy as np

REL = 1e-12


def dev(a, dtype=None):
    import torch
    t = torch.from_numpy(np.ascontiguousarray(a))
    if dtype is not None:
        t = t.to(dtype)
    return t.to("cuda")


def _fingerprint(got, want):
    """Where two histograms differ, in terms that tell failure kinds apart:
    events lost (bins only low, total short), events mis-binned (as many
    units gained as lost, total unchanged) or extra events (total long)."""
    d = np.asarray(got, dtype=np.float64) - np.asarray(want, dtype=np.float64)
    hi = np.nonzero(d > 0)[0]
    lo = np.nonzero(d < 0)[0]
    return ("%d bins high (+%.6g), %d bins low (%.6g); total got %.17g want %.17g "
            "(diff %.6g); first high %s, first low %s"
            % (hi.size, float(d[hi].sum()) if hi.size else 0.0, lo.size,
               float(d[lo].sum()) if lo.size else 0.0, math.fsum(np.asarray(got, np.float64)),
               math.fsum(np.asarray(want, np.float64)),
               math.fsum(np.asarray(got, np.float64)) - math.fsum(np.asarray(want, np.float64)),
               hi[:8].tolist(), lo[:8].tolist()))


def assert_bins_equal(got, want, what="bins"):
    got = np.asarray(got)
    want = np.asarray(want)
    assert got.shape == want.shape, what
    bad = np.nonzero(got != want)[0]
    if bad.size:
        i = bad[0]
        raise AssertionError("%s differ at %d of %d places; first at %d: got %d want %d; %s"
                             % (what, bad.size, got.size, i, got[i], want[i],
                                _fingerprint(got, want)))


def assert_sums_close(got, want, rel=REL, what="sums"):
    got = np.asarray(got)
    want = np.asarray(want)
    err = np.abs(got - want)
    lim = rel * np.abs(want)
    bad = np.nonzero(err > lim)[0]
    if bad.size:
        i = bad[0]
        raise AssertionError("%s differ at %d bins; first at %d: got %r want %r (rel %.3g); "
                             "largest rel %.3g; %s"
                             % (what, bad.size, i, got[i], want[i],
                                err[i] / max(abs(want[i]), 1e-300),
                                float(np.max(err[bad] / np.maximum(np.abs(want[bad]), 1e-300))),
                                _fingerprint(got, want)))


def assert_stats_close(got, want, abs_scale, rel=REL):
    for k, (g, o, s) in enumerate(zip(got, want, abs_scale)):
        lim = rel * max(abs(o), s)
        assert abs(g - o) <= lim, "stat %d: got %r want %r (scale %r)" % (k, g, o, s)


def max_rel_err(got, want):
    got = np.asarray(got, dtype=np.float64)
    want = np.asarray(want, dtype=np.float64)
    nz = want != 0
    if not nz.any():
        return 0.0
    return float(np.max(np.abs(got[nz] - want[nz]) / np.abs(want[nz])))
