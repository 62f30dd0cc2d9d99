"""The seeded generators: determinism, shapes, dtypes and the recipe facts the
workloads rely on."""
import numpy as np

import synth


def test_deterministic_and_seeded():
    a = synth.plain_1d(1000)
    b = synth.plain_1d(1000)
    assert np.array_equal(a["coords"][0], b["coords"][0])
    assert np.array_equal(a["weights"], b["weights"])
    c = synth.plain_1d(1000, seed=99)
    assert not np.array_equal(a["coords"][0], c["coords"][0])


def test_shapes_and_dtypes():
    wl = synth.plain_1d(5000)
    assert wl["coords"][0].dtype == np.float64 and wl["coords"][0].shape == (5000,)
    assert np.all((wl["weights"] >= 0.5) & (wl["weights"] < 1.5))
    v = synth.variable_1d(1000)
    e = v["axes"][0]["edges"]
    assert e.shape == (100_000,) and v["axes"][0]["nbins"] == 99_999
    assert np.all(np.diff(e) > 0) and e[0] == 1e-3 and e[-1] == 1e3
    assert v["weights"] is None
    c = synth.corr_3d(20_000)
    X = np.stack(c["coords"])
    r = np.corrcoef(X)
    assert np.allclose(r[np.triu_indices(3, 1)], 0.5, atol=0.03)
    xs, ws = next(synth.precision_slices(n=3000, slice_len=1000))
    assert xs.dtype == np.float32 and ws.dtype == np.float32 and xs.shape == (1000,)


def test_precision_slices_cover_n():
    sizes = [x.size for x, _ in synth.precision_slices(n=10_500, slice_len=4096)]
    assert sizes == [4096, 4096, 2308]


def test_batched_members_recipe():
    ms = synth.batched_64(n_scale=1e-3)
    assert len(ms) == 64
    for m in ms:
        d = len(m["axes"])
        assert 1 <= d <= 3 and len(m["coords"]) == d
        T = 1
        for ax in m["axes"]:
            assert ax["nbins"] >= 1
            if "edges" in ax:
                assert ax["edges"].shape == (ax["nbins"] + 1,)
                assert np.all(np.diff(ax["edges"]) > 0)
            T *= ax["nbins"] + 2
        assert T <= 1_100_000
        assert np.all((m["weights"] >= 0) & (m["weights"] < 2))
    full = synth.batched_64(n_scale=0.0)   # draws the same sizes without data
    assert all(len(m["weights"]) == 0 for m in full)


def test_special_values_include_edges_and_neighbours():
    e = np.array([0.0, 0.5, 1.0])
    v = synth.special_values(e, count_near=1)
    assert set(e).issubset(set(v[np.isfinite(v)]))
    assert np.nextafter(0.5, 1.0) in v and np.nextafter(0.5, 0.0) in v
    assert np.isnan(v).sum() == 1
