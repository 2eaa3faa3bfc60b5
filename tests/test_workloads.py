import math

import numpy as np

import workloads as wl


def _distinct(xy):
    k = xy[:, 0].astype(np.int64) * (1 << 31) + xy[:, 1]
    return len(np.unique(k)) == len(k)


def test_zero_sum_exact():
    rng = np.random.default_rng(0)
    for n in (1, 2, 17, 1000, 100_000):
        f = wl.zero_sum_loads(rng.standard_normal(n))
        k = np.rint(f * 2.0 ** 32).astype(np.int64)
        assert np.array_equal(k.astype(np.float64) / 2.0 ** 32, f)   # on the 2^-32 grid
        assert int(k.sum()) == 0                                      # exactly zero sum


def test_small_uniform():
    xy, f = wl.config_small_uniform()
    assert xy.shape == (1000, 2) and xy.dtype == np.int32
    assert xy.min() >= 0 and xy.max() < 256 and _distinct(xy)
    assert np.rint(f * 2.0 ** 32).astype(np.int64).sum() == 0
    xy2, f2 = wl.config_small_uniform()
    assert np.array_equal(xy, xy2) and np.array_equal(f, f2)          # seeded


def test_clusters_small():
    xy, f = wl.config_clusters(n=20_000, n_clusters=8)
    assert len(xy) == 20_000 and _distinct(xy)
    assert xy.min() >= 0 and xy.max() < (1 << 20)


def test_batched_sizes():
    sizes = wl.generators.batched_sizes()
    assert len(sizes) == 512 and sizes.min() >= 1000 and sizes.max() <= 100_000
    assert 0.9e7 < sizes.sum() < 1.4e7


def test_serving_request():
    xy, f, layout = wl.config_serving_request(5, 3, lo=1e2, hi=1e4)
    assert layout in ("uniform", "clusters") and _distinct(xy) and len(xy) == len(f)


def test_sample_targets():
    s = wl.sample_targets(20, 1000, 100)
    assert len(s) == 100 and len(np.unique(s)) == 100 and s.max() < 1000
    assert len(wl.sample_targets(1, 10, 100)) == 10
