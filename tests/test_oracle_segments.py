"""Pins of the segmented periodic-search oracle.

* One segment at offset 0 is the plain periodic search exactly.
* Assembly: cells land at their offsets, gap cells are invalid-encoded,
  overlapping segments are rejected.
* Two sectors far apart (a gap of 3000 slots), the same planet injected in
  both on one lattice-periodic train: the combined search finds its period
  and phase, with a higher SNR than either sector alone.
"""
import numpy as np
import pytest

from oracle import gp as ogp, linear as olin, periodic as oper, segments as oseg


def _grid(rng, n_d, n):
    var = rng.uniform(1e-7, 3e-7, (n_d, n))
    depth = rng.standard_normal((n_d, n)) * np.sqrt(var)
    return depth, var, 0.5 * depth ** 2 / var, np.ones((n_d, n), np.uint8)


def test_single_segment_is_the_plain_search():
    rng = np.random.default_rng(3)
    g = _grid(rng, 2, 150)
    periods = np.linspace(5.0, 40.0, 30)
    a = oseg.periodic_search_segments([g], [0], 1.0, periods)
    b = oper.periodic_search(*g, 1.0, periods)
    for k in a:
        np.testing.assert_array_equal(a[k], b[k])


def test_assembly_and_overlap():
    rng = np.random.default_rng(4)
    g1, g2 = _grid(rng, 2, 40), _grid(rng, 2, 30)
    d, v, l, ok = oseg.assemble([g1, g2], [5, 100])
    assert d.shape == (2, 130)
    np.testing.assert_array_equal(d[:, 5:45], g1[0])
    np.testing.assert_array_equal(v[:, 100:130], g2[1])
    gap = np.r_[0:5, 45:100]
    assert np.all(ok[:, gap] == 0) and np.all(np.isinf(v[:, gap])) and np.all(d[:, gap] == 0)
    with pytest.raises(ValueError):
        oseg.assemble([g1, g2], [5, 30])


def test_two_sectors_combine():
    dt, sig = 0.02, 1e-3
    rng = np.random.default_rng(11)
    periods = np.arange(30.0, 120.0, 1.0) * dt
    p_slots, s0, nd, dep = 71, 23, 4, 1.5e-3
    grids, offsets = [], [0, 3400]
    for off in offsets:
        n = 500
        f = 1.0 + sig * rng.standard_normal(n)
        lat = np.arange(n, dtype=np.int64)
        for c in range(s0, off + n, p_slots):
            if c >= off:
                lo = c - off - nd // 2
                f[max(0, lo):max(0, lo + nd)] -= dep
        L = np.linalg.cholesky(ogp.covariance(lat * dt, {"amp": 0.0, "omega": 1.0, "q": 5.0, "sigma_w": sig}))
        ls = olin.linear_search(f, np.ones((n, 1)), L, lat, np.array([4], np.int32))
        grids.append((ls["depth"], ls["var"], ls["dll"], ls["valid"]))
    both = oseg.periodic_search_segments(grids, offsets, dt, periods)
    ip = oper.first_argmax(both["q_snr"])
    assert periods[ip] == pytest.approx(p_slots * dt) and both["best_phase"][ip] == s0
    single = [oper.periodic_search(*g, dt, periods) for g in grids]
    assert both["q_snr"][ip] > max(s["q_snr"].max() for s in single)
