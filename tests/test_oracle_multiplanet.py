"""Pins of the multi-candidate oracle (mask the found transits, search again).

* The window test against rational arithmetic over a wide range of k (with
  the reading's single rounding of k p), including windows wider than half
  the period (overlapping), phases near both ends of the grid, and a slot at
  distance exactly 3 after that rounding (p = 9.6, k = 5).
* The invalid encoding on masked slots, untouched elsewhere, idempotence.
* Two planets injected on the lattice into white noise: the first search
  finds the deeper one at its true period and phase, the search after
  masking finds the other.
"""
from fractions import Fraction

import numpy as np
import pytest

from oracle import gp as ogp, linear as olin, multiplanet as omp, periodic as oper


def _brute(n, p, m, h):
    # the reading's one rounding (of k p), everything else exact, over a wide range of k
    out = np.zeros(n, dtype=bool)
    for i in range(n):
        for k in range(-200, 201):
            if abs(Fraction(i - m) - Fraction(float(k) * p)) < h:
                out[i] = True
                break
    return out


@pytest.mark.parametrize("n,p,m,h", [(60, 7.0, 3, 2), (60, 7.25, 0, 2), (80, 9.6, 9, 3), (50, 4.4, 2, 3),
                                     (40, 3.0, 1, 2), (70, 23.7, 60, 5), (30, 100.0, 29, 4), (45, 5.5, 44, 1)])
def test_window_matches_exact_arithmetic(n, p, m, h):
    got = omp.masked_slots(n, p, m, h)
    np.testing.assert_array_equal(got, _brute(n, p, m, h))


def test_integer_period_window_counts():
    # p = 10, h = 2: slots m + 10 k + {-1, 0, 1} -> 3 per transit
    got = omp.masked_slots(100, 10.0, 4, 2)
    assert got.sum() == 30
    assert all(got[4 + 10 * k + d] for k in range(10) for d in (-1, 0, 1) if 0 <= 4 + 10 * k + d < 100)


def test_mask_encoding_and_idempotence():
    rng = np.random.default_rng(1)
    n_d, n_t = 3, 90
    depth = rng.standard_normal((n_d, n_t))
    var = rng.uniform(1, 2, (n_d, n_t))
    dll = rng.uniform(0, 3, (n_d, n_t))
    valid = np.ones((n_d, n_t), np.uint8)
    a = omp.mask_transit(depth, var, dll, valid, 0.5, 6.5, 2, 3)   # p = 13 slots
    sel = omp.masked_slots(n_t, 13.0, 2, 3)
    assert sel.any() and not sel.all()
    assert np.all(a[0][:, sel] == 0) and np.all(np.isinf(a[1][:, sel])) and np.all(a[2][:, sel] == 0)
    assert np.all(a[3][:, sel] == 0)
    np.testing.assert_array_equal(a[0][:, ~sel], depth[:, ~sel])
    np.testing.assert_array_equal(a[1][:, ~sel], var[:, ~sel])
    np.testing.assert_array_equal(a[3][:, ~sel], 1)
    b = omp.mask_transit(*a, 0.5, 6.5, 2, 3)
    for x, y in zip(a, b):
        np.testing.assert_array_equal(x, y)


def test_two_injected_planets_found_in_turn():
    # white noise (K = sigma^2 I), constant trend; two lattice boxes of different depth
    n, sig = 600, 1e-3
    rng = np.random.default_rng(7)
    lattice = np.arange(n, dtype=np.int64)
    t = lattice * 0.02
    f = 1.0 + sig * rng.standard_normal(n)
    planets = [(4e-3, 5, 47, 4), (2.5e-3, 31, 83, 4)]   # depth, slot0, period in slots, duration
    for dep, s0, pp, nd in planets:
        for c in range(s0, n, pp):
            f[max(0, c - nd // 2):c - nd // 2 + nd] -= dep
    A = np.ones((n, 1))
    L = np.linalg.cholesky(ogp.covariance(t, {"amp": 0.0, "omega": 1.0, "q": 5.0, "sigma_w": sig}))
    durs = np.array([2, 4, 6], np.int32)
    ls = olin.linear_search(f, A, L, lattice, durs)
    periods = np.arange(20.0, 100.0, 1.0) * 0.02   # integer slot periods 20..99
    found = omp.search_planets(ls["depth"], ls["var"], ls["dll"], ls["valid"], 0.02, periods, durs, 2)
    assert len(found) == 2
    (d1, s1, p1, n1), (d2, s2, p2, n2) = planets
    assert found[0]["period"] == pytest.approx(p1 * 0.02) and found[0]["phase"] == s1 % p1
    assert durs[found[0]["dur_index"]] == n1
    assert found[1]["period"] == pytest.approx(p2 * 0.02) and found[1]["phase"] == s2 % p2
    assert found[1]["snr"] > 5
