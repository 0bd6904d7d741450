"""Pins for the oracle's linear search (Section 2.2, Eqs. 5-6).

Independent references: the closed-form box least squares of white noise
(mean out-of-transit minus mean in-transit, with its variance), weighted
means for a heteroscedastic diagonal, exact rational arithmetic and 50-digit
brute force for small dense problems, the Frisch-Waugh-Lovell identity,
invariances of the fit, the Cauchy-Schwarz recovery of a noiseless box, and
the null distribution of depth/sigma.
"""
import math
from fractions import Fraction

import mpmath
import numpy as np
import pytest
import scipy.stats

from oracle import gp, linear
from synth import lattice_box_mask


def _lattice_with_gap(n, after, missing):
    steps = np.ones(n, dtype=np.int64)
    steps[0] = 0
    steps[after + 1] += missing
    return np.cumsum(steps)


def test_box_range_matches_enumeration():
    lat = _lattice_with_gap(40, 17, 6)
    for n_dur in (1, 2, 3, 4, 7):
        for slot in range(-3, int(lat[-1]) + 4):
            lo, hi = linear.box_sample_range(lat, slot, n_dur)
            members = [n for n in range(40) if slot - n_dur // 2 <= lat[n] < slot - n_dur // 2 + n_dur]
            if members:
                assert (lo, hi) == (members[0], members[-1] + 1)
                assert members == list(range(lo, hi))
            else:
                assert lo == hi
            np.testing.assert_array_equal(lattice_box_mask(lat, slot, n_dur).nonzero()[0], members)


def test_white_noise_reduces_to_box_least_squares():
    rng = np.random.default_rng(1)
    n, s = 120, 2e-3
    lat = _lattice_with_gap(n, 60, 5)
    f = 1.0 + s * rng.standard_normal(n)
    A = np.ones((n, 1))
    L = np.eye(n) * s
    out = linear.linear_search(f, A, L, lat, [1, 4, 9])
    checked = 0
    for j, nd in enumerate([1, 4, 9]):
        for i in range(int(lat[-1]) + 1):
            m = lattice_box_mask(lat, i, nd)
            n_in = int(m.sum())
            if n_in == 0:
                assert out["valid"][j, i] == 0 and out["var"][j, i] == np.inf
                continue
            depth = f[~m].mean() - f[m].mean()
            var = s * s * (1.0 / n_in + 1.0 / (n - n_in))
            assert out["valid"][j, i] == 1
            assert out["depth"][j, i] == pytest.approx(depth, rel=1e-9, abs=1e-13)
            assert out["var"][j, i] == pytest.approx(var, rel=1e-10)
            checked += 1
    assert checked > 300


def test_heteroscedastic_diagonal_gives_weighted_means():
    rng = np.random.default_rng(2)
    n = 80
    lat = np.arange(n)
    sig = rng.uniform(5e-4, 3e-3, n)
    f = 1.0 + sig * rng.standard_normal(n)
    L = np.diag(sig)
    out = linear.linear_search(f, np.ones((n, 1)), L, lat, [5])
    w = 1.0 / sig ** 2
    for i in range(n):
        m = lattice_box_mask(lat, i, 5)
        mean_in = (w[m] * f[m]).sum() / w[m].sum()
        mean_out = (w[~m] * f[~m]).sum() / w[~m].sum()
        assert out["depth"][0, i] == pytest.approx(mean_out - mean_in, rel=1e-9, abs=1e-13)
        assert out["var"][0, i] == pytest.approx(1 / w[m].sum() + 1 / w[~m].sum(), rel=1e-10)


def _frac_solve(M, B):
    """Exact Gauss-Jordan solve of M X = B over the rationals."""
    n = len(M)
    aug = [list(M[r]) + list(B[r]) for r in range(n)]
    for c in range(n):
        piv = next(r for r in range(c, n) if aug[r][c] != 0)
        aug[c], aug[piv] = aug[piv], aug[c]
        pv = aug[c][c]
        aug[c] = [x / pv for x in aug[c]]
        for r in range(n):
            if r != c and aug[r][c] != 0:
                fac = aug[r][c]
                aug[r] = [x - fac * y for x, y in zip(aug[r], aug[c])]
    return [row[n:] for row in aug]


def test_exact_rational_gls_small_dense():
    # K = 4 I + u u^T + v v^T with small integers: SPD and exactly rational
    n = 9
    u = [1, 2, 0, -1, 1, 3, 0, 1, -2]
    v = [0, 1, 1, 2, -1, 0, 2, 1, 1]
    Kq = [[Fraction(4 if r == c else 0) + u[r] * u[c] + v[r] * v[c] for c in range(n)] for r in range(n)]
    fq = [Fraction(x) for x in (3, -1, 4, 1, -5, 9, 2, -6, 5)]
    lat = np.array([0, 1, 2, 4, 5, 6, 7, 9, 10])  # two one-slot gaps
    Aq = [[Fraction(1), Fraction(r)] for r in range(n)]
    K = np.array([[float(x) for x in row] for row in Kq])
    A = np.array([[float(x) for x in row] for row in Aq])
    f = np.array([float(x) for x in fq])
    L = gp.cholesky(K)
    durs = [1, 2, 3]
    out = linear.linear_search(f, A, L, lat, durs)
    # trend-only chi2 for dll
    Kinv_f = [r[0] for r in _frac_solve(Kq, [[x] for x in fq])]

    def gls(X):
        KiX = _frac_solve(Kq, [list(r) for r in X])
        M = len(X[0])
        G = [[sum(X[n_][a] * KiX[n_][b] for n_ in range(n)) for b in range(M)] for a in range(M)]
        rhs = [[sum(X[n_][a] * Kinv_f[n_] for n_ in range(n))] for a in range(M)]
        w = [r[0] for r in _frac_solve(G, rhs)]
        cov = _frac_solve(G, [[Fraction(int(a == b)) for b in range(M)] for a in range(M)])
        r = [fq[n_] - sum(X[n_][a] * w[a] for a in range(M)) for n_ in range(n)]
        Kir = [x[0] for x in _frac_solve(Kq, [[x] for x in r])]
        chi2 = sum(a * b for a, b in zip(r, Kir))
        return w, cov, chi2

    _, _, chi2_0 = gls(Aq)
    for j, nd in enumerate(durs):
        for i in range(int(lat[-1]) + 1):
            m = lattice_box_mask(lat, i, nd)
            if not m.any():
                assert out["valid"][j, i] == 0
                continue
            X = [Aq[r] + [Fraction(-1 if m[r] else 0)] for r in range(n)]
            w, cov, chi2 = gls(X)
            assert out["depth"][j, i] == pytest.approx(float(w[-1]), rel=1e-11, abs=1e-12)
            assert out["var"][j, i] == pytest.approx(float(cov[-1][-1]), rel=1e-11)
            assert out["dll"][j, i] == pytest.approx(float((chi2_0 - chi2) / 2), rel=1e-9, abs=1e-11)


def test_mpmath_brute_force_sho_kernel():
    mpmath.mp.dps = 50
    rng = np.random.default_rng(3)
    lat = _lattice_with_gap(36, 20, 3)
    t = lat * (2 / 1440)
    th = {"amp": 0.01, "omega": 40.0, "q": 5.0, "sigma_w": 1e-3}
    K = gp.covariance(t, th)
    A = np.stack([np.ones(36), (t - t.mean()) / np.ptp(t), ((t - t.mean()) / np.ptp(t)) ** 2], 1)
    f = A @ [1.0, 2e-3, -1e-3] + np.linalg.cholesky(K) @ rng.standard_normal(36)
    L = gp.cholesky(K)
    durs = [2, 5]
    out = linear.linear_search(f, A, L, lat, durs)
    Km = mpmath.matrix(K.tolist())
    fm = mpmath.matrix(f.tolist())

    def gls(X):
        Xm = mpmath.matrix(X.tolist())
        KiX = mpmath.matrix(Xm.rows, Xm.cols)
        for c in range(Xm.cols):  # lu_solve takes one right-hand side at a time
            col = mpmath.lu_solve(Km, Xm[:, c])
            for r in range(Xm.rows):
                KiX[r, c] = col[r]
        Kif = mpmath.lu_solve(Km, fm)
        G = Xm.T * KiX
        w = mpmath.lu_solve(G, Xm.T * Kif)
        cov = G ** -1
        r = fm - Xm * w
        chi2 = (r.T * mpmath.lu_solve(Km, r))[0]
        return w, cov, chi2

    _, _, chi2_0 = gls(A)
    for j, nd in enumerate(durs):
        for i in range(0, int(lat[-1]) + 1, 3):
            m = lattice_box_mask(lat, i, nd)
            if not m.any():
                continue
            X = np.concatenate([A, -m[:, None].astype(float)], 1)
            w, cov, chi2 = gls(X)
            M = X.shape[1]
            assert out["depth"][j, i] == pytest.approx(float(w[M - 1]), rel=1e-8, abs=1e-12)
            assert out["var"][j, i] == pytest.approx(float(cov[M - 1, M - 1]), rel=1e-9)
            assert out["dll"][j, i] == pytest.approx(float((chi2_0 - chi2) / 2), rel=1e-7, abs=1e-9)


def _sho_problem(n=150, seed=4, gap=True):
    rng = np.random.default_rng(seed)
    lat = _lattice_with_gap(n, n // 2, 7) if gap else np.arange(n)
    t = lat * (2 / 1440)
    th = {"amp": 0.008, "omega": 25.0, "q": 5.0, "sigma_w": 8e-4}
    K = gp.covariance(t, th)
    x = (t - t.mean()) / np.ptp(t)
    A = np.stack([np.ones(n), x, x * x], 1)
    f = A @ [1.0, 1e-3, -5e-4] + np.linalg.cholesky(K) @ rng.standard_normal(n)
    return lat, K, A, f


def test_fwl_identity_dll_equals_half_snr_squared():
    lat, K, A, f = _sho_problem()
    out = linear.linear_search(f, A, gp.cholesky(K), lat, [3, 8])
    v = out["valid"].astype(bool)
    fwl = 0.5 * out["depth"][v] ** 2 / out["var"][v]
    np.testing.assert_allclose(out["dll"][v], fwl, rtol=1e-7, atol=1e-9)


def test_invariances():
    lat, K, A, f = _sho_problem(seed=5)
    L = gp.cholesky(K)
    base = linear.linear_search(f, A, L, lat, [4])
    v = base["valid"].astype(bool)
    # trend added to the flux is absorbed by the trend columns
    shifted = linear.linear_search(f + A @ [0.3, -0.02, 0.01], A, L, lat, [4])
    np.testing.assert_allclose(shifted["depth"][v], base["depth"][v], rtol=1e-6, atol=1e-12)
    np.testing.assert_allclose(shifted["dll"][v], base["dll"][v], rtol=1e-5, atol=1e-7)
    # flux scaled by s: depth x s, dll x s^2, var unchanged
    s = 3.0
    sc = linear.linear_search(s * f, A, L, lat, [4])
    np.testing.assert_allclose(sc["depth"][v], s * base["depth"][v], rtol=1e-9, atol=1e-13)
    np.testing.assert_allclose(sc["dll"][v], s * s * base["dll"][v], rtol=1e-7, atol=1e-9)
    np.testing.assert_allclose(sc["var"][v], base["var"][v], rtol=1e-12)
    # covariance scaled by c^2: var x c^2, dll / c^2, depth unchanged
    c = 0.5
    kc = linear.linear_search(f, A, c * L, lat, [4])
    np.testing.assert_allclose(kc["var"][v], c * c * base["var"][v], rtol=1e-12)
    np.testing.assert_allclose(kc["dll"][v], base["dll"][v] / (c * c), rtol=1e-7, atol=1e-9)
    np.testing.assert_allclose(kc["depth"][v], base["depth"][v], rtol=1e-9, atol=1e-13)


def test_noiseless_injection_recovered_exactly():
    lat, K, A, _ = _sho_problem(seed=6)
    L = gp.cholesky(K)
    durs = [3, 6, 9]
    true_j, true_i, delta = 1, 40, 1.7e-3
    f = A @ [1.0, 1e-3, -5e-4] - delta * lattice_box_mask(lat, true_i, durs[true_j])
    out = linear.linear_search(f, A, L, lat, durs)
    assert out["depth"][true_j, true_i] == pytest.approx(delta, rel=1e-8)
    flat = np.argmax(np.where(out["valid"] == 1, out["dll"], -np.inf))
    assert np.unravel_index(flat, out["dll"].shape) == (true_j, true_i)
    d = out["dll"].copy()
    d[true_j, true_i] = -np.inf
    assert d.max() < out["dll"][true_j, true_i] * (1 - 1e-6)


def test_null_calibration_depth_over_sigma_is_standard_normal():
    rng = np.random.default_rng(11)
    lat, K, A, _ = _sho_problem(n=90, seed=7, gap=False)
    L = gp.cholesky(K)
    cells = [(0, 20), (1, 55)]
    z, ll = [], []
    for _ in range(400):
        f = A @ [1.0, 0.0, 0.0] + L @ rng.standard_normal(90)
        out = linear.linear_search(f, A, L, lat, [4, 10], cells=cells)
        z.extend(out["depth"] / np.sqrt(out["var"]))
        ll.extend(2 * out["dll"])
    assert scipy.stats.kstest(z, "norm").pvalue > 1e-3
    assert scipy.stats.kstest(ll, scipy.stats.chi2(1).cdf).pvalue > 1e-3


def test_lnl0_is_eq5_of_trend_only_fit():
    lat, K, A, f = _sho_problem(n=60, seed=8)
    L = gp.cholesky(K)
    out = linear.linear_search(f, A, L, lat, [3])
    Ki = np.linalg.inv(K)
    w = np.linalg.solve(A.T @ Ki @ A, A.T @ Ki @ f)
    r = f - A @ w
    _, ld = np.linalg.slogdet(K)
    ref = -0.5 * r @ Ki @ r - 0.5 * ld - 0.5 * 60 * math.log(2 * math.pi)
    assert out["lnl0"] == pytest.approx(ref, rel=1e-9)


def test_box_in_the_span_of_the_trend_is_invalid():
    """A box over every sample equals minus the constant trend column: X^T K^-1 X is singular and the
    cell is invalid, whatever the rounding of its last pivot. A box that leaves one sample out is not in
    the span and stays valid, with the exactly determined fit of that case (depth = difference of the
    two means weighted by K)."""
    rng = np.random.default_rng(4)
    n = 6
    t = np.arange(n) * 0.01
    theta = {"amp": 0.01, "omega": 8.0, "q": 3.0, "sigma_w": 1e-3}
    L = gp.cholesky(gp.covariance(t, theta))
    f = 1.0 + rng.normal(0, 1e-3, n)
    A = np.ones((n, 1))
    lattice = np.arange(n)
    out = linear.linear_search(f, A, L, lattice, [n, n - 1], cells=[(0, n // 2), (1, (n - 1) // 2)])
    assert out["valid"].tolist() == [0, 1]
    assert out["var"][0] == np.inf and out["dll"][0] == 0.0 and out["depth"][0] == 0.0
    assert np.isfinite(out["var"][1]) and out["var"][1] > 0
