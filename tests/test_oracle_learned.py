"""Pins for the learned-part oracle: the counter-based generator, the GP
sampler, the CNN input, the network's gradient, Adam, and the two
likelihoods of the trend-only model (Eq. 5 with the trend profiled).

Each check is independent of the formula it pins: Philox against its
published known answers; the sampler against the SHO covariance of Appendix
A (itself pinned to the oscillator's stationary solution); the convolution
against SciPy's correlation; the backward pass against central differences;
the Kalman likelihood against the dense Cholesky likelihood (two derivations
of one number) and both against the white-noise closed form.
"""
import json
import math
import os

import numpy as np
import pytest
import scipy.optimize
import scipy.signal
import scipy.stats

from oracle import gp, learned as ol

HERE = os.path.dirname(os.path.abspath(__file__))


def test_philox_known_answers():
    kat = json.load(open(os.path.join(HERE, "golden", "philox4x32_10_kat.json")))
    for v in kat["vectors"]:
        ctr = [int(x, 16) for x in v["ctr"]]
        key = [int(x, 16) for x in v["key"]]
        assert ol.philox4x32_10(ctr, key) == [int(x, 16) for x in v["out"]]


def test_uniforms_and_normals():
    key = [12345, 678]
    u, z = [], []
    for n in range(6000):
        w = ol.philox4x32_10([n, 7, 0, 1], key)
        u.append(ol.uniform01(w[0], w[1]))
        z.extend(ol.normal_pair(w))
    u, z = np.array(u), np.array(z)
    assert u.min() > 0.0 and u.max() < 1.0
    assert scipy.stats.kstest(u, "uniform").pvalue > 1e-3
    assert scipy.stats.kstest(z, "norm").pvalue > 1e-3
    assert abs(z.mean()) < 5 / math.sqrt(z.size) and abs(z.var() - 1) < 5 * math.sqrt(2 / z.size)
    # the extremes of the 52-bit grid stay strictly inside (0, 1)
    assert ol.uniform01(0, 0) == 2.0 ** -53 and ol.uniform01(0xFFFFFFFF, 0xFFFFFFFF) == 1.0 - 2.0 ** -53


def test_sampler_ensemble_covariance_matches_the_sho_kernel():
    # 2000 independent curves of 12 samples with a gap: the empirical covariance of
    # f - 1 must be K = k_SHO + sigma_w^2 I within sampling error
    t = np.array([0.0, 0.01, 0.02, 0.03, 0.05, 0.08, 0.13, 0.21, 0.34, 0.55, 0.56, 0.57])
    th = {"amp": 0.02, "omega": ol.omega_from_rotation(0.4, 5.0), "q": 5.0, "sigma_w": 0.005}
    F = np.array([ol.sample_curve(t, th, 99, c) for c in range(2000)]) - 1.0
    C = F.T @ F / F.shape[0]
    K = gp.covariance(t, th)
    se = np.sqrt((K ** 2 + np.outer(np.diag(K), np.diag(K))) / F.shape[0])  # std error of a Gaussian covariance
    assert np.all(np.abs(C - K) < 5 * se), np.max(np.abs(C - K) / se)


def test_sampler_is_a_function_of_seed_and_curve():
    t = np.arange(20) * 0.01
    th = {"amp": 0.01, "omega": 5.0, "q": 2.0, "sigma_w": 1e-3}
    a = ol.sample_curve(t, th, 5, 3)
    assert np.array_equal(a, ol.sample_curve(t, th, 5, 3))
    assert not np.array_equal(a, ol.sample_curve(t, th, 5, 4))
    assert not np.array_equal(a, ol.sample_curve(t, th, 6, 3))


def test_theta_prior_draws():
    th = [ol.draw_theta(3, c) for c in range(3000)]
    for name in ol.TARGET_KEYS:
        lo, hi = ol.PRIOR[name]
        v = np.log([d[name] for d in th])
        assert v.min() >= math.log(lo) and v.max() <= math.log(hi)
        u = (v - math.log(lo)) / (math.log(hi) - math.log(lo))
        assert scipy.stats.kstest(u, "uniform").pvalue > 1e-3


def test_bin_input_by_hand():
    # 10 samples, 5 bins of width 9/5: bins get samples {0,1}, {2,3}, {4}, {5,6,7}, {8,9}
    t = np.arange(10.0)
    f = np.array([1.0, 1.2, 0.9, 0.9, 1.1, 1.0, 1.0, 1.0, 2.0, 1.0])
    assert list(ol.bin_index(t, 5)) == [0, 0, 1, 1, 2, 2, 3, 3, 4, 4]
    # means 1.1, 0.9, 1.05, 1.0, 1.5 -> median 1.05
    x = ol.bin_input(t, f, 5)
    np.testing.assert_allclose(x, 100 * (np.array([1.1, 0.9, 1.05, 1.0, 1.5]) / 1.05 - 1), rtol=1e-13, atol=1e-12)
    # a gap leaves empty bins at 0 and the median is over the non-empty ones
    t2 = np.array([0.0, 1.0, 2.0, 8.0, 9.0, 10.0])
    f2 = np.array([1.0, 1.0, 2.0, 3.0, 1.0, 1.0])
    x2 = ol.bin_input(t2, f2, 5)
    assert x2[2] == 0.0 and x2[3] == 0.0


def test_standardise_roundtrip():
    th = {"amp": 0.012, "prot": 0.77, "q": 13.0, "sigma_w": 9e-4}
    back = ol.unstandardise(ol.standardise(th))
    for k in th:
        assert back[k] == pytest.approx(th[k], rel=1e-13)


def test_conv1d_matches_scipy_correlation():
    rng = np.random.default_rng(0)
    x = rng.standard_normal((2, 3, 32))
    W = rng.standard_normal((5, 3, 7))
    b = rng.standard_normal(5)
    z = ol.conv1d(x, W, b)
    for bb in range(2):
        for co in range(5):
            full = sum(scipy.signal.correlate(np.pad(x[bb, ci], 3), W[co, ci], mode="valid") for ci in range(3))
            np.testing.assert_allclose(z[bb, co], full[::2][:16] + b[co], rtol=1e-12, atol=1e-12)


def test_cnn_param_count():
    assert ol.n_params() == 512 + 3 * (64 * 64 * 7 + 64) + 4 * 64 + 4


def test_cnn_gradient_against_central_differences():
    rng = np.random.default_rng(1)
    p = ol.init_params(2)
    x = rng.standard_normal((3, 512))
    y = rng.standard_normal((3, 4))
    loss, g = ol.cnn_backward(p, x, y)
    idx = np.concatenate([rng.choice(np.arange(0, 512), 12, replace=False),
                          rng.choice(np.arange(512, ol.n_params()), 40, replace=False),
                          np.arange(ol.n_params() - 260, ol.n_params(), 13)])
    h = 1e-6
    for i in idx:
        e = np.zeros_like(p)
        e[i] = h
        fd = (ol.mse(ol.cnn_forward(p + e, x)[0], y) - ol.mse(ol.cnn_forward(p - e, x)[0], y)) / (2 * h)
        assert fd == pytest.approx(g[i], rel=1e-5, abs=1e-9), i
    assert loss == pytest.approx(ol.mse(ol.cnn_forward(p, x)[0], y), rel=1e-15)


def test_adam_first_step_closed_form():
    p = np.array([1.0, -2.0, 0.5])
    g = np.array([0.3, -1e-3, 4.0])
    p1, m, v = ol.adam_step(p, g, np.zeros(3), np.zeros(3), 1, lr=1e-2)
    # bias-corrected first step: m^ = g, v^ = g^2, so the step is lr * g / (|g| + eps)
    np.testing.assert_allclose(p1, p - 1e-2 * g / (np.abs(g) + 1e-8), rtol=1e-13)


@pytest.mark.parametrize("q", [5.0, 0.5, 0.3])
def test_kalman_likelihood_equals_dense(q):
    rng = np.random.default_rng(3)
    t = np.sort(np.concatenate([np.arange(150) * 0.004, 0.8 + np.arange(100) * 0.004]))
    th = {"amp": 0.01, "omega": 9.0, "q": q, "sigma_w": 1.5e-3}
    f = 1.0 + 0.01 * rng.standard_normal(t.size)
    x = (t - t.mean()) / (np.ptp(t) / 2)
    A = np.column_stack([np.ones_like(x), x, x * x])
    d = ol.nll_dense(t, f, A, th)
    k = ol.nll_kalman(t, f, A, th)
    assert k == pytest.approx(d, rel=1e-10, abs=1e-8)
    assert ol.nll_kalman(t, f, A[:, :0], th) == pytest.approx(ol.nll_dense(t, f, A[:, :0], th), rel=1e-10)


def test_white_noise_likelihood_closed_form_and_optimum():
    rng = np.random.default_rng(4)
    n = 400
    t = np.arange(n) * 0.01
    A = np.column_stack([np.ones(n), t])
    f = 1.0 + 0.02 * t + 0.003 * rng.standard_normal(n)
    w, *_ = np.linalg.lstsq(A, f, rcond=None)
    rss = float(np.sum((f - A @ w) ** 2))
    th = {"amp": 0.0, "omega": 1.0, "q": 1.0, "sigma_w": 0.004}
    closed = rss / (2 * 0.004 ** 2) + n * math.log(0.004) + 0.5 * n * math.log(2 * math.pi)
    assert ol.nll_dense(t, f, A, th) == pytest.approx(closed, rel=1e-12)
    assert ol.nll_kalman(t, f, A, th) == pytest.approx(closed, rel=1e-12)
    best = scipy.optimize.minimize_scalar(
        lambda s: ol.nll_kalman(t, f, A, {**th, "sigma_w": s}), bounds=(1e-4, 1e-2), method="bounded",
        options={"xatol": 1e-12})
    assert best.x == pytest.approx(math.sqrt(rss / n), rel=1e-6)


def test_bfgs_optimum_is_stationary_and_beats_the_truth():
    t = np.arange(300) * (10 / 1440)
    truth = {"amp": 0.012, "prot": 0.6, "q": 8.0, "sigma_w": 1e-3}
    th = {"amp": truth["amp"], "omega": ol.omega_from_rotation(truth["prot"], truth["q"]), "q": truth["q"],
          "sigma_w": truth["sigma_w"]}
    f = ol.sample_curve(t, th, 11, 0)
    A = np.ones((t.size, 1))
    res = ol.fit_bfgs(t, f, A, truth)
    assert res.fun <= ol.nll_kalman(t, f, A, th) + 1e-9
    g = scipy.optimize.approx_fprime(res.x, lambda x: ol.nll_kalman(t, f, A, ol.theta_from_x(x)), 1e-6)
    assert np.max(np.abs(g)) < 1e-2


# ---------------------------------------------------------------------------
# The plain start (Section 3.3: the rotation period from a Lomb-Scargle
# periodogram; amp and sigma_w from the curve's moments). Each part is pinned
# to a closed form or a sampling law, not to the formula it uses.

def test_plain_init_sigma_w_closed_forms():
    """Second differences of a sampled polynomial on a uniform grid of step h:
    zero for a line, 2 c h^2 everywhere for c t^2, so the white-noise level is
    exactly 2 c h^2 / sqrt(6) and 0 (up to rounding)."""
    h = 2.0 / 1440
    t = np.arange(5000) * h
    grid = np.linspace(0.3, 2.0, 50)
    line = ol.plain_init(t, 1.0 + 3e-3 * t, grid)
    assert line["sigma_w"] <= 1e-14
    c = 4e-4
    quad = ol.plain_init(t, 1.0 + c * t * t, grid)
    assert quad["sigma_w"] == pytest.approx(2.0 * c * h * h / math.sqrt(6.0), rel=1e-6)
    assert quad["q"] == 5.0 and line["q"] == 5.0


def test_plain_init_amp_of_a_sinusoid_over_whole_cycles():
    """Discrete orthogonality: N equally spaced samples over c whole cycles
    (2c not a multiple of N) of a sin(2 pi c n / N + phi) have mean 0 and mean
    square a^2 / 2, so the amplitude estimate is exactly a / sqrt(2)."""
    n, cycles, a = 3000, 7, 0.02
    idx = np.arange(n)
    t = idx * (10 / 1440)
    f = 1.0 + a * np.sin(2 * np.pi * cycles * idx / n + 0.4)
    out = ol.plain_init(t, f, np.linspace(0.3, 5.0, 100))
    assert out["amp"] == pytest.approx(a / math.sqrt(2.0), rel=1e-12)


def test_plain_init_sigma_w_of_white_noise_within_its_sampling_law():
    """On white noise of sigma, d_n = e_n - 2 e_{n+1} + e_{n+2} has variance
    6 sigma^2; the squares have variance 72 sigma^4 and lag-1 and lag-2
    covariances 32 and 2 sigma^4, so mean(d^2) has relative standard error
    sqrt(140 / N) / 6 and its square root half that. The estimate must lie
    within five standard errors of sigma."""
    n, sigma = 200000, 1.3e-3
    rng = np.random.default_rng(17)
    t = np.arange(n) * (2 / 1440)
    f = 1.0 + sigma * rng.standard_normal(n)
    out = ol.plain_init(t, f, np.linspace(0.3, 2.0, 20))
    se = 0.5 * math.sqrt(140.0 / (n - 2)) / 6.0
    assert abs(out["sigma_w"] / sigma - 1.0) < 5.0 * se


@pytest.mark.parametrize("p_true", [0.45, 1.2, 3.3])
def test_plain_init_lomb_scargle_finds_a_noiseless_rotation_on_the_grid(p_true):
    """A noiseless sinusoid whose period is a grid point, sampled with a gap:
    the periodogram's first maximum is that grid point."""
    t = np.arange(9000) * (2 / 1440)
    t = np.concatenate([t[:4000], t[4700:]])
    grid = np.linspace(0.3, 4.0, 371)
    p = grid[np.argmin(np.abs(grid - p_true))]
    f = 1.0 + 0.01 * np.sin(2 * np.pi * t / p + 1.1)
    out = ol.plain_init(t, f, grid)
    assert out["prot"] == p
