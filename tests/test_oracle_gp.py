"""Pins for the oracle's covariance and Cholesky (Appendix A; Eq. 5's ln|Sigma|).

Each check is independent of the oracle's own formulas: the SHO covariance
is compared with the stationary solution of the oscillator's stochastic
differential equation (matrix exponential of its drift), the branches with
their limits, the factor with a textbook loop and with closed forms.
"""
import math

import numpy as np
import pytest
import scipy.linalg

from oracle import gp
from synth import sho_omega_from_rotation


def _sde_covariance(tau, amp, omega, q):
    # stationary covariance of x'' + (omega/Q) x' + omega^2 x = noise:
    # k(tau) = [expm(F tau) Pinf]_00, Pinf = diag(amp^2, amp^2 omega^2)
    F = np.array([[0.0, 1.0], [-omega * omega, -omega / q]])
    Pinf = np.diag([amp * amp, amp * amp * omega * omega])
    return np.array([(scipy.linalg.expm(F * t) @ Pinf)[0, 0] for t in np.atleast_1d(tau)])


@pytest.mark.parametrize("q", [0.2, 0.45, 0.5, 0.7, 5.0, 45.0])
def test_sho_matches_sde_stationary_covariance(q):
    amp, omega = 0.013, 7.3
    tau = np.array([0.0, 1e-3, 0.05, 0.3, 1.1, 2.9])
    k = gp.sho_kernel(tau, amp, omega, q)
    ref = _sde_covariance(tau, amp, omega, q)
    np.testing.assert_allclose(k, ref, rtol=1e-10, atol=1e-12 * amp * amp)


def test_sho_zero_lag_is_amplitude_squared():
    for q in (0.3, 0.5, 5.0):
        assert gp.sho_kernel(0.0, 0.02, 3.0, q) == pytest.approx(0.02 ** 2, rel=1e-15)


def test_sho_branches_continuous_at_half():
    tau = np.linspace(0.0, 2.0, 17)
    mid = gp.sho_kernel(tau, 1.0, 4.0, 0.5)
    # dk/dQ is O(omega tau), so a step of 1e-8 in Q moves k by ~1e-7 at most
    for eps in (1e-8, -1e-8):
        np.testing.assert_allclose(gp.sho_kernel(tau, 1.0, 4.0, 0.5 + eps), mid, rtol=1e-6, atol=1e-12)


def test_rotation_parametrisation_oscillates_at_prot():
    # the Q > 1/2 branch oscillates as cos(g omega tau / 2Q): one full turn at tau = P_rot
    for prot, q in ((1.2, 5.0), (0.3, 45.0), (2.0, 0.8)):
        om = sho_omega_from_rotation(prot, q)
        g = math.sqrt(4 * q * q - 1)
        assert g * om * prot / (2 * q) == pytest.approx(2 * math.pi, rel=1e-14)


def test_covariance_spd_and_white_only():
    t = np.sort(np.random.default_rng(0).uniform(0, 3, 60))
    th = {"amp": 0.01, "omega": 9.0, "q": 5.0, "sigma_w": 1e-3}
    K = gp.covariance(t, th)
    assert np.allclose(K, K.T)
    assert np.linalg.eigvalsh(K).min() > 0
    thw = dict(th, amp=0.0)
    np.testing.assert_array_equal(gp.covariance(t, thw), np.eye(60) * 1e-6)


def test_cholesky_white_noise_closed_form():
    s = 3e-3
    K = np.eye(50) * s * s
    L = gp.cholesky(K)
    np.testing.assert_allclose(L, np.eye(50) * s, rtol=1e-15)
    assert gp.logdet(L) == pytest.approx(2 * 50 * math.log(s), rel=1e-14)


def test_cholesky_second_opinion_and_reconstruction():
    t = np.arange(40) * (2 / 1440)
    K = gp.covariance(t, {"amp": 0.02, "omega": 10.0, "q": 45.0, "sigma_w": 1e-3})
    L1 = gp.cholesky(K)
    L2 = gp.cholesky_textbook(K)
    np.testing.assert_allclose(L1, L2, rtol=1e-9, atol=1e-12)
    np.testing.assert_allclose(L1 @ L1.T, K, rtol=0, atol=1e-14)
    sign, ld = np.linalg.slogdet(K)  # LU-based, a different route
    assert sign > 0 and gp.logdet(L1) == pytest.approx(ld, rel=1e-11)


def test_cholesky_textbook_flags_non_pd():
    K = np.ones((4, 4))  # rank one
    with pytest.raises(np.linalg.LinAlgError):
        gp.cholesky_textbook(K)


# ---------------------------------------------------------------------------
# The Section 3.2 stellar-variability kernel (sum of terms)

def test_single_sho_term_is_the_sho_covariance():
    from oracle import gp as g
    t = np.sort(np.random.default_rng(1).uniform(0, 5, 60))
    th = {"amp": 0.01, "omega": 3.1, "q": 4.0, "sigma_w": 1e-3}
    a = g.covariance(t, th)
    b = g.covariance_terms(t, {"sho": [(0.01, 3.1, 4.0)]}, 1e-3)
    np.testing.assert_array_equal(a, b)


def test_rotation_terms_variance_split_and_periods():
    from oracle import gp as g
    sigma, P, q0, dq, f = 0.02, 1.3, 2.0, 3.0, 0.4
    terms = g.rotation_terms(sigma, P, q0, dq, f, 0.003, 0.05, 0.005, 7.0)
    (a1, w1, q1), (a2, w2, q2) = terms["sho"]
    # k1(0) + k2(0) = sigma^2, split 1 : f
    assert a1 ** 2 + a2 ** 2 == pytest.approx(sigma ** 2, rel=1e-14)
    assert a2 ** 2 / a1 ** 2 == pytest.approx(f, rel=1e-14)
    assert q1 == 0.5 + q0 + dq and q2 == 0.5 + q0 and w2 == 2 * w1
    # the damped oscillation of k1 has period P: sin/cos argument g omega tau / (2 Q) = 2 pi tau / P
    gq = np.sqrt(4 * q1 ** 2 - 1)
    assert gq * w1 / (2 * q1) == pytest.approx(2 * np.pi / P, rel=1e-14)
    K = g.covariance_terms(np.array([0.0]), terms, 0.001)
    assert K[0, 0] == pytest.approx(sigma ** 2 + 0.003 ** 2 + 0.005 ** 2 + 0.001 ** 2, rel=1e-14)


def test_exponential_term_has_a_tridiagonal_inverse():
    # an exponential covariance on any grid is Markov (AR(1)): its precision matrix is tridiagonal,
    # which pins exp(-|tau|/ell) against e.g. a squared exponential
    from oracle import gp as g
    t = np.sort(np.random.default_rng(2).uniform(0, 3, 40))
    K = g.covariance_terms(t, {"exp": [(0.7, 0.4)]}, 0.0)
    Pm = np.linalg.inv(K)
    off = np.abs(np.triu(Pm, 2)).max() / np.abs(Pm).max()
    assert off < 1e-10


def test_rotation_covariance_is_positive_definite():
    from oracle import gp as g
    rng = np.random.default_rng(3)
    t = np.arange(300) * (2 / 1440)
    for _ in range(5):
        terms = g.rotation_terms(rng.uniform(0.005, 0.03), rng.uniform(0.3, 3), rng.uniform(0.1, 5),
                                 rng.uniform(0.01, 5), rng.uniform(0.05, 1), rng.uniform(1e-4, 2e-3),
                                 rng.uniform(0.005, 0.05), rng.uniform(1e-4, 5e-3), rng.uniform(1, 20))
        K = g.covariance_terms(t, terms, rng.uniform(3e-4, 2e-3))
        g.cholesky(K)
