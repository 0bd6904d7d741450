"""Oracle: GP covariance of the light curve and its Cholesky factor.

TEST INFRASTRUCTURE ONLY (see ``oracle/__init__.py``).

* ``sho_kernel`` is the SHO covariance of Appendix A written out branch by
  branch: k(tau) = sigma^2 exp(-omega tau / 2Q) times
  (1 + omega tau) for Q = 1/2, cosh(f omega tau/2Q) + sinh(f omega tau/2Q)/f
  for Q < 1/2, cos(g omega tau/2Q) + sin(g omega tau/2Q)/g for Q > 1/2,
  with f = sqrt(1-4Q^2) and g = sqrt(4Q^2-1).
* ``covariance`` adds the white-noise variance on the diagonal (Section 1.1,
  principle-dataset caption; Section 3.2: the diagonal is a free term).
* ``cholesky`` is the lower factor K = L L^T (a library routine), and
  ``cholesky_textbook`` the Cholesky-Banachiewicz loop, as a second opinion.
* ``logdet`` = 2 sum log L_nn, the ln|Sigma| term of Eq. 5.
* ``rotation_terms`` is the stellar-variability kernel of Section 3.2,
  k = k1 + k2 + k3 + k4: two SHO terms at the rotation period P and at P/2,
      Q1 = 1/2 + Q0 + dQ, omega1 = 4 pi Q1 / (P sqrt(4 Q1^2 - 1)),
      S1 = sigma^2 / ((1 + f) omega1 Q1),
      Q2 = 1/2 + Q0, omega2 = 2 omega1, S2 = f sigma^2 / ((1 + f) omega2 Q2),
  and two exponential terms sigma_i^2 exp(-|tau| / ell_i). An SHO term with
  power S0 has k(0) = S0 omega Q (the form Appendix A writes with sigma^2),
  so amp1^2 = sigma^2 / (1 + f) and amp2^2 = f sigma^2 / (1 + f).
  ``covariance_terms`` sums the terms and adds sigma_w^2 on the diagonal.
"""
from __future__ import annotations

import math

import numpy as np
import scipy.linalg


def sho_kernel(tau, amp: float, omega: float, q: float) -> np.ndarray:
    """SHO covariance k(tau) of Appendix A (sigma = amp)."""
    tau = np.abs(np.asarray(tau, dtype=np.float64))
    x = omega * tau / (2.0 * q)
    env = amp * amp * np.exp(-x)
    if q == 0.5:
        return env * (1.0 + omega * tau)
    if q < 0.5:
        f = math.sqrt(1.0 - 4.0 * q * q)
        return env * (np.cosh(f * x) + np.sinh(f * x) / f)
    g = math.sqrt(4.0 * q * q - 1.0)
    return env * (np.cos(g * x) + np.sin(g * x) / g)


def covariance(t: np.ndarray, theta: dict) -> np.ndarray:
    """Dense K[n, m] = k_SHO(|t_n - t_m|) + sigma_w^2 delta_nm."""
    t = np.asarray(t, dtype=np.float64)
    tau = np.abs(t[:, None] - t[None, :])
    K = sho_kernel(tau, theta["amp"], theta["omega"], theta["q"])
    K[np.diag_indices_from(K)] += theta["sigma_w"] ** 2
    return K


def cholesky(K: np.ndarray) -> np.ndarray:
    """Lower Cholesky factor (LAPACK via SciPy)."""
    return scipy.linalg.cholesky(K, lower=True)


def cholesky_textbook(K: np.ndarray) -> np.ndarray:
    """Cholesky-Banachiewicz, row by row; slow, for small N only."""
    n = K.shape[0]
    L = np.zeros_like(K, dtype=np.float64)
    for i in range(n):
        for j in range(i + 1):
            s = K[i, j] - np.dot(L[i, :j], L[j, :j])
            if i == j:
                if s <= 0.0:
                    raise np.linalg.LinAlgError(f"not positive definite at pivot {i}")
                L[i, i] = math.sqrt(s)
            else:
                L[i, j] = s / L[j, j]
    return L


def logdet(L: np.ndarray) -> float:
    """ln|K| = 2 sum_n ln L_nn."""
    return float(2.0 * np.sum(np.log(np.diag(L))))


def exp_kernel(tau, sigma: float, ell: float) -> np.ndarray:
    """Exponential covariance sigma^2 exp(-|tau| / ell) (Section 3.2, k3 and k4)."""
    return sigma * sigma * np.exp(-np.abs(np.asarray(tau, dtype=np.float64)) / ell)


def rotation_terms(sigma: float, period: float, q0: float, dq: float, f: float,
                   sigma3: float, ell3: float, sigma4: float, ell4: float) -> dict:
    """The terms of the Section 3.2 kernel: {"sho": [(amp, omega, q), ...], "exp": [(sigma, ell), ...]}."""
    q1 = 0.5 + q0 + dq
    w1 = 4.0 * math.pi * q1 / (period * math.sqrt(4.0 * q1 * q1 - 1.0))
    s1 = sigma * sigma / ((1.0 + f) * w1 * q1)
    q2 = 0.5 + q0
    w2 = 2.0 * w1
    s2 = f * sigma * sigma / ((1.0 + f) * w2 * q2)
    # k(0) = S0 omega Q for an SHO term of power S0
    return {"sho": [(math.sqrt(s1 * w1 * q1), w1, q1), (math.sqrt(s2 * w2 * q2), w2, q2)],
            "exp": [(sigma3, ell3), (sigma4, ell4)]}


def covariance_terms(t: np.ndarray, terms: dict, sigma_w: float) -> np.ndarray:
    """Dense K[n, m] = sum of the terms at |t_n - t_m| + sigma_w^2 delta_nm."""
    t = np.asarray(t, dtype=np.float64)
    tau = np.abs(t[:, None] - t[None, :])
    K = np.zeros_like(tau)
    for amp, omega, q in terms.get("sho", []):
        K += sho_kernel(tau, amp, omega, q)
    for sig, ell in terms.get("exp", []):
        K += exp_kernel(tau, sig, ell)
    K[np.diag_indices_from(K)] += sigma_w * sigma_w
    return K
