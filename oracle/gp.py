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
