"""Oracle: the linear search (Section 2.2, Eqs. 5-6).

TEST INFRASTRUCTURE ONLY (see ``oracle/__init__.py``).

For every trial epoch slot i and duration j the design matrix is
X = [A | b_ij], the trend columns followed by a unit box (Section 2.1), and
the generalised least-squares fit of Eq. 6 is solved in full:

    w   = (X^T K^-1 X)^-1 X^T K^-1 f,     Cov(w) = (X^T K^-1 X)^-1,
    depth = w_M,  var = Cov(w)_MM,
    chi2  = (f - Xw)^T K^-1 (f - Xw),
    ln L  = -chi2/2 - ln|K|/2 - (N/2) ln 2 pi              (Eq. 5)

with K^-1 applied through the Cholesky factor (whitening by L^-1). The
returned ``dll`` is the log-likelihood gain over the trend-only fit,
dll = (chi2_0 - chi2)/2 = ln L - ln L_0; ``lnl0`` is ln L_0.

Readings (the paper is silent on these):

* box sign and edges: b = -1 on samples whose lattice index lies in
  [i - floor(n_j/2), i - floor(n_j/2) + n_j), 0 elsewhere, so a dip has a
  positive depth; the epoch grid is every lattice slot from the first to
  the last sample (the time array itself when there are no gaps);
* invalid cells (no sample in the box, or X^T K^-1 X not positive definite):
  depth = 0, var = +inf, dll = 0, valid = 0. X^T K^-1 X is singular when the
  box lies in the span of the trend columns (a box over every sample, with a
  constant trend); in floating point its last pivot is then rounding noise,
  so a cell counts as singular when the Schur complement of the trend block,
  S = 1 / var, is at most 1e-12 times q = b^T K^-1 b;
* var is the variance (the square of the depth uncertainty of Eq. 6).
"""
from __future__ import annotations

import math
from typing import Optional

import numpy as np
import scipy.linalg


def box_sample_range(lattice: np.ndarray, slot: int, n_dur: int):
    """[lo, hi): samples whose lattice index lies in the box window of ``slot``.

    Written as an explicit scan, not a search, so it is checkable by eye."""
    a = slot - n_dur // 2
    inside = np.nonzero((lattice >= a) & (lattice < a + n_dur))[0]
    if inside.size == 0:
        return 0, 0
    return int(inside[0]), int(inside[-1]) + 1


def whiten(L: np.ndarray, Y: np.ndarray) -> np.ndarray:
    """L^-1 Y by triangular solve."""
    return scipy.linalg.solve_triangular(L, Y, lower=True, check_finite=False)


def null_fit(L: np.ndarray, f: np.ndarray, A: np.ndarray):
    """Trend-only GLS: returns (chi2_0, w0)."""
    ft = whiten(L, f)
    if A.shape[1] == 0:
        return float(ft @ ft), np.zeros(0)
    At = whiten(L, A)
    G = At.T @ At
    w0 = np.linalg.solve(G, At.T @ ft)
    r = ft - At @ w0
    return float(r @ r), w0


def _fit_cells(At: np.ndarray, ft: np.ndarray, Bt: np.ndarray):
    """Full GLS for each whitened box column Bt[:, c] with whitened trend At.

    Returns depth, var, chi2, ok arrays over the columns."""
    n, m1 = At.shape
    nb = Bt.shape[1]
    M = m1 + 1
    depth = np.zeros(nb)
    var = np.full(nb, np.inf)
    chi2 = np.full(nb, np.nan)
    ok = np.zeros(nb, dtype=bool)
    for c in range(nb):
        Xt = np.empty((n, M))
        Xt[:, :m1] = At
        Xt[:, m1] = Bt[:, c]
        G = Xt.T @ Xt                      # X^T K^-1 X
        rhs = Xt.T @ ft                    # X^T K^-1 f
        try:
            cf = scipy.linalg.cho_factor(G, lower=True)
        except np.linalg.LinAlgError:
            continue
        w = scipy.linalg.cho_solve(cf, rhs)
        cov_last = scipy.linalg.cho_solve(cf, np.eye(M)[:, m1])[m1]
        if not (cov_last > 0.0 and math.isfinite(cov_last)):
            continue
        if not (1.0 / cov_last > 1e-12 * G[m1, m1]):   # box in the span of the trend: singular
            continue
        r = ft - Xt @ w
        depth[c] = w[m1]
        var[c] = cov_last
        chi2[c] = float(r @ r)
        ok[c] = True
    return depth, var, chi2, ok


def linear_search(f: np.ndarray, A: np.ndarray, L: np.ndarray, lattice: np.ndarray,
                  durations, n_epochs: Optional[int] = None, cells=None,
                  batch: int = 512) -> dict:
    """Run the linear search over all (duration j, slot i) cells, or over the
    listed ``cells`` = [(j, i), ...] only.

    Returns a dict with ``depth``, ``var``, ``dll`` (float64) and ``valid``
    (uint8), shaped [n_d, n_epochs] (or [len(cells)] when ``cells`` is
    given), plus ``lnl0``, ``chi2_0``, ``logdet``.
    """
    f = np.asarray(f, dtype=np.float64)
    A = np.asarray(A, dtype=np.float64).reshape(f.shape[0], -1)
    lattice = np.asarray(lattice, dtype=np.int64)
    durations = [int(d) for d in durations]
    n = f.shape[0]
    if n_epochs is None:
        n_epochs = int(lattice[-1]) + 1
    if cells is None:
        cells = [(j, i) for j in range(len(durations)) for i in range(n_epochs)]
        shape = (len(durations), n_epochs)
    else:
        shape = (len(cells),)
    ft = whiten(L, f)
    At = whiten(L, A) if A.shape[1] else np.zeros((n, 0))
    chi2_0, _ = null_fit(L, f, A)
    ld = float(2.0 * np.sum(np.log(np.diag(L))))
    lnl0 = -0.5 * chi2_0 - 0.5 * ld - 0.5 * n * math.log(2.0 * math.pi)

    ncell = len(cells)
    depth = np.zeros(ncell)
    var = np.full(ncell, np.inf)
    dll = np.zeros(ncell)
    valid = np.zeros(ncell, dtype=np.uint8)
    ranges = [box_sample_range(lattice, i, durations[j]) for (j, i) in cells]
    todo = [c for c in range(ncell) if ranges[c][1] > ranges[c][0]]
    for s in range(0, len(todo), batch):
        idx = todo[s:s + batch]
        B = np.zeros((n, len(idx)))
        for col, c in enumerate(idx):
            lo, hi = ranges[c]
            B[lo:hi, col] = -1.0
        Bt = whiten(L, B)
        d, v, c2, ok = _fit_cells(At, ft, Bt)
        for col, c in enumerate(idx):
            if ok[col]:
                depth[c] = d[col]
                var[c] = v[col]
                dll[c] = 0.5 * (chi2_0 - c2[col])
                valid[c] = 1
    return {
        "depth": depth.reshape(shape), "var": var.reshape(shape), "dll": dll.reshape(shape),
        "valid": valid.reshape(shape), "lnl0": lnl0, "chi2_0": chi2_0, "logdet": ld,
        "ranges": np.array(ranges, dtype=np.int64).reshape(shape + (2,)),
    }
