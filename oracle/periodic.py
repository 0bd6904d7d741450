"""Oracle: the periodic search and the periodogram (Sections 2.3-2.4).

TEST INFRASTRUCTURE ONLY (see ``oracle/__init__.py``).

For each trial period P (steps in the paper's order):

1. The linear-search grid is interpolated onto a common grid of transit
   phases (Section 2.3): phases m = 0 .. ceil(p)-1 in lattice slots, with
   p = P / dt; the k-th transit of phase m sits at slot position m + k p.
   With base_k = floor(k p) and w_k = k p - base_k the event value of each
   quantity V is (1 - w_k) V[m + base_k] + w_k V[m + base_k + 1]
   (or V[m + base_k] when w_k = 0).
2. The K events of each (phase, duration) cell are combined with a common
   depth (Eq. 8) using the biased estimates of Eq. B4:
       1/sigma^2 = sum_k 1/var_k,   depth = sigma^2 sum_k depth_k/var_k,
       lnP = sum_k dll_k - 1/2 sum_k [ s (ln var_k - ln(sigma^2 + var_k))
                                       + (depth_k - depth)^2 / (var_k + sigma^2) ]
   with s = +1 for the sign printed in Eq. 8 and s = -1 for the sign the
   derivation of Appendix B gives (the two disagree; both are offered).
3. The argmax of lnP over (phase, duration) (Eq. 9) gives Q(P) = depth/sigma
   at that cell (Section 2.4).

The best candidate is the period of largest Q (Section 2.4).

Readings (the paper is silent or inconsistent on these):

* dll_k, the gain of the single-event fit over the trend-only fit, stands
  for ln L_k of Eq. 8 (with the absolute ln L_k every event adds ln L_0, so
  phases with more events would win whatever the data);
* interpolation is linear in the lattice index, of (dll, depth, var); an
  event needs its slot(s) inside [0, n_T - 1] and valid, otherwise it is
  skipped; a cell with no event is excluded;
* phases are in lattice steps from slot 0 (the first sample), so the epoch
  of phase m is t_first + m dt;
* argmax order is phase outer, duration inner, and the first maximum wins
  (strict >); NaN never wins; with no valid cell Q = 0 and indices are -1;
* sums over events run in increasing k;
* a trial period shorter than one cadence (p < 1), or not finite, has no
  event: Section 2.3 places one phase grid step of one cadence under every
  period, and a period below it would put several transits into one
  lattice step;
* phases at or beyond the last slot hold no event (their k = 0 event is
  already past the grid), so only phases below n_T are formed.
"""
from __future__ import annotations

import math

import numpy as np


def _events(n_epochs: int, p: float):
    """(base_k, w_k) for k = 0, 1, ... while base_k <= n_epochs - 1."""
    out = []
    k = 0
    while True:
        kp = float(k) * p
        base = math.floor(kp)
        if base > n_epochs - 1:
            break
        out.append((base, kp - base))
        k += 1
    return out


def fold_period(depth, var, dll, valid, dt: float, period: float, sign: int = 1):
    """lnP, combined depth and sigma^2 for every (phase, duration) cell of one
    period. Returns (lnp, dep, sig2, nev) each shaped [n_phase, n_d]."""
    n_d, n_t = depth.shape
    p = period / dt
    if not (math.isfinite(p) and p >= 1.0):
        # no phase grid below one cadence: no event, no cell
        z = np.zeros((0, n_d))
        return z, z.copy(), z.copy(), np.zeros((0, n_d), dtype=np.int64)
    n_ph = min(int(math.ceil(p)), n_t)
    m = np.arange(n_ph)
    ok = valid.astype(bool)
    ev = _events(n_t, p)
    lnp = np.full((n_ph, n_d), np.nan)
    dep = np.zeros((n_ph, n_d))
    sig2 = np.full((n_ph, n_d), np.nan)
    nev = np.zeros((n_ph, n_d), dtype=np.int64)
    for j in range(n_d):
        # gather the interpolated events once per (j, k): arrays over phases
        gathered = []
        for base, w in ev:
            i0 = m + base
            if w == 0.0:
                use = i0 <= n_t - 1
                i0c = np.minimum(i0, n_t - 1)
                use = use & ok[j, i0c]
                d_k = depth[j, i0c]
                v_k = var[j, i0c]
                l_k = dll[j, i0c]
            else:
                use = i0 + 1 <= n_t - 1
                i0c = np.minimum(i0, n_t - 2)
                use = use & ok[j, i0c] & ok[j, i0c + 1]
                d_k = (1.0 - w) * depth[j, i0c] + w * depth[j, i0c + 1]
                v_k = (1.0 - w) * var[j, i0c] + w * var[j, i0c + 1]
                l_k = (1.0 - w) * dll[j, i0c] + w * dll[j, i0c + 1]
            gathered.append((use, d_k, v_k, l_k))
        # pass 1: combined estimates (Eq. B4) and the sum of single-event terms
        s_w = np.zeros(n_ph)
        s_wd = np.zeros(n_ph)
        s_ll = np.zeros(n_ph)
        cnt = np.zeros(n_ph, dtype=np.int64)
        for use, d_k, v_k, l_k in gathered:
            with np.errstate(divide="ignore", invalid="ignore"):
                s_w = np.where(use, s_w + 1.0 / v_k, s_w)
                s_wd = np.where(use, s_wd + d_k / v_k, s_wd)
            s_ll = np.where(use, s_ll + l_k, s_ll)
            cnt = cnt + use
        with np.errstate(divide="ignore", invalid="ignore"):
            s2 = 1.0 / s_w
            dc = s2 * s_wd
        # pass 2: the common-depth correction of Eq. 8
        corr = np.zeros(n_ph)
        for use, d_k, v_k, l_k in gathered:
            with np.errstate(divide="ignore", invalid="ignore"):
                term = sign * (np.log(v_k) - np.log(s2 + v_k)) + (d_k - dc) ** 2 / (v_k + s2)
            corr = np.where(use, corr + term, corr)
        has = cnt > 0
        lnp[:, j] = np.where(has, s_ll - 0.5 * corr, np.nan)
        dep[:, j] = np.where(has, dc, 0.0)
        sig2[:, j] = np.where(has, s2, np.nan)
        nev[:, j] = cnt
    return lnp, dep, sig2, nev


def first_argmax(values: np.ndarray) -> int:
    """Index of the first strict maximum; NaN never wins; -1 if none."""
    best = -1
    bv = -math.inf
    for i, v in enumerate(np.asarray(values).ravel()):
        if v > bv:  # False for NaN
            bv = v
            best = i
    return best


def periodic_search(depth, var, dll, valid, dt: float, periods, sign: int = 1) -> dict:
    """Q(P) periodogram and the per-period best (phase, duration, depth, sigma, lnP)."""
    depth = np.asarray(depth, dtype=np.float64)
    var = np.asarray(var, dtype=np.float64)
    dll = np.asarray(dll, dtype=np.float64)
    valid = np.asarray(valid)
    periods = np.asarray(periods, dtype=np.float64)
    n_p = periods.shape[0]
    n_d = depth.shape[0]
    out = {
        "q_snr": np.zeros(n_p), "best_phase": np.full(n_p, -1, dtype=np.int64),
        "best_dur": np.full(n_p, -1, dtype=np.int32), "best_depth": np.zeros(n_p),
        "best_sigma": np.zeros(n_p), "best_lnp": np.full(n_p, -np.inf),
    }
    for ip, P in enumerate(periods):
        lnp, dep, sig2, _ = fold_period(depth, var, dll, valid, dt, float(P), sign)
        flat = first_argmax(lnp.ravel())  # phase outer, duration inner
        if flat < 0:
            continue
        m, j = divmod(flat, n_d)
        s = math.sqrt(sig2[m, j])
        out["q_snr"][ip] = dep[m, j] / s
        out["best_phase"][ip] = m
        out["best_dur"][ip] = j
        out["best_depth"][ip] = dep[m, j]
        out["best_sigma"][ip] = s
        out["best_lnp"][ip] = lnp[m, j]
    return out


def best_candidate(search: dict, periods, t_first: float, dt: float, durations) -> dict:
    """The candidate of largest Q (first maximum; Section 2.4)."""
    ip = first_argmax(search["q_snr"])
    if ip < 0:
        return {"index": -1}
    j = int(search["best_dur"][ip])
    return {
        "index": ip, "period": float(periods[ip]),
        "t0": t_first + float(search["best_phase"][ip]) * dt,
        "duration": float(durations[j]) * dt, "depth": float(search["best_depth"][ip]),
        "sigma": float(search["best_sigma"][ip]), "snr": float(search["q_snr"][ip]),
    }
