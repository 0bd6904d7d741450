"""Oracle: the iterative search for several transiting candidates (Section 3.3,
the search of TOI-540).

TEST INFRASTRUCTURE ONLY (see ``oracle/__init__.py``).

The linear search is done once. After a periodic search has found a
candidate, the trial epochs in windows of width 2 D centred on its periodic
transits are masked in the linear-search products (the log-likelihood gains,
the depths and their uncertainties), and the periodic search runs again on
the masked products; each further candidate repeats the two steps.

Readings (the paper states the window width and what is masked, not the
rest):

* the candidate's transits sit at slot positions m + k p, p = P / dt, for
  every integer k (also below the first sample), where m is the best phase
  of the best period: the positions the fold combines;
* D is the candidate's duration n_j dt, so the window half-width is n_j
  slots, and slot i is masked when |i - (m + k p)| < n_j for some k (strict);
  the distance is evaluated as (i - m) - k p in FP64, one rounding for k p;
* a masked slot is masked for every duration, with the invalid-cell encoding
  of the linear search (depth 0, var +inf, dll 0, valid 0);
* the search stops early when a periodic search finds no candidate.
"""
from __future__ import annotations

import math

import numpy as np

from . import periodic


def masked_slots(n_epochs: int, period_slots: float, phase: int, half_width: int) -> np.ndarray:
    """Boolean mask of the slots within half_width of a transit m + k p."""
    p, m, h = float(period_slots), int(phase), int(half_width)
    out = np.zeros(n_epochs, dtype=bool)
    for i in range(n_epochs):
        x = float(i - m)
        k_lo = math.floor((x - h) / p) - 1
        k_hi = math.ceil((x + h) / p) + 1
        for k in range(k_lo, k_hi + 1):
            if abs(x - float(k) * p) < h:
                out[i] = True
                break
    return out


def mask_transit(depth, var, dll, valid, dt: float, period: float, phase: int, half_width: int):
    """Copies of the linear-search products with the candidate's windows masked."""
    depth = np.array(depth, dtype=np.float64)
    var = np.array(var, dtype=np.float64)
    dll = np.array(dll, dtype=np.float64)
    valid = np.array(valid, dtype=np.uint8)
    sel = masked_slots(depth.shape[1], period / dt, phase, half_width)
    depth[:, sel] = 0.0
    var[:, sel] = np.inf
    dll[:, sel] = 0.0
    valid[:, sel] = 0
    return depth, var, dll, valid


def search_planets(depth, var, dll, valid, dt: float, periods, durations, n_planets: int, sign: int = 1) -> list:
    """Up to n_planets candidates: periodic search, mask the best candidate's transits, repeat."""
    periods = np.asarray(periods, dtype=np.float64)
    cur = (np.array(depth, dtype=np.float64), np.array(var, dtype=np.float64),
           np.array(dll, dtype=np.float64), np.array(valid, dtype=np.uint8))
    found = []
    for _ in range(n_planets):
        s = periodic.periodic_search(*cur, dt, periods, sign)
        ip = periodic.first_argmax(s["q_snr"])
        if ip < 0 or s["best_phase"][ip] < 0:
            break
        m, j = int(s["best_phase"][ip]), int(s["best_dur"][ip])
        found.append({"index": ip, "period": float(periods[ip]), "phase": m, "dur_index": j,
                      "snr": float(s["q_snr"][ip]), "depth": float(s["best_depth"][ip]),
                      "lnp": float(s["best_lnp"][ip])})
        cur = mask_transit(*cur, dt, float(periods[ip]), m, int(durations[j]))
    return found
