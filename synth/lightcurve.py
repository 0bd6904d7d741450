"""Seeded synthetic light curves shaped like the paper's workloads.

A light curve is drawn as  f = trend + g + e - depth * box  (Section 1.1,
Eq. 1: a Gaussian-process sample around a linear mean), where

* trend  = [1, x, x^2] @ c, with x the time rescaled to [-1, 1];
* g      = stellar variability from a stochastically driven damped harmonic
           oscillator (SHO, Appendix A). It is simulated here as the 2-state
           linear stochastic differential equation the SHO is, with its exact
           discretisation between samples; the covariance formula of
           Appendix A is *not* used, so this module shares no arithmetic
           with the search (which builds its covariance from that formula);
* e      = white noise of standard deviation sigma_w;
* box    = 1 on samples inside an injected periodic transit.

Random numbers are drawn from ``numpy.random.default_rng(seed)`` in a fixed
order, so every array is a pure function of the seed.

Workloads (all times in days, TESS-like 2-min or 10-min cadence):

* ``config1``: N=1440 at 10 min (10 d), P_rot=1.2 d, Q=5, amp=1%,
  sigma_w=1e-3; injected depth 2e-3, D=1 h, P=2.3 d; 3 durations
  (3/6/9 samples); 2000 periods in [0.5, 5] d.
* ``config2``: N=18000 at 2 min with a 720-slot (1 d) gap after sample
  9000; P_rot log-uniform in [0.3, 2] d, amp log-uniform in [0.5%, 3%],
  Q=5, sigma_w=8e-4; injected depth 1e-3, D=36 samples, P uniform in
  [0.5, 10] d; 10 durations 9..90 samples; 20000 periods in [0.3, 13] d.
* ``config3``: 64 curves, N uniform in {4000..20000} at 2 min, no gap,
  hyperparameters as config2, an injection with probability 1/2
  (depth U[5e-4, 5e-3], D U[0.5, 2] h, P U[0.5, 10] d); 8 durations
  [15, 21, 28, 34, 41, 47, 54, 60] samples; 20000 periods in [0.3, 13] d.
* ``principle_e1``: the dataset of the paper's principle figure (4 d at
  2 min, P=0.7 d, D=1.2 h, depth 2%, SHO omega=pi/(6D), Q=45, amp=depth,
  white noise 0.1%).
"""
from __future__ import annotations

from dataclasses import dataclass, field
from typing import Optional, Sequence

import numpy as np
import scipy.linalg

MINUTE = 1.0 / 1440.0  # one minute in days


@dataclass
class Workload:
    """One light curve plus the search grids to run on it."""

    name: str
    seed: int
    t: np.ndarray  # (N,) float64 times [d], t = t0 + lattice * dt
    lattice: np.ndarray  # (N,) int64 strictly increasing, lattice[0] == 0
    dt: float  # cadence [d]
    f: np.ndarray  # (N,) float64 flux
    A: np.ndarray  # (N, m1) float64 trend design (column-major when copied to C)
    theta: dict  # {"amp", "omega", "q", "sigma_w"} of the SHO + white noise
    durations: np.ndarray  # (n_d,) int32 box durations in samples (lattice slots)
    periods: np.ndarray  # (n_p,) float64 trial periods [d]
    injection: Optional[dict] = None
    extra: dict = field(default_factory=dict)

    @property
    def n(self) -> int:
        return int(self.t.shape[0])

    @property
    def n_epochs(self) -> int:
        return int(self.lattice[-1]) + 1


# ---------------------------------------------------------------------------
# SHO as a stochastic differential equation
# ---------------------------------------------------------------------------

def sho_omega_from_rotation(prot: float, q: float) -> float:
    """Angular frequency omega of an SHO whose damped oscillation has period
    ``prot`` (for Q > 1/2 the covariance oscillates at omega*sqrt(1-1/(4Q^2));
    for Q <= 1/2 there is no oscillation and omega = 2*pi/prot is used)."""
    if q > 0.5:
        return 4.0 * np.pi * q / (prot * np.sqrt(4.0 * q * q - 1.0))
    return 2.0 * np.pi / prot


def _sho_sde(amp: float, omega: float, q: float):
    """Drift matrix F and stationary state covariance of the oscillator
    x'' + (omega/Q) x' + omega^2 x = white forcing, scaled so Var(x) = amp^2."""
    F = np.array([[0.0, 1.0], [-omega * omega, -omega / q]])
    Pinf = np.diag([amp * amp, amp * amp * omega * omega])
    return F, Pinf


def sample_sho_state_space(t: np.ndarray, amp: float, omega: float, q: float,
                           rng: np.random.Generator) -> np.ndarray:
    """Exact O(N) draw of the SHO process at times ``t`` (sorted).

    Between samples the state evolves as s_{n+1} = Phi s_n + w_n with
    Phi = expm(F dt_n) and Cov(w_n) = Pinf - Phi Pinf Phi^T.
    """
    F, Pinf = _sho_sde(amp, omega, q)
    n = t.shape[0]
    z = rng.standard_normal((n, 2))
    out = np.empty(n)
    s = np.linalg.cholesky(Pinf) @ z[0]
    out[0] = s[0]
    cache: dict = {}
    for i in range(1, n):
        h = float(t[i] - t[i - 1])
        key = round(h / MINUTE * 1e6)
        if key not in cache:
            Phi = scipy.linalg.expm(F * h)
            Qd = Pinf - Phi @ Pinf @ Phi.T
            Qd = 0.5 * (Qd + Qd.T)
            # Qd is PSD but can be numerically rank-deficient for tiny h
            w, V = np.linalg.eigh(Qd)
            C = V @ np.diag(np.sqrt(np.clip(w, 0.0, None)))
            cache[key] = (Phi, C)
        Phi, C = cache[key]
        s = Phi @ s + C @ z[i]
        out[i] = s[0]
    return out


# ---------------------------------------------------------------------------
# Grids, trend, injections
# ---------------------------------------------------------------------------

def linspace_periods(pmin: float, pmax: float, n: int) -> np.ndarray:
    return np.linspace(pmin, pmax, n)


def quadratic_trend(t: np.ndarray) -> np.ndarray:
    """Design columns [1, x, x^2] with x = (t - t_mid) / half_span."""
    t_first, t_last = float(t[0]), float(t[-1])
    half = 0.5 * (t_last - t_first) if t_last > t_first else 1.0
    x = (t - 0.5 * (t_first + t_last)) / half
    return np.stack([np.ones_like(x), x, x * x], axis=1)


def lattice_box_mask(lattice: np.ndarray, slot: int, n_dur: int) -> np.ndarray:
    """Samples whose lattice index lies in [slot - n_dur//2, slot - n_dur//2 + n_dur)."""
    a = slot - n_dur // 2
    return (lattice >= a) & (lattice < a + n_dur)


def _continuous_box(t: np.ndarray, period: float, t0: float, dur: float) -> np.ndarray:
    """1 on samples with |t - (t0 + k P)| < D/2 for some integer k."""
    k = np.round((t - t0) / period)
    return (np.abs(t - (t0 + k * period)) < 0.5 * dur).astype(np.float64)


def make_workload(name: str, seed: int, n: int, dt: float, theta: dict,
                  durations: Sequence[int], periods: np.ndarray,
                  gaps: Sequence[tuple] = (), trend_coef=(1.0, 1e-3, -5e-4),
                  injection: Optional[dict] = None,
                  rng: Optional[np.random.Generator] = None) -> Workload:
    """Assemble one workload.

    ``gaps`` is a list of (after_sample, n_missing_slots): the lattice jumps
    by n_missing_slots + 1 after that sample. ``injection`` holds
    {"depth", "period", "t0", "duration"} in days (continuous-time box) or
    {"depth", "slot0", "p_slots", "n_dur"} (a box on lattice windows).
    """
    if rng is None:
        rng = np.random.default_rng(seed)
    steps = np.ones(n, dtype=np.int64)
    steps[0] = 0
    for after, missing in gaps:
        steps[after + 1] += missing
    lattice = np.cumsum(steps)
    t = lattice * dt
    A = quadratic_trend(t)
    trend = A @ np.asarray(trend_coef, dtype=np.float64)
    g = sample_sho_state_space(t, theta["amp"], theta["omega"], theta["q"], rng)
    e = rng.standard_normal(n) * theta["sigma_w"]
    f = trend + g + e
    inj = None
    if injection is not None:
        inj = dict(injection)
        if "slot0" in inj:
            box = np.zeros(n)
            s = int(inj["slot0"])
            while s - inj["n_dur"] // 2 <= lattice[-1]:
                box[lattice_box_mask(lattice, s, int(inj["n_dur"]))] = 1.0
                s += int(inj["p_slots"])
        else:
            box = _continuous_box(t, inj["period"], inj["t0"], inj["duration"])
        f = f - inj["depth"] * box
        inj["n_in_transit"] = int(box.sum())
    return Workload(name=name, seed=seed, t=t, lattice=lattice.astype(np.int64), dt=dt,
                    f=f, A=np.ascontiguousarray(A), theta=dict(theta),
                    durations=np.asarray(durations, dtype=np.int32),
                    periods=np.asarray(periods, dtype=np.float64), injection=inj)


def _log_uniform(rng, lo, hi):
    return float(np.exp(rng.uniform(np.log(lo), np.log(hi))))


# ---------------------------------------------------------------------------
# The named workloads
# ---------------------------------------------------------------------------

def config1(seed: int = 1) -> Workload:
    """Plain FP64 single light curve (10-min cadence, 10 d)."""
    rng = np.random.default_rng(seed)
    dt = 10 * MINUTE
    q = 5.0
    theta = {"amp": 0.01, "omega": sho_omega_from_rotation(1.2, q), "q": q, "sigma_w": 1e-3}
    period = 2.3
    inj = {"depth": 2e-3, "period": period, "duration": 1.0 / 24.0,
           "t0": float(rng.uniform(0.0, period))}
    return make_workload("plain-fp64-N1440", seed, 1440, dt, theta, [3, 6, 9],
                         linspace_periods(0.5, 5.0, 2000), injection=inj, rng=rng)


def config2(seed: int = 2) -> Workload:
    """TESS-sector-shaped curve: N=18000 at 2 min with a 1-d gap mid-sector."""
    rng = np.random.default_rng(seed)
    dt = 2 * MINUTE
    q = 5.0
    prot = _log_uniform(rng, 0.3, 2.0)
    amp = _log_uniform(rng, 0.005, 0.03)
    theta = {"amp": amp, "omega": sho_omega_from_rotation(prot, q), "q": q, "sigma_w": 8e-4}
    period = float(rng.uniform(0.5, 10.0))
    inj = {"depth": 1e-3, "period": period, "duration": 36 * dt,
           "t0": float(rng.uniform(0.0, period))}
    w = make_workload("tess-sector-N18000", seed, 18000, dt, theta, [9 * k for k in range(1, 11)],
                      linspace_periods(0.3, 13.0, 20000), gaps=[(8999, 720)], injection=inj, rng=rng)
    w.extra["prot"] = prot
    return w


def two_sectors(seed: int = 8, gap_slots: int = 262800):
    """Two TESS-sector-shaped curves (as config2: N = 18000 at 2 min, 1-d mid-sector gap) a year apart
    (gap_slots empty slots between them), each with its own rotation GP, and one planet through both:
    depth 1e-3, duration 36 samples, period = the trial period of index 7402 (5.0005 d; on the grid, since
    over a one-year baseline a period between grid points drifts the later transits out of their box),
    first transit at global time 1234 dt. Returns the two workloads (each on its own lattice from 0, its
    injection epoch shifted into it) and their global slot offsets."""
    rng = np.random.default_rng(seed)
    dt = 2 * MINUTE
    q = 5.0
    periods = linspace_periods(0.3, 13.0, 20000)
    period, t0_global = float(periods[7402]), 1234 * dt
    out, offs = [], []
    off = 0
    for c in range(2):
        prot = _log_uniform(rng, 0.3, 2.0)
        amp = _log_uniform(rng, 0.005, 0.03)
        theta = {"amp": amp, "omega": sho_omega_from_rotation(prot, q), "q": q, "sigma_w": 8e-4}
        inj = {"depth": 1e-3, "period": period, "duration": 36 * dt,
               "t0": float((t0_global - off * dt) % period), "global_t0": t0_global}
        w = make_workload(f"sector-{c}", seed * 10 + c, 18000, dt, theta, [9 * k for k in range(1, 11)],
                          periods, gaps=[(8999, 720)], injection=inj, rng=rng)
        w.extra["prot"] = prot
        out.append(w)
        offs.append(off)
        off += int(w.n_epochs) + gap_slots
    return out, offs


def config3(n_curves: int = 64, base_seed: int = 3000):
    """Uneven batch: curves of N uniform in {4000..20000} samples at 2 min."""
    out = []
    dt = 2 * MINUTE
    q = 5.0
    for c in range(n_curves):
        seed = base_seed + c
        rng = np.random.default_rng(seed)
        n = int(rng.integers(4000, 20001))
        prot = _log_uniform(rng, 0.3, 2.0)
        amp = _log_uniform(rng, 0.005, 0.03)
        theta = {"amp": amp, "omega": sho_omega_from_rotation(prot, q), "q": q, "sigma_w": 8e-4}
        inj = None
        if rng.uniform() < 0.5:
            period = float(rng.uniform(0.5, 10.0))
            inj = {"depth": float(rng.uniform(5e-4, 5e-3)), "period": period,
                   "duration": float(rng.uniform(0.5, 2.0)) / 24.0,
                   "t0": float(rng.uniform(0.0, period))}
        w = make_workload(f"batch-{c}-N{n}", seed, n, dt, theta, [15, 21, 28, 34, 41, 47, 54, 60],
                          linspace_periods(0.3, 13.0, 20000), injection=inj, rng=rng)
        w.extra["prot"] = prot
        out.append(w)
    return out


def principle_e1(seed: int = 7, periods=None, durations=(36,)) -> Workload:
    """The principle dataset: 4 d at 2 min, P=0.7 d, D=1.2 h, depth 2%,
    SHO omega = pi/(6D), Q=45, amp = depth, white noise 0.1%.

    Times in days, so omega is in rad/day with D in days. The injected
    transit sits on lattice windows (36 slots = 1.2 h at 2 min) with a
    period of 504 slots (0.7 d), so it is on the search grid.
    """
    rng = np.random.default_rng(seed)
    dt = 2 * MINUTE
    depth = 0.02
    dur = 1.2 / 24.0
    theta = {"amp": depth, "omega": np.pi / (6.0 * dur), "q": 45.0, "sigma_w": 1e-3}
    slot0 = int(rng.integers(0, 504))
    inj = {"depth": depth, "slot0": slot0, "p_slots": 504, "n_dur": 36}
    if periods is None:
        periods = np.array([0.35, 0.7])
    return make_workload("principle-E1", seed, 2880, dt, theta, list(durations), np.asarray(periods),
                         injection=inj, rng=rng)
