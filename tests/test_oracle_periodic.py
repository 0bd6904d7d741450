"""Pins for the oracle's periodic search (Sections 2.3-2.4, Eq. 8, Eq. B4, Eq. 9).

Independent references: closed forms of Eq. 8 for one event and for K
identical events (for both signs of the log-ratio term), a scalar
enumeration of the fold on tiny grids, exact interpolation of linear data,
the reduction of Eq. B4 to the least-squares fit of one periodic box under
white noise without trend, noiseless recovery of an on-grid periodic
transit, the argmax rules, and the alias property of the paper's principle
figure.
"""
import json
import math
import os

import numpy as np
import pytest

from oracle import gp, linear, periodic
from synth import lattice_box_mask, principle_e1, make_workload

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _grid(n_d, n_t, seed=0, pvalid=1.0):
    rng = np.random.default_rng(seed)
    depth = rng.normal(1e-3, 5e-4, (n_d, n_t))
    var = rng.uniform(1e-7, 4e-7, (n_d, n_t))
    dll = 0.5 * depth ** 2 / var
    valid = (rng.uniform(size=(n_d, n_t)) < pvalid).astype(np.uint8)
    var[valid == 0] = np.inf
    depth[valid == 0] = 0.0
    dll[valid == 0] = 0.0
    return depth, var, dll, valid


@pytest.mark.parametrize("sign", [1, -1])
def test_single_event_closed_form(sign):
    depth, var, dll, valid = _grid(2, 10, seed=1)
    # period longer than the grid: exactly one event per phase
    lnp, dep, s2, nev = periodic.fold_period(depth, var, dll, valid, 1.0, 25.0, sign)
    for m in range(10):
        for j in range(2):
            assert nev[m, j] == 1
            assert dep[m, j] == pytest.approx(depth[j, m], rel=1e-15)
            assert s2[m, j] == pytest.approx(var[j, m], rel=1e-15)
            assert lnp[m, j] == pytest.approx(dll[j, m] + sign * 0.5 * math.log(2.0), rel=1e-14)


@pytest.mark.parametrize("sign", [1, -1])
@pytest.mark.parametrize("K", [2, 3, 7])
def test_identical_events_closed_form(sign, K):
    p = 5
    n_t = p * K
    d0, v0 = 1.3e-3, 2e-7
    l0 = 0.5 * d0 * d0 / v0
    depth = np.full((1, n_t), d0)
    var = np.full((1, n_t), v0)
    dll = np.full((1, n_t), l0)
    valid = np.ones((1, n_t), dtype=np.uint8)
    lnp, dep, s2, nev = periodic.fold_period(depth, var, dll, valid, 0.1, 0.1 * p, sign)
    assert (nev[:, 0] == K).all()
    np.testing.assert_allclose(dep[:, 0], d0, rtol=1e-14)
    np.testing.assert_allclose(s2[:, 0], v0 / K, rtol=1e-14)
    ref = K * l0 + sign * 0.5 * K * math.log(1 + 1 / K)
    np.testing.assert_allclose(lnp[:, 0], ref, rtol=1e-13)


def _brute_fold(depth, var, dll, valid, dt, P, sign):
    n_d, n_t = depth.shape
    p = P / dt
    out = {}
    for m in range(int(math.ceil(p))):
        for j in range(n_d):
            evs = []
            k = 0
            while True:
                kp = k * p
                base = math.floor(kp)
                if base > n_t - 1:
                    break
                w = kp - base
                i0 = m + base
                if w == 0.0:
                    if i0 <= n_t - 1 and valid[j, i0]:
                        evs.append((depth[j, i0], var[j, i0], dll[j, i0]))
                elif i0 + 1 <= n_t - 1 and valid[j, i0] and valid[j, i0 + 1]:
                    evs.append(tuple((1 - w) * a[j, i0] + w * a[j, i0 + 1] for a in (depth, var, dll)))
                k += 1
            if not evs:
                out[m, j] = None
                continue
            sw = swd = sll = 0.0
            for d, v, l in evs:
                sw += 1 / v
                swd += d / v
                sll += l
            s2 = 1 / sw
            dc = s2 * swd
            corr = 0.0
            for d, v, l in evs:
                corr += sign * (math.log(v) - math.log(s2 + v)) + (d - dc) ** 2 / (v + s2)
            out[m, j] = (sll - 0.5 * corr, dc, s2, len(evs))
    return out


@pytest.mark.parametrize("P", [3.0, 2.5, 3.7, 0.9, 13.3, 40.0])
@pytest.mark.parametrize("sign", [1, -1])
def test_fold_matches_scalar_enumeration(P, sign):
    depth, var, dll, valid = _grid(3, 31, seed=2, pvalid=0.8)
    lnp, dep, s2, nev = periodic.fold_period(depth, var, dll, valid, 1.0, P, sign)
    ref = _brute_fold(depth, var, dll, valid, 1.0, P, sign)
    if P < 1.0:  # below one cadence: no phase grid, no cell (reading of Section 2.3)
        assert lnp.shape[0] == 0
        return
    # phases at or past the last slot hold no event and are not formed
    assert lnp.shape[0] == min(int(math.ceil(P)), 31)
    for (m, j), r in ref.items():
        if m >= lnp.shape[0]:
            assert r is None
        elif r is None:
            assert nev[m, j] == 0 and math.isnan(lnp[m, j])
        else:
            assert nev[m, j] == r[3]
            assert lnp[m, j] == pytest.approx(r[0], rel=1e-13, abs=1e-13)
            assert dep[m, j] == pytest.approx(r[1], rel=1e-13)
            assert s2[m, j] == pytest.approx(r[2], rel=1e-13)


def test_half_integer_period_interpolates_linear_data_exactly():
    n_t = 40
    idx = np.arange(n_t, dtype=float)
    depth = (1e-3 + 1e-5 * idx)[None, :]
    var = (1e-7 + 1e-9 * idx)[None, :]
    dll = (2.0 + 0.25 * idx)[None, :]
    valid = np.ones((1, n_t), dtype=np.uint8)
    p = 6.5
    lnp, dep, s2, nev = periodic.fold_period(depth, var, dll, valid, 1.0, p, 1)
    for m in range(7):
        pos = []
        for k in range(n_t):
            last = m + math.ceil(k * p)  # the right-hand slot an event reads
            if last <= n_t - 1:
                pos.append(m + k * p)
        v = 1e-7 + 1e-9 * np.array(pos)
        d = 1e-3 + 1e-5 * np.array(pos)
        s2_ref = 1 / np.sum(1 / v)
        assert nev[m, 0] == len(pos)
        assert s2[m, 0] == pytest.approx(s2_ref, rel=1e-12)
        assert dep[m, 0] == pytest.approx(s2_ref * np.sum(d / v), rel=1e-12)


def test_white_noise_no_trend_equals_periodic_box_gls():
    # Eq. B4's combination of single events equals the least-squares fit of
    # one periodic box when the events are independent (diagonal covariance)
    rng = np.random.default_rng(5)
    n, s = 200, 1e-3
    lat = np.arange(n)
    f = s * rng.standard_normal(n) - 2e-3 * sum(lattice_box_mask(lat, c, 5) for c in (7, 47, 87, 127, 167))
    L = np.eye(n) * s
    out = linear.linear_search(f, np.zeros((n, 0)), L, lat, [5])
    p_slots = 40
    lnp, dep, s2, nev = periodic.fold_period(out["depth"], out["var"], out["dll"], out["valid"], 1.0,
                                             float(p_slots), 1)
    for m in range(p_slots):
        box = np.zeros(n, dtype=bool)
        for c in range(m, n, p_slots):  # event slots inside the epoch grid
            box |= lattice_box_mask(lat, c, 5)
        n_tot = box.sum()
        assert dep[m, 0] == pytest.approx(-f[box].sum() / n_tot, rel=1e-10, abs=1e-15)
        assert s2[m, 0] == pytest.approx(s * s / n_tot, rel=1e-10)


def test_noiseless_periodic_injection_recovered_on_grid():
    lat = np.arange(700)
    dt = 10 / 1440
    t = lat * dt
    th = {"amp": 0.01, "omega": 4 * math.pi * 5 / (1.2 * math.sqrt(99)), "q": 5.0, "sigma_w": 1e-3}
    K = gp.covariance(t, th)
    x = (t - t.mean()) / (np.ptp(t) / 2)
    A = np.stack([np.ones(700), x, x * x], 1)
    durs = [3, 6, 9]
    p_slots, slot0, jtrue, delta = 173, 61, 1, 2e-3
    box = np.zeros(700)
    for c in range(slot0, 720, p_slots):
        box[lattice_box_mask(lat, c, durs[jtrue])] = 1.0
    f = A @ [1.0, 1e-3, -5e-4] - delta * box
    out = linear.linear_search(f, A, gp.cholesky(K), lat, durs)
    periods = np.array([p_slots * dt * r for r in (0.5, 0.77, 1.0, 1.31, 2.0)])
    res = periodic.periodic_search(out["depth"], out["var"], out["dll"], out["valid"], dt, periods)
    best = periodic.best_candidate(res, periods, 0.0, dt, durs)
    assert best["index"] == 2
    assert res["best_phase"][2] == slot0 and res["best_dur"][2] == jtrue
    assert best["depth"] == pytest.approx(delta, rel=0.05)


def test_argmax_rules():
    assert periodic.first_argmax([1.0, 3.0, 3.0, 2.0]) == 1
    assert periodic.first_argmax([np.nan, 2.0, np.nan, 2.0]) == 1
    assert periodic.first_argmax([np.nan, np.nan]) == -1
    depth, var, dll, valid = _grid(2, 12, seed=3)
    valid[:] = 0
    res = periodic.periodic_search(depth, np.full_like(var, np.inf), np.zeros_like(dll), valid, 1.0, [3.0, 5.5])
    assert (res["q_snr"] == 0).all() and (res["best_phase"] == -1).all() and (res["best_dur"] == -1).all()
    # exact ties: identical columns -> the first phase, then the first duration wins
    depth = np.ones((2, 12)) * 1e-3
    var = np.ones((2, 12)) * 1e-7
    dll = np.ones((2, 12)) * 5.0
    res = periodic.periodic_search(depth, var, dll, np.ones((2, 12), np.uint8), 1.0, [4.0])
    assert res["best_phase"][0] == 0 and res["best_dur"][0] == 0


def test_principle_dataset_alias_scores_lower():
    with open(os.path.join(GOLDEN, "principle_e1.json")) as fh:
        g = json.load(fh)
    w = principle_e1(periods=np.array([g["alias_claim"]["alias_period_days"], g["alias_claim"]["period_days"]]))
    # the synthetic dataset is the one the caption prints
    assert w.n == int(g["span_days"] * 1440 / g["cadence_minutes"])
    assert w.dt == pytest.approx(g["cadence_minutes"] / 1440)
    assert w.injection["depth"] == g["transit_depth"] and w.theta["amp"] == g["transit_depth"]
    assert w.injection["p_slots"] * w.dt == pytest.approx(g["transit_period_days"])
    assert w.durations[0] * w.dt == pytest.approx(g["transit_duration_hours"] / 24)
    assert w.theta["omega"] == pytest.approx(math.pi / (6 * g["transit_duration_hours"] / 24))
    assert w.theta["q"] == g["sho_Q"] and w.theta["sigma_w"] == g["white_noise_std"]
    L = gp.cholesky(gp.covariance(w.t, w.theta))
    out = linear.linear_search(w.f, w.A, L, w.lattice, w.durations)
    for sign in (1, -1):
        best = []
        for P in w.periods:
            lnp, *_ = periodic.fold_period(out["depth"], out["var"], out["dll"], out["valid"], w.dt, float(P), sign)
            best.append(np.nanmax(lnp))
        assert best[1] > best[0], (sign, best)


@pytest.mark.parametrize("sign", [1, -1])
def test_period_of_one_cadence_combines_every_valid_slot(sign):
    """p = 1 (Section 2.3): one phase, an event on every slot (w_k = 0), so
    Eq. B4 is the inverse-variance mean over all valid slots of a duration, and
    Eq. 8's log term is the closed form of K independent events."""
    depth, var, dll, valid = _grid(2, 40, seed=7, pvalid=0.7)
    lnp, dep, s2, nev = periodic.fold_period(depth, var, dll, valid, 0.25, 0.25, sign)
    assert lnp.shape == (1, 2)
    for j in range(2):
        ok = valid[j].astype(bool)
        w = 1.0 / var[j, ok]
        sig2 = 1.0 / w.sum()
        d = sig2 * (w * depth[j, ok]).sum()
        ref = dll[j, ok].sum() - 0.5 * (sign * np.log(var[j, ok] / (sig2 + var[j, ok]))
                                        + (depth[j, ok] - d) ** 2 / (var[j, ok] + sig2)).sum()
        assert nev[0, j] == ok.sum()
        assert s2[0, j] == pytest.approx(sig2, rel=1e-13)
        assert dep[0, j] == pytest.approx(d, rel=1e-12)
        assert lnp[0, j] == pytest.approx(ref, rel=1e-12)


@pytest.mark.parametrize("period", [0.5, 0.999999, 0.0, -1.0, float("nan"), float("inf"), float("-inf")])
def test_periods_below_one_cadence_or_not_finite_have_no_event(period):
    """Reading of Section 2.3's phase grid (one cadence per step): a period
    shorter than one cadence, or not finite, forms no (phase, duration) cell;
    the periodogram reports Q = 0 and indices -1 for it."""
    depth, var, dll, valid = _grid(2, 30, seed=3)
    lnp, dep, s2, nev = periodic.fold_period(depth, var, dll, valid, 1.0, period, 1)
    assert lnp.shape == (0, 2) and nev.sum() == 0
    out = periodic.periodic_search(depth, var, dll, valid, 1.0, [period, 3.0])
    assert out["best_phase"][0] == -1 and out["best_dur"][0] == -1 and out["q_snr"][0] == 0.0
    assert out["best_lnp"][0] == -np.inf
    assert out["best_phase"][1] >= 0


def test_period_far_beyond_the_grid_leaves_single_events():
    """A period longer than the grid by any factor gives one event per phase
    (k = 0 only); phases past the grid hold none, so only n_T phases form."""
    depth, var, dll, valid = _grid(1, 12, seed=5)
    for P in (13.0, 1e6, 1e300):
        lnp, dep, s2, nev = periodic.fold_period(depth, var, dll, valid, 1.0, P, 1)
        assert lnp.shape == (12, 1)
        np.testing.assert_array_equal(nev[:, 0], np.ones(12, dtype=np.int64))
        np.testing.assert_allclose(dep[:, 0], depth[0], rtol=1e-15)
