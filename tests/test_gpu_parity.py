"""GPU parity: the HIP path (through the C ABI) against the CPU oracle.

Bars (FP64 path): valid flags and every index bit-exact; dll within 1e-9 of
max(|dll_ref|, 1 nat); depth within 1e-9 of the reference sigma; var within
1e-9 relative; the fold's Q within 1e-12 relative of the oracle on identical
inputs (only log() differs) and argmax indices identical unless the oracle's
own lnP values of the two cells are tied within 1e-12 (certified tie).
"""
import math

import numpy as np
import pytest

from oracle import gp as ogp, linear as olin, periodic as oper
from synth import config1, config2, lattice_box_mask, make_workload, sho_omega_from_rotation

pytestmark = pytest.mark.gpu

DLL_TOL = 1e-9
DEPTH_TOL = 1e-9
VAR_TOL = 1e-9


def say(msg):
    print(f"[gpu-case] {msg}", flush=True)


@pytest.fixture(scope="module")
def api():
    import torch
    from paper_2402_06835_amd import _lib, api as a
    _lib.lib()  # fails loudly when the library is missing
    assert torch.cuda.is_available()
    return a


@pytest.fixture(scope="module")
def ctx(api):
    return api.Context(0)


def _host(ls):
    return {k: ls[k].cpu().numpy() for k in ("depth", "var", "dll", "valid")}


def assert_linear_close(gpu, ref, tag=""):
    v = ref["valid"].astype(bool)
    np.testing.assert_array_equal(gpu["valid"].astype(bool), v, err_msg=f"valid {tag}")
    assert np.all(gpu["var"][~v] == np.inf) and np.all(gpu["depth"][~v] == 0) and np.all(gpu["dll"][~v] == 0)
    if not v.any():
        return {}
    e_dll = np.abs(gpu["dll"][v] - ref["dll"][v]) / np.maximum(np.abs(ref["dll"][v]), 1.0)
    e_dep = np.abs(gpu["depth"][v] - ref["depth"][v]) / np.sqrt(ref["var"][v])
    e_var = np.abs(gpu["var"][v] - ref["var"][v]) / ref["var"][v]
    errs = {"dll": e_dll.max(), "depth": e_dep.max(), "var": e_var.max()}
    say(f"{tag} max errors {errs}")
    assert errs["dll"] <= DLL_TOL, (tag, errs)
    assert errs["depth"] <= DEPTH_TOL, (tag, errs)
    assert errs["var"] <= VAR_TOL, (tag, errs)
    return errs


def _case(n, m1, durs, gap=None, seed=0, q=5.0):
    th = {"amp": 0.01, "omega": sho_omega_from_rotation(1.2, q), "q": q, "sigma_w": 1e-3}
    gaps = [gap] if gap else []
    w = make_workload(f"case-N{n}", seed, n, 10 / 1440, th, durs, np.linspace(0.3, 2.0, 50), gaps=gaps,
                      injection={"depth": 2e-3, "period": 0.61, "t0": 0.13, "duration": 0.05} if n > 20 else None)
    if m1 < 3:
        w.A = np.ascontiguousarray(w.A[:, :m1])
    return w


LINEAR_CASES = [
    ("N1-m0", dict(n=1, m1=0, durs=[1])),
    ("N5-m1", dict(n=5, m1=1, durs=[1, 2])),
    ("N128-m3", dict(n=128, m1=3, durs=[1, 3, 8])),
    ("N129-m3-gap", dict(n=129, m1=3, durs=[2, 5], gap=(60, 4))),
    ("N700-m3-gap", dict(n=700, m1=3, durs=[1, 4, 9, 17], gap=(333, 25))),
    ("N300-m2-Qhalf", dict(n=300, m1=2, durs=[3, 7], q=0.5)),
    ("N300-m3-Qlow", dict(n=300, m1=3, durs=[3, 7], q=0.3)),
    # one past the column chunk of the row products (2048) and of the row chunks of the
    # transposed products (512) and of the box sums (256)
    ("N2049-m3-gap", dict(n=2049, m1=3, durs=[1, 6, 40], gap=(1024, 30), seed=2)),
    # several chunks of each, with a last chunk of 4 rows / columns
    ("N4100-m3", dict(n=4100, m1=3, durs=[2, 13, 64], seed=3)),
]


@pytest.mark.parametrize("name,kw", LINEAR_CASES, ids=[c[0] for c in LINEAR_CASES])
def test_linear_search_parity(api, ctx, name, kw):
    import torch
    w = _case(**kw)
    say(f"linear {name}: N={w.n} m1={w.A.shape[1]} durs={list(w.durations)} n_epochs={w.n_epochs}")
    fac = api.gp_factor(ctx, w.t, w.theta)
    ls = api.linear_search(ctx, fac, w.f, w.A if w.A.shape[1] else None, w.lattice, w.n_epochs, w.durations)
    torch.cuda.synchronize()
    L = ogp.cholesky(ogp.covariance(w.t, w.theta))
    ref = olin.linear_search(w.f, w.A, L, w.lattice, w.durations)
    assert fac.logdet == pytest.approx(ref["logdet"], rel=1e-12, abs=1e-9)
    null = ls["null"].cpu().numpy()
    assert null[0] == pytest.approx(ref["lnl0"], rel=1e-11, abs=1e-9)
    assert null[1] == pytest.approx(ref["chi2_0"], rel=1e-9, abs=1e-9)
    assert_linear_close(_host(ls), ref, name)


def _certify_ties(gpu, ref, depth, var, dll, valid, dt, periods, sign, rtol=1e-12):
    """Indices must agree, except where the oracle's lnP at the GPU's cell ties its maximum."""
    n_d = depth.shape[0]
    bad = np.nonzero((gpu["best_phase"] != ref["best_phase"]) | (gpu["best_dur"] != ref["best_dur"]))[0]
    for ip in bad:
        lnp, *_ = oper.fold_period(depth, var, dll, valid, dt, float(periods[ip]), sign)
        mx = np.nanmax(lnp)
        g = lnp[gpu["best_phase"][ip], gpu["best_dur"][ip]]
        assert abs(g - mx) <= rtol * max(abs(mx), 1.0), f"period {ip}: not a tie ({g} vs {mx})"
    return len(bad)


def _fold_host(ps):
    return {k: ps[k].cpu().numpy() for k in ("q_snr", "best_phase", "best_dur", "best_depth", "best_sigma",
                                             "best_lnp", "best_index")}


@pytest.mark.parametrize("sign", [1, -1])
def test_fold_parity_on_oracle_grid(api, ctx, sign):
    import torch
    w = config1()
    say(f"fold on oracle grid, cfg1 N={w.n}, sign={sign}")
    L = ogp.cholesky(ogp.covariance(w.t, w.theta))
    ref_ls = olin.linear_search(w.f, w.A, L, w.lattice, w.durations)
    ps = api.periodic_search(ctx, ref_ls["depth"], ref_ls["var"], ref_ls["dll"], ref_ls["valid"], w.dt, w.periods,
                             sign)
    torch.cuda.synchronize()
    gpu = _fold_host(ps)
    ref = oper.periodic_search(ref_ls["depth"], ref_ls["var"], ref_ls["dll"], ref_ls["valid"], w.dt, w.periods, sign)
    ties = _certify_ties(gpu, ref, ref_ls["depth"], ref_ls["var"], ref_ls["dll"], ref_ls["valid"], w.dt, w.periods,
                         sign)
    same = (gpu["best_phase"] == ref["best_phase"]) & (gpu["best_dur"] == ref["best_dur"])
    np.testing.assert_allclose(gpu["q_snr"][same], ref["q_snr"][same], rtol=1e-12, atol=1e-12)
    np.testing.assert_allclose(gpu["best_lnp"], ref["best_lnp"], rtol=1e-12, atol=1e-12)
    np.testing.assert_allclose(gpu["best_sigma"][same], ref["best_sigma"][same], rtol=1e-13)
    assert gpu["best_index"][0] == oper.first_argmax(ref["q_snr"]) or ties
    say(f"fold sign={sign}: certified ties {ties}")


@pytest.mark.parametrize("sign", [1, -1])
@pytest.mark.parametrize("kind", ["constant", "noise-plus-event"])
def test_fold_second_pass_skipping_keeps_the_argmax(api, ctx, kind, sign):
    """Grids built to stress the fold's bound-based skipping of its second pass: a constant
    grid (the cells of a period tie up to rounding, so nothing near the best may be skipped)
    and chi-square noise with one strong event (most cells skipped)."""
    import torch
    rng = np.random.default_rng(12 if kind == "constant" else 13)
    n_d, n_t, dt = 3, 700, 0.01
    if kind == "constant":
        depth = np.full((n_d, n_t), 1e-3)
        var = np.full((n_d, n_t), 4e-7)
        dll = 0.5 * depth ** 2 / var
    else:
        var = rng.uniform(2e-7, 6e-7, (n_d, n_t))
        depth = rng.standard_normal((n_d, n_t)) * np.sqrt(var)
        depth[1, 100::137] += 4e-3
        dll = 0.5 * depth ** 2 / var
    valid = np.ones((n_d, n_t), np.uint8)
    valid[:, 350:360] = 0
    periods = np.concatenate([np.linspace(0.5, 3.0, 120), [1.37]])
    say(f"fold skipping {kind} sign={sign}")
    ps = api.periodic_search(ctx, depth, var, dll, valid, dt, periods, sign)
    torch.cuda.synchronize()
    gpu = _fold_host(ps)
    ref = oper.periodic_search(depth, var, dll, valid, dt, periods, sign)
    # cells whose lnP differ only by rounding may be picked differently: certified as ties
    ties = _certify_ties(gpu, ref, depth, var, dll, valid, dt, periods, sign)
    same = (gpu["best_phase"] == ref["best_phase"]) & (gpu["best_dur"] == ref["best_dur"])
    np.testing.assert_allclose(gpu["best_lnp"], ref["best_lnp"], rtol=1e-12, atol=1e-12)
    np.testing.assert_allclose(gpu["q_snr"][same], ref["q_snr"][same], rtol=1e-12, atol=1e-12)
    say(f"fold skipping {kind} sign={sign}: certified ties {ties}")
    if kind != "constant":
        assert ties <= 2


def test_end_to_end_config1(api, ctx):
    import torch
    w = config1()
    say(f"end-to-end cfg1 N={w.n} n_p={w.periods.size}")
    fac = api.gp_factor(ctx, w.t, w.theta)
    ls = api.linear_search(ctx, fac, w.f, w.A, w.lattice, w.n_epochs, w.durations)
    ps = api.periodic_search(ctx, ls["depth"], ls["var"], ls["dll"], ls["valid"], w.dt, w.periods)
    torch.cuda.synchronize()
    L = ogp.cholesky(ogp.covariance(w.t, w.theta))
    ref_ls = olin.linear_search(w.f, w.A, L, w.lattice, w.durations)
    assert_linear_close(_host(ls), ref_ls, "cfg1")
    ref = oper.periodic_search(ref_ls["depth"], ref_ls["var"], ref_ls["dll"], ref_ls["valid"], w.dt, w.periods)
    gpu = _fold_host(ps)
    # inputs differ by <= 1e-9, so compare Q to 1e-7 and the argmax up to ties at that level
    ties = _certify_ties(gpu, ref, ref_ls["depth"], ref_ls["var"], ref_ls["dll"], ref_ls["valid"], w.dt, w.periods,
                         1, rtol=1e-7)
    same = (gpu["best_phase"] == ref["best_phase"]) & (gpu["best_dur"] == ref["best_dur"])
    np.testing.assert_allclose(gpu["q_snr"][same], ref["q_snr"][same], rtol=1e-7, atol=1e-7)
    assert int(gpu["best_index"][0]) == oper.first_argmax(ref["q_snr"])
    say(f"cfg1 best period {w.periods[gpu['best_index'][0]]:.4f} d (injected {w.injection['period']}), ties {ties}")


def test_noiseless_periodic_injection_recovered(api, ctx):
    import torch
    n = 900
    lat = np.arange(n)
    dt = 10 / 1440
    th = {"amp": 0.01, "omega": sho_omega_from_rotation(1.2, 5.0), "q": 5.0, "sigma_w": 1e-3}
    t = lat * dt
    x = (t - t.mean()) / (np.ptp(t) / 2)
    A = np.stack([np.ones(n), x, x * x], 1)
    durs = np.array([3, 6, 9], dtype=np.int32)
    p_slots, slot0, jtrue, delta = 211, 47, 2, 2e-3
    box = np.zeros(n)
    for c in range(slot0, n + 10, p_slots):
        box[lattice_box_mask(lat, c, int(durs[jtrue]))] = 1.0
    f = A @ [1.0, 1e-3, -5e-4] - delta * box
    periods = np.array([p_slots * dt * r for r in (0.5, 0.8, 1.0, 1.25, 2.0)])
    say("noiseless periodic injection N=900")
    fac = api.gp_factor(ctx, t, th)
    ls = api.linear_search(ctx, fac, f, A, lat, n, durs)
    ps = api.periodic_search(ctx, ls["depth"], ls["var"], ls["dll"], ls["valid"], dt, periods)
    torch.cuda.synchronize()
    gpu = _fold_host(ps)
    assert gpu["best_index"][0] == 2
    assert gpu["best_phase"][2] == slot0 and gpu["best_dur"][2] == jtrue


def test_not_positive_definite_reports_pivot(api, ctx):
    from paper_2402_06835_amd._lib import NU_ERR_NOT_PD, NuanceError
    t = np.array([0.0, 0.1, 0.1, 0.3])  # duplicate time, no white noise: K singular
    say("not-PD covariance (duplicate time, sigma_w = 0)")
    with pytest.raises(NuanceError) as ei:
        api.gp_factor(ctx, t, {"amp": 0.01, "omega": 3.0, "q": 5.0, "sigma_w": 0.0})
    assert ei.value.status == NU_ERR_NOT_PD
    assert ei.value.pivot == 2


def test_argument_errors_enqueue_nothing(api, ctx):
    from paper_2402_06835_amd._lib import NuanceError
    w = _case(n=50, m1=3, durs=[2])
    say("argument validation")
    fac = api.gp_factor(ctx, w.t, w.theta)
    with pytest.raises(NuanceError):
        api.linear_search(ctx, fac, w.f, w.A, w.lattice, w.n_epochs, [0])
    with pytest.raises(NuanceError):
        api.linear_search(ctx, fac, w.f, w.A, w.lattice, w.n_epochs, [2000])
    with pytest.raises(NuanceError):
        api.gp_factor(ctx, w.t, {"amp": 0.01, "omega": -1.0, "q": 5.0, "sigma_w": 1e-3})
    ls = api.linear_search(ctx, fac, w.f, w.A, w.lattice, w.n_epochs, [2])
    with pytest.raises(NuanceError):
        api.periodic_search(ctx, ls["depth"], ls["var"], ls["dll"], ls["valid"], 0.0, [1.0])
    with pytest.raises(NuanceError):
        api.periodic_search(ctx, ls["depth"], ls["var"], ls["dll"], ls["valid"], w.dt, [1.0], sign=0)


def test_lattice_that_breaks_the_rules_gives_no_cell(api, ctx):
    """The lattice is checked on the device: lattice[0] == 0, strictly increasing, lattice[-1] ==
    n_epochs - 1. One that breaks a rule leaves every cell invalid and ln L_0 = NaN (dense and
    state-space searches, boxes and templates); a good lattice afterwards gives the oracle's cells."""
    import torch
    w = _case(n=300, m1=2, durs=[2, 5], gap=(150, 9))
    say("lattice check")
    fac = api.gp_factor(ctx, w.t, w.theta)
    kern = api.Kernel(sho=[(w.theta["amp"], w.theta["omega"], w.theta["q"])], sigma_w=w.theta["sigma_w"])
    shapes = [np.ones(2), np.linspace(0.2, 1.0, 5)]
    swapped = w.lattice.copy()
    swapped[[40, 41]] = swapped[[41, 40]]
    repeated = w.lattice.copy()
    repeated[100] = repeated[99]
    shifted = w.lattice + 1
    short_end = w.lattice.copy()
    short_end[-1] -= 1  # n_epochs then exceeds lattice[-1] + 1
    for tag, lat in (("swapped", swapped), ("repeated", repeated), ("shifted", shifted), ("short end", short_end)):
        outs = [api.linear_search(ctx, fac, w.f, w.A, lat, w.n_epochs, w.durations),
                api.linear_search(ctx, fac, w.f, w.A, lat, w.n_epochs, w.durations, shapes=shapes),
                api.linear_search_ss(ctx, w.t, kern, w.f, w.A, lat, w.n_epochs, w.durations, check=False)]
        torch.cuda.synchronize()
        for ls in outs:
            h = _host(ls)
            assert not h["valid"].any(), tag
            assert np.all(h["var"] == np.inf) and np.all(h["depth"] == 0) and np.all(h["dll"] == 0), tag
            assert math.isnan(float(ls["null"][0].item())), tag
    ls = api.linear_search(ctx, fac, w.f, w.A, w.lattice, w.n_epochs, w.durations)
    torch.cuda.synchronize()
    ref = olin.linear_search(w.f, w.A, ogp.cholesky(ogp.covariance(w.t, w.theta)), w.lattice, w.durations)
    assert_linear_close(_host(ls), ref, "after a bad lattice")


def test_periods_at_and_below_one_cadence_match_the_oracle(api, ctx):
    """Section 2.3's phase grid at its edge: a period below one cadence (p < 1) or
    not finite has no event on both sides; p = 1 folds every slot into phase 0;
    a period far beyond the grid leaves single events."""
    import torch
    w = _case(n=64, m1=1, durs=[2, 3])
    say("periods at and below one cadence, against the oracle")
    fac = api.gp_factor(ctx, w.t, w.theta)
    ls = api.linear_search(ctx, fac, w.f, w.A, w.lattice, w.n_epochs, w.durations)
    periods = np.array([0.5 * w.dt, w.dt, float("nan"), float("inf"), -w.dt, 0.0, 1.5 * w.dt, 3 * w.dt,
                        1e20 * w.dt, 0.999999 * w.dt])
    for sign in (1, -1):
        ps = api.periodic_search(ctx, ls["depth"], ls["var"], ls["dll"], ls["valid"], w.dt, periods, sign=sign)
        torch.cuda.synchronize()
        g = _fold_host(ps)
        h = _host(ls)
        ref = oper.periodic_search(h["depth"], h["var"], h["dll"], h["valid"], w.dt, periods, sign)
        for k in ("best_phase", "best_dur"):
            np.testing.assert_array_equal(g[k], ref[k], err_msg=k)
        for k in ("q_snr", "best_depth", "best_sigma", "best_lnp"):
            np.testing.assert_allclose(g[k], ref[k], rtol=1e-12, atol=0, err_msg=k)
        none = [0, 2, 3, 4, 5, 9]
        assert np.all(g["best_phase"][none] == -1) and np.all(g["q_snr"][none] == 0)
        assert np.all(g["best_phase"][[1, 6, 7, 8]] >= 0)


def test_deterministic(api, ctx):
    import torch
    w = _case(n=700, m1=3, durs=[1, 4, 9], gap=(333, 25), seed=3)
    say("determinism N=700")
    outs = []
    for _ in range(2):
        fac = api.gp_factor(ctx, w.t, w.theta)
        ls = api.linear_search(ctx, fac, w.f, w.A, w.lattice, w.n_epochs, w.durations)
        ps = api.periodic_search(ctx, ls["depth"], ls["var"], ls["dll"], ls["valid"], w.dt, w.periods)
        torch.cuda.synchronize()
        outs.append((_host(ls), _fold_host(ps)))
    for k in ("depth", "var", "dll", "valid"):
        np.testing.assert_array_equal(outs[0][0][k], outs[1][0][k])
    for k in outs[0][1]:
        np.testing.assert_array_equal(outs[0][1][k], outs[1][1][k])


def test_nuance_object_paper_interface(api):
    w = config1()
    say("Nuance object on cfg1")
    nu = api.Nuance(w.t, w.f, gp=api.SHO.from_dict(w.theta), X=w.A)
    nu.linear_search(w.t.copy(), w.durations * w.dt)
    search = nu.periodic_search(w.periods)
    P, T0, D, depth, sigma = search.best
    assert search.Q_snr.shape == w.periods.shape
    assert abs(P - w.injection["period"]) < 0.02 or abs(2 * P - w.injection["period"]) < 0.02 or \
        abs(P - 2 * w.injection["period"]) < 0.02
    assert depth > 0 and sigma > 0


# ---------------------------------------------------------------------------
# Full size (the TESS-sector workload, N = 18000, 10 durations, 20000 periods)
# ---------------------------------------------------------------------------

def test_full_size_linear_search_sampled(api, ctx):
    import torch
    w = config2()
    say(f"full-size linear search N={w.n} n_epochs={w.n_epochs} n_d={w.durations.size}")
    fac = api.gp_factor(ctx, w.t, w.theta)
    ls = api.linear_search(ctx, fac, w.f, w.A, w.lattice, w.n_epochs, w.durations)
    torch.cuda.synchronize()
    gpu = _host(ls)
    say("oracle Cholesky at N=18000 (CPU)")
    L = ogp.cholesky(ogp.covariance(w.t, w.theta))
    rng = np.random.default_rng(99)
    n_d, n_t = gpu["dll"].shape
    # sampled cells: random, both gap edges, the grid edges
    cells = [(int(rng.integers(n_d)), int(rng.integers(n_t))) for _ in range(120)]
    for i in (0, 1, 8999, 9000, 9001, 9719, 9720, 9721, n_t - 2, n_t - 1):
        for j in (0, n_d - 1):
            cells.append((j, i))
    ref = olin.linear_search(w.f, w.A, L, w.lattice, w.durations, cells=cells)
    assert fac.logdet == pytest.approx(ref["logdet"], rel=1e-11)
    sel = {k: np.array([gpu[k][j, i] for (j, i) in cells]) for k in gpu}
    assert_linear_close(sel, ref, "full-size sampled")


def test_full_size_fold_sampled(api, ctx):
    import torch
    w = config2()
    rng = np.random.default_rng(5)
    n_d, n_t = w.durations.size, w.n_epochs
    # synthetic single-event grid of the full shape (not from the HIP path)
    depth = rng.normal(2e-4, 3e-4, (n_d, n_t))
    var = rng.uniform(4e-8, 1.2e-7, (n_d, n_t)) / np.arange(1, n_d + 1)[:, None]
    dll = 0.5 * depth ** 2 / var
    valid = np.ones((n_d, n_t), dtype=np.uint8)
    valid[:, 9000 - 20:9720 + 20] = 0
    depth[valid == 0] = 0
    var[valid == 0] = np.inf
    dll[valid == 0] = 0
    say(f"full-size fold n_p={w.periods.size} n_d={n_d} n_t={n_t}")
    ps = api.periodic_search(ctx, depth, var, dll, valid, w.dt, w.periods)
    torch.cuda.synchronize()
    gpu = _fold_host(ps)
    idx = np.sort(np.concatenate([rng.choice(w.periods.size, 24, replace=False), [0, w.periods.size - 1]]))
    say(f"oracle fold on {idx.size} sampled periods")
    sub = oper.periodic_search(depth, var, dll, valid, w.dt, w.periods[idx])
    g = {k: v[idx] for k, v in gpu.items() if k != "best_index"}
    ties = _certify_ties(g, sub, depth, var, dll, valid, w.dt, w.periods[idx], 1)
    same = (g["best_phase"] == sub["best_phase"]) & (g["best_dur"] == sub["best_dur"])
    np.testing.assert_allclose(g["q_snr"][same], sub["q_snr"][same], rtol=1e-12, atol=1e-12)
    np.testing.assert_allclose(g["best_lnp"], sub["best_lnp"], rtol=1e-12)
    say(f"full-size fold: certified ties {ties}")


# ---------------------------------------------------------------------------
# Reduced-precision inverse (FP32 level products + FP64 band Newton step +
# iterative refinement of the small solves): the bar is 1e-6 on dll (and on
# depth in sigma units and var), against the FP64 oracle.
# ---------------------------------------------------------------------------
MIXED_TOL = 1e-6


def assert_linear_close_tol(gpu, ref, tol, tag=""):
    v = ref["valid"].astype(bool)
    np.testing.assert_array_equal(gpu["valid"].astype(bool), v, err_msg=f"valid {tag}")
    e_dll = np.abs(gpu["dll"][v] - ref["dll"][v]) / np.maximum(np.abs(ref["dll"][v]), 1.0)
    e_dep = np.abs(gpu["depth"][v] - ref["depth"][v]) / np.sqrt(ref["var"][v])
    e_var = np.abs(gpu["var"][v] - ref["var"][v]) / ref["var"][v]
    errs = {"dll": e_dll.max(), "depth": e_dep.max(), "var": e_var.max(), "dll_p999": np.quantile(e_dll, 0.999)}
    say(f"{tag} max errors {errs}")
    assert errs["dll"] <= tol and errs["depth"] <= tol and errs["var"] <= tol, (tag, errs)
    return errs


@pytest.mark.parametrize("precision", ["fp32_refine", "bf16x3_refine"])
@pytest.mark.parametrize("name,kw", [("N700-m3-gap", dict(n=700, m1=3, durs=[1, 4, 9, 17], gap=(333, 25))),
                                     ("N1000-m3", dict(n=1000, m1=3, durs=[3, 9, 20], seed=4)),
                                     ("N2300-m2-gap", dict(n=2300, m1=2, durs=[5, 30, 90], gap=(1500, 120), seed=6))],
                         ids=["N700-m3-gap", "N1000-m3", "N2300-m2-gap"])
def test_linear_search_reduced_precision_parity(api, ctx, name, kw, precision):
    import torch
    w = _case(**kw)
    say(f"{precision} {name}: N={w.n}")
    fac = api.gp_factor(ctx, w.t, w.theta)
    ls = api.linear_search(ctx, fac, w.f, w.A, w.lattice, w.n_epochs, w.durations, precision=precision)
    torch.cuda.synchronize()
    L = ogp.cholesky(ogp.covariance(w.t, w.theta))
    ref = olin.linear_search(w.f, w.A, L, w.lattice, w.durations)
    assert_linear_close_tol(_host(ls), ref, MIXED_TOL, f"{precision} {name}")


def test_precision_switch_and_factor_reuse(api, ctx):
    import torch
    w = _case(n=700, m1=3, durs=[2, 6], gap=(200, 11), seed=8)
    w2 = _case(n=700, m1=3, durs=[2, 6], gap=(200, 11), seed=9)
    say("precision switch and factor reuse N=700")
    fac = api.gp_factor(ctx, w.t, w.theta)
    a = _host(api.linear_search(ctx, fac, w.f, w.A, w.lattice, w.n_epochs, w.durations))
    b = _host(api.linear_search(ctx, fac, w.f, w.A, w.lattice, w.n_epochs, w.durations, precision="fp32_refine"))
    c = _host(api.linear_search(ctx, fac, w.f, w.A, w.lattice, w.n_epochs, w.durations))
    d = _host(api.linear_search(ctx, fac, w.f, w.A, w.lattice, w.n_epochs, w.durations, precision="bf16x3_refine"))
    e = _host(api.linear_search(ctx, fac, w.f, w.A, w.lattice, w.n_epochs, w.durations, precision="fp32_refine"))
    torch.cuda.synchronize()
    for k in a:
        np.testing.assert_array_equal(a[k], c[k])  # back to FP64: identical to the first FP64 run
        np.testing.assert_array_equal(b[k], e[k])  # FP32 after BF16 (wider band kept): identical
    v = a["valid"].astype(bool)
    for r in (b, d):
        assert np.max(np.abs(r["dll"][v] - a["dll"][v]) / np.maximum(np.abs(a["dll"][v]), 1)) < MIXED_TOL
    # refill the same factor with another curve: same results as a fresh factor
    api.gp_factor(ctx, w2.t, w2.theta, out=fac)
    r1 = _host(api.linear_search(ctx, fac, w2.f, w2.A, w2.lattice, w2.n_epochs, w2.durations))
    fresh = api.gp_factor(ctx, w2.t, w2.theta)
    r2 = _host(api.linear_search(ctx, fresh, w2.f, w2.A, w2.lattice, w2.n_epochs, w2.durations))
    torch.cuda.synchronize()
    for k in r1:
        np.testing.assert_array_equal(r1[k], r2[k])


def test_full_size_reduced_precision_sampled(api, ctx):
    import torch
    w = config2()
    say(f"full-size reduced precision N={w.n}")
    fac = api.gp_factor(ctx, w.t, w.theta)
    ls64 = _host(api.linear_search(ctx, fac, w.f, w.A, w.lattice, w.n_epochs, w.durations))
    got = {}
    for prec in ("fp32_refine", "bf16x3_refine"):
        got[prec] = _host(api.linear_search(ctx, fac, w.f, w.A, w.lattice, w.n_epochs, w.durations, precision=prec))
    torch.cuda.synchronize()
    v = ls64["valid"].astype(bool)
    e_all = {}
    for prec, ls in got.items():
        e_all[prec] = np.abs(ls["dll"][v] - ls64["dll"][v]) / np.maximum(np.abs(ls64["dll"][v]), 1.0)
        say(f"{prec} vs fp64 (all {v.sum()} cells): max {e_all[prec].max():.2e} "
            f"p99.9 {np.quantile(e_all[prec], 0.999):.2e}")
    say("oracle Cholesky at N=18000 (CPU)")
    L = ogp.cholesky(ogp.covariance(w.t, w.theta))
    rng = np.random.default_rng(7)
    n_d, n_t = ls64["dll"].shape
    cells = [(int(rng.integers(n_d)), int(rng.integers(n_t))) for _ in range(100)]
    ref = olin.linear_search(w.f, w.A, L, w.lattice, w.durations, cells=cells)
    for prec, ls in got.items():
        sel = {k: np.array([ls[k][j, i] for (j, i) in cells]) for k in ls}
        assert_linear_close_tol(sel, ref, MIXED_TOL, f"full-size {prec} sampled")
        assert e_all[prec].max() <= MIXED_TOL, prec
