"""GPU: batch search of uneven light curves, captured graphs and the tile
policy, all through the C ABI.

The batch and the graph run the same kernels as the single-curve calls, on
the same per-curve problems, so their outputs must equal the single-curve
outputs bit for bit (those are parity-tested against the oracle elsewhere);
two curves are also compared with the oracle directly. The tile policy only
changes the shape of the output tiles: every element sums the same products
in the same order, so a search under forced 64 x 64 tiles must equal one
under forced 128 x 128 tiles bit for bit.
"""
import copy

import numpy as np
import pytest

from oracle import gp as ogp, linear as olin
from synth import make_workload, sho_omega_from_rotation

pytestmark = pytest.mark.gpu

CELL_KEYS = ("depth", "var", "dll", "valid")
PERIOD_KEYS = ("q_snr", "best_phase", "best_dur", "best_depth", "best_sigma", "best_lnp")


def say(msg):
    print(f"[gpu-case] {msg}", flush=True)


@pytest.fixture(scope="module")
def api():
    import torch
    from paper_2402_06835_amd import _lib, api as a
    _lib.lib()
    assert torch.cuda.is_available()
    return a


@pytest.fixture(scope="module")
def ctx(api):
    return api.Context(0)


DURS = [1, 4, 9, 17]
PERIODS = np.linspace(0.3, 2.0, 60)
DT = 10 / 1440


def _curve(n, seed, prot, gap=None):
    th = {"amp": 0.01, "omega": sho_omega_from_rotation(prot, 5.0), "q": 5.0, "sigma_w": 1e-3}
    w = make_workload(f"batch-N{n}-s{seed}", seed, n, DT, th, DURS, PERIODS, gaps=[gap] if gap else [],
                      injection={"depth": 2e-3, "period": 0.61, "t0": 0.13, "duration": 0.05})
    return w


def _curves():
    # uneven lengths: several tiles, ragged tails, one gap, one curve shorter than a tile
    return [_curve(700, 11, 1.2, gap=(333, 25)), _curve(300, 12, 0.8), _curve(1000, 13, 1.6),
            _curve(129, 14, 1.0), _curve(515, 15, 0.5)]


def _as_batch_input(w):
    return {"t": w.t, "f": w.f, "A": w.A, "lattice": w.lattice, "n_epochs": w.n_epochs, "theta": w.theta,
            "dt": DT}


def _single(api, ctx, w, precision):
    import torch
    fac = api.gp_factor(ctx, w.t, w.theta)
    ls = api.linear_search(ctx, fac, w.f, w.A, w.lattice, w.n_epochs, DURS, precision)
    ps = api.periodic_search(ctx, ls["depth"], ls["var"], ls["dll"], ls["valid"], DT, PERIODS)
    torch.cuda.synchronize()
    out = {k: ls[k].cpu().numpy() for k in CELL_KEYS}
    out.update({k: ps[k].cpu().numpy() for k in PERIOD_KEYS})
    out["null"] = ls["null"].cpu().numpy()
    out["best_index"] = int(ps["best_index"].cpu().item())
    out["logdet"] = fac.logdet
    fac.close()
    return out


def _assert_same(a, b, tag):
    for k in CELL_KEYS + PERIOD_KEYS + ("null",):
        np.testing.assert_array_equal(np.asarray(a[k]), np.asarray(b[k]), err_msg=f"{tag}: {k}")
    assert a["best_index"] == b["best_index"], tag


@pytest.mark.parametrize("precision", ["fp64", "fp32_refine", "bf16x3_refine"])
def test_batch_equals_single_curve_calls(api, ctx, precision):
    import torch
    ws = _curves()
    say(f"batch of {len(ws)} curves, N={[w.n for w in ws]}, {precision}")
    res = api.search_batch(ctx, [_as_batch_input(w) for w in ws], DURS, PERIODS, precision=precision)
    torch.cuda.synchronize()
    assert np.all(res["fail_pivot"] == -1)
    best = res["best_index"].cpu().numpy()
    for c, w in enumerate(ws):
        single = _single(api, ctx, w, precision)
        got = {k: res["cells"][c][k].cpu().numpy() for k in CELL_KEYS}
        got.update({k: res["periods"][c][k].cpu().numpy() for k in PERIOD_KEYS})
        got["null"] = res["null"][c].cpu().numpy()
        got["best_index"] = int(best[c])
        _assert_same(got, single, f"curve {c} N={w.n}")
        assert res["logdet"][c] == single["logdet"]


def test_batch_against_oracle(api, ctx):
    import torch
    ws = [_curve(300, 21, 0.9), _curve(129, 22, 1.3, gap=(60, 4))]
    say("batch of 2 curves vs the oracle, fp64")
    res = api.search_batch(ctx, [_as_batch_input(w) for w in ws], DURS, PERIODS, precision="fp64")
    torch.cuda.synchronize()
    for c, w in enumerate(ws):
        L = ogp.cholesky(ogp.covariance(w.t, w.theta))
        ref = olin.linear_search(w.f, w.A, L, w.lattice, DURS)
        got = {k: res["cells"][c][k].cpu().numpy() for k in CELL_KEYS}
        v = ref["valid"].astype(bool)
        np.testing.assert_array_equal(got["valid"].astype(bool), v)
        e = np.abs(got["dll"][v] - ref["dll"][v]) / np.maximum(np.abs(ref["dll"][v]), 1.0)
        assert e.max() <= 1e-9
        assert res["logdet"][c] == pytest.approx(ref["logdet"], rel=1e-12)


def test_batch_waves_under_a_small_budget(api, ctx):
    import torch
    ws = _curves()
    say("batch split into waves by a small memory budget")
    one = api.search_batch(ctx, [_as_batch_input(w) for w in ws], DURS, PERIODS, precision="fp64")
    # room for the largest factor (N=1000: at most 2.25 * 1024^2 doubles) and a little more: several waves
    budget = 20 << 20
    many = api.search_batch(ctx, [_as_batch_input(w) for w in ws], DURS, PERIODS, precision="fp64",
                            memory_budget=budget)
    torch.cuda.synchronize()
    for k in CELL_KEYS + PERIOD_KEYS + ("null", "best_index"):
        np.testing.assert_array_equal(one[k].cpu().numpy(), many[k].cpu().numpy(), err_msg=k)


def test_batch_arena_kept_across_budgets(api, ctx):
    """Budgets that grow a little from call to call: a later call may plan its waves within the arena the
    context already holds instead of growing it; every call's outputs equal the single-wave call's."""
    import torch
    ws = _curves()
    say("batch under growing budgets on one context")
    one = api.search_batch(ctx, [_as_batch_input(w) for w in ws], DURS, PERIODS, precision="fp64")
    ctx.release_memory()
    for budget in ((20 << 20), (21 << 20), (23 << 20), (26 << 20), (30 << 20)):
        got = api.search_batch(ctx, [_as_batch_input(w) for w in ws], DURS, PERIODS, precision="fp64",
                               memory_budget=budget)
        torch.cuda.synchronize()
        for k in CELL_KEYS + PERIOD_KEYS + ("null", "best_index"):
            np.testing.assert_array_equal(one[k].cpu().numpy(), got[k].cpu().numpy(), err_msg=f"{k} {budget}")


def test_batch_budget_too_small_is_oom(api, ctx):
    from paper_2402_06835_amd._lib import NU_ERR_OOM, NuanceError
    ws = _curves()[:2]
    say("batch with a budget below one factor")
    with pytest.raises(NuanceError) as ei:
        api.search_batch(ctx, [_as_batch_input(w) for w in ws], DURS, PERIODS, precision="fp64",
                         memory_budget=1024)
    assert ei.value.status == NU_ERR_OOM


def test_batch_not_positive_definite_curve(api, ctx):
    import torch
    from paper_2402_06835_amd._lib import NU_ERR_NOT_PD, NuanceError
    ws = [_curve(300, 31, 0.9), _curve(200, 32, 1.1), _curve(150, 33, 0.7)]
    ws[1].theta = {"amp": 0.0, "omega": 3.0, "q": 5.0, "sigma_w": 0.0}  # K = 0: first pivot fails
    say("batch with a zero covariance in the middle")
    with pytest.raises(NuanceError) as ei:
        api.search_batch(ctx, [_as_batch_input(w) for w in ws], DURS, PERIODS, precision="fp64")
    assert ei.value.status == NU_ERR_NOT_PD
    res = api.search_batch(ctx, [_as_batch_input(w) for w in ws], DURS, PERIODS, precision="fp64",
                           raise_not_pd=False)
    torch.cuda.synchronize()
    assert list(res["fail_pivot"]) == [-1, 0, -1]
    bad = res["cells"][1]
    assert not bad["valid"].any().item() and bool(torch.isinf(bad["var"]).all().item())
    assert bool((res["periods"][1]["best_phase"] == -1).all().item())
    assert int(res["best_index"][1].item()) == -1
    for c in (0, 2):
        single = _single(api, ctx, ws[c], "fp64")
        np.testing.assert_array_equal(res["cells"][c]["dll"].cpu().numpy(), single["dll"])
        np.testing.assert_array_equal(res["periods"][c]["q_snr"].cpu().numpy(), single["q_snr"])


def _batch_host(out, nc):
    got = {k: out[k].cpu().numpy() for k in CELL_KEYS + PERIOD_KEYS + ("null", "best_index")}
    return got


@pytest.mark.parametrize("precision", ["fp64", "fp32_refine"])
def test_batch_graph_replays_match_eager(api, ctx, precision):
    """The captured batch (one graph launch per batch) against the eager batch call, bit for bit, over three
    replays with new hyperparameters, with eager batches and synchronisations between the replays; a
    small budget forces several waves into the graph."""
    import torch
    ws = _curves()
    curves = [_as_batch_input(w) for w in ws]
    say(f"batch graph of {len(ws)} curves, N={[w.n for w in ws]}, {precision}, three replays")
    batch = api.prepare_batch(ctx, curves)
    # room for the largest factor (N = 1000) and a little more: several waves
    budget = (20 if precision == "fp64" else 48) << 20
    g = api.BatchGraph(ctx, batch, DURS, PERIODS, precision=precision, memory_budget=budget)
    for rep in range(3):
        thetas = []
        for c, w in enumerate(ws):
            th = dict(w.theta)
            th["amp"] = w.theta["amp"] * (1.0 + 0.25 * rep + 0.05 * c)
            th["sigma_w"] = w.theta["sigma_w"] * (1.0 + 0.1 * rep)
            thetas.append(th)
        g.set_theta(thetas)
        out = g.launch()
        torch.cuda.synchronize()
        assert np.all(g.status.cpu().numpy() == -1)
        got = _batch_host(out, len(ws))
        eager_curves = [dict(cv, theta=th) for cv, th in zip(curves, thetas)]
        ref = api.search_batch(ctx, eager_curves, DURS, PERIODS, precision=precision)
        torch.cuda.synchronize()
        for k in got:
            np.testing.assert_array_equal(got[k], ref[k].cpu().numpy(), err_msg=f"replay {rep}: {k}")
        np.testing.assert_array_equal(g.logdet.cpu().numpy(), ref["logdet"])
    g.close()


def test_batch_graph_reports_not_pd_without_sync(api, ctx):
    import torch
    ws = [_curve(300, 31, 0.9), _curve(200, 32, 1.1), _curve(150, 33, 0.7)]
    curves = [_as_batch_input(w) for w in ws]
    say("batch graph with a zero covariance in the middle on the second launch")
    g = api.BatchGraph(ctx, curves, DURS, PERIODS, precision="fp64")
    g.launch()
    torch.cuda.synchronize()
    assert list(g.status.cpu().numpy()) == [-1, -1, -1]
    g.set_theta([ws[0].theta, {"amp": 0.0, "omega": 3.0, "q": 5.0, "sigma_w": 0.0}, ws[2].theta])
    out = g.launch()
    torch.cuda.synchronize()
    assert list(g.status.cpu().numpy()) == [-1, 0, -1]
    bad = out["cells"][1]
    assert not bad["valid"].any().item() and bool(torch.isinf(bad["var"]).all().item())
    assert bool((out["periods"][1]["best_phase"] == -1).all().item())
    assert int(out["best_index"][1].item()) == -1
    for c in (0, 2):
        single = _single(api, ctx, ws[c], "fp64")
        np.testing.assert_array_equal(out["cells"][c]["dll"].cpu().numpy(), single["dll"])
    g.close()


@pytest.mark.parametrize("precision", ["fp64", "fp32_refine", "bf16x3_refine"])
@pytest.mark.parametrize("n", [700, 2000])
def test_graph_replays_match_eager(api, ctx, precision, n):
    # N = 2000 has trailing updates beyond the next panel (the eager step loop
    # splits them across two streams; the captured one keeps one stream)
    import torch
    w = _curve(n, 41, 1.2, gap=(333, 25))
    say(f"graph N={n}, {precision}: three replays with new theta and flux")
    g = api.Graph(ctx, w.t, w.f, w.A, w.lattice, w.n_epochs, DURS, w.theta, DT, PERIODS, precision=precision)
    rng = np.random.default_rng(5)
    for rep in range(3):
        theta = dict(w.theta)
        theta["amp"] = w.theta["amp"] * (1.0 + 0.3 * rep)
        theta["sigma_w"] = w.theta["sigma_w"] * (1.0 + 0.2 * rep)
        f = w.f + 1e-4 * rng.standard_normal(w.n)
        g.set_inputs(theta=theta, f=f)
        out = g.launch()
        torch.cuda.synchronize()
        assert int(g.status.item()) == -1
        got = {k: out[k].cpu().numpy() for k in CELL_KEYS + PERIOD_KEYS + ("null",)}
        got["best_index"] = int(out["best_index"].item())
        # eager run of the same inputs between replays
        w2 = copy.copy(w)
        w2.theta, w2.f = theta, f
        _assert_same(got, _single(api, ctx, w2, precision), f"replay {rep}")
    g.close()


def test_graph_reports_not_pd_without_sync(api, ctx):
    import torch
    w = _curve(300, 42, 1.0)
    say("graph with a zero covariance on the second launch")
    g = api.Graph(ctx, w.t, w.f, w.A, w.lattice, w.n_epochs, DURS, w.theta, DT, PERIODS)
    g.launch()
    torch.cuda.synchronize()
    assert int(g.status.item()) == -1
    g.set_inputs(theta={"amp": 0.0, "omega": 3.0, "q": 5.0, "sigma_w": 0.0})
    g.launch()
    torch.cuda.synchronize()
    assert int(g.status.item()) == 0
    g.set_inputs(theta=w.theta)
    out = g.launch()
    torch.cuda.synchronize()
    assert int(g.status.item()) == -1
    np.testing.assert_array_equal(out["dll"].cpu().numpy(), _single(api, ctx, w, "fp64")["dll"])
    g.close()


@pytest.mark.parametrize("precision", ["fp64", "fp32_refine", "bf16x3_refine"])
def test_tile_policy_does_not_change_results(api, ctx, precision):
    from paper_2402_06835_amd._lib import TUNE_CLASSES
    w = _curve(1000, 51, 1.3, gap=(400, 30))
    say(f"tile policy: all 128 vs all 64, N=1000, {precision}")
    c = api.Context(0)
    c.set_tuning(**{k: 0 for k in TUNE_CLASSES})
    big = _single(api, c, w, precision)
    c.set_tuning(**{k: 1 << 30 for k in TUNE_CLASSES})
    small = _single(api, c, w, precision)
    _assert_same(big, small, "64 vs 128 tiles")
    assert big["logdet"] == small["logdet"]
    c.close()


def test_autotune_keeps_results(api, ctx):
    w = _curve(700, 61, 1.1)
    say("autotune at n=2048, fp32_refine")
    c = api.Context(0)
    before = _single(api, c, w, "fp32_refine")
    tuned = c.autotune(2048, "fp32_refine")
    say(f"tuned thresholds {tuned}")
    assert set(tuned.values()) <= {0, 256, 512, 1024, 2048, 1 << 30}
    after = _single(api, c, w, "fp32_refine")
    _assert_same(before, after, "autotuned")
    c.close()


def test_batch_many_curves_under_load(api, ctx):
    """Regression: a loaded batch (many merged tiles per launch, late steps with few curves left) gives
    every curve exactly its single-curve result; an in-place panel product split across tiles of the
    same rows once made this fail at random."""
    import torch
    rng = np.random.default_rng(77)
    ns = [int(n) for n in rng.integers(2500, 6000, size=16)]
    ws = [_curve(n, 100 + i, float(rng.uniform(0.3, 2.0))) for i, n in enumerate(ns)]
    say(f"loaded batch of {len(ws)} curves, N={ns}, fp64, small budget (several waves)")
    budget = 3 * (6000 + 128) ** 2 * 8 * 3
    res = api.search_batch(ctx, [_as_batch_input(w) for w in ws], DURS, PERIODS, precision="fp64",
                           memory_budget=budget)
    torch.cuda.synchronize()
    assert np.all(res["fail_pivot"] == -1)
    for c, w in enumerate(ws):
        single = _single(api, ctx, w, "fp64")
        np.testing.assert_array_equal(res["cells"][c]["dll"].cpu().numpy(), single["dll"], err_msg=f"curve {c}")
        assert res["logdet"][c] == single["logdet"]


def test_batch_split_precision_per_output_errors(api, ctx):
    """The uneven batch with the split-BF16 inverse against the FP64 batch, output by output
    (dll, depth in sigma units, var, per-period SNR), on curves long enough that the FP64 band
    step does not cover them; one curve also against the oracle on sampled cells."""
    import torch
    dt = 2 / 1440
    ws = []
    for c, n in enumerate((2600, 4100, 5000)):
        rng = np.random.default_rng(7000 + c)
        prot = float(np.exp(rng.uniform(np.log(0.3), np.log(2.0))))
        amp = float(np.exp(rng.uniform(np.log(0.005), np.log(0.03))))
        th = {"amp": amp, "omega": sho_omega_from_rotation(prot, 5.0), "q": 5.0, "sigma_w": 8e-4}
        ws.append(make_workload(f"split-N{n}", 7000 + c, n, dt, th, [15, 28, 41, 60], np.linspace(0.5, 3.0, 200),
                                injection={"depth": 2e-3, "period": 1.3, "t0": 0.4, "duration": 40 * dt}))
    say(f"split-BF16 batch N={[w.n for w in ws]}")
    curves = [{"t": w.t, "f": w.f, "A": w.A, "lattice": w.lattice, "n_epochs": w.n_epochs, "theta": w.theta,
               "dt": dt} for w in ws]
    durs, periods = ws[0].durations, ws[0].periods
    ref = api.search_batch(ctx, curves, durs, periods, precision="fp64")
    got = api.search_batch(ctx, curves, durs, periods, precision="bf16x3_refine")
    torch.cuda.synchronize()
    v = ref["valid"].cpu().numpy().astype(bool)
    np.testing.assert_array_equal(got["valid"].cpu().numpy().astype(bool), v)
    g = {k: got[k].cpu().numpy() for k in ("depth", "var", "dll", "q_snr", "best_phase", "best_dur")}
    r = {k: ref[k].cpu().numpy() for k in ("depth", "var", "dll", "q_snr", "best_phase", "best_dur")}
    errs = {"dll": np.max(np.abs(g["dll"][v] - r["dll"][v]) / np.maximum(np.abs(r["dll"][v]), 1.0)),
            "depth": np.max(np.abs(g["depth"][v] - r["depth"][v]) / np.sqrt(r["var"][v])),
            "var": np.max(np.abs(g["var"][v] - r["var"][v]) / r["var"][v])}
    ok = r["best_phase"] >= 0
    errs["q_snr"] = np.max(np.abs(g["q_snr"][ok] - r["q_snr"][ok]) / np.maximum(np.abs(r["q_snr"][ok]), 1.0))
    same = np.mean((g["best_phase"][ok] == r["best_phase"][ok]) & (g["best_dur"][ok] == r["best_dur"][ok]))
    say(f"split-BF16 vs FP64 batch: {errs}, best cell agreement {same:.4f}")
    assert max(errs.values()) <= 1e-6, errs
    assert same >= 0.99
    np.testing.assert_array_equal(got["best_index"].cpu().numpy(), ref["best_index"].cpu().numpy())
    # the longest curve against the oracle on sampled cells
    w = ws[2]
    L = ogp.cholesky(ogp.covariance(w.t, w.theta))
    rng = np.random.default_rng(3)
    cells = [(int(rng.integers(len(durs))), int(rng.integers(w.n_epochs))) for _ in range(60)]
    oref = olin.linear_search(w.f, w.A, L, w.lattice, durs, cells=cells)
    gc = {k: got["cells"][2][k].cpu().numpy() for k in CELL_KEYS}
    sel = {k: np.array([gc[k][j, i] for (j, i) in cells]) for k in gc}
    vv = oref["valid"].astype(bool)
    np.testing.assert_array_equal(sel["valid"].astype(bool), vv)
    e = np.abs(sel["dll"][vv] - oref["dll"][vv]) / np.maximum(np.abs(oref["dll"][vv]), 1.0)
    say(f"split-BF16 longest curve vs oracle (sampled): dll max {e.max():.2e}")
    assert e.max() <= 1e-6
