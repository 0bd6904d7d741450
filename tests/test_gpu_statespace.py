"""GPU: the state-space linear search (entry point 2b) against the oracle.

The path never forms K: it runs the Kalman filter of the state-space form of
the covariance (the quasiseparable route of Section 3.2 and Appendix A). What
it computes has a plain definition, the dense GLS linear search of Section
2.2 on K, so the reference is the oracle's dense search
(``oracle.linear.linear_search`` on the Cholesky factor of
``oracle.gp.covariance_terms`` / ``oracle.gp.covariance``), at the FP64 bar of
the dense path (1e-9 on dll relative to max(|dll|, 1), depth in units of its
sigma, var relative).

* The rotation kernel of Section 3.2 with and without a gap, plus an
  overdamped term; kernels of every term shape (critical, overdamped and
  underdamped SHO, exponential only, the widest 4 + 4); the single SHO of
  Appendix A on the small configuration; no trend; durations 1 and 1024.
* ln L_0, chi2_0 and ln|K| against the oracle's.
* The TESS-sector size (N = 18000) with the rotation kernel on sampled cells.
* A covariance that is not positive definite is reported (index of the first
  failing sample), or, unchecked, leaves every cell invalid and ln L_0 NaN.
* Argument errors are reported before any launch.
"""
import math

import numpy as np
import pytest

from oracle import gp as ogp, linear as olin
from synth import config1, config2, make_workload, sho_omega_from_rotation

pytestmark = pytest.mark.gpu

DLL_TOL, DEPTH_TOL, VAR_TOL = 1e-9, 1e-9, 1e-9


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


ROT = dict(sigma=0.012, period=0.9, q0=1.5, dq=2.0, f=0.5, sigma_short=8e-4, ell_short=0.02,
           sigma_long=3e-3, ell_long=4.0, sigma_w=1e-3)


def _rot_terms():
    return ogp.rotation_terms(ROT["sigma"], ROT["period"], ROT["q0"], ROT["dq"], ROT["f"], ROT["sigma_short"],
                              ROT["ell_short"], ROT["sigma_long"], ROT["ell_long"])


def _curve(n, seed, gap=None, durations=(1, 4, 9)):
    th = {"amp": 0.01, "omega": sho_omega_from_rotation(0.9, 5.0), "q": 5.0, "sigma_w": 1e-3}
    return make_workload(f"ss-N{n}", seed, n, 10 / 1440, th, list(durations), np.linspace(0.3, 2.0, 50),
                         gaps=[gap] if gap else [],
                         injection={"depth": 2e-3, "period": 0.61, "t0": 0.13, "duration": 0.05})


def _host(ls):
    return {k: ls[k].cpu().numpy() for k in ("depth", "var", "dll", "valid")}


def _close(gpu, ref, tag):
    v = ref["valid"].astype(bool)
    np.testing.assert_array_equal(gpu["valid"].astype(bool), v)
    inv = ~v
    assert np.all(gpu["dll"][inv] == 0.0) and np.all(np.isinf(gpu["var"][inv]))
    if not v.any():
        return
    e = {"dll": float(np.max(np.abs(gpu["dll"][v] - ref["dll"][v]) / np.maximum(np.abs(ref["dll"][v]), 1.0))),
         "depth": float(np.max(np.abs(gpu["depth"][v] - ref["depth"][v]) / np.sqrt(ref["var"][v]))),
         "var": float(np.max(np.abs(gpu["var"][v] - ref["var"][v]) / ref["var"][v]))}
    say(f"{tag} max errors {e}")
    assert e["dll"] <= DLL_TOL and e["depth"] <= DEPTH_TOL and e["var"] <= VAR_TOL, (tag, e)


def _null_close(ls, ref, tag):
    null = ls["null"].cpu().numpy()
    say(f"{tag} null {null} oracle {ref['lnl0']}, {ref['chi2_0']}, {ref['logdet']}")
    assert null[2] == pytest.approx(ref["logdet"], rel=1e-11, abs=1e-9)
    assert null[1] == pytest.approx(ref["chi2_0"], rel=1e-9)
    assert null[0] == pytest.approx(ref["lnl0"], rel=1e-11, abs=1e-8)


def _run(api, ctx, w, kernel, terms, sw, A="trend"):
    import torch
    trend = w.A if A == "trend" else None
    ls = api.linear_search_ss(ctx, w.t, kernel, w.f, trend, w.lattice, w.n_epochs, w.durations)
    torch.cuda.synchronize()
    L = ogp.cholesky(ogp.covariance_terms(w.t, terms, sw))
    ref = olin.linear_search(w.f, trend if trend is not None else np.zeros((w.n, 0)), L, w.lattice, w.durations,
                             n_epochs=w.n_epochs)
    return ls, ref


@pytest.mark.parametrize("n,gap,extra", [(300, None, False), (900, (450, 30), False), (1500, (700, 45), True)])
def test_rotation_kernel_matches_oracle(api, ctx, n, gap, extra):
    w = _curve(n, 41, gap)
    terms = _rot_terms()
    k = api.rotation_kernel(**ROT)
    if extra:  # an overdamped oscillator on top (the hyperbolic branch)
        terms["sho"].append((0.004, 30.0, 0.3))
        k.sho.append((0.004, 30.0, 0.3))
    say(f"state-space rotation kernel N={n} gap={gap} extra={extra}")
    ls, ref = _run(api, ctx, w, k, terms, ROT["sigma_w"])
    _close(_host(ls), ref, f"ss rotation N={n}")
    _null_close(ls, ref, f"ss rotation N={n}")


KERNELS = {
    "critical": {"sho": [(0.01, 20.0, 0.5)], "exp": []},
    "overdamped": {"sho": [(0.01, 20.0, 0.2)], "exp": []},
    "exp-only": {"sho": [], "exp": [(0.006, 0.1)]},
    "two-exp": {"sho": [], "exp": [(0.006, 0.1), (0.002, 0.01)]},
    "widest": {"sho": [(0.006, 8.0, 3.0), (0.003, 16.0, 1.2), (0.002, 40.0, 0.5), (0.002, 25.0, 0.3)],
               "exp": [(0.001, 0.02), (0.002, 0.3), (0.0015, 2.0), (0.001, 0.05)]},
}


@pytest.mark.parametrize("name", sorted(KERNELS))
def test_term_shapes_match_oracle(api, ctx, name):
    terms = KERNELS[name]
    w = _curve(420, 43, (200, 17))
    k = api.Kernel(sho=list(terms["sho"]), exp=list(terms["exp"]), sigma_w=1.5e-3)
    say(f"state-space kernel {name} N={w.n}")
    ls, ref = _run(api, ctx, w, k, terms, 1.5e-3)
    _close(_host(ls), ref, f"ss {name}")
    _null_close(ls, ref, f"ss {name}")


def test_single_sho_small_configuration(api, ctx):
    import torch
    w = config1()
    say(f"state-space single SHO on the small configuration N={w.n}")
    ls = api.linear_search_ss(ctx, w.t, api.SHO.from_dict(w.theta), w.f, w.A, w.lattice, w.n_epochs, w.durations)
    torch.cuda.synchronize()
    L = ogp.cholesky(ogp.covariance(w.t, w.theta))
    ref = olin.linear_search(w.f, w.A, L, w.lattice, w.durations, n_epochs=w.n_epochs)
    _close(_host(ls), ref, "ss config1")
    _null_close(ls, ref, "ss config1")


def test_no_trend_and_extreme_durations(api, ctx):
    w = _curve(1300, 47, (600, 40), durations=(1, 1024, 37))
    terms = _rot_terms()
    say(f"state-space no trend, durations {w.durations.tolist()}")
    ls, ref = _run(api, ctx, w, api.rotation_kernel(**ROT), terms, ROT["sigma_w"], A=None)
    _close(_host(ls), ref, "ss no trend")
    _null_close(ls, ref, "ss no trend")


def test_full_size_rotation_sampled(api, ctx):
    import torch
    w = config2()
    terms = _rot_terms()
    say(f"state-space full size N={w.n} n_epochs={w.n_epochs} n_d={w.durations.size}")
    ls = api.linear_search_ss(ctx, w.t, api.rotation_kernel(**ROT), w.f, w.A, w.lattice, w.n_epochs, w.durations)
    torch.cuda.synchronize()
    gpu = _host(ls)
    say("oracle Cholesky of the rotation kernel at N=18000 (CPU)")
    L = ogp.cholesky(ogp.covariance_terms(w.t, terms, ROT["sigma_w"]))
    rng = np.random.default_rng(17)
    n_d, n_t = gpu["dll"].shape
    cells = [(int(rng.integers(n_d)), int(rng.integers(n_t))) for _ in range(100)]
    for i in (0, 1, 8999, 9000, 9001, 9719, 9720, 9721, n_t - 2, n_t - 1):
        for j in (0, n_d - 1):
            cells.append((j, i))
    ref = olin.linear_search(w.f, w.A, L, w.lattice, w.durations, cells=cells)
    sel = {k: np.array([gpu[k][j, i] for (j, i) in cells]) for k in gpu}
    _close(sel, ref, "ss full size sampled")
    _null_close(ls, ref, "ss full size")


def test_not_positive_definite_is_reported(api, ctx):
    import torch
    from paper_2402_06835_amd._lib import NU_ERR_NOT_PD, NuanceError
    w = _curve(200, 53)
    k = api.Kernel(sho=[(0.0, 10.0, 2.0)], sigma_w=0.0)  # K = 0
    say("state-space K = 0, checked")
    with pytest.raises(NuanceError) as ei:
        api.linear_search_ss(ctx, w.t, k, w.f, w.A, w.lattice, w.n_epochs, w.durations)
    assert ei.value.status == NU_ERR_NOT_PD and ei.value.index == 0
    say("state-space K = 0, unchecked")
    ls = api.linear_search_ss(ctx, w.t, k, w.f, w.A, w.lattice, w.n_epochs, w.durations, check=False)
    torch.cuda.synchronize()
    assert math.isnan(float(ls["null"][0])) and math.isnan(float(ls["null"][2]))
    assert int(ls["valid"].sum()) == 0
    # the context still works afterwards
    ok = api.linear_search_ss(ctx, w.t, api.rotation_kernel(**ROT), w.f, w.A, w.lattice, w.n_epochs, w.durations)
    torch.cuda.synchronize()
    assert int(ok["valid"].sum()) > 0


def test_argument_errors(api, ctx):
    from paper_2402_06835_amd._lib import NU_ERR_ARG, NuanceError
    w = _curve(100, 59)
    bad = [api.Kernel(sigma_w=1e-3),                                  # no term
           api.Kernel(sho=[(0.01, -1.0, 1.0)], sigma_w=1e-3),           # omega <= 0
           api.Kernel(exp=[(0.01, 0.0)], sigma_w=1e-3),                 # ell <= 0
           api.Kernel(sho=[(0.01, 1.0, 1.0)], sigma_w=float("nan"))]    # sigma_w not finite
    for k in bad:
        with pytest.raises(NuanceError) as ei:
            api.linear_search_ss(ctx, w.t, k, w.f, w.A, w.lattice, w.n_epochs, w.durations)
        assert ei.value.status == NU_ERR_ARG
    with pytest.raises(NuanceError) as ei:  # a duration beyond 1024 slots
        api.linear_search_ss(ctx, w.t, api.rotation_kernel(**ROT), w.f, w.A, w.lattice, w.n_epochs, [4, 2000])
    assert ei.value.status == NU_ERR_ARG


def test_nuance_object_statespace_solver(api):
    w = config1()
    say("Nuance object, state-space solver against the dense one on the small configuration")
    dense = api.Nuance(w.t, w.f, gp=api.SHO.from_dict(w.theta), X=w.A)
    ss = api.Nuance(w.t, w.f, gp=api.SHO.from_dict(w.theta), X=w.A, solver="statespace")
    a = dense.linear_search(w.t.copy(), w.durations * w.dt)
    b = ss.linear_search(w.t.copy(), w.durations * w.dt)
    ga, gb = _host(a), _host(b)
    np.testing.assert_array_equal(ga["valid"], gb["valid"])
    v = ga["valid"].astype(bool)
    assert np.max(np.abs(ga["dll"][v] - gb["dll"][v]) / np.maximum(np.abs(ga["dll"][v]), 1.0)) <= DLL_TOL
    ra, rb = dense.periodic_search(w.periods), ss.periodic_search(w.periods)
    assert ra.best[0] == rb.best[0]
    with pytest.raises(ValueError):
        api.Nuance(w.t, w.f, gp=api.SHO.from_dict(w.theta), solver="banded")


def test_chunked_and_sequential_filters_agree(api, ctx):
    """The chunked (parallel-in-time) filter runs for kernels of at most 6 states with white noise and
    positive term variances, the one-wave sequential filter otherwise. An extra SHO term of zero amplitude
    leaves K unchanged but sends the search down the sequential path: both must give the same cells."""
    import torch
    w = config2()
    k = api.rotation_kernel(**ROT)
    k_seq = api.Kernel(sho=list(k.sho) + [(0.0, 5.0, 2.0)], exp=list(k.exp), sigma_w=k.sigma_w)
    say(f"chunked against sequential filter at N={w.n}")
    a = _host(api.linear_search_ss(ctx, w.t, k, w.f, w.A, w.lattice, w.n_epochs, w.durations))
    b_ls = api.linear_search_ss(ctx, w.t, k_seq, w.f, w.A, w.lattice, w.n_epochs, w.durations)
    b = _host(b_ls)
    torch.cuda.synchronize()
    np.testing.assert_array_equal(a["valid"], b["valid"])
    v = a["valid"].astype(bool)
    e = float(np.max(np.abs(a["dll"][v] - b["dll"][v]) / np.maximum(np.abs(b["dll"][v]), 1.0)))
    say(f"chunked vs sequential max dll error {e}")
    assert e <= 1e-10


def test_no_white_noise_sequential_path(api, ctx):
    """sigma_w = 0 (the chunked filter needs white noise): an exponential kernel is still positive definite."""
    terms = {"sho": [], "exp": [(0.006, 0.1), (0.002, 0.02)]}
    w = _curve(500, 73, (240, 11))
    k = api.Kernel(exp=list(terms["exp"]), sigma_w=0.0)
    say("state-space exponential kernel without white noise")
    ls, ref = _run(api, ctx, w, k, terms, 0.0)
    _close(_host(ls), ref, "ss no white noise")


@pytest.mark.parametrize("n", [1, 2, 3, 191, 192, 193, 384, 385])
def test_chunk_boundary_sizes(api, ctx, n):
    """Sizes around the chunk length of the chunked filter (192 samples), and the smallest curves (where
    boxes over every sample are collinear with the constant trend: invalid on both sides)."""
    import torch
    terms = _rot_terms()
    k = api.rotation_kernel(**ROT)
    rng = np.random.default_rng(100 + n)
    t = np.arange(n) * (10 / 1440)
    lattice = np.arange(n, dtype=np.int64)
    f = 1.0 + rng.normal(0, 2e-3, n)
    A = np.ones((n, 1)) if n >= 2 else np.zeros((n, 0))
    durs = np.array([1, 4, 9][: max(1, min(3, n))], dtype=np.int32)
    say(f"state-space chunk-boundary size N={n}")
    ls = api.linear_search_ss(ctx, t, k, f, A if A.shape[1] else None, lattice, n, durs)
    torch.cuda.synchronize()
    L = ogp.cholesky(ogp.covariance_terms(t, terms, ROT["sigma_w"]))
    ref = olin.linear_search(f, A, L, lattice, durs, n_epochs=n)
    _close(_host(ls), ref, f"ss N={n}")
    _null_close(ls, ref, f"ss N={n}")
