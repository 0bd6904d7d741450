"""GPU: the single-event search with a non-box base model (entry point 2c,
and the shapes argument of the state-space search 2b) against the oracle
(``oracle.templates.linear_search_template``).

* Dense factor, FP64: limb-darkened (central and grazing) and exocomet shapes
  on a curve with a gap, durations 1 to 13 slots, at the FP64 bar (1e-9 on
  dll relative to max(|dll|, 1), depth in units of its sigma, var relative);
  FP32_REFINE and BF16X3_REFINE at the reduced-precision bar (1e-6).
* State-space path: the same shapes with the rotation kernel of Section 3.2
  and with one SHO term, at the FP64 bar.
* The unit shape gives the box search of (2); a one-slot shape of value c
  gives the box depth divided by c.
* The TESS-sector size (N = 18000) on sampled cells: dense FP32_REFINE with
  the limb-darkened shape, and the state-space path with the exocomet shape.
* Shapes over 2048 values, or with a non-finite value, are argument errors.
"""
import numpy as np
import pytest

from oracle import gp as ogp, templates as otpl
from synth import config2, make_workload, sho_omega_from_rotation
from synth import templates as stpl

pytestmark = pytest.mark.gpu

FP64_TOL, MIXED_TOL = 1e-9, 1e-6

ROT = dict(sigma=0.012, period=0.9, q0=1.5, dq=2.0, f=0.5, sigma_short=8e-4, ell_short=0.02,
           sigma_long=3e-3, ell_long=4.0, sigma_w=1e-3)


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


def _curve(n=700, seed=61, gap=(330, 23), durations=(1, 6, 13)):
    th = {"amp": 0.008, "omega": sho_omega_from_rotation(0.8, 4.0), "q": 4.0, "sigma_w": 1e-3}
    return make_workload(f"tpl-N{n}", seed, n, 10 / 1440, th, list(durations), np.linspace(0.3, 2.0, 40),
                         gaps=[gap] if gap else [],
                         injection={"depth": 2e-3, "period": 0.55, "t0": 0.21, "duration": 0.06})


SHAPES = {
    "limb_darkened": lambda d: stpl.limb_darkened(d),
    "grazing": lambda d: stpl.limb_darkened(d, u1=0.3, u2=0.3, b=0.7),
    "exocomet": lambda d: stpl.exocomet(d),
}


def _host(ls):
    return {k: ls[k].cpu().numpy() for k in ("depth", "var", "dll", "valid")}


def _close(gpu, ref, tol, tag):
    v = ref["valid"].astype(bool)
    np.testing.assert_array_equal(gpu["valid"].astype(bool), v, err_msg=tag)
    assert v.any()
    e = {"dll": float(np.max(np.abs(gpu["dll"][v] - ref["dll"][v]) / np.maximum(np.abs(ref["dll"][v]), 1.0))),
         "depth": float(np.max(np.abs(gpu["depth"][v] - ref["depth"][v]) / np.sqrt(ref["var"][v]))),
         "var": float(np.max(np.abs(gpu["var"][v] - ref["var"][v]) / ref["var"][v]))}
    say(f"{tag} max errors {e}")
    assert max(e.values()) <= tol, (tag, e)
    inv = ~v
    assert np.all(gpu["dll"][inv] == 0.0) and np.all(np.isinf(gpu["var"][inv]))


@pytest.mark.parametrize("kind", sorted(SHAPES))
@pytest.mark.parametrize("precision,tol", [("fp64", FP64_TOL), ("fp32_refine", MIXED_TOL),
                                           ("bf16x3_refine", MIXED_TOL)])
def test_dense_template_matches_oracle(api, ctx, kind, precision, tol):
    import torch
    w = _curve()
    shapes = [SHAPES[kind](int(d)) for d in w.durations]
    say(f"dense template {kind} {precision} N={w.n}")
    fac = api.gp_factor(ctx, w.t, w.theta)
    ls = api.linear_search(ctx, fac, w.f, w.A, w.lattice, w.n_epochs, w.durations, precision, shapes=shapes)
    torch.cuda.synchronize()
    L = ogp.cholesky(ogp.covariance(w.t, w.theta))
    ref = otpl.linear_search_template(w.f, w.A, L, w.lattice, shapes, n_epochs=w.n_epochs)
    _close(_host(ls), ref, tol, f"dense {kind} {precision}")


@pytest.mark.parametrize("kind", sorted(SHAPES))
@pytest.mark.parametrize("kernel", ["rotation", "sho"])
def test_statespace_template_matches_oracle(api, ctx, kind, kernel):
    import torch
    w = _curve(seed=67)
    shapes = [SHAPES[kind](int(d)) for d in w.durations]
    if kernel == "rotation":
        k = api.rotation_kernel(**ROT)
        terms = ogp.rotation_terms(ROT["sigma"], ROT["period"], ROT["q0"], ROT["dq"], ROT["f"], ROT["sigma_short"],
                                   ROT["ell_short"], ROT["sigma_long"], ROT["ell_long"])
        K = ogp.covariance_terms(w.t, terms, ROT["sigma_w"])
    else:
        k = api.SHO.from_dict(w.theta)
        K = ogp.covariance(w.t, w.theta)
    say(f"state-space template {kind} kernel={kernel} N={w.n}")
    ls = api.linear_search_ss(ctx, w.t, k, w.f, w.A, w.lattice, w.n_epochs, w.durations, shapes=shapes)
    torch.cuda.synchronize()
    ref = otpl.linear_search_template(w.f, w.A, ogp.cholesky(K), w.lattice, shapes, n_epochs=w.n_epochs)
    _close(_host(ls), ref, FP64_TOL, f"ss {kind} {kernel}")


def test_unit_and_scaled_shapes(api, ctx):
    import torch
    w = _curve(n=500, seed=71, durations=(1, 5, 12))
    fac = api.gp_factor(ctx, w.t, w.theta)
    say("unit shapes against the box search; a one-slot shape of value c")
    box = _host(api.linear_search(ctx, fac, w.f, w.A, w.lattice, w.n_epochs, w.durations))
    unit = _host(api.linear_search(ctx, fac, w.f, w.A, w.lattice, w.n_epochs, w.durations,
                                   shapes=[np.ones(int(d)) for d in w.durations]))
    ss_unit = _host(api.linear_search_ss(ctx, w.t, api.SHO.from_dict(w.theta), w.f, w.A, w.lattice, w.n_epochs,
                                         w.durations, shapes=[np.ones(int(d)) for d in w.durations]))
    c = 2.5
    scaled = _host(api.linear_search(ctx, fac, w.f, w.A, w.lattice, w.n_epochs, w.durations,
                                     shapes=[np.full(int(d), c) for d in w.durations]))
    torch.cuda.synchronize()
    v = box["valid"].astype(bool)
    for got, tag in ((unit, "dense unit"), (ss_unit, "state-space unit")):
        np.testing.assert_array_equal(got["valid"], box["valid"], err_msg=tag)
        assert np.max(np.abs(got["dll"][v] - box["dll"][v]) / np.maximum(np.abs(box["dll"][v]), 1.0)) <= FP64_TOL
        assert np.max(np.abs(got["depth"][v] - box["depth"][v]) / np.sqrt(box["var"][v])) <= FP64_TOL
    np.testing.assert_allclose(scaled["depth"][v], box["depth"][v] / c, rtol=1e-9, atol=1e-15)
    np.testing.assert_allclose(scaled["var"][v], box["var"][v] / c ** 2, rtol=1e-9)


def _sampled_cells(n_d, n_t, seed):
    rng = np.random.default_rng(seed)
    cells = [(int(rng.integers(n_d)), int(rng.integers(n_t))) for _ in range(80)]
    for i in (0, 1, 8999, 9000, 9001, 9719, 9720, 9721, n_t - 2, n_t - 1):
        for j in (0, n_d - 1):
            cells.append((j, i))
    return cells


def test_full_size_sampled(api, ctx):
    import torch
    w = config2()
    ld = [stpl.limb_darkened(int(d)) for d in w.durations]
    com = [stpl.exocomet(int(d)) for d in w.durations]
    say(f"full-size templates N={w.n}: dense FP32_REFINE limb-darkened, state-space exocomet")
    fac = api.gp_factor(ctx, w.t, w.theta)
    dense = _host(api.linear_search(ctx, fac, w.f, w.A, w.lattice, w.n_epochs, w.durations, "fp32_refine",
                                    shapes=ld))
    ss = _host(api.linear_search_ss(ctx, w.t, api.SHO.from_dict(w.theta), w.f, w.A, w.lattice, w.n_epochs,
                                    w.durations, shapes=com))
    torch.cuda.synchronize()
    del fac
    say("oracle Cholesky at N=18000 (CPU)")
    L = ogp.cholesky(ogp.covariance(w.t, w.theta))
    n_d, n_t = dense["dll"].shape
    cells = _sampled_cells(n_d, n_t, 23)
    for got, shapes, tol, tag in ((dense, ld, MIXED_TOL, "dense fp32_refine limb-darkened"),
                                  (ss, com, FP64_TOL, "state-space exocomet")):
        ref = otpl.linear_search_template(w.f, w.A, L, w.lattice, shapes, cells=cells)
        sel = {k: np.array([got[k][j, i] for (j, i) in cells]) for k in got}
        _close(sel, ref, tol, f"full size {tag}")


def test_shape_argument_errors(api, ctx):
    from paper_2402_06835_amd._lib import NU_ERR_ARG, NuanceError
    w = _curve(n=300, gap=None, durations=(4, 9))
    fac = api.gp_factor(ctx, w.t, w.theta)
    bad_nan = [np.ones(4), np.array([1.0] * 8 + [np.nan])]
    for call in (lambda s: api.linear_search(ctx, fac, w.f, w.A, w.lattice, w.n_epochs, w.durations, shapes=s),
                 lambda s: api.linear_search_ss(ctx, w.t, api.SHO.from_dict(w.theta), w.f, w.A, w.lattice,
                                                w.n_epochs, w.durations, shapes=s)):
        with pytest.raises(NuanceError) as ei:
            call(bad_nan)
        assert ei.value.status == NU_ERR_ARG
        with pytest.raises(ValueError):
            call([np.ones(4)])                     # one shape per duration
        with pytest.raises(ValueError):
            call([np.ones(4), np.ones(8)])         # shape 1 needs 9 values
    long_durs = [1000, 1000, 100]                  # 2100 values together
    with pytest.raises(NuanceError) as ei:
        api.linear_search(ctx, fac, w.f, w.A, w.lattice, w.n_epochs, long_durs,
                          shapes=[np.ones(d) for d in long_durs])
    assert ei.value.status == NU_ERR_ARG
