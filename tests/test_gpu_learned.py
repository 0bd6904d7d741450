"""GPU parity of the learned warm start and the hyperparameter fit (entry point 7)
against the oracle: the sampler (same Philox draws, so the same curves), the CNN
input, the trend-profiled likelihood (Kalman on the GPU against the dense
Cholesky likelihood of the oracle and of the GPU's own search), the plain start,
BFGS, and the network's forward pass, gradient and Adam step.

Bars: sampler flux within 1e-10 (transcendental functions and the closed-form
transition differ from the oracle's in the last bits; the recursion contracts);
integer decisions (bins, prior draws' ordering) exact; the likelihood within
1e-10 relative; the FP32 network within 1e-4 relative on outputs, the gradient
within 1e-3 relative in norm with cosine >= 0.9999 against the FP64 oracle.
"""
import math

import numpy as np
import pytest

from oracle import learned as ol

pytestmark = pytest.mark.gpu


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


def _t_with_gap(n, dt=2 / 1440, gap_after=None, gap=0):
    t = np.arange(n) * dt
    if gap_after is not None:
        t[gap_after:] += gap * dt
    return t


def test_sampler_matches_oracle_given_theta(api, ctx):
    t = _t_with_gap(300, gap_after=140, gap=60)
    thetas = [{"amp": 0.01, "omega": ol.omega_from_rotation(0.4, 5.0), "q": 5.0, "sigma_w": 1e-3},
              {"amp": 0.02, "omega": 3.0, "q": 0.5, "sigma_w": 5e-4},
              {"amp": 0.005, "omega": 7.0, "q": 0.3, "sigma_w": 2e-3}]
    say("sampler, 3 given thetas (Q > 1/2, = 1/2, < 1/2), N=300 with a gap")
    out = api.gp_sample(ctx, t, 3, theta=thetas, seed=1234, curve_base=10, n_bins=64, flux=True)
    flux = out["flux"].cpu().numpy()
    for c, th in enumerate(thetas):
        ref = ol.sample_curve(t, th, 1234, 10 + c)
        np.testing.assert_allclose(flux[c], ref, rtol=0, atol=1e-10)
        x = ol.bin_input(t, ref, 64)
        np.testing.assert_allclose(out["input"].cpu().numpy()[c], x, rtol=1e-5, atol=1e-5)


def test_sampler_prior_draws_and_targets(api, ctx):
    t = _t_with_gap(200)
    say("sampler, 8 curves with prior draws")
    out = api.gp_sample(ctx, t, 8, theta=None, seed=77, curve_base=5, n_bins=32, flux=True)
    th = out["theta"].cpu().numpy()
    tg = out["target"].cpu().numpy()
    for c in range(8):
        d = ol.draw_theta(77, 5 + c)
        om = ol.omega_from_rotation(d["prot"], d["q"])
        np.testing.assert_allclose(th[c], [d["amp"], om, d["q"], d["sigma_w"]], rtol=1e-13)
        np.testing.assert_allclose(tg[c], ol.standardise(d), rtol=1e-6, atol=1e-6)
        ref = ol.sample_curve(t, {"amp": d["amp"], "omega": om, "q": d["q"], "sigma_w": d["sigma_w"]}, 77, 5 + c)
        np.testing.assert_allclose(out["flux"].cpu().numpy()[c], ref, rtol=0, atol=1e-10)


def _batch(api, ctx, curves):
    return api.prepare_batch(ctx, [{"t": t, "f": f, "A": A, "lattice": np.arange(t.size), "n_epochs": t.size,
                                    "theta": {"amp": 1.0, "omega": 1.0, "q": 1.0, "sigma_w": 1.0}, "dt": 1.0}
                                   for t, f, A in curves])


def _trend(t, m):
    x = (t - t.mean()) / (np.ptp(t) / 2)
    return np.column_stack([x ** k for k in range(m)]) if m else np.zeros((t.size, 0))


@pytest.mark.parametrize("m1", [0, 1, 3])
def test_kalman_likelihood_matches_oracle_dense(api, ctx, m1):
    rng = np.random.default_rng(m1)
    curves = []
    for n, gap in ((300, 40), (450, 0), (129, 10)):
        t = _t_with_gap(n, dt=5 / 1440, gap_after=n // 2, gap=gap)
        f = 1.0 + 0.01 * np.sin(t * 9.0) + 1e-3 * rng.standard_normal(n)
        curves.append((t, f, _trend(t, m1)))
    thetas = [{"amp": 0.01, "omega": 9.0, "q": 5.0, "sigma_w": 1.2e-3},
              {"amp": 0.02, "omega": 4.0, "q": 0.5, "sigma_w": 8e-4},
              {"amp": 0.004, "omega": 20.0, "q": 0.3, "sigma_w": 2e-3}]
    say(f"Kalman likelihood, m1={m1}, 3 curves x 3 thetas")
    b = _batch(api, ctx, curves)
    nll = api.gp_nll(ctx, b, [th for _ in curves for th in thetas], n_eval=3).cpu().numpy()
    for c, (t, f, A) in enumerate(curves):
        for e, th in enumerate(thetas):
            ref = ol.nll_dense(t, f, A, th)
            assert nll[c, e] == pytest.approx(ref, rel=1e-10, abs=1e-7), (c, e)


def test_kalman_likelihood_matches_the_searchs_dense_null_fit(api, ctx):
    import torch
    # two independent GPU derivations of Eq. 5 for the trend-only model: the Kalman
    # innovations and the dense Cholesky of the linear search (ln L_0)
    t = _t_with_gap(700, dt=10 / 1440, gap_after=333, gap=25)
    rng = np.random.default_rng(9)
    f = 1.0 + 2e-3 * rng.standard_normal(t.size)
    A = _trend(t, 3)
    th = {"amp": 0.01, "omega": ol.omega_from_rotation(1.2, 5.0), "q": 5.0, "sigma_w": 1e-3}
    say("Kalman likelihood vs the search's ln L_0, N=700")
    b = _batch(api, ctx, [(t, f, A)])
    nll = float(api.gp_nll(ctx, b, [th]).cpu().numpy()[0, 0])
    fac = api.gp_factor(ctx, t, th)
    lat = np.rint((t - t[0]) / (10 / 1440)).astype(np.int64)
    ls = api.linear_search(ctx, fac, f, A, lat, int(lat[-1]) + 1, [3])
    torch.cuda.synchronize()
    assert -float(ls["null"][0].item()) == pytest.approx(nll, rel=1e-10)


def test_plain_init_matches_oracle(api, ctx):
    rng = np.random.default_rng(5)
    grid = np.exp(np.linspace(math.log(0.2), math.log(3.0), 400))
    curves = []
    for c, n in enumerate((800, 1200)):
        t = np.arange(n) * (2 / 1440) * 10
        th = {"amp": 0.01, "omega": ol.omega_from_rotation(0.5 + 0.4 * c, 5.0), "q": 5.0, "sigma_w": 1e-3}
        curves.append((t, ol.sample_curve(t, th, 3, c), np.ones((n, 1))))
    say("plain start: Lomb-Scargle, moments")
    b = _batch(api, ctx, curves)
    x0 = api.plain_init(ctx, b, grid).cpu().numpy()
    for c, (t, f, _) in enumerate(curves):
        ref = ol.plain_init(t, f, grid)
        np.testing.assert_allclose(np.exp(x0[c]), [ref["amp"], ref["prot"], ref["q"], ref["sigma_w"]], rtol=1e-10)


def test_fit_reaches_the_oracle_optimum(api, ctx):
    say("BFGS fit of 3 curves vs SciPy BFGS on the oracle likelihood")
    curves, starts = [], []
    for c in range(3):
        t = np.arange(500) * (10 / 1440)
        truth = {"amp": 0.01 + 0.005 * c, "prot": 0.6 + 0.3 * c, "q": 6.0, "sigma_w": 1e-3}
        th = {"amp": truth["amp"], "omega": ol.omega_from_rotation(truth["prot"], truth["q"]), "q": truth["q"],
              "sigma_w": truth["sigma_w"]}
        curves.append((t, ol.sample_curve(t, th, 21, c), np.ones((t.size, 1))))
        starts.append({k: v * 1.3 for k, v in truth.items()})
    b = _batch(api, ctx, curves)
    x0 = np.log([[s["amp"], s["prot"], s["q"], s["sigma_w"]] for s in starts])
    res = api.fit_hyper(ctx, b, x0, max_iter=200, gtol=1e-4)
    for c, (t, f, A) in enumerate(curves):
        ref = ol.fit_bfgs(t, f, A, starts[c])
        say(f"curve {c}: gpu nll {res['nll'][c]:.6f} ({res['n_eval'][c]} evals), oracle {ref.fun:.6f}")
        assert res["nll"][c] <= ref.fun + 1e-3
        assert ol.nll_kalman(t, f, A, ol.theta_from_x(res["x"][c])) == pytest.approx(res["nll"][c], rel=1e-10)


def _cnn_case(seed, batch=6):
    rng = np.random.default_rng(seed)
    p = ol.init_params(seed)
    x = rng.standard_normal((batch, 512))
    y = rng.standard_normal((batch, 4))
    return p, x, y


def test_cnn_forward_fp32_and_fp16(api, ctx):
    import torch
    p, x, y = _cnn_case(1)
    say("CNN forward, FP32 and FP16 products")
    ref, _ = ol.cnn_forward(p, x)
    xt = torch.as_tensor(x, dtype=torch.float32, device="cuda")
    for half, tol in ((False, 1e-4), (True, 3e-2)):
        m = api.CNN(ctx, half=half, max_batch=8, params=p)
        out, xlog = m.forward(xt)
        torch.cuda.synchronize()
        got = out.cpu().numpy()
        err = np.abs(got - ref).max() / np.abs(ref).max()
        say(f"half={half}: max rel error {err:.2e}")
        assert err < tol
        # fit coordinates: the prior's log-uniform centre and scale applied to the outputs
        y0 = ol.unstandardise(got[0])
        np.testing.assert_allclose(np.exp(xlog.cpu().numpy()[0]), [y0[k] for k in ol.TARGET_KEYS], rtol=1e-6)
        m.close()


def test_cnn_gradient_against_oracle(api, ctx):
    import torch
    p, x, y = _cnn_case(2, batch=5)
    say("CNN gradient, FP32 and FP16 products vs the FP64 oracle")
    loss_ref, g_ref = ol.cnn_backward(p, x, y)
    xt = torch.as_tensor(x, dtype=torch.float32, device="cuda")
    yt = torch.as_tensor(y, dtype=torch.float32, device="cuda")
    for half, rel, cos_min in ((False, 1e-3, 0.9999), (True, 5e-2, 0.999)):
        m = api.CNN(ctx, half=half, max_batch=8, params=p)
        g, loss = m.gradient(xt, yt)
        torch.cuda.synchronize()
        g = g.cpu().numpy().astype(np.float64)
        e = np.linalg.norm(g - g_ref) / np.linalg.norm(g_ref)
        cos = g @ g_ref / (np.linalg.norm(g) * np.linalg.norm(g_ref))
        say(f"half={half}: rel norm error {e:.2e}, cosine {cos:.8f}, loss {loss.item():.6f} vs {loss_ref:.6f}")
        assert e < rel and cos > cos_min
        assert loss.item() == pytest.approx(loss_ref, rel=1e-4 if not half else 3e-2)
        # every parameter block gets its gradient (no block left at zero)
        off = 0
        for name, shp in ol.param_shapes():
            k = int(np.prod(shp))
            assert np.linalg.norm(g[off:off + k] - g_ref[off:off + k]) <= 10 * rel * np.linalg.norm(g_ref[off:off + k]) + 1e-7, name
            off += k
        m.close()


def test_cnn_adam_step_matches_oracle(api, ctx):
    import torch
    p, x, y = _cnn_case(3, batch=4)
    say("CNN train step (gradient + Adam), FP32")
    _, g_ref = ol.cnn_backward(p, x, y)
    p1, _, _ = ol.adam_step(p, g_ref, np.zeros_like(p), np.zeros_like(p), 1, lr=1e-3)
    m = api.CNN(ctx, half=False, max_batch=8, params=p)
    m.train_step(torch.as_tensor(x, dtype=torch.float32, device="cuda"),
                 torch.as_tensor(y, dtype=torch.float32, device="cuda"), lr=1e-3)
    got = m.get_params().astype(np.float64)
    # the first Adam step moves each parameter by about lr * sign(g); compare the moves
    step, step_ref = got - p.astype(np.float32), p1 - p
    big = np.abs(g_ref) > 1e-4 * np.abs(g_ref).max()
    np.testing.assert_allclose(step[big], step_ref[big], rtol=2e-2, atol=2e-6)
    m.close()


def test_cnn_training_reduces_the_loss(api, ctx):
    import torch
    say("CNN training on sampled curves, 150 steps of 128, FP16 products")
    t = np.arange(3000) * (2 / 1440) * 4
    data = api.gp_sample(ctx, t, 2048, theta=None, seed=5, n_bins=512)
    m = api.CNN(ctx, half=True, max_batch=128, params=ol.init_params(7))
    loss = torch.empty(1, dtype=torch.float32, device="cuda")
    x, y = data["input"], data["target"]
    first = last = None
    for step in range(150):
        i = (step * 128) % 2048
        m.train_step(x[i:i + 128], y[i:i + 128], lr=1e-3, loss=loss)
        if step < 10:
            first = loss.item() if first is None else first + loss.item()
        if step >= 140:
            last = loss.item() if last is None else last + loss.item()
    say(f"mean loss of the first 10 steps {first / 10:.4f}, of the last 10 {last / 10:.4f}")
    assert last / 10 < 0.7 * first / 10
    m.close()


def test_learned_warm_start_gain(api, ctx):
    """What the trained network gains over the plain start, at the TESS-sector shape:
    the network is trained on the GPU on 100000 curves drawn from the GP, then both
    starts seed the same BFGS fit on 128 held-out curves. The reference is the best optimum
    found from the plain, learned and true starts."""
    import torch
    dt = 2 / 1440
    t = np.arange(18000) * dt
    t[9000:] += 720 * dt
    say("learned warm start: sample 100000 curves N=18000, train 12 epochs, fit 128 held-out curves")
    ntr, bs = 100000, 256
    X = torch.empty((ntr, 512), dtype=torch.float32, device="cuda")
    Y = torch.empty((ntr, 4), dtype=torch.float32, device="cuda")
    for base in range(0, ntr, 8192):
        k = min(8192, ntr - base)
        d = api.gp_sample(ctx, t, k, theta=None, seed=5_000_000, curve_base=base)
        X[base:base + k] = d["input"]
        Y[base:base + k] = d["target"]
    m = api.CNN(ctx, half=True, max_batch=bs, seed=1)
    steps = ntr // bs
    for ep in range(12):
        lr = 2e-3 * 0.5 ** (ep // 4)
        for s in range(steps):
            j = ((s + 37 * ep) % steps) * bs  # a different order each epoch, deterministic
            m.train_step(X[j:j + bs], Y[j:j + bs], lr=lr)
    torch.cuda.synchronize()
    nev = 128
    d = api.gp_sample(ctx, t, nev, theta=None, seed=6000, curve_base=0, flux=True)
    th = d["theta"].cpu().numpy()
    prot = 4 * np.pi * th[:, 2] / (th[:, 1] * np.sqrt(4 * th[:, 2] ** 2 - 1))
    x_true = np.log(np.column_stack([th[:, 0], prot, th[:, 2], th[:, 3]]))
    x = (t - t.mean()) / (np.ptp(t) / 2)
    A1 = np.concatenate([np.stack([np.ones_like(x), x, x * x])] * nev).reshape(-1)
    batch = {"n_curves": nev, "sample_off": np.arange(nev + 1, dtype=np.int64) * t.size,
             "t": torch.as_tensor(np.tile(t, nev), device="cuda"), "f": d["flux"].reshape(-1).contiguous(),
             "A": torch.as_tensor(A1, device="cuda"), "m1": 3}
    grid = np.exp(np.linspace(math.log(0.1), math.log(5.0), 1000))
    x_plain = api.plain_init(ctx, batch, grid)
    x_learned = m.warm_start(d["input"], x_plain)
    starts = {"plain": x_plain.cpu().numpy(), "learned": x_learned.cpu().numpy(), "truth": x_true}
    fits = {k: api.fit_hyper(ctx, batch, v, max_iter=300, gtol=1e-3) for k, v in starts.items()}
    best = np.min(np.stack([f["nll"] for f in fits.values()]), axis=0)

    def start_gap(x0):
        rows = []
        for r in x0:
            amp, p_rot, q, sw = np.exp(r)
            rows.append([amp, ol.omega_from_rotation(p_rot, q), q, sw])
        return api.gp_nll(ctx, batch, torch.as_tensor(np.array(rows), device="cuda")).cpu().numpy()[:, 0] - best

    stats = {}
    for k in ("plain", "learned"):
        gap = fits[k]["nll"] - best
        stats[k] = {"success": float(np.mean(gap < 0.1)), "evals": float(fits[k]["n_eval"].mean()),
                    "start_gap": float(np.median(start_gap(starts[k]))),
                    "q_err": float(np.median(np.abs(starts[k][:, 2] - x_true[:, 2])))}
        say(f"{k}: {stats[k]}")
    assert stats["learned"]["success"] >= stats["plain"]["success"]
    assert stats["learned"]["start_gap"] < stats["plain"]["start_gap"] / 5
    assert stats["learned"]["q_err"] < stats["plain"]["q_err"] / 2
    assert stats["learned"]["evals"] < 0.95 * stats["plain"]["evals"]
    m.close()
