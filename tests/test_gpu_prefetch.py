"""GPU: the inverse prefetch (``nu_ctx_set_inverse_prefetch``) changes when the
reduced-precision inverse is computed, not what it is.

A context with prefetch and one without factor the same curve; the linear
search (Section 2.2) on each must agree bit for bit, at the prefetched
precision, at the other reduced precision and in FP64, for a single-block
curve, small curves of a few blocks and the TESS-sector size (N = 18000),
and after a refactor into the same factor. The prefetched results are also
held to the oracle at the reduced-precision bar.
"""
import numpy as np
import pytest

from oracle import gp as ogp, linear as olin
from synth import config2, make_workload, sho_omega_from_rotation

pytestmark = pytest.mark.gpu

MIXED_TOL = 1e-6


def say(msg):
    print(f"[gpu-case] {msg}", flush=True)


@pytest.fixture(scope="module")
def api():
    import torch
    from paper_2402_06835_amd import _lib, api as a
    _lib.lib()
    assert torch.cuda.is_available()
    return a


def _curve(n, seed):
    th = {"amp": 0.008, "omega": sho_omega_from_rotation(0.8, 4.0), "q": 4.0, "sigma_w": 1e-3}
    return make_workload(f"prefetch-N{n}", seed, n, 2 / 1440, th, [1, 5, 13], np.linspace(0.3, 2.0, 40),
                         gaps=[(n // 3, 17)] if n > 200 else [],
                         injection={"depth": 2e-3, "period": 0.37, "t0": 0.11, "duration": 0.04})


def _host(ls):
    return {k: ls[k].cpu().numpy() for k in ("depth", "var", "dll", "valid")}


def _same(a, b, tag):
    for k in a:
        assert np.array_equal(a[k], b[k], equal_nan=True), (tag, k)


@pytest.mark.parametrize("n,cus", [(100, 0), (700, 0), (700, 16), (2000, 0), (2000, 1000)])
@pytest.mark.parametrize("prefetch", ["fp32_refine", "bf16x3_refine"])
def test_prefetch_bit_identical(api, n, cus, prefetch):
    import torch
    w = _curve(n, 80 + n % 7)
    on, off = api.Context(0), api.Context(0)
    on.set_inverse_prefetch(prefetch, cus)
    say(f"prefetch {prefetch} N={n}")
    f_on = api.gp_factor(on, w.t, w.theta)
    f_off = api.gp_factor(off, w.t, w.theta)
    assert f_on.logdet == f_off.logdet
    for prec in ("fp32_refine", "bf16x3_refine", "fp64"):
        got = _host(api.linear_search(on, f_on, w.f, w.A, w.lattice, w.n_epochs, w.durations, prec))
        ref = _host(api.linear_search(off, f_off, w.f, w.A, w.lattice, w.n_epochs, w.durations, prec))
        torch.cuda.synchronize()
        _same(got, ref, f"N={n} prefetch {prefetch} search {prec}")
    # a refit into the same factor prefetches again
    th2 = dict(w.theta, amp=w.theta["amp"] * 1.3)
    api.gp_factor(on, w.t, th2, out=f_on)
    api.gp_factor(off, w.t, th2, out=f_off)
    got = _host(api.linear_search(on, f_on, w.f, w.A, w.lattice, w.n_epochs, w.durations, prefetch))
    ref = _host(api.linear_search(off, f_off, w.f, w.A, w.lattice, w.n_epochs, w.durations, prefetch))
    torch.cuda.synchronize()
    _same(got, ref, f"N={n} refit")
    # and the prefetched search meets the oracle
    L = ogp.cholesky(ogp.covariance(w.t, th2))
    o = olin.linear_search(w.f, w.A, L, w.lattice, w.durations, n_epochs=w.n_epochs)
    v = o["valid"].astype(bool)
    np.testing.assert_array_equal(got["valid"].astype(bool), v)
    err = np.max(np.abs(got["dll"][v] - o["dll"][v]) / np.maximum(np.abs(o["dll"][v]), 1.0))
    say(f"N={n} refit vs oracle: dll {err:.2e}")
    assert err <= MIXED_TOL


def test_prefetch_full_size(api):
    import torch
    w = config2()
    on, off = api.Context(0), api.Context(0)
    on.set_inverse_prefetch("fp32_refine")
    say(f"prefetch fp32_refine N={w.n}")
    f_on = api.gp_factor(on, w.t, w.theta)
    got = _host(api.linear_search(on, f_on, w.f, w.A, w.lattice, w.n_epochs, w.durations, "fp32_refine"))
    torch.cuda.synchronize()
    del f_on
    f_off = api.gp_factor(off, w.t, w.theta)
    ref = _host(api.linear_search(off, f_off, w.f, w.A, w.lattice, w.n_epochs, w.durations, "fp32_refine"))
    torch.cuda.synchronize()
    _same(got, ref, "full size")


def test_prefetch_argument_errors(api):
    from paper_2402_06835_amd import _lib
    from paper_2402_06835_amd._lib import NU_ERR_ARG
    ctx = api.Context(0)
    with pytest.raises(ValueError):
        ctx.set_inverse_prefetch("fp64")
    assert _lib.lib().nu_ctx_set_inverse_prefetch(ctx.ptr, 0, 0) == NU_ERR_ARG
    assert _lib.lib().nu_ctx_set_inverse_prefetch(ctx.ptr, 3, 0) == NU_ERR_ARG
    assert _lib.lib().nu_ctx_set_inverse_prefetch(ctx.ptr, 1, -1) == NU_ERR_ARG
    ctx.set_inverse_prefetch("bf16x3_refine", 64)
    ctx.set_inverse_prefetch(None)
