"""The allocation-free periodic search (nu_periodic_search_noalloc) against
nu_periodic_search, through the C ABI: two calls in a row on one context, the
second on a smaller grid and fewer periods (the fixed scratch array keeps the
first call's contents), each bitwise equal to the allocating call; a grid
beyond the array is refused before any launch."""
import ctypes

import numpy as np
import pytest

from synth import make_workload, sho_omega_from_rotation

pytestmark = pytest.mark.gpu

KEYS = ("q_snr", "best_phase", "best_dur", "best_depth", "best_sigma", "best_lnp", "best_index")


def say(msg):
    print(f"[gpu-case] {msg}", flush=True)


@pytest.fixture(scope="module")
def api():
    import torch
    from paper_2402_06835_amd import _lib, api as a
    _lib.lib()
    assert torch.cuda.is_available()
    return a


def _noalloc(api, ctx, ls, dt, periods, sign=1):
    import torch
    from paper_2402_06835_amd._lib import NU_OK, lib
    dev = ctx.device
    per = torch.as_tensor(np.ascontiguousarray(periods), dtype=torch.float64, device=dev)
    n_d, n_t = ls["depth"].shape
    n_p = per.numel()
    out = {"q_snr": torch.empty(n_p, dtype=torch.float64, device=dev),
           "best_phase": torch.empty(n_p, dtype=torch.int64, device=dev),
           "best_dur": torch.empty(n_p, dtype=torch.int32, device=dev),
           "best_depth": torch.empty(n_p, dtype=torch.float64, device=dev),
           "best_sigma": torch.empty(n_p, dtype=torch.float64, device=dev),
           "best_lnp": torch.empty(n_p, dtype=torch.float64, device=dev),
           "best_index": torch.empty(1, dtype=torch.int64, device=dev)}
    st = lib().nu_periodic_search_noalloc(
        ctx.ptr, *[ctypes.c_void_p(ls[k].data_ptr()) for k in ("depth", "var", "dll", "valid")], n_d, n_t,
        float(dt), ctypes.c_void_p(per.data_ptr()), n_p, int(sign),
        *[ctypes.c_void_p(out[k].data_ptr()) for k in KEYS])
    return st, out, per


def _curve(n, seed, durs):
    th = {"amp": 0.01, "omega": sho_omega_from_rotation(1.1, 5.0), "q": 5.0, "sigma_w": 1e-3}
    return make_workload(f"noalloc-N{n}", seed, n, 10 / 1440, th, durs, np.linspace(0.3, 3.0, 300),
                         gaps=[(n // 2, 17)], injection={"depth": 2e-3, "period": 0.83, "t0": 0.21, "duration": 0.05})


def test_noalloc_periodic_search_equals_the_allocating_call(api):
    import torch
    from paper_2402_06835_amd._lib import NU_ERR_ARG, NU_OK
    ctx = api.Context(0)
    results = []
    for n, seed, durs, n_per, sign in ((3000, 1, [2, 5, 9, 14], 300, 1), (900, 2, [3, 6], 120, -1)):
        w = _curve(n, seed, durs)
        say(f"noalloc periodic search N={n} n_d={len(durs)} periods={n_per} sign={sign}")
        fac = api.gp_factor(ctx, w.t, w.theta)
        ls = api.linear_search(ctx, fac, w.f, w.A, w.lattice, w.n_epochs, w.durations)
        periods = w.periods[:n_per]
        ref = api.periodic_search(ctx, ls["depth"], ls["var"], ls["dll"], ls["valid"], w.dt, periods, sign=sign)
        st, got, _ = _noalloc(api, ctx, ls, w.dt, periods, sign)
        torch.cuda.synchronize()
        assert st == NU_OK
        for k in KEYS:
            np.testing.assert_array_equal(got[k].cpu().numpy(), ref[k].cpu().numpy(), err_msg=k)
        assert int(got["best_phase"].max().item()) >= 0
        results.append(got)
    # a grid beyond the fixed array: refused, nothing launched
    big = {k: torch.zeros((16, 200000), dtype=torch.float64 if k != "valid" else torch.uint8, device=ctx.device)
           for k in ("depth", "var", "dll", "valid")}
    st, _, _ = _noalloc(api, ctx, big, 1.0, [3.0])
    assert st == NU_ERR_ARG
    ctx.close()
