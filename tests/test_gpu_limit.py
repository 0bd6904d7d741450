"""GPU: the context's workspace limit, through the C ABI.

A context created with a limit counts the device memory the library
allocates on it (search workspace, batch arena, fold grids, factors, graphs)
and returns NU_ERR_OOM, allocating nothing more, for a call that would go past
it. Within the limit the outputs are those of an unlimited context, bit for
bit: the limit changes where memory comes from and how a batch is cut into
waves, never the arithmetic.
"""
import numpy as np
import pytest

from synth import make_workload, sho_omega_from_rotation

pytestmark = pytest.mark.gpu

DURS = [1, 4, 9, 17]
PERIODS = np.linspace(0.3, 2.0, 40)
DT = 10 / 1440
CELL_KEYS = ("depth", "var", "dll", "valid")


def say(msg):
    print(f"[gpu-case] {msg}", flush=True)


@pytest.fixture(scope="module")
def api():
    import torch
    from paper_2402_06835_amd import _lib, api as a
    _lib.lib()
    assert torch.cuda.is_available()
    return a


def _curve(n, seed, prot):
    th = {"amp": 0.01, "omega": sho_omega_from_rotation(prot, 5.0), "q": 5.0, "sigma_w": 1e-3}
    return make_workload(f"limit-N{n}-s{seed}", seed, n, DT, th, DURS, PERIODS, gaps=[],
                         injection={"depth": 2e-3, "period": 0.61, "t0": 0.13, "duration": 0.05})


def _search(api, ctx, w):
    import torch
    fac = api.gp_factor(ctx, w.t, w.theta)
    try:
        ls = api.linear_search(ctx, fac, w.f, w.A, w.lattice, w.n_epochs, DURS, "fp64")
        torch.cuda.synchronize()
        return {k: ls[k].cpu().numpy() for k in CELL_KEYS}
    finally:
        fac.close()


def test_single_curve_calls_within_and_beyond_the_limit(api):
    from paper_2402_06835_amd._lib import NU_ERR_OOM, NuanceError
    w = _curve(1000, 41, 1.1)
    say("single-curve factor + linear search, N=1000, unlimited context")
    free = api.Context(0)
    fac = api.gp_factor(free, w.t, w.theta)
    b_factor = free.device_bytes()
    assert b_factor >= 2 * 1024 * 1024 * 8  # L and X at least
    fac.close()
    assert free.device_bytes() == 0
    ref = _search(api, free, w)
    b_ws = free.device_bytes()  # the search workspace the context keeps
    assert b_ws > 0
    free.release_memory()
    assert free.device_bytes() == 0
    free.close()

    say("a limit below one factor: NU_ERR_OOM, nothing left counted")
    tight = api.Context(0, workspace_limit=1 << 20)
    with pytest.raises(NuanceError) as ei:
        api.gp_factor(tight, w.t, w.theta)
    assert ei.value.status == NU_ERR_OOM
    assert tight.device_bytes() == 0
    tight.close()

    say("a limit that holds the factor but not the search workspace")
    mid = api.Context(0, workspace_limit=b_factor + b_ws // 2)
    fac = api.gp_factor(mid, w.t, w.theta)
    with pytest.raises(NuanceError) as ei:
        api.linear_search(mid, fac, w.f, w.A, w.lattice, w.n_epochs, DURS, "fp64")
    assert ei.value.status == NU_ERR_OOM
    assert mid.device_bytes() == b_factor
    fac.close()
    mid.close()

    say("a limit that holds both: outputs equal the unlimited context's")
    fit = api.Context(0, workspace_limit=b_factor + b_ws)
    got = _search(api, fit, w)
    assert fit.device_bytes() == b_ws
    for k in CELL_KEYS:
        np.testing.assert_array_equal(got[k], ref[k], err_msg=k)
    fit.close()


def test_batch_plans_its_waves_within_the_limit(api):
    import torch
    from paper_2402_06835_amd._lib import NU_ERR_OOM, NuanceError
    ws = [_curve(700, 51, 1.2), _curve(300, 52, 0.8), _curve(1000, 53, 1.6), _curve(129, 54, 1.0)]
    curves = [{"t": w.t, "f": w.f, "A": w.A, "lattice": w.lattice, "n_epochs": w.n_epochs, "theta": w.theta,
               "dt": DT} for w in ws]
    say("batch of 4 curves, unlimited context")
    free = api.Context(0)
    one = api.search_batch(free, curves, DURS, PERIODS, precision="fp64")
    torch.cuda.synchronize()
    whole = free.device_bytes()  # workspace + one arena holding every factor
    free.close()

    say("batch of 4 curves under a limit of 75 % of that: several waves, same outputs")
    limit = int(whole * 0.75)
    ctx = api.Context(0, workspace_limit=limit)
    many = api.search_batch(ctx, curves, DURS, PERIODS, precision="fp64")
    torch.cuda.synchronize()
    assert 0 < ctx.device_bytes() <= limit
    for k in CELL_KEYS + ("q_snr", "best_phase", "best_dur", "best_depth", "best_sigma", "best_lnp", "null",
                          "best_index"):
        np.testing.assert_array_equal(one[k].cpu().numpy(), many[k].cpu().numpy(), err_msg=k)
    ctx.close()

    say("batch under a limit below its largest curve: NU_ERR_OOM")
    small = api.Context(0, workspace_limit=4 << 20)
    with pytest.raises(NuanceError) as ei:
        api.search_batch(small, curves, DURS, PERIODS, precision="fp64")
    assert ei.value.status == NU_ERR_OOM
    small.close()
