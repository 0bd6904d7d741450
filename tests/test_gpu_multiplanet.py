"""GPU: the search for further candidates (mask a found candidate's transits in
the linear-search products, search again; Section 3.3) through the C ABI,
against the oracle (``oracle.multiplanet``).

* The mask kernel equals the oracle's mask bit for bit, including a slot at
  distance exactly h after the rounding of k p, overlapping windows and phases
  at both ends of the grid.
* Argument errors are reported before any launch.
* Two planets injected on the lattice: the GPU's iterative search and the
  oracle's, on the same linear-search grid, pick the same candidates, which are
  the injected planets.
"""
import numpy as np
import pytest

from oracle import multiplanet as omp, periodic as oper
from synth import make_workload, sho_omega_from_rotation

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


def _grid(rng, n_d, n_t):
    var = rng.uniform(1e-7, 4e-7, (n_d, n_t))
    depth = rng.standard_normal((n_d, n_t)) * np.sqrt(var)
    dll = 0.5 * depth ** 2 / var
    valid = (rng.uniform(size=(n_d, n_t)) > 0.05).astype(np.uint8)
    depth[valid == 0] = 0.0
    var[valid == 0] = np.inf
    dll[valid == 0] = 0.0
    return depth, var, dll, valid


@pytest.mark.parametrize("period,dt,phase,h", [(9.6, 1.0, 9, 3), (0.96, 0.1, 9, 3), (4.4, 1.0, 2, 3),
                                               (7.0, 1.0, 0, 4), (23.7, 1.0, 299, 5), (500.0, 1.0, 150, 7),
                                               (1.0, 1.0, 0, 1), (3.3, 1.0, 299, 2)])
def test_mask_matches_oracle(api, ctx, period, dt, phase, h):
    import torch
    rng = np.random.default_rng(int(period * 10) + phase + h)
    n_d, n_t = 3, 300
    depth, var, dll, valid = _grid(rng, n_d, n_t)
    say(f"mask P={period} dt={dt} m={phase} h={h}")
    dev = {k: torch.as_tensor(np.ascontiguousarray(v), device="cuda") for k, v in
           (("depth", depth), ("var", var), ("dll", dll), ("valid", valid))}
    api.mask_transit(ctx, dev, dt, period, phase, h)
    torch.cuda.synchronize()
    ref = omp.mask_transit(depth, var, dll, valid, dt, period, phase, h)
    for k, r in zip(("depth", "var", "dll", "valid"), ref):
        np.testing.assert_array_equal(dev[k].cpu().numpy(), r, err_msg=k)


def test_mask_argument_errors(api, ctx):
    import torch
    from paper_2402_06835_amd._lib import NuanceError
    dev = {k: torch.zeros((2, 50), dtype=t, device="cuda") for k, t in
           (("depth", torch.float64), ("var", torch.float64), ("dll", torch.float64), ("valid", torch.uint8))}
    before = {k: v.clone() for k, v in dev.items()}
    for args in ((1.0, 0.5, 0, 2), (1.0, 2.0, 50, 2), (1.0, 2.0, -1, 2), (1.0, 2.0, 0, 0), (1.0, 2.0, 0, 2000),
                 (0.0, 2.0, 0, 2), (1.0, float("nan"), 0, 2)):
        with pytest.raises(NuanceError):
            api.mask_transit(ctx, dev, *args)
    torch.cuda.synchronize()
    for k in dev:
        assert torch.equal(dev[k], before[k])


def test_two_injected_planets_found_in_turn(api, ctx):
    import torch
    dt = 10 / 1440
    th = {"amp": 0.004, "omega": sho_omega_from_rotation(1.1, 5.0), "q": 5.0, "sigma_w": 1e-3}
    durs = [3, 6, 9]
    periods = np.linspace(0.6, 4.0, 700)
    w = make_workload("two-planets", 91, 2000, dt, th, durs, periods,
                      injection={"depth": 4e-3, "slot0": 37, "p_slots": 293, "n_dur": 6})
    # the second, shallower planet on the lattice as well
    second = {"depth": 2.5e-3, "slot0": 120, "p_slots": 411, "n_dur": 6}
    f = w.f.copy()
    s = second["slot0"]
    while s - 3 <= w.lattice[-1]:
        f[(w.lattice >= s - 3) & (w.lattice < s + 3)] -= second["depth"]
        s += second["p_slots"]
    say(f"two planets N={w.n}: periods 293 and 411 slots")
    fac = api.gp_factor(ctx, w.t, w.theta)
    ls = api.linear_search(ctx, fac, f, w.A, w.lattice, w.n_epochs, durs)
    found = api.search_planets(ctx, ls, dt, periods, durs, 2)
    torch.cuda.synchronize()
    host = {k: ls[k].cpu().numpy() for k in ("depth", "var", "dll", "valid")}
    ref = omp.search_planets(host["depth"], host["var"], host["dll"], host["valid"], dt, periods, durs, 2)
    say(f"gpu {[(c['index'], c['phase'], c['dur_index'], round(c['snr'], 2)) for c in found]}")
    say(f"oracle {[(c['index'], c['phase'], c['dur_index'], round(c['snr'], 2)) for c in ref]}")
    assert len(found) == len(ref) == 2
    for g, r in zip(found, ref):
        assert (g["index"], g["phase"], g["dur_index"]) == (r["index"], r["phase"], r["dur_index"])
        assert g["snr"] == pytest.approx(r["snr"], rel=1e-10)
    for c, (p_slots, s0) in zip(found, ((293, 37), (411, 120))):
        assert abs(c["period"] / dt - p_slots) < 0.01 * p_slots
        assert abs(c["phase"] - s0 % p_slots) <= 3
    # the input grid is untouched (the search masks copies)
    assert torch.equal(ls["valid"].cpu(), torch.as_tensor(host["valid"]))


def test_nuance_search_planets(api):
    dt = 10 / 1440
    th = {"amp": 0.004, "omega": sho_omega_from_rotation(1.1, 5.0), "q": 5.0, "sigma_w": 1e-3}
    w = make_workload("nuance-planets", 92, 1200, dt, th, [6], np.linspace(0.6, 3.0, 300),
                      injection={"depth": 5e-3, "slot0": 50, "p_slots": 257, "n_dur": 6})
    nu = api.Nuance(w.t, w.f, gp=api.SHO(amp=th["amp"], omega=th["omega"], q=th["q"], sigma_w=th["sigma_w"]),
                    X=w.A, dt=dt)
    nu.linear_search(Ds=[6 * dt])
    cands = nu.search_planets(w.periods, n_planets=2)
    say(f"nuance candidates {[(round(c[0], 4), round(c[4], 2)) for c in cands]}")
    assert len(cands) == 2
    assert abs(cands[0][0] - 257 * dt) < 0.01 * 257 * dt
