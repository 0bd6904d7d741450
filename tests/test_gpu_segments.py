"""GPU: the periodic search over segments of one light curve, each with its own
linear search (entry point 3c), against the oracle's definition (the plain
fold on one global grid with the gaps invalid; ``oracle.segments``).

* Random grids in three segments with a large and a minimum (64-slot) gap,
  both signs of Eq. 8's log term: indices agree up to certified ties, values
  to 1e-12.
* One segment at offset 0 is the single-grid fold bit for bit.
* Two sectors with different GPs, one planet in both: the segmented search
  on the GPU's per-sector linear searches recovers it, as the oracle does.
* Argument errors are reported before any launch.
"""
import numpy as np
import pytest

from oracle import periodic as oper, segments as oseg
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


def _grid(rng, n_d, n):
    var = rng.uniform(1e-7, 4e-7, (n_d, n))
    depth = rng.standard_normal((n_d, n)) * np.sqrt(var)
    valid = (rng.uniform(size=(n_d, n)) > 0.03).astype(np.uint8)
    depth[valid == 0] = 0.0
    var[valid == 0] = np.inf
    dll = np.where(valid == 1, 0.5 * depth ** 2 / var, 0.0)
    return depth, var, dll, valid


def _host(ps):
    return {k: ps[k].cpu().numpy() for k in ("q_snr", "best_phase", "best_dur", "best_depth", "best_sigma",
                                             "best_lnp", "best_index")}


def _compare(gpu, ref, glob, dt, periods, sign):
    bad = np.nonzero((gpu["best_phase"] != ref["best_phase"]) | (gpu["best_dur"] != ref["best_dur"]))[0]
    for ip in bad:  # certified ties only
        lnp, *_ = oper.fold_period(*glob, dt, float(periods[ip]), sign)
        mx = np.nanmax(lnp)
        g = lnp[gpu["best_phase"][ip], gpu["best_dur"][ip]]
        assert abs(g - mx) <= 1e-12 * max(abs(mx), 1.0), f"period {ip}: not a tie"
    same = (gpu["best_phase"] == ref["best_phase"]) & (gpu["best_dur"] == ref["best_dur"])
    np.testing.assert_allclose(gpu["best_lnp"], ref["best_lnp"], rtol=1e-12, atol=1e-12)
    np.testing.assert_allclose(gpu["q_snr"][same], ref["q_snr"][same], rtol=1e-12, atol=1e-12)
    return len(bad)


@pytest.mark.parametrize("sign", [1, -1])
def test_segments_match_oracle(api, ctx, sign):
    import torch
    rng = np.random.default_rng(21 + sign)
    n_d, dt = 3, 0.01
    lens, offs = [400, 250, 300], [7, 5407, 5721]   # gaps of 5000 and 64 slots
    grids = [_grid(rng, n_d, n) for n in lens]
    # a weak periodic signal through all three segments
    for g, o, n in zip(grids, offs, lens):
        for c in range(37, o + n, 173):
            if c >= o:
                g[0][1, c - o] += 6e-4
                g[2][1, c - o] = 0.5 * g[0][1, c - o] ** 2 / g[1][1, c - o]
    periods = np.concatenate([np.linspace(0.05, 4.0, 250), [1.73]])
    say(f"segments {lens} at {offs}, sign={sign}")
    dev = [{k: torch.as_tensor(np.ascontiguousarray(v), device="cuda") for k, v in
            zip(("depth", "var", "dll", "valid"), g)} for g in grids]
    gpu = _host(api.periodic_search_segments(ctx, dev, offs, dt, periods, sign))
    torch.cuda.synchronize()
    ref = oseg.periodic_search_segments(grids, offs, dt, periods, sign)
    ties = _compare(gpu, ref, oseg.assemble(grids, offs), dt, periods, sign)
    say(f"segments sign={sign}: certified ties {ties}")
    assert gpu["best_index"][0] == oper.first_argmax(ref["q_snr"]) or ties


def test_single_segment_is_the_plain_fold(api, ctx):
    import torch
    rng = np.random.default_rng(5)
    g = _grid(rng, 2, 600)
    periods = np.linspace(0.3, 3.0, 150)
    dev = {k: torch.as_tensor(np.ascontiguousarray(v), device="cuda") for k, v in
           zip(("depth", "var", "dll", "valid"), g)}
    a = _host(api.periodic_search_segments(ctx, [dev], [0], 0.01, periods))
    b = _host(api.periodic_search(ctx, dev["depth"], dev["var"], dev["dll"], dev["valid"], 0.01, periods))
    torch.cuda.synchronize()
    for k in a:
        np.testing.assert_array_equal(a[k], b[k], err_msg=k)


def test_two_sectors_recover_planet(api, ctx):
    import torch
    dt = 10 / 1440
    durs = [3, 6]
    p_slots, s0 = 247, 61
    # the true period on the grid: over a 5500-slot span a grid step of ~1 slot would drift the
    # later transits out of their boxes
    periods = np.concatenate([np.linspace(0.8, 3.0, 300), [p_slots * dt]])
    grids, offs = [], [0, 4000]
    for c, (off, prot, amp) in enumerate(zip(offs, (0.9, 1.6), (0.003, 0.006))):
        th = {"amp": amp, "omega": sho_omega_from_rotation(prot, 5.0), "q": 5.0, "sigma_w": 1e-3}
        first = s0 + ((off - s0 + p_slots - 1) // p_slots) * p_slots - off   # first transit in the sector
        w = make_workload(f"sector{c}", 300 + c, 1500, dt, th, durs, periods,
                          injection={"depth": 2.5e-3, "slot0": first, "p_slots": p_slots, "n_dur": 6})
        fac = api.gp_factor(ctx, w.t, w.theta)
        ls = api.linear_search(ctx, fac, w.f, w.A, w.lattice, w.n_epochs, durs)
        grids.append(ls)
    say("two sectors of 1500 samples, 2500 slots apart")
    gpu = _host(api.periodic_search_segments(ctx, grids, offs, dt, periods))
    torch.cuda.synchronize()
    host = [tuple(g[k].cpu().numpy() for k in ("depth", "var", "dll", "valid")) for g in grids]
    ref = oseg.periodic_search_segments(host, offs, dt, periods)
    _compare(gpu, ref, oseg.assemble(host, offs), dt, periods, 1)
    ip = int(gpu["best_index"][0])
    say(f"best period {periods[ip]:.4f} d (injected {p_slots * dt:.4f}), phase {gpu['best_phase'][ip]}, "
        f"snr {gpu['q_snr'][ip]:.2f}")
    assert abs(periods[ip] / dt - p_slots) < 0.01 * p_slots
    assert abs(gpu["best_phase"][ip] - s0) <= 3


def test_segment_argument_errors(api, ctx):
    import torch
    from paper_2402_06835_amd._lib import NuanceError
    z = {k: torch.zeros((2, 50), dtype=t, device="cuda") for k, t in
         (("depth", torch.float64), ("var", torch.float64), ("dll", torch.float64), ("valid", torch.uint8))}
    for offs in ([0, 60], [0, 113], [100, 0], [-1, 200]):   # overlap, gap < 64, descending, negative
        with pytest.raises(NuanceError):
            api.periodic_search_segments(ctx, [z, z], offs, 0.01, [0.5])
    with pytest.raises(NuanceError):
        api.periodic_search_segments(ctx, [z] * 33, [200 * i for i in range(33)], 0.01, [0.5])
    api.periodic_search_segments(ctx, [z, z], [0, 114], 0.01, [0.5])  # exactly 64 apart
    torch.cuda.synchronize()
