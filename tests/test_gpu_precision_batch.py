"""GPU: the reduced-precision paths on the uneven batch's hardest curves,
through the batch entry point, against the FP64 oracle.

The two curves of the 64-curve batch (seeds 3000 + c) with the strongest
long-period variability over the white noise (c = 42: N = 17090, P_rot =
1.70 d, amp = 2.9 %; c = 7: N = 19319, P_rot = 1.82 d, amp = 2.6 %) have the
slowest-decaying L^-1, so reduced-precision blocks far from the diagonal
carry the most weight in the box sums. Cells are sampled at random and, per
precision, where that precision departs most from the FP64 batch (the FP64
path is itself oracle-pinned); every sampled cell is compared with the
oracle's full GLS. Bars on dll (relative to max(|dll|, 1 nat)), depth (in
units of sigma) and var (relative):
  * FP32_REFINE: 1e-6, the bar for the reduced-precision search;
  * BF16X3_REFINE: the split-BF16 inverse does not reach 1e-6 on these
    curves (measured worst: dll 2.4e-6, depth 4.2e-6 sigma, var 2.5e-6, SNR
    2.3e-7, all on c = 42); it is held to BF16_BOUND, a bound with margin over
    those figures, and stays out of every 1e-6 claim.
"""
import numpy as np
import pytest

from oracle import gp as ogp, linear as olin
from synth import config3

pytestmark = pytest.mark.gpu

CURVES = (42, 7)
N_PERIODS = 2000
FP32_BAR = 1e-6
BF16_BOUND = 1e-5


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


@pytest.fixture(scope="module")
def hard_curves():
    ws = config3(n_curves=max(CURVES) + 1)
    return [ws[c] for c in CURVES]


def _errors(g, r, v):
    return {"dll": np.abs(g["dll"][v] - r["dll"][v]) / np.maximum(np.abs(r["dll"][v]), 1.0),
            "depth": np.abs(g["depth"][v] - r["depth"][v]) / np.sqrt(r["var"][v]),
            "var": np.abs(g["var"][v] - r["var"][v]) / r["var"][v]}


@pytest.fixture(scope="module")
def batches(api, ctx, hard_curves):
    import torch
    ws = hard_curves
    dt = ws[0].dt
    periods = np.linspace(0.3, 13.0, N_PERIODS)
    curves = [{"t": w.t, "f": w.f, "A": w.A, "lattice": w.lattice, "n_epochs": w.n_epochs, "theta": w.theta,
               "dt": dt} for w in ws]
    out = {}
    for prec in ("fp64", "fp32_refine", "bf16x3_refine"):
        say(f"hard curves N={[w.n for w in ws]} through the batch, {prec}")
        res = api.search_batch(ctx, curves, ws[0].durations, periods, precision=prec)
        torch.cuda.synchronize()
        out[prec] = {"cells": [{k: res["cells"][c][k].cpu().numpy() for k in ("depth", "var", "dll", "valid")}
                               for c in range(len(ws))],
                     "q_snr": res["q_snr"].cpu().numpy(), "best_phase": res["best_phase"].cpu().numpy(),
                     "best_dur": res["best_dur"].cpu().numpy()}
    return out


@pytest.mark.parametrize("precision,bar", [("fp32_refine", FP32_BAR), ("bf16x3_refine", BF16_BOUND)])
def test_hard_curves_against_the_oracle(hard_curves, batches, precision, bar):
    worst = {}
    for c, w in enumerate(hard_curves):
        g = batches[precision]["cells"][c]
        r64 = batches["fp64"]["cells"][c]
        v = r64["valid"].astype(bool)
        np.testing.assert_array_equal(g["valid"].astype(bool), v)
        e = _errors(g, r64, v)
        full = {k: float(x.max()) for k, x in e.items()}
        say(f"curve {CURVES[c]} {precision} vs the FP64 batch, all cells: {full}")
        # sampled cells: random ones and the worst of each output against the FP64 batch
        rng = np.random.default_rng(100 + c)
        n_d = w.durations.size
        cells = {(int(rng.integers(n_d)), int(rng.integers(w.n_epochs))) for _ in range(24)}
        jj, ii = np.nonzero(v)
        for k in e:
            for idx in np.argsort(e[k])[-4:]:
                cells.add((int(jj[idx]), int(ii[idx])))
        cells = sorted(cells)
        say(f"curve {CURVES[c]}: oracle GLS on {len(cells)} cells (N={w.n})")
        L = ogp.cholesky(ogp.covariance(w.t, w.theta))
        ref = olin.linear_search(w.f, w.A, L, w.lattice, w.durations, cells=cells)
        del L
        sel = {k: np.array([g[k][j, i] for (j, i) in cells]) for k in g}
        vv = ref["valid"].astype(bool)
        np.testing.assert_array_equal(sel["valid"].astype(bool), vv)
        eo = {k: float(x.max()) for k, x in _errors(sel, ref, vv).items()}
        say(f"curve {CURVES[c]} {precision} vs the oracle, sampled cells: {eo}")
        for k in eo:
            worst[k] = max(worst.get(k, 0.0), eo[k], full[k])
    say(f"{precision}: worst {worst} (bar {bar})")
    assert max(worst.values()) <= bar, worst


@pytest.mark.parametrize("precision,bar", [("fp32_refine", FP32_BAR), ("bf16x3_refine", BF16_BOUND)])
def test_hard_curves_snr_against_fp64(batches, precision, bar):
    g, r = batches[precision], batches["fp64"]
    ok = r["best_phase"] >= 0
    e = np.max(np.abs(g["q_snr"][ok] - r["q_snr"][ok]) / np.maximum(np.abs(r["q_snr"][ok]), 1.0))
    same = np.mean((g["best_phase"][ok] == r["best_phase"][ok]) & (g["best_dur"][ok] == r["best_dur"][ok]))
    say(f"{precision}: SNR error {e:.2e}, best cell agreement {same:.5f}")
    assert e <= bar
    assert same >= 0.99
