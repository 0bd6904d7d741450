"""Benchmark of the transit-search hot path on one MI355X.

One step = the whole hot path over one light curve already resident in HBM:
gp_factor (covariance build + FP64 Cholesky) -> linear_search (triangular
inverse, trend fit, every (epoch, duration) box fit) -> periodic_search (fold
over all periods, best period). Workload: the TESS-sector-shaped curve
(N = 18000 samples at 2-min cadence with a 1-d gap, 18720 epoch slots,
10 durations of 9..90 samples, 20000 periods in [0.3, 13] d), synthetic and
seeded.

Prints one JSON line: value = valid (t0, D) fits per second of whole-step
wall time (plus light curves per second), the roofline of the dominant
kernel from HIP events recorded by the library around its launches inside
the timed region, and the CPU oracle timed on a bounded sample of the same
workload.

Default precision: FP32_REFINE (FP64 Cholesky, FP32 inverse products with an
FP64 band Newton step and one refinement step), the fastest path that meets
the 1e-6 dll bar; its dll error against the FP64 path on the same curve is
measured after the timed region and reported. The FP32 inverse is started
inside the factorisation (the context's inverse prefetch: its early phases
on three quarters of the CUs beside the late, latency-bound Cholesky steps;
bit-identical results). Other modes:
  --inverse-prefetch off  the inverse after the factorisation, inside linear_search
  --mode graph          the same step as one captured-graph launch
  --workload batch-64   64 curves of 4000..20000 samples in one batch call per step
                        (--mode loop: the same curves through the single-curve calls)
  --autotune            tile policy tuned on the device before warming up
  --workload learned    the learned warm start: GP sampling, CNN training, and BFGS fits of 256
                        held-out curves from the plain and from the learned start
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

# gemm_bf16x3 counts each product once (FP32-equivalent flops); it takes three BF16 products at the
# 2.5 PFLOP/s dense BF16 peak
# MI355X peaks: dense MFMA per type (TFLOP/s; split BF16 counts its three products as one), FP64 vector ALU
# (256 CUs x 4 SIMDs x 16 lanes x 2 flops per FMA x 2.4 GHz, TFLOP/s) and HBM (GB/s)
PEAKS = {"gemm_f64": 78.6, "gemm_f32": 157.3, "gemm_bf16x3": 2500.0 / 3, "fp64_alu": 78.6, "hbm_gbs": 8000.0}


# the stellar-variability kernel of Section 3.2 at a 2-d rotation period (variance split between the modes,
# a short and a long exponential term) with the white noise of the TESS-sector curve
ROTATION_KERNEL = dict(sigma=1e-2, period=2.0, q0=1.0, dq=3.0, f=0.4, sigma_short=3e-4, ell_short=0.02,
                       sigma_long=8e-4, ell_long=3.0, sigma_w=8e-4)


def log(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def workload(name: str):
    from synth import config1, config2
    return {"tess-sector": config2, "plain-1440": config1}[name]()


def run_step(api, ctx, dev_in, w, precision, fac=None, planets=1, solver="dense", kernel=None, shapes=None):
    """gp_factor + linear_search + periodic_search (solver "statespace": the state-space linear search, no
    factor); with planets > 1, the periodic search is repeated on the same linear-search grid with each found
    candidate's transits masked (Section 3.3). Returns the factor, the grid, the first periodic search and the
    candidates (None for planets == 1)."""
    if solver == "statespace":
        ls = api.linear_search_ss(ctx, dev_in["t"], kernel, dev_in["f"], dev_in["A"], dev_in["lattice"],
                                  w.n_epochs, w.durations, check=False, shapes=shapes)
    else:
        fac = api.gp_factor(ctx, dev_in["t"], w.theta if kernel is None else kernel,
                            out=fac if kernel is None else None)
        ls = api.linear_search(ctx, fac, dev_in["f"], dev_in["A"], dev_in["lattice"], w.n_epochs, w.durations,
                               precision, shapes=shapes)
    ps = api.periodic_search(ctx, ls["depth"], ls["var"], ls["dll"], ls["valid"], w.dt, dev_in["periods"])
    if planets <= 1:
        return fac, ls, ps, None
    # the first candidate comes from ps; the next ones from masked copies of the grid
    ip = int(ps["best_index"].item())
    cands = []
    if ip >= 0:
        m, j = int(ps["best_phase"][ip].item()), int(ps["best_dur"][ip].item())
        cands.append({"period": float(w.periods[ip]), "phase": m, "dur_index": j, "snr": float(ps["q_snr"][ip].item())})
        masked = api.mask_transit(ctx, {k: ls[k].clone() for k in ("depth", "var", "dll", "valid")}, w.dt,
                                  float(w.periods[ip]), m, int(w.durations[j]))
        cands += api.search_planets(ctx, masked, w.dt, dev_in["periods"], w.durations, planets - 1, copy=False)
    return fac, ls, ps, cands


def cpu_baseline(w, n_valid: int, budget_cells: int = 192, budget_periods: int = 4, kernel: str = "sho",
                 shapes=None):
    """The oracle on a bounded sample of the same workload, scaled to whole-step fits/s. The oracle is the
    dense definition whichever solver the GPU step uses."""
    import numpy as np
    from threadpoolctl import threadpool_info

    from oracle import gp as ogp, linear as olin, periodic as oper, templates as otpl

    threads = max([d.get("num_threads", 1) for d in threadpool_info()] or [1])
    log(f"cpu baseline: oracle K build + Cholesky at N={w.n} ({threads} BLAS threads)")
    t0 = time.perf_counter()
    if kernel == "rotation":
        rk = ROTATION_KERNEL
        terms = ogp.rotation_terms(rk["sigma"], rk["period"], rk["q0"], rk["dq"], rk["f"], rk["sigma_short"],
                                   rk["ell_short"], rk["sigma_long"], rk["ell_long"])
        K = ogp.covariance_terms(w.t, terms, rk["sigma_w"])
    else:
        K = ogp.covariance(w.t, w.theta)
    L = ogp.cholesky(K)
    del K
    t_factor = time.perf_counter() - t0
    rng = np.random.default_rng(0)
    n_d, n_t = w.durations.size, w.n_epochs
    cells = [(int(rng.integers(n_d)), int(rng.integers(n_t))) for _ in range(budget_cells)]
    log(f"cpu baseline: oracle GLS on {budget_cells} sampled cells")
    t0 = time.perf_counter()
    if shapes is None:
        olin.linear_search(w.f, w.A, L, w.lattice, w.durations, cells=cells)
    else:
        otpl.linear_search_template(w.f, w.A, L, w.lattice, shapes, cells=cells)
    t_cells = time.perf_counter() - t0
    # the fold needs the single-event grid; a synthetic one of the full shape costs the same
    depth = rng.normal(2e-4, 3e-4, (n_d, n_t))
    var = rng.uniform(4e-8, 1.2e-7, (n_d, n_t))
    dll = 0.5 * depth ** 2 / var
    valid = np.ones((n_d, n_t), dtype=np.uint8)
    pidx = np.linspace(0, w.periods.size - 1, budget_periods).astype(int)
    log(f"cpu baseline: oracle fold on {budget_periods} sampled periods")
    t0 = time.perf_counter()
    oper.periodic_search(depth, var, dll, valid, w.dt, w.periods[pidx])
    t_fold = time.perf_counter() - t0
    total = t_factor + t_cells / budget_cells * (n_d * n_t) + t_fold / budget_periods * w.periods.size
    return {
        "value": n_valid / total, "unit": "(t0,D) fits/s", "cores": int(threads), "kind": "oracle",
        "sample": (f"K build + Cholesky of the full N={w.n} covariance ({t_factor:.1f} s), GLS of {budget_cells} "
                   f"random cells ({t_cells:.1f} s), fold of {budget_periods} periods ({t_fold:.1f} s); "
                   f"extrapolated to {n_d * n_t} cells and {w.periods.size} periods = {total:.0f} s per curve"),
        "seconds_per_curve": total,
    }


def roofline_of(timings):
    """Dominant kernel (by accumulated time, among the kernels with algorithmic work: a set-up kernel's first
    launch can include the loading of its code object) and its achieved rate against the MI355X peak."""
    merged = {}
    for k, v in timings.items():
        if k.startswith("host:"):  # host-side phases, not kernels
            continue
        base = k.split(":")[0]
        m = merged.setdefault(base, {"launches": 0, "ms": 0.0, "work": 0.0})
        for f in m:
            m[f] += v[f]
    cand = {k: v for k, v in merged.items() if v["work"] > 0} or merged
    name, tk = max(cand.items(), key=lambda kv: kv[1]["ms"])
    common = {"kernel": name, "traffic": None, "launches": tk["launches"], "avg_launch_ms": tk["ms"] / tk["launches"],
              "work_per_launch": tk["work"] / tk["launches"]}
    if name.startswith("gemm_"):
        achieved = tk["work"] / (tk["ms"] * 1e-3) / 1e12
        roof = {"bound": "mfma", "achieved": achieved, "peak": PEAKS[name], "unit": "TFLOP/s",
                "frac": achieved / PEAKS[name], "work_unit": "flop (algorithmic)"}
    elif name == "fold":
        # FP64 arithmetic on a cache-resident grid: bound by the vector ALU, not HBM
        achieved = tk["work"] / (tk["ms"] * 1e-3) / 1e12
        roof = {"bound": "alu", "achieved": achieved, "peak": PEAKS["fp64_alu"], "unit": "TFLOP/s",
                "frac": achieved / PEAKS["fp64_alu"], "work_unit": "flop (algorithmic, FP64)"}
    else:
        achieved = tk["work"] / (tk["ms"] * 1e-3) / 1e9
        roof = {"bound": "hbm", "achieved": achieved, "peak": PEAKS["hbm_gbs"], "unit": "GB/s",
                "frac": achieved / PEAKS["hbm_gbs"], "work_unit": "byte (algorithmic)"}
    roof.update(common)
    gemms = {k: {"tflops": v["work"] / (v["ms"] * 1e-3) / 1e12, "ms": v["ms"]}
             for k, v in merged.items() if k.startswith("gemm_")}
    return roof, gemms


# the kernel and the schedule of its launches
TRAFFIC_SOURCES = ["paper_2402_06835_amd/csrc/gemm.hip", "paper_2402_06835_amd/csrc/engine.cpp"]


def measured_traffic(roof, workload, precision):
    """HBM bytes per launch of the dominant kernel from the committed counter summary, if it was taken on
    this workload, precision and the current kernel sources (else None)."""
    import hashlib
    path = os.path.join(ROOT, "profiles", f"traffic_{roof['kernel']}_{workload}_{precision}.json")
    if not os.path.exists(path):
        return None
    rec = json.load(open(path))
    h = hashlib.sha256()
    for src in TRAFFIC_SOURCES:
        h.update(open(os.path.join(ROOT, src), "rb").read())
    if rec.get("sources_sha256") != h.hexdigest():
        log(f"traffic record {os.path.basename(path)} predates the current kernel sources: traffic = null")
        return None
    return rec["bytes_per_launch"]


def _stats(err):
    import torch
    if err.numel() == 0:
        return {"max": 0.0, "p999": 0.0}
    e = err.float()
    if e.numel() > 1 << 24:  # quantile's input limit
        e = e[torch.randperm(e.numel(), device=e.device)[:1 << 24]]
    return {"max": float(err.max().item()), "p999": float(torch.quantile(e, 0.999).item())}


def output_errors(got, ref):
    """Per-output error of a reduced-precision search against the FP64 path on the same inputs:
    dll relative to max(|dll|, 1), depth in units of its FP64 sigma, var relative, the per-period
    SNR relative to max(|SNR|, 1), and how many per-period best (phase, duration) picks agree."""
    import torch
    v = ref["valid"].bool()
    out = {"dll": _stats((got["dll"][v] - ref["dll"][v]).abs() / ref["dll"][v].abs().clamp(min=1.0)),
           "depth": _stats((got["depth"][v] - ref["depth"][v]).abs() / ref["var"][v].sqrt()),
           "var": _stats((got["var"][v] - ref["var"][v]).abs() / ref["var"][v])}
    out["valid_same"] = bool(torch.equal(got["valid"], ref["valid"]))
    if "q_snr" in ref:
        ok = ref["best_phase"] >= 0
        q, qr = got["q_snr"][ok], ref["q_snr"][ok]
        out["q_snr"] = _stats((q - qr).abs() / qr.abs().clamp(min=1.0))
        same = (got["best_phase"][ok] == ref["best_phase"][ok]) & (got["best_dur"][ok] == ref["best_dur"][ok])
        out["best_cell_same"] = f"{int(same.sum().item())}/{int(ok.sum().item())}"
    return out


def bench_batch(args, api, ctx, torch):
    """The uneven 64-curve batch in one batch call per step."""
    from synth import config3
    t0 = time.perf_counter()
    ws = config3()
    log(f"batch of {len(ws)} curves generated in {time.perf_counter() - t0:.1f} s; N from "
        f"{min(w.n for w in ws)} to {max(w.n for w in ws)}")
    curves = [{"t": w.t, "f": w.f, "A": w.A, "lattice": w.lattice, "n_epochs": w.n_epochs, "theta": w.theta,
               "dt": w.dt} for w in ws]
    durs, periods = ws[0].durations, ws[0].periods
    batch = api.prepare_batch(ctx, curves)
    per = torch.as_tensor(periods, device=ctx.device)
    dev_in = [{"t": torch.as_tensor(w.t, device=ctx.device), "f": torch.as_tensor(w.f, device=ctx.device),
               "A": torch.as_tensor(w.A, device=ctx.device), "lattice": torch.as_tensor(w.lattice, device=ctx.device),
               "periods": per} for w in ws] if args.mode == "loop" else None
    graph = None
    if args.mode == "graph":
        t0 = time.perf_counter()
        graph = api.BatchGraph(ctx, batch, durs, per, precision=args.precision)
        log(f"batch graph captured in {time.perf_counter() - t0:.1f} s")

    def one_step():
        if graph is not None:
            return graph.launch()
        if dev_in is None:
            return api.search_batch(ctx, batch, durs, per, precision=args.precision)
        # the same curves one by one through the single-curve entry points
        valid = []
        for w, d in zip(ws, dev_in):
            fac, ls, _, _ = run_step(api, ctx, d, w, args.precision)
            valid.append(ls["valid"].reshape(-1))
            fac.close()
        return {"valid": torch.cat(valid)}

    for i in range(max(args.warmup, 1)):
        res = one_step()
        torch.cuda.synchronize()
        log(f"warmup {i + 1}/{args.warmup} done")
    ctx.enable_timing(True)
    ctx.reset_timing()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for i in range(args.steps):
        res = one_step()
        log(f"step {i + 1}/{args.steps} done")
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    timings = ctx.timings()
    ctx.enable_timing(False)
    n_valid = int(res["valid"].sum().item())
    if dev_in is not None:
        log(f"{args.steps} loops of {len(ws)} single-curve searches in {elapsed:.3f} s: "
            f"{n_valid * args.steps / elapsed:.4g} fits/s, {len(ws) * args.steps / elapsed:.4g} curves/s")
        cfg = {"workload": "uneven-batch-64x(4000..20000)", "n_curves": len(ws), "valid_cells": n_valid,
               "precision": args.precision, "mode": "loop of single-curve calls"}
        return elapsed, n_valid, len(ws), timings, None, cfg, {}
    dll_err = None
    if args.precision != "fp64" and not args.no_dll_check:
        if graph is not None:
            graph.close()
        ref = api.search_batch(ctx, batch, durs, per, precision="fp64")
        dll_err = output_errors(res, ref)
        log(f"errors vs fp64: {dll_err}")
    best = res["best_index"].cpu().numpy()
    found = sum(1 for c, w in enumerate(ws) if w.injection and best[c] >= 0 and
                abs(periods[best[c]] - w.injection["period"]) < 0.01 * w.injection["period"])
    n_inj = sum(1 for w in ws if w.injection)
    log(f"{args.steps} batches in {elapsed:.3f} s: {n_valid * args.steps / elapsed:.4g} fits/s, "
        f"{len(ws) * args.steps / elapsed:.4g} curves/s; injected periods recovered {found}/{n_inj}")
    cfg = {"workload": "uneven-batch-64x(4000..20000)", "n_curves": len(ws),
           "n_samples_total": int(sum(w.n for w in ws)), "n_durations": int(len(durs)),
           "n_periods": int(len(periods)), "valid_cells": n_valid, "precision": args.precision,
           "mode": "batch graph launch" if graph is not None else "batch call"}
    return elapsed, n_valid, len(ws), timings, dll_err, cfg, {"injected_recovered": f"{found}/{n_inj}"}


def bench_two_sectors(args, api, ctx, torch):
    """Two TESS-sector curves a year apart, one star: per step, each sector's gp_factor + linear_search, then
    one segmented periodic search over both (the fold skips the year-long gap)."""
    from synth.lightcurve import two_sectors
    ws, offs = two_sectors()
    dev = ctx.device
    dev_in = [{"t": torch.as_tensor(w.t, device=dev), "f": torch.as_tensor(w.f, device=dev),
               "A": torch.as_tensor(w.A, device=dev), "lattice": torch.as_tensor(w.lattice, device=dev)} for w in ws]
    per = torch.as_tensor(ws[0].periods, device=dev)
    dt, durs = ws[0].dt, ws[0].durations
    facs = [None, None]
    prefetch = args.inverse_prefetch == "on" and args.precision != "fp64"
    if prefetch:
        ctx.set_inverse_prefetch(args.precision, args.prefetch_cus)

    def one_step(precision):
        grids = []
        for i, (w, d) in enumerate(zip(ws, dev_in)):
            facs[i] = api.gp_factor(ctx, d["t"], w.theta, out=facs[i])
            grids.append(api.linear_search(ctx, facs[i], d["f"], d["A"], d["lattice"], w.n_epochs, durs, precision))
        ps = api.periodic_search_segments(ctx, grids, offs, dt, per)
        return grids, ps

    for i in range(max(args.warmup, 1)):
        one_step(args.precision)
        torch.cuda.synchronize()
        log(f"warmup {i + 1}/{args.warmup} done")
    ctx.enable_timing(True)
    ctx.reset_timing()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for i in range(args.steps):
        grids, ps = one_step(args.precision)
        log(f"step {i + 1}/{args.steps} enqueued")
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    timings = ctx.timings()
    ctx.enable_timing(False)
    n_valid = int(sum(int(g["valid"].sum().item()) for g in grids))
    best = int(ps["best_index"].item())
    err = None
    if args.precision != "fp64" and not args.no_dll_check:
        ctx.set_inverse_prefetch(None)
        ref_grids, ref_ps = one_step("fp64")
        got = {k: torch.cat([g[k].reshape(-1) for g in grids]) for k in ("depth", "var", "dll", "valid")}
        ref = {k: torch.cat([g[k].reshape(-1) for g in ref_grids]) for k in ("depth", "var", "dll", "valid")}
        got.update({k: ps[k] for k in ("q_snr", "best_phase", "best_dur")})
        ref.update({k: ref_ps[k] for k in ("q_snr", "best_phase", "best_dur")})
        err = output_errors(got, ref)
        log(f"errors vs fp64: {err}")
    p_true = ws[0].injection["period"]
    log(f"{args.steps} steps in {elapsed:.3f} s: {n_valid * args.steps / elapsed:.4g} fits/s; best period "
        f"{float(ws[0].periods[best]) if best >= 0 else None} (injected {p_true:.4f})")
    cfg = {"workload": "two-tess-sectors-N2x18000-gap1yr", "sectors": 2, "n_samples": [w.n for w in ws],
           "offsets_slots": offs, "n_durations": int(len(durs)), "n_periods": int(len(ws[0].periods)),
           "valid_cells": n_valid, "precision": args.precision, "mode": "eager"}
    if prefetch:
        cfg["inverse_prefetch_cus"] = args.prefetch_cus
    extra = {"best_period_days": float(ws[0].periods[best]) if best >= 0 else None, "injected_period_days": p_true,
             "best_t0_days": float(ps["best_phase"][best].item()) * dt if best >= 0 else None,
             "injected_t0_days": float(ws[0].injection["global_t0"])}
    return elapsed, n_valid, 2, timings, err, cfg, extra


def bench_learned(args, api, ctx, torch):
    """The learned warm start at the TESS-sector shape: 100000 training curves drawn from the
    GP on the device, the CNN trained on them, then 256 held-out curves fitted by BFGS from the
    plain start and from the learned one (the reference: the best optimum of those and of the true start)."""
    import numpy as np
    dt = 2 / 1440
    t = np.arange(18000) * dt
    t[9000:] += 720 * dt
    ntr, bs, nev = 100000, 256, 256
    X = torch.empty((ntr, 512), dtype=torch.float32, device=ctx.device)
    Y = torch.empty((ntr, 4), dtype=torch.float32, device=ctx.device)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for base in range(0, ntr, 8192):
        k = min(8192, ntr - base)
        d = api.gp_sample(ctx, t, k, theta=None, seed=5_000_000, curve_base=base)
        X[base:base + k] = d["input"]
        Y[base:base + k] = d["target"]
    torch.cuda.synchronize()
    t_sample = time.perf_counter() - t0
    log(f"sampled {ntr} curves of N=18000 in {t_sample:.2f} s")
    m = api.CNN(ctx, half=True, max_batch=bs, seed=1)
    steps = ntr // bs
    loss = torch.empty(1, dtype=torch.float32, device=ctx.device)
    ctx.enable_timing(True)
    ctx.reset_timing()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for ep in range(args.epochs):
        lr = 2e-3 * 0.5 ** (ep // 4)
        for s in range(steps):
            j = ((s + 37 * ep) % steps) * bs
            m.train_step(X[j:j + bs], Y[j:j + bs], lr=lr, loss=loss)
        log(f"epoch {ep + 1}/{args.epochs}: loss of the last batch {loss.item():.4f}")
    torch.cuda.synchronize()
    t_train = time.perf_counter() - t0
    train_timings = ctx.timings()
    d = api.gp_sample(ctx, t, nev, theta=None, seed=6000, curve_base=0, flux=True)
    th = d["theta"].cpu().numpy()
    prot = 4 * np.pi * th[:, 2] / (th[:, 1] * np.sqrt(4 * th[:, 2] ** 2 - 1))
    x_true = np.log(np.column_stack([th[:, 0], prot, th[:, 2], th[:, 3]]))
    x = (t - t.mean()) / (np.ptp(t) / 2)
    A1 = np.concatenate([np.stack([np.ones_like(x), x, x * x])] * nev).reshape(-1)
    batch = {"n_curves": nev, "sample_off": np.arange(nev + 1, dtype=np.int64) * t.size,
             "t": torch.as_tensor(np.tile(t, nev), device=ctx.device), "f": d["flux"].reshape(-1).contiguous(),
             "A": torch.as_tensor(A1, device=ctx.device), "m1": 3}
    grid = np.exp(np.linspace(math.log(0.1), math.log(5.0), 1000))
    ctx.reset_timing()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    x_plain = api.plain_init(ctx, batch, grid)
    t_plain_init = time.perf_counter() - t0
    t0 = time.perf_counter()
    x_learned = m.warm_start(d["input"], x_plain)
    torch.cuda.synchronize()
    t_infer = time.perf_counter() - t0
    fits, t_fit = {}, {}
    for k, x0 in (("plain", x_plain), ("learned", x_learned), ("truth", x_true)):
        t0 = time.perf_counter()
        fits[k] = api.fit_hyper(ctx, batch, x0, max_iter=300, gtol=1e-3)
        t_fit[k] = time.perf_counter() - t0
        log(f"fit from the {k} start: {t_fit[k]:.2f} s, {fits[k]['n_eval'].mean():.1f} likelihood evaluations per curve")
    timings = ctx.timings()
    ctx.enable_timing(False)
    best = np.min(np.stack([f["nll"] for f in fits.values()]), axis=0)
    summary = {}
    for k in ("plain", "learned"):
        gap = fits[k]["nll"] - best
        x0 = (x_plain if k == "plain" else x_learned).cpu().numpy()
        summary[k] = {"success_rate": float(np.mean(gap < 0.1)), "mean_evaluations": float(fits[k]["n_eval"].mean()),
                      "fit_seconds": t_fit[k], "curves_per_s": nev / t_fit[k],
                      "median_abs_log_error_at_start": np.median(np.abs(x0 - x_true), axis=0).round(4).tolist()}
    cfg = {"workload": "learned-warm-start-tess-sector", "train_curves": ntr, "epochs": args.epochs,
           "batch": bs, "eval_curves": nev, "n_samples": int(t.size), "precision": "cnn fp16/fp32, fit fp64"}
    extra = {"sampler_curves_per_s": ntr / t_sample, "train_samples_per_s": ntr * args.epochs / t_train,
             "train_seconds": t_train, "plain_start_seconds": t_plain_init, "learned_start_seconds": t_infer,
             "fit": summary, "train_kernels": {k: v["ms"] for k, v in train_timings.items()}}
    return t_fit["learned"], nev, nev, timings, None, cfg, extra


def bench_curve(args, api, ctx, torch):
    """One TESS-sector-shaped curve per step (eager calls, or one captured-graph launch)."""
    w = workload(args.workload)
    dev = ctx.device
    dev_in = {
        "t": torch.as_tensor(w.t, device=dev), "f": torch.as_tensor(w.f, device=dev),
        "A": torch.as_tensor(w.A, device=dev), "lattice": torch.as_tensor(w.lattice, device=dev),
        "periods": torch.as_tensor(w.periods, device=dev),
    }
    fac = None
    g = None
    kernel = None
    shapes = None
    if args.template != "box":
        from synth import templates as stpl
        shapes = stpl.shapes_for(args.template, w.durations)
    if args.kernel == "rotation":
        kernel = api.rotation_kernel(**ROTATION_KERNEL)
    elif args.solver == "statespace":
        kernel = api.SHO.from_dict(w.theta)
    ctx_prefetch = args.inverse_prefetch == "on" and args.mode == "eager" and args.solver == "dense" \
        and args.precision != "fp64"
    if ctx_prefetch:
        ctx.set_inverse_prefetch(args.precision, args.prefetch_cus)
    if args.mode == "graph":
        g = api.Graph(ctx, dev_in["t"], dev_in["f"], dev_in["A"], dev_in["lattice"], w.n_epochs, w.durations,
                      w.theta, w.dt, dev_in["periods"], precision=args.precision)
    full = None  # every launch of the last warm-up step timed: the per-kernel breakdown
    for i in range(max(args.warmup, 1)):
        last = i == max(args.warmup, 1) - 1
        if g is None:
            if last:
                ctx.enable_timing(True)
                ctx.reset_timing()
            fac, _, _, _ = run_step(api, ctx, dev_in, w, args.precision, fac, args.planets, args.solver, kernel,
                                    shapes)
            if last:
                full = ctx.timings()
                ctx.enable_timing(False)
        else:
            g.launch()
        torch.cuda.synchronize()
        log(f"warmup {i + 1}/{args.warmup} done")
    # the timed steps record events only around the launches of the dominant kernel
    # (the roofline's), so that the other launches run as they do untimed
    dominant = roofline_of(full)[0]["kernel"] if full else None
    ctx.enable_timing(g is None)
    if dominant:
        ctx.set_timing_filter(dominant)
    ctx.reset_timing()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    keep = None
    for i in range(args.steps):
        # one curve per step; the factor's device buffers are reused across curves of one length
        if g is None:
            keep = run_step(api, ctx, dev_in, w, args.precision, fac, args.planets, args.solver, kernel, shapes)
        else:
            g.launch()
        log(f"step {i + 1}/{args.steps} enqueued")
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    timings = ctx.timings()
    ctx.enable_timing(False)
    ctx.set_timing_filter("")
    cands = None
    if g is None:
        fac, ls, ps, cands = keep
        got = dict(ls)
        got.update(ps)
    else:
        assert int(g.status.item()) == -1
        got = g.out
        fac = api.gp_factor(ctx, dev_in["t"], w.theta)
    valid, best = got["valid"], int(got["best_index"].item())
    n_valid = int(valid.sum().item())
    dll_err = None
    if (args.precision != "fp64" or args.solver == "statespace") and not args.no_dll_check:
        # accuracy of this path against the dense FP64 path on the same curve (outside the timed region)
        if fac is None:
            fac = api.gp_factor(ctx, dev_in["t"], w.theta if kernel is None or args.kernel != "rotation" else kernel)
        ref = dict(api.linear_search(ctx, fac, dev_in["f"], dev_in["A"], dev_in["lattice"], w.n_epochs,
                                     w.durations, shapes=shapes))
        ref.update(api.periodic_search(ctx, ref["depth"], ref["var"], ref["dll"], ref["valid"], w.dt,
                                       dev_in["periods"]))
        dll_err = output_errors(got, ref)
        log(f"errors vs fp64: {dll_err}")
    log(f"{args.steps} steps in {elapsed:.3f} s: {n_valid * args.steps / elapsed:.4g} fits/s, "
        f"{args.steps / elapsed:.4g} curves/s; best period {w.periods[best] if best >= 0 else None}")
    cfg = {"workload": w.name, "n_samples": w.n, "n_epochs": w.n_epochs, "n_durations": int(w.durations.size),
           "n_periods": int(w.periods.size), "valid_cells": n_valid,
           "precision": args.precision if args.solver == "dense" else "fp64", "mode": args.mode,
           "solver": args.solver, "kernel": args.kernel, "template": args.template}
    if ctx_prefetch:
        cfg["inverse_prefetch_cus"] = args.prefetch_cus
    extra = {"best_period_days": float(w.periods[best]) if best >= 0 else None,
             "injected_period_days": w.injection["period"] if w.injection else None}
    if full:
        extra["_one_step_timings"] = full
    if args.planets > 1:
        cfg["planets"] = args.planets
        extra["candidates"] = cands
    return elapsed, n_valid, 1, timings, dll_err, cfg, extra, w


def bench_extras(args, api, ctx, torch):
    """Beside the headline curve: the uneven 64-curve batch, FP32_REFINE against FP64, each one captured
    batch graph per step and one eager batch call per step (seconds per batch, curves/s, fits/s, the
    per-kernel time and dominant-kernel roofline of one timed eager call, and the FP32_REFINE errors against
    the FP64 batch over every cell); and the 1440-sample curve in FP64 with its per-stage microseconds."""
    import numpy as np

    from synth import config1, config3
    out = {}
    t0 = time.perf_counter()
    ws = config3()
    curves = [{"t": w.t, "f": w.f, "A": w.A, "lattice": w.lattice, "n_epochs": w.n_epochs, "theta": w.theta,
               "dt": w.dt} for w in ws]
    durs, per = ws[0].durations, torch.as_tensor(ws[0].periods, device=ctx.device)
    batch = api.prepare_batch(ctx, curves)
    log(f"extras: 64-curve batch generated in {time.perf_counter() - t0:.1f} s")
    ctx.release_memory()
    res = {}
    for prec in ("fp32_refine", "fp64"):
        g = api.BatchGraph(ctx, batch, durs, per, precision=prec)
        g.launch()
        torch.cuda.synchronize()
        steps = args.extra_steps
        t0 = time.perf_counter()
        for _ in range(steps):
            o = g.launch()
        torch.cuda.synchronize()
        el = (time.perf_counter() - t0) / steps
        n_valid = int(o["valid"].sum().item())
        res[prec] = {k: (o[k].clone() if hasattr(o[k], "clone") else o[k]) for k in
                     ("depth", "var", "dll", "valid", "q_snr", "best_phase", "best_dur")}
        out[prec] = {"s_per_batch": el, "curves_per_s": len(ws) / el, "fits_per_s": n_valid / el,
                     "valid_cells": n_valid, "mode": "one captured batch graph launch per step", "steps": steps}
        log(f"extras: batch-64 {prec}: {el:.3f} s per batch, {n_valid / el:.4g} fits/s")
        g.close()
        del g
        # the same batch through the eager batch call (one wait at its end)
        api.search_batch(ctx, batch, durs, per, precision=prec)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(steps):
            api.search_batch(ctx, batch, durs, per, precision=prec)
        torch.cuda.synchronize()
        out[prec]["eager_call_s_per_batch"] = (time.perf_counter() - t0) / steps
        log(f"extras: batch-64 {prec}, eager call: {out[prec]['eager_call_s_per_batch']:.3f} s per batch")
        # one more eager call with every launch timed (HIP events on the launch streams): the batch's
        # per-kernel time and the roofline of its dominant kernel (durations overlapped, as in the headline)
        ctx.enable_timing(True)
        ctx.reset_timing()
        api.search_batch(ctx, batch, durs, per, precision=prec)
        torch.cuda.synchronize()
        tm = ctx.timings()
        ctx.enable_timing(False)
        roof, _ = roofline_of(tm)
        out[prec]["roofline"] = {k: roof[k] for k in ("kernel", "bound", "achieved", "peak", "unit", "frac",
                                                      "launches", "avg_launch_ms")}
        out[prec]["kernels_ms_per_batch"] = {k: v["ms"] for k, v in sorted(tm.items(), key=lambda kv: -kv[1]["ms"])
                                             if not k.startswith("host:")}
        ctx.release_memory()  # the eager call's arena, before the next graph takes its own
    out["errors_fp32_refine_vs_fp64"] = output_errors(res["fp32_refine"], res["fp64"])
    out["fp32_refine_speedup_vs_fp64"] = out["fp64"]["s_per_batch"] / out["fp32_refine"]["s_per_batch"]
    del res, batch
    ctx.release_memory()
    # the 1440-sample curve, FP64: per-stage microseconds (kernel time per step, HIP events)
    w = config1()
    dev_in = {"t": torch.as_tensor(w.t, device=ctx.device), "f": torch.as_tensor(w.f, device=ctx.device),
              "A": torch.as_tensor(w.A, device=ctx.device), "lattice": torch.as_tensor(w.lattice, device=ctx.device),
              "periods": torch.as_tensor(w.periods, device=ctx.device)}
    run_step(api, ctx, dev_in, w, "fp64")
    torch.cuda.synchronize()
    steps = 10
    ctx.enable_timing(True)
    ctx.reset_timing()
    t0 = time.perf_counter()
    for _ in range(steps):
        fac, ls, ps, _ = run_step(api, ctx, dev_in, w, "fp64")
    torch.cuda.synchronize()
    el = (time.perf_counter() - t0) / steps
    tm = ctx.timings()
    ctx.enable_timing(False)
    stages = {"K build": ["kbuild"], "Cholesky": ["potrf_diag", "gemm_f64:panel", "gemm_f64:panel_update",
                                                  "gemm_f64:trailing"],
              "inverse": ["gemm_f64:inverse"], "trend fit and passes": ["rows_matvec", "null_solve", "cols_matvec"],
              "box sums": ["q_partial"], "cell normal equations": ["cell_epilogue"], "fold": ["fold"],
              "best period": ["best_period"]}
    out["plain_1440_fp64"] = {
        "workload": "plain-fp64-N1440", "us_per_step": el * 1e6,
        "stage_kernel_us": {k: sum(tm[n]["ms"] for n in v if n in tm) / steps * 1e3 for k, v in stages.items()},
        "launches_per_step": sum(v["launches"] for v in tm.values()) / steps}
    log(f"extras: plain-1440 fp64 {el * 1e6:.0f} us per step")
    return out


def main(argv=None):
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--workload", default="tess-sector",
                    choices=["tess-sector", "plain-1440", "batch-64", "learned", "two-sectors"])
    ap.add_argument("--epochs", type=int, default=12, help="training epochs of the learned workload")
    ap.add_argument("--precision", default="fp32_refine", choices=["fp64", "fp32_refine", "bf16x3_refine"])
    ap.add_argument("--mode", default="eager", choices=["eager", "graph", "loop"])
    ap.add_argument("--solver", default="dense", choices=["dense", "statespace"],
                    help="linear search from the dense factor, or from the state-space (Kalman) form of the "
                         "covariance (FP64; single-curve eager mode)")
    ap.add_argument("--template", default="box", choices=["box", "limb_darkened", "exocomet"],
                    help="single-event base model in the last column of the design (Section 4.4, prospects)")
    ap.add_argument("--kernel", default="sho", choices=["sho", "rotation"],
                    help="covariance: the workload's SHO, or the stellar-variability kernel of Section 3.2")
    ap.add_argument("--planets", type=int, default=1,
                    help="candidates per curve: after each periodic search the found transits are masked in the "
                         "linear-search products and the periodic search is repeated (single-curve eager mode)")
    ap.add_argument("--autotune", action="store_true", help="tune the tile policy before warming up")
    ap.add_argument("--inverse-prefetch", default="on", choices=["on", "off"],
                    help="compute the reduced-precision inverse inside the factorisation (dense solver, "
                         "single-curve eager steps)")
    ap.add_argument("--prefetch-cus", type=int, default=0,
                    help="compute units of the inverse started inside the factorisation (0: three quarters)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-extras", action="store_true",
                    help="headline curve only: skip the 64-curve batch (FP32_REFINE and FP64) and the "
                         "1440-sample per-stage timings")
    ap.add_argument("--extra-steps", type=int, default=2, help="timed batch launches per precision in the extras")
    ap.add_argument("--no-dll-check", action="store_true",
                    help="skip the FP64 reference search that measures the dll error of a reduced precision "
                         "(keeps a profiled run to the timed kernels)")
    ap.add_argument("--copy-probe-mib", type=int, default=0,
                    help="before the workload, one plain device copy of this many MiB (a kernel of known "
                         "traffic, to scale hardware byte counters)")
    args = ap.parse_args(argv)
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for --gpus {args.gpus}); curves shard across GPUs with no "
              "communication, and the timed step is one GPU's share", file=sys.stderr)
        return 2

    import torch

    from paper_2402_06835_amd import _lib, api

    _lib.lib()
    assert torch.cuda.is_available(), "bench needs a GPU"
    log(f"workload {args.workload}, precision {args.precision}, mode {args.mode}")
    if args.copy_probe_mib > 0:
        n = args.copy_probe_mib * (1 << 20) // 8
        src = torch.ones(n, dtype=torch.float64, device="cuda")
        dst = torch.empty_like(src)
        torch.cuda.synchronize()
        dst.copy_(src)
        torch.cuda.synchronize()
        log(f"copy probe: {args.copy_probe_mib} MiB read + {args.copy_probe_mib} MiB written")
        del src, dst
    ctx = api.Context(0)
    tuning = None
    if args.autotune:
        t0 = time.perf_counter()
        tuning = ctx.autotune(18000 if args.workload != "plain-1440" else 1440, args.precision)
        log(f"autotuned in {time.perf_counter() - t0:.1f} s: {tuning}")
    w = None
    if args.workload == "learned":
        elapsed, n_valid, curves, timings, dll_err, cfg, extra = bench_learned(args, api, ctx, torch)
        out = {"metric": "ML hyperparameter fits/s from the learned warm start", "value": n_valid / elapsed,
               "unit": "curves/s", "n_gpus": 1, "steps": 1, "warmup": 0, "ms_per_step": elapsed * 1e3,
               "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f16+f32 (cnn), f64 (fit)",
               "data": "synthetic", "config": cfg, "roofline": None,
               "kernels": {k: {"launches": v["launches"], "ms": v["ms"]} for k, v in timings.items()}}
        out.update(extra)
        print(json.dumps(out), flush=True)
        return 0
    if args.workload == "batch-64":
        elapsed, n_valid, curves, timings, dll_err, cfg, extra = bench_batch(args, api, ctx, torch)
    elif args.workload == "two-sectors":
        if args.mode != "eager" or args.planets > 1:
            raise SystemExit("the two-sector search runs eager, one candidate")
        elapsed, n_valid, curves, timings, dll_err, cfg, extra = bench_two_sectors(args, api, ctx, torch)
    else:
        if args.mode == "loop":
            raise SystemExit("--mode loop compares against the batch (--workload batch-64)")
        if args.planets > 1 and args.mode != "eager":
            raise SystemExit("--planets applies to the eager single-curve step")
        if (args.solver == "statespace" or args.kernel == "rotation" or args.template != "box") and \
                args.mode != "eager":
            raise SystemExit("--solver statespace, --kernel rotation and --template run the eager single-curve step")
        elapsed, n_valid, curves, timings, dll_err, cfg, extra, w = bench_curve(args, api, ctx, torch)
    roof, gemms = (roofline_of(timings) if timings else (None, None))
    if roof is not None:
        roof["traffic"] = measured_traffic(roof, args.workload, args.precision)
    kernels = {k: {"launches": v["launches"], "ms_per_step": v["ms"] / args.steps} for k, v in timings.items()}
    one = extra.pop("_one_step_timings", None)
    kernels_from = "the timed steps"
    if one:
        # the breakdown of every kernel comes from the last warm-up step, which timed every launch
        _, gemms_one = roofline_of(one)
        gemms = {k: {"tflops": v["tflops"], "ms": v["ms"] * args.steps} for k, v in gemms_one.items()}
        kernels = {k: {"launches": v["launches"], "ms_per_step": v["ms"]} for k, v in one.items()}
        kernels_from = ("the last warm-up step, every launch timed (the timed steps record events only around "
                        f"the launches of {roof['kernel'] if roof else 'the dominant kernel'})")
    out = {
        "metric": "(t0,D) GLS fits/s and light curves/s at Δll err ≤1e-6 vs FP64",
        "value": n_valid * args.steps / elapsed, "unit": "(t0,D) fits/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": elapsed / args.steps * 1e3, "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None,
        "dtype": "f64" if args.solver == "statespace" else
        {"fp64": "f64", "fp32_refine": "f64+f32", "bf16x3_refine": "f64+bf16x3"}[args.precision], "data": "synthetic",
        "config": cfg,
        "light_curves_per_s": curves * args.steps / elapsed,
        "errors_vs_fp64": dll_err,
        "gemm_by_type": {k: {"tflops": v["tflops"], "ms_per_step": v["ms"] / args.steps} for k, v in gemms.items()}
        if gemms else None,
        "roofline": roof,
        "kernels": kernels,
        "kernels_from": kernels_from,
        "tuning": tuning,
    }
    out.update(extra)
    if (not args.no_extras and args.workload == "tess-sector" and args.mode == "eager" and args.solver == "dense"
            and args.kernel == "sho" and args.template == "box" and args.planets == 1):
        out["batch_64"] = bench_extras(args, api, ctx, torch)
        out["plain_1440_fp64"] = out["batch_64"].pop("plain_1440_fp64")
    if not args.no_cpu_baseline and w is not None:
        shapes = None
        if args.template != "box":
            from synth import templates as stpl
            shapes = stpl.shapes_for(args.template, w.durations)
        out["cpu_baseline"] = cpu_baseline(w, n_valid, kernel=args.kernel, shapes=shapes)
        out["cpu_baseline"]["unit"] = out["unit"]
    print(json.dumps(out), flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
