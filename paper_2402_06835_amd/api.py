"""Python binding of the transit-search library (argument marshalling only).

Functional layer with the C ABI's names (``Context``, ``gp_factor``,
``linear_search``, ``periodic_search``) over torch device tensors, plus a
``Nuance`` object shaped like the paper's interface (Section 2.5):
``Nuance(time, flux, gp=..., X=...)``, ``.linear_search(t0s, Ds)``,
``.periodic_search(periods)`` with ``.best`` and ``.Q_snr``.

Every step of the search runs in the HIP library; this module only checks
and converts arguments, allocates outputs with torch and passes pointers.
"""
from __future__ import annotations

import atexit
import ctypes
import weakref
from dataclasses import dataclass, field
from typing import Optional

import numpy as np
import torch

from ._lib import NU_ERR_NOT_PD, NU_OK, PRECISIONS, TUNE_CLASSES, NuanceError, NuKernel, NuSho, lib


# Live library handles. Every handle the binding creates is closed by an exit
# hook, in dependency order (factors, graphs and networks before the contexts
# whose streams and events they use), while the HIP runtime is still up: left to
# __del__, a handle held at module scope is released only during interpreter
# teardown, after the runtime may have begun to tear down its own state.
_LIVE = {0: weakref.WeakSet(), 1: weakref.WeakSet()}  # 0: factors, graphs, networks; 1: contexts


def _register(obj, rank: int):
    _LIVE[rank].add(obj)


@atexit.register
def _close_live_handles():
    for rank in (0, 1):
        for obj in list(_LIVE[rank]):
            try:
                obj.close()
            except Exception:
                pass


def _check(ctx_ptr, status: int):
    if status != NU_OK:
        msg = lib().nu_ctx_last_error(ctx_ptr)
        raise NuanceError(status, msg.decode() if msg else "")


def _dev_tensor(x, dtype, device) -> torch.Tensor:
    if isinstance(x, torch.Tensor):
        t = x.to(device=device, dtype=dtype)
    else:
        t = torch.as_tensor(np.ascontiguousarray(x), dtype=dtype, device=device)
    return t.contiguous()


@dataclass
class SHO:
    """SHO covariance (Appendix A) + white noise: amp = sigma, omega, Q, sigma_w."""

    amp: float
    omega: float
    q: float
    sigma_w: float = 0.0

    @classmethod
    def from_dict(cls, d: dict) -> "SHO":
        return cls(float(d["amp"]), float(d["omega"]), float(d["q"]), float(d["sigma_w"]))

    def c(self) -> NuSho:
        return NuSho(self.amp, self.omega, self.q, self.sigma_w)


class Context:
    """Library context bound to one device and (by default) torch's current stream."""

    def __init__(self, device: int = 0, stream: Optional[torch.cuda.Stream] = None, workspace_limit: int = 0):
        """workspace_limit: bytes of device memory the library may allocate on this
        context (0: no limit); a call that would exceed it raises NuanceError
        with NU_ERR_OOM."""
        if not torch.cuda.is_available():
            raise RuntimeError("no GPU visible: the transit-search library runs on the device only")
        self.device = torch.device("cuda", device)
        if stream is None:
            stream = torch.cuda.current_stream(self.device)
        self.stream = stream
        p = ctypes.c_void_p()
        st = lib().nu_ctx_create(device, ctypes.c_void_p(stream.cuda_stream), int(workspace_limit), ctypes.byref(p))
        if st != NU_OK:
            raise NuanceError(st, "nu_ctx_create failed")
        self.ptr = p
        _register(self, 1)

    def close(self):
        if getattr(self, "ptr", None):
            lib().nu_ctx_destroy(self.ptr)
            self.ptr = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def release_memory(self):
        """Free the device memory the context keeps between calls (workspace, batch arena)."""
        _check(self.ptr, lib().nu_ctx_release_memory(self.ptr))

    def device_bytes(self) -> int:
        """Device bytes counted against the workspace limit right now."""
        return int(lib().nu_ctx_device_bytes(self.ptr))

    def set_inverse_prefetch(self, precision: Optional[str], compute_units: int = 0):
        """Compute the factor's reduced-precision inverse inside every later
        ``gp_factor`` ("fp32_refine" or "bf16x3_refine"; None turns it off), its
        early phases on ``compute_units`` CUs beside the factorisation (0: three quarters of the chip)."""
        if precision is not None and precision not in ("fp32_refine", "bf16x3_refine"):
            raise ValueError("inverse prefetch is for fp32_refine or bf16x3_refine")
        code = -1 if precision is None else PRECISIONS[precision]
        _check(self.ptr, lib().nu_ctx_set_inverse_prefetch(self.ptr, code, int(compute_units)))

    def enable_timing(self, on: bool = True):
        _check(self.ptr, lib().nu_ctx_enable_timing(self.ptr, int(on)))

    def set_timing_filter(self, prefix: str = ""):
        """Time only the launches whose kernel name starts with prefix ("" for all)."""
        _check(self.ptr, lib().nu_ctx_set_timing_filter(self.ptr, prefix.encode()))

    def reset_timing(self):
        _check(self.ptr, lib().nu_ctx_timing_reset(self.ptr))

    def timings(self) -> dict:
        """{kernel name: {"launches", "ms", "work"}} accumulated since the last reset."""
        out = {}
        n = lib().nu_ctx_timing_count(self.ptr)
        for i in range(n):
            name = ctypes.c_char_p()
            launches = ctypes.c_int64()
            ms = ctypes.c_double()
            work = ctypes.c_double()
            _check(self.ptr, lib().nu_ctx_timing_entry(self.ptr, i, ctypes.byref(name), ctypes.byref(launches),
                                                       ctypes.byref(ms), ctypes.byref(work)))
            out[name.value.decode()] = {"launches": launches.value, "ms": ms.value, "work": work.value}
        return out


    # tile policy of the dense launches (entry point 6 of the C ABI)
    def autotune(self, n: int, precision: str = "fp64") -> dict:
        """Time six tile thresholds per launch class on a synthetic covariance of size n; keep the fastest."""
        _check(self.ptr, lib().nu_ctx_autotune(self.ptr, int(n), PRECISIONS[precision]))
        return self.tuning()

    def tuning(self) -> dict:
        out = {}
        for i, name in enumerate(TUNE_CLASSES):
            v = ctypes.c_int()
            _check(self.ptr, lib().nu_ctx_get_tuning(self.ptr, i, ctypes.byref(v)))
            out[name] = v.value
        return out

    def set_tuning(self, **thresholds):
        for name, v in thresholds.items():
            _check(self.ptr, lib().nu_ctx_set_tuning(self.ptr, TUNE_CLASSES.index(name), int(v)))


class Factor:
    """Device Cholesky factor of K (and, once a search ran, its inverse)."""

    def __init__(self, ptr, n: int, logdet: float):
        self.ptr = ptr
        self.n = n
        self.logdet = logdet
        _register(self, 0)

    def close(self):
        if getattr(self, "ptr", None):
            lib().nu_factor_destroy(self.ptr)
            self.ptr = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


@dataclass
class Kernel:
    """A covariance as a sum of terms (entry point 1b): SHO terms (amp, omega, q), exponential terms
    (sigma, ell): sigma^2 exp(-|tau| / ell), and sigma_w^2 on the diagonal."""

    sho: list = field(default_factory=list)
    exp: list = field(default_factory=list)
    sigma_w: float = 0.0

    def c(self) -> NuKernel:
        if len(self.sho) > 4 or len(self.exp) > 4:
            raise ValueError("at most 4 SHO and 4 exponential terms")
        k = NuKernel()
        k.n_sho, k.n_exp = len(self.sho), len(self.exp)
        for i, (a, w, q) in enumerate(self.sho):
            k.sho_amp[i], k.sho_omega[i], k.sho_q[i] = float(a), float(w), float(q)
        for i, (sg, ell) in enumerate(self.exp):
            k.exp_sigma[i], k.exp_ell[i] = float(sg), float(ell)
        k.sigma_w = float(self.sigma_w)
        return k


def rotation_kernel(sigma: float, period: float, q0: float, dq: float, f: float, sigma_short: float,
                    ell_short: float, sigma_long: float, ell_long: float, sigma_w: float) -> Kernel:
    """The stellar-variability kernel of Section 3.2, k = k1 + k2 + k3 + k4 (8 hyperparameters, plus the
    white-noise diagonal), parametrised by the library (``nu_rotation_kernel``): SHO terms at the rotation
    period and at half of it, and the short and long exponential terms."""
    k = NuKernel()
    st = lib().nu_rotation_kernel(float(sigma), float(period), float(q0), float(dq), float(f), float(sigma_short),
                                  float(ell_short), float(sigma_long), float(ell_long), float(sigma_w),
                                  ctypes.byref(k))
    if st != NU_OK:
        raise NuanceError(st, "rotation_kernel: invalid hyperparameters")
    return Kernel(sho=[(k.sho_amp[i], k.sho_omega[i], k.sho_q[i]) for i in range(k.n_sho)],
                  exp=[(k.exp_sigma[i], k.exp_ell[i]) for i in range(k.n_exp)], sigma_w=k.sigma_w)


def gp_factor(ctx: Context, t, theta, out: Optional[Factor] = None) -> Factor:
    """K = k_SHO + sigma_w^2 I (``theta``: SHO or dict), or a sum of terms (``theta``: Kernel), built and
    factored on the device (one stream sync).

    With ``out`` (a factor of the same length; SHO only) its device buffers are reused."""
    t_dev = _dev_tensor(t, torch.float64, ctx.device)
    logdet = ctypes.c_double()
    pivot = ctypes.c_int64(-1)
    if isinstance(theta, Kernel):
        if out is not None:
            raise ValueError("a sum-of-terms kernel factors into a new factor (out is for SHO refits)")
        kc = theta.c()
        p = ctypes.c_void_p()
        st = lib().nu_gp_factor_kernel(ctx.ptr, ctypes.c_void_p(t_dev.data_ptr()), t_dev.numel(), ctypes.byref(kc),
                                       ctypes.byref(p), ctypes.byref(logdet), ctypes.byref(pivot))
        if st != NU_OK:
            err = NuanceError(st, lib().nu_ctx_last_error(ctx.ptr).decode())
            err.pivot = pivot.value
            raise err
        return Factor(p, t_dev.numel(), logdet.value)
    sho = theta if isinstance(theta, SHO) else SHO.from_dict(theta)
    c = sho.c()
    if out is not None:
        st = lib().nu_gp_factor_into(ctx.ptr, out.ptr, ctypes.c_void_p(t_dev.data_ptr()), t_dev.numel(),
                                     ctypes.byref(c), ctypes.byref(logdet), ctypes.byref(pivot))
        p = None
    else:
        p = ctypes.c_void_p()
        st = lib().nu_gp_factor(ctx.ptr, ctypes.c_void_p(t_dev.data_ptr()), t_dev.numel(), ctypes.byref(c),
                                ctypes.byref(p), ctypes.byref(logdet), ctypes.byref(pivot))
    if st != NU_OK:
        msg = lib().nu_ctx_last_error(ctx.ptr).decode()
        err = NuanceError(st, msg)
        err.pivot = pivot.value
        raise err
    if out is not None:
        out.logdet = logdet.value
        return out
    return Factor(p, t_dev.numel(), logdet.value)


def _shapes_arg(shapes, durs):
    """Concatenated template shapes (one per duration, d_j values each) as a contiguous host array, or None."""
    if shapes is None:
        return None
    if len(shapes) != durs.size:
        raise ValueError("one shape per duration")
    parts = [np.asarray(s, dtype=np.float64).reshape(-1) for s in shapes]
    for p_, d in zip(parts, durs):
        if p_.size != int(d):
            raise ValueError("shape j must hold durations[j] values (one per slot of the window)")
    return np.ascontiguousarray(np.concatenate(parts))


def linear_search(ctx: Context, factor: Factor, f, A, lattice, n_epochs: int, durations,
                  precision: str = "fp64", shapes=None) -> dict:
    """Single-event GLS fits over every (duration, epoch slot) cell.

    f: (N,), A: (N, m1) trend design or None, lattice: (N,) int64 slot of each
    sample (lattice[0] == 0, strictly increasing), durations: box lengths in
    slots. Returns device tensors depth, var, dll (float64) and valid (uint8),
    shaped (n_d, n_epochs), and ``null`` = [ln L_0, chi2_0, ln|K|].

    ``shapes``: one shape per duration (``durations[j]`` values, one per slot of
    the window) in place of the box (entry point 2c): limb-darkened transits,
    exocomets, any single-event base model.
    """
    dev = ctx.device
    f_d = _dev_tensor(f, torch.float64, dev)
    n = f_d.numel()
    if A is None:
        m1 = 0
        A_d = None
    else:
        A_t = A if isinstance(A, torch.Tensor) else torch.as_tensor(np.asarray(A, dtype=np.float64))
        if A_t.ndim == 1:
            A_t = A_t[:, None]
        if A_t.shape[0] != n:
            raise ValueError("A must be (N, m1)")
        m1 = int(A_t.shape[1])
        A_d = A_t.to(device=dev, dtype=torch.float64).t().contiguous()  # column-major N x m1
    lat = _dev_tensor(lattice, torch.int64, dev)
    if lat.numel() != n:
        raise ValueError("lattice must have N entries")
    durs = np.ascontiguousarray(np.asarray(durations, dtype=np.int32))
    n_d = int(durs.size)
    shape = (n_d, int(n_epochs))
    depth = torch.empty(shape, dtype=torch.float64, device=dev)
    var = torch.empty(shape, dtype=torch.float64, device=dev)
    dll = torch.empty(shape, dtype=torch.float64, device=dev)
    valid = torch.empty(shape, dtype=torch.uint8, device=dev)
    null = torch.empty(3, dtype=torch.float64, device=dev)
    if precision not in PRECISIONS:
        raise ValueError(f"precision must be one of {sorted(PRECISIONS)}")
    shp = _shapes_arg(shapes, durs)
    if shp is None:
        st = lib().nu_linear_search(
            ctx.ptr, factor.ptr, ctypes.c_void_p(f_d.data_ptr()),
            ctypes.c_void_p(A_d.data_ptr() if A_d is not None else 0), m1, ctypes.c_void_p(lat.data_ptr()),
            int(n_epochs), durs.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)), n_d, PRECISIONS[precision],
            ctypes.c_void_p(depth.data_ptr()), ctypes.c_void_p(var.data_ptr()), ctypes.c_void_p(dll.data_ptr()),
            ctypes.c_void_p(valid.data_ptr()), ctypes.c_void_p(null.data_ptr()))
    else:
        st = lib().nu_linear_search_template(
            ctx.ptr, factor.ptr, ctypes.c_void_p(f_d.data_ptr()),
            ctypes.c_void_p(A_d.data_ptr() if A_d is not None else 0), m1, ctypes.c_void_p(lat.data_ptr()),
            int(n_epochs), durs.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)), n_d,
            shp.ctypes.data_as(ctypes.POINTER(ctypes.c_double)), PRECISIONS[precision],
            ctypes.c_void_p(depth.data_ptr()), ctypes.c_void_p(var.data_ptr()), ctypes.c_void_p(dll.data_ptr()),
            ctypes.c_void_p(valid.data_ptr()), ctypes.c_void_p(null.data_ptr()))
    _check(ctx.ptr, st)
    # keep the inputs alive until the enqueued work has consumed them
    return {"depth": depth, "var": var, "dll": dll, "valid": valid, "null": null,
            "_keep": (f_d, A_d, lat)}


def _as_kernel(theta) -> "Kernel":
    if isinstance(theta, Kernel):
        return theta
    sho = theta if isinstance(theta, SHO) else SHO.from_dict(theta)
    return Kernel(sho=[(sho.amp, sho.omega, sho.q)], sigma_w=sho.sigma_w)


def linear_search_ss(ctx: Context, t, theta, f, A, lattice, n_epochs: int, durations, check: bool = True,
                     shapes=None) -> dict:
    """The linear search of ``linear_search`` from the state-space (Kalman) form of the covariance
    (entry point 2b): no N x N factor, O(N J^2) work. ``theta``: Kernel, SHO or SHO dict.

    With ``check`` the call waits for the filter and raises NU_ERR_NOT_PD (with ``.index``, the first
    failing sample) if an innovation variance is not positive; without it nothing waits, and a failure
    shows as NaN in ``null`` and every cell invalid. ``shapes`` as in ``linear_search``."""
    dev = ctx.device
    kc = _as_kernel(theta).c()
    t_d = _dev_tensor(t, torch.float64, dev)
    f_d = _dev_tensor(f, torch.float64, dev)
    n = f_d.numel()
    if t_d.numel() != n:
        raise ValueError("t and f must have the same length")
    m1, A_d = _trend_colmajor(A, n, dev)
    lat = _dev_tensor(lattice, torch.int64, dev)
    if lat.numel() != n:
        raise ValueError("lattice must have N entries")
    durs = np.ascontiguousarray(np.asarray(durations, dtype=np.int32))
    n_d = int(durs.size)
    shape = (n_d, int(n_epochs))
    depth = torch.empty(shape, dtype=torch.float64, device=dev)
    var = torch.empty(shape, dtype=torch.float64, device=dev)
    dll = torch.empty(shape, dtype=torch.float64, device=dev)
    valid = torch.empty(shape, dtype=torch.uint8, device=dev)
    null = torch.empty(3, dtype=torch.float64, device=dev)
    fail = ctypes.c_int64(-1)
    shp = _shapes_arg(shapes, durs)
    st = lib().nu_linear_search_ss(
        ctx.ptr, ctypes.c_void_p(t_d.data_ptr()), n, ctypes.byref(kc), ctypes.c_void_p(f_d.data_ptr()),
        ctypes.c_void_p(A_d.data_ptr() if A_d is not None else 0), m1, ctypes.c_void_p(lat.data_ptr()),
        int(n_epochs), durs.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)), n_d,
        shp.ctypes.data_as(ctypes.POINTER(ctypes.c_double)) if shp is not None else None,
        ctypes.c_void_p(depth.data_ptr()),
        ctypes.c_void_p(var.data_ptr()), ctypes.c_void_p(dll.data_ptr()), ctypes.c_void_p(valid.data_ptr()),
        ctypes.c_void_p(null.data_ptr()), ctypes.byref(fail) if check else None)
    if st != NU_OK:
        err = NuanceError(st, lib().nu_ctx_last_error(ctx.ptr).decode())
        err.index = fail.value
        raise err
    return {"depth": depth, "var": var, "dll": dll, "valid": valid, "null": null,
            "_keep": (t_d, f_d, A_d, lat)}


def periodic_search(ctx: Context, depth, var, dll, valid, dt: float, periods, sign: int = 1) -> dict:
    """Fold of the single-event grid over periods x phases (Eq. 8, Eq. 9)."""
    dev = ctx.device
    depth = _dev_tensor(depth, torch.float64, dev)
    var = _dev_tensor(var, torch.float64, dev)
    dll = _dev_tensor(dll, torch.float64, dev)
    valid = _dev_tensor(valid, torch.uint8, dev)
    if not (depth.shape == var.shape == dll.shape == valid.shape) or depth.ndim != 2:
        raise ValueError("depth, var, dll, valid must share one (n_d, n_epochs) shape")
    per = _dev_tensor(periods, torch.float64, dev)
    n_d, n_t = depth.shape
    n_p = per.numel()
    out = {
        "q_snr": torch.empty(n_p, dtype=torch.float64, device=dev),
        "best_phase": torch.empty(n_p, dtype=torch.int64, device=dev),
        "best_dur": torch.empty(n_p, dtype=torch.int32, device=dev),
        "best_depth": torch.empty(n_p, dtype=torch.float64, device=dev),
        "best_sigma": torch.empty(n_p, dtype=torch.float64, device=dev),
        "best_lnp": torch.empty(n_p, dtype=torch.float64, device=dev),
        "best_index": torch.empty(1, dtype=torch.int64, device=dev),
    }
    st = lib().nu_periodic_search(
        ctx.ptr, ctypes.c_void_p(depth.data_ptr()), ctypes.c_void_p(var.data_ptr()),
        ctypes.c_void_p(dll.data_ptr()), ctypes.c_void_p(valid.data_ptr()), n_d, n_t, float(dt),
        ctypes.c_void_p(per.data_ptr()), n_p, int(sign),
        *[ctypes.c_void_p(out[k].data_ptr()) for k in ("q_snr", "best_phase", "best_dur", "best_depth",
                                                       "best_sigma", "best_lnp", "best_index")])
    _check(ctx.ptr, st)
    out["_keep"] = (depth, var, dll, valid, per)
    return out


def periodic_search_segments(ctx: Context, grids, offsets, dt: float, periods, sign: int = 1) -> dict:
    """Fold over segments of one light curve, each with its own linear search (entry point 3c).

    grids: a list of per-segment linear-search outputs (dicts with depth, var, dll, valid of shape
    (n_d, n_s)); offsets: the global lattice slot of each segment's first slot (ascending, at least 64
    slots apart). Phases in the result are global slots."""
    dev = ctx.device
    if len(grids) < 1:
        raise ValueError("need at least one segment")
    n_d = None
    parts = {k: [] for k in ("depth", "var", "dll", "valid")}
    lens = []
    for g in grids:
        d = _dev_tensor(g["depth"], torch.float64, dev)
        if d.ndim != 2:
            raise ValueError("segment grids must be (n_d, n_s)")
        n_d = d.shape[0] if n_d is None else n_d
        if d.shape[0] != n_d:
            raise ValueError("segments must share the durations")
        for k, t in (("depth", torch.float64), ("var", torch.float64), ("dll", torch.float64), ("valid", torch.uint8)):
            x = _dev_tensor(g[k], t, dev)
            if tuple(x.shape) != tuple(d.shape):
                raise ValueError("depth, var, dll, valid must share one shape per segment")
            parts[k].append(x.reshape(-1))
        lens.append(d.shape[1])
    cat = {k: torch.cat(v).contiguous() for k, v in parts.items()}
    lens_h = np.ascontiguousarray(lens, dtype=np.int64)
    offs_h = np.ascontiguousarray([int(o) for o in offsets], dtype=np.int64)
    if offs_h.size != lens_h.size:
        raise ValueError("one offset per segment")
    per = _dev_tensor(periods, torch.float64, dev)
    n_p = per.numel()
    out = {
        "q_snr": torch.empty(n_p, dtype=torch.float64, device=dev),
        "best_phase": torch.empty(n_p, dtype=torch.int64, device=dev),
        "best_dur": torch.empty(n_p, dtype=torch.int32, device=dev),
        "best_depth": torch.empty(n_p, dtype=torch.float64, device=dev),
        "best_sigma": torch.empty(n_p, dtype=torch.float64, device=dev),
        "best_lnp": torch.empty(n_p, dtype=torch.float64, device=dev),
        "best_index": torch.empty(1, dtype=torch.int64, device=dev),
    }
    P64 = ctypes.POINTER(ctypes.c_int64)
    st = lib().nu_periodic_search_segments(
        ctx.ptr, ctypes.c_void_p(cat["depth"].data_ptr()), ctypes.c_void_p(cat["var"].data_ptr()),
        ctypes.c_void_p(cat["dll"].data_ptr()), ctypes.c_void_p(cat["valid"].data_ptr()), int(n_d), len(lens),
        lens_h.ctypes.data_as(P64), offs_h.ctypes.data_as(P64), float(dt), ctypes.c_void_p(per.data_ptr()), n_p,
        int(sign), *[ctypes.c_void_p(out[k].data_ptr()) for k in ("q_snr", "best_phase", "best_dur", "best_depth",
                                                                  "best_sigma", "best_lnp", "best_index")])
    _check(ctx.ptr, st)
    out["_keep"] = (cat, per)
    return out


_PERIOD_KEYS = ("q_snr", "best_phase", "best_dur", "best_depth", "best_sigma", "best_lnp")
_PERIOD_DTYPES = (torch.float64, torch.int64, torch.int32, torch.float64, torch.float64, torch.float64)


def _trend_colmajor(A, n, dev):
    if A is None:
        return 0, None
    A_t = A if isinstance(A, torch.Tensor) else torch.as_tensor(np.asarray(A, dtype=np.float64))
    if A_t.ndim == 1:
        A_t = A_t[:, None]
    if A_t.shape[0] != n:
        raise ValueError("A must be (N, m1)")
    return int(A_t.shape[1]), A_t.to(device=dev, dtype=torch.float64).t().contiguous()


def prepare_batch(ctx: Context, curves) -> dict:
    """Concatenate a batch of light curves into device arrays (done once, outside any timing).

    curves: list of dicts with t, f, A (N x m1 or None; the same m1 for all),
    lattice (int64 slots, starting at 0), n_epochs, theta (SHO or dict) and dt.
    """
    dev = ctx.device
    nc = len(curves)
    if nc < 1:
        raise ValueError("empty batch")
    ns = [int(np.asarray(c["lattice"]).size) for c in curves]
    nes = [int(c["n_epochs"]) for c in curves]
    soff = np.zeros(nc + 1, dtype=np.int64)
    soff[1:] = np.cumsum(ns)
    eoff = np.zeros(nc + 1, dtype=np.int64)
    eoff[1:] = np.cumsum(nes)
    m1s = set()
    cols = []
    for c, n in zip(curves, ns):
        m1, Ac = _trend_colmajor(c.get("A"), n, torch.device("cpu"))
        m1s.add(m1)
        cols.append(Ac)
    if len(m1s) != 1:
        raise ValueError("every curve needs the same number of trend columns")
    m1 = m1s.pop()
    return {
        "n_curves": nc, "n_epochs": nes, "sample_off": soff, "epoch_off": eoff, "m1": m1,
        "t": _dev_tensor(np.concatenate([np.asarray(c["t"], dtype=np.float64) for c in curves]), torch.float64, dev),
        "f": _dev_tensor(np.concatenate([np.asarray(c["f"], dtype=np.float64) for c in curves]), torch.float64, dev),
        "lattice": _dev_tensor(np.concatenate([np.asarray(c["lattice"], dtype=np.int64) for c in curves]),
                               torch.int64, dev),
        "A": torch.cat([a.reshape(-1) for a in cols]).to(dev) if m1 > 0 else None,
        "theta": (NuSho * nc)(*[(c["theta"] if isinstance(c["theta"], SHO) else SHO.from_dict(c["theta"])).c()
                                for c in curves]),
        "dt": np.ascontiguousarray([float(c["dt"]) for c in curves], dtype=np.float64),
    }


def mask_transit(ctx: Context, ls: dict, dt: float, period: float, phase: int, half_width: int) -> dict:
    """Mask a found candidate's transit windows in the linear-search outputs ``ls`` in place (entry point 3b,
    Section 3.3): slots within ``half_width`` of phase + k period/dt, every duration. Returns ``ls``."""
    depth, var, dll, valid = ls["depth"], ls["var"], ls["dll"], ls["valid"]
    n_d, n_epochs = depth.shape
    for x, dt_ in ((depth, torch.float64), (var, torch.float64), (dll, torch.float64), (valid, torch.uint8)):
        if x.dtype != dt_ or not x.is_cuda or not x.is_contiguous() or tuple(x.shape) != (n_d, n_epochs):
            raise ValueError("mask_transit: ls must hold the contiguous device outputs of linear_search")
    _check(ctx.ptr, lib().nu_mask_transit(ctx.ptr, ctypes.c_void_p(depth.data_ptr()), ctypes.c_void_p(var.data_ptr()),
                                          ctypes.c_void_p(dll.data_ptr()), ctypes.c_void_p(valid.data_ptr()), n_d,
                                          n_epochs, float(dt), float(period), int(phase), int(half_width)))
    return ls


def search_planets(ctx: Context, ls: dict, dt: float, periods, durations, n_planets: int, sign: int = 1,
                   copy: bool = True) -> list:
    """Up to ``n_planets`` candidates from one linear search (Section 3.3): periodic search, mask the best
    candidate's transits (windows of width 2 D), repeat. ``durations``: the box lengths in slots passed to
    linear_search. With ``copy`` the masking works on copies of the grid, else ``ls`` is masked in place.
    One stream synchronisation per candidate (to read its period, phase and duration)."""
    if copy:
        ls = {k: ls[k].clone() for k in ("depth", "var", "dll", "valid")}
    durs = np.asarray(durations, dtype=np.int64)
    per_host = periods.cpu().numpy() if isinstance(periods, torch.Tensor) else np.asarray(periods, dtype=np.float64)
    found = []
    for _ in range(int(n_planets)):
        ps = periodic_search(ctx, ls["depth"], ls["var"], ls["dll"], ls["valid"], dt, periods, sign)
        ip = int(ps["best_index"].item())
        if ip < 0:
            break
        m = int(ps["best_phase"][ip].item())
        if m < 0:
            break
        j = int(ps["best_dur"][ip].item())
        found.append({"index": ip, "period": float(per_host[ip]), "phase": m, "dur_index": j,
                      "snr": float(ps["q_snr"][ip].item()), "depth": float(ps["best_depth"][ip].item()),
                      "lnp": float(ps["best_lnp"][ip].item())})
        mask_transit(ctx, ls, dt, float(per_host[ip]), m, int(durs[j]))
    return found


def search_batch(ctx: Context, curves, durations, periods, precision: str = "fp32_refine", sign: int = 1,
                 memory_budget: int = 0, raise_not_pd: bool = True) -> dict:
    """Linear + periodic search of a batch of light curves of uneven length (entry point 4).

    curves: a list of curve dicts (see ``prepare_batch``) or a prepared batch.
    Returns the concatenated device outputs and, per curve, views:
    ``cells[c]`` (depth, var, dll, valid shaped (n_d, n_epochs_c)) and
    ``periods[c]`` (the per-period arrays), plus host ``logdet``,
    ``fail_pivot`` and the device ``best_index`` (one per curve).
    """
    dev = ctx.device
    b = curves if isinstance(curves, dict) else prepare_batch(ctx, curves)
    nc, nes, soff, eoff = b["n_curves"], b["n_epochs"], b["sample_off"], b["epoch_off"]
    durs = np.ascontiguousarray(np.asarray(durations, dtype=np.int32))
    n_d = int(durs.size)
    per = _dev_tensor(periods, torch.float64, dev)
    n_p = per.numel()
    cells = n_d * int(eoff[-1])
    out = {k: torch.empty(cells, dtype=dt_, device=dev)
           for k, dt_ in (("depth", torch.float64), ("var", torch.float64), ("dll", torch.float64),
                          ("valid", torch.uint8))}
    out["null"] = torch.empty((nc, 3), dtype=torch.float64, device=dev)
    for k, dt_ in zip(_PERIOD_KEYS, _PERIOD_DTYPES):
        out[k] = torch.empty((nc, n_p), dtype=dt_, device=dev)
    out["best_index"] = torch.empty(nc, dtype=torch.int64, device=dev)
    logdet = np.zeros(nc, dtype=np.float64)
    pivot = np.full(nc, -1, dtype=np.int64)
    if precision not in PRECISIONS:
        raise ValueError(f"precision must be one of {sorted(PRECISIONS)}")
    P64 = ctypes.POINTER(ctypes.c_int64)
    A = b["A"]
    st = lib().nu_search_batch(
        ctx.ptr, nc, soff.ctypes.data_as(P64), eoff.ctypes.data_as(P64), ctypes.c_void_p(b["t"].data_ptr()),
        ctypes.c_void_p(b["f"].data_ptr()), ctypes.c_void_p(A.data_ptr() if A is not None else 0), b["m1"],
        ctypes.c_void_p(b["lattice"].data_ptr()), b["theta"], b["dt"].ctypes.data_as(ctypes.POINTER(ctypes.c_double)),
        durs.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)), n_d, ctypes.c_void_p(per.data_ptr()), n_p,
        PRECISIONS[precision], int(sign), int(memory_budget),
        *[ctypes.c_void_p(out[k].data_ptr()) for k in ("depth", "var", "dll", "valid", "null")],
        *[ctypes.c_void_p(out[k].data_ptr()) for k in _PERIOD_KEYS],
        ctypes.c_void_p(out["best_index"].data_ptr()),
        logdet.ctypes.data_as(ctypes.POINTER(ctypes.c_double)), pivot.ctypes.data_as(P64))
    if st != NU_OK and not (st == NU_ERR_NOT_PD and not raise_not_pd):
        _check(ctx.ptr, st)
    out["logdet"] = logdet
    out["fail_pivot"] = pivot
    out["cells"] = [{k: out[k][n_d * int(eoff[c]):n_d * int(eoff[c + 1])].view(n_d, nes[c])
                     for k in ("depth", "var", "dll", "valid")} for c in range(nc)]
    out["periods"] = [{k: out[k][c] for k in _PERIOD_KEYS} for c in range(nc)]
    out["_keep"] = (b, per)
    return out


class BatchGraph:
    """Captured graph of the batch search (entry point 4b): every stage of every wave of ``search_batch``
    recorded once; ``launch()`` replays the whole batch in one graph launch on the context's stream, with no
    synchronisation. Inputs are read from the prepared batch's device arrays and ``theta`` (device, one SHO per
    curve; ``set_theta`` rewrites it); ``status`` receives -1 or the failing pivot per curve, ``logdet`` ln|K|.
    Outputs as in ``search_batch``."""

    def __init__(self, ctx: Context, curves, durations, periods, precision: str = "fp32_refine", sign: int = 1,
                 memory_budget: int = 0):
        dev = ctx.device
        self.ctx = ctx
        b = curves if isinstance(curves, dict) else prepare_batch(ctx, curves)
        self.batch = b
        nc, nes, soff, eoff = b["n_curves"], b["n_epochs"], b["sample_off"], b["epoch_off"]
        self.durs = np.ascontiguousarray(np.asarray(durations, dtype=np.int32))
        n_d = int(self.durs.size)
        self.per = _dev_tensor(periods, torch.float64, dev)
        n_p = self.per.numel()
        cells = n_d * int(eoff[-1])
        out = {k: torch.empty(cells, dtype=dt_, device=dev)
               for k, dt_ in (("depth", torch.float64), ("var", torch.float64), ("dll", torch.float64),
                              ("valid", torch.uint8))}
        out["null"] = torch.empty((nc, 3), dtype=torch.float64, device=dev)
        for k, dt_ in zip(_PERIOD_KEYS, _PERIOD_DTYPES):
            out[k] = torch.empty((nc, n_p), dtype=dt_, device=dev)
        out["best_index"] = torch.empty(nc, dtype=torch.int64, device=dev)
        self.status = torch.empty(nc, dtype=torch.int64, device=dev)
        self.logdet = torch.empty(nc, dtype=torch.float64, device=dev)
        self.theta = torch.empty((nc, 4), dtype=torch.float64, device=dev)
        self.theta.copy_(torch.tensor([[t.amp, t.omega, t.q, t.sigma_w] for t in b["theta"]], dtype=torch.float64))
        if precision not in PRECISIONS:
            raise ValueError(f"precision must be one of {sorted(PRECISIONS)}")
        P64 = ctypes.POINTER(ctypes.c_int64)
        A = b["A"]
        p = ctypes.c_void_p()
        st = lib().nu_batch_graph_create(
            ctx.ptr, nc, soff.ctypes.data_as(P64), eoff.ctypes.data_as(P64), ctypes.c_void_p(b["t"].data_ptr()),
            ctypes.c_void_p(b["f"].data_ptr()), ctypes.c_void_p(A.data_ptr() if A is not None else 0), b["m1"],
            ctypes.c_void_p(b["lattice"].data_ptr()), ctypes.c_void_p(self.theta.data_ptr()),
            b["dt"].ctypes.data_as(ctypes.POINTER(ctypes.c_double)),
            self.durs.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)), n_d, ctypes.c_void_p(self.per.data_ptr()), n_p,
            PRECISIONS[precision], int(sign), int(memory_budget),
            *[ctypes.c_void_p(out[k].data_ptr()) for k in ("depth", "var", "dll", "valid", "null")],
            *[ctypes.c_void_p(out[k].data_ptr()) for k in _PERIOD_KEYS],
            ctypes.c_void_p(out["best_index"].data_ptr()), ctypes.c_void_p(self.status.data_ptr()),
            ctypes.c_void_p(self.logdet.data_ptr()), ctypes.byref(p))
        _check(ctx.ptr, st)
        self.ptr = p
        _register(self, 0)
        out["cells"] = [{k: out[k][n_d * int(eoff[c]):n_d * int(eoff[c + 1])].view(n_d, nes[c])
                         for k in ("depth", "var", "dll", "valid")} for c in range(nc)]
        out["periods"] = [{k: out[k][c] for k in _PERIOD_KEYS} for c in range(nc)]
        self.out = out

    def set_theta(self, thetas):
        """Rewrite the per-curve hyperparameters the next launch reads (stream-ordered copy)."""
        rows = [t if isinstance(t, SHO) else SHO.from_dict(t) for t in thetas]
        self.theta.copy_(torch.tensor([[t.amp, t.omega, t.q, t.sigma_w] for t in rows], dtype=torch.float64))

    def launch(self) -> dict:
        _check(self.ctx.ptr, lib().nu_batch_graph_launch(self.ctx.ptr, self.ptr))
        return self.out

    def close(self):
        if getattr(self, "ptr", None):
            lib().nu_batch_graph_destroy(self.ptr)
            self.ptr = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Graph:
    """Captured graph of the whole search of one light curve (entry point 5).

    The graph is bound to device buffers owned by this object: write new
    inputs with ``set_inputs`` (same shapes) and ``launch()`` replays factor,
    inverse, linear and periodic search on the context's stream without any
    synchronisation; ``status`` holds -1 or the failing pivot of the launch.
    """

    def __init__(self, ctx: Context, t, f, A, lattice, n_epochs: int, durations, theta, dt: float, periods,
                 precision: str = "fp64", sign: int = 1):
        dev = ctx.device
        self.ctx = ctx
        self.t = _dev_tensor(t, torch.float64, dev)
        n = self.t.numel()
        self.f = _dev_tensor(f, torch.float64, dev)
        self.m1, self.A = _trend_colmajor(A, n, dev)
        self.lattice = _dev_tensor(lattice, torch.int64, dev)
        self.periods = _dev_tensor(periods, torch.float64, dev)
        self.theta = torch.empty(4, dtype=torch.float64, device=dev)
        self.status = torch.empty(1, dtype=torch.int64, device=dev)
        self.set_inputs(theta=theta)
        self.durs = np.ascontiguousarray(np.asarray(durations, dtype=np.int32))
        n_d = int(self.durs.size)
        shape = (n_d, int(n_epochs))
        self.out = {"depth": torch.empty(shape, dtype=torch.float64, device=dev),
                    "var": torch.empty(shape, dtype=torch.float64, device=dev),
                    "dll": torch.empty(shape, dtype=torch.float64, device=dev),
                    "valid": torch.empty(shape, dtype=torch.uint8, device=dev),
                    "null": torch.empty(3, dtype=torch.float64, device=dev),
                    "best_index": torch.empty(1, dtype=torch.int64, device=dev)}
        n_p = self.periods.numel()
        for k, dt_ in zip(_PERIOD_KEYS, _PERIOD_DTYPES):
            self.out[k] = torch.empty(n_p, dtype=dt_, device=dev)
        p = ctypes.c_void_p()
        st = lib().nu_graph_create(
            ctx.ptr, ctypes.c_void_p(self.t.data_ptr()), n, ctypes.c_void_p(self.theta.data_ptr()),
            ctypes.c_void_p(self.f.data_ptr()), ctypes.c_void_p(self.A.data_ptr() if self.A is not None else 0),
            self.m1, ctypes.c_void_p(self.lattice.data_ptr()), int(n_epochs),
            self.durs.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)), n_d, PRECISIONS[precision], float(dt),
            ctypes.c_void_p(self.periods.data_ptr()), n_p, int(sign),
            *[ctypes.c_void_p(self.out[k].data_ptr()) for k in ("depth", "var", "dll", "valid", "null")],
            *[ctypes.c_void_p(self.out[k].data_ptr()) for k in _PERIOD_KEYS],
            ctypes.c_void_p(self.out["best_index"].data_ptr()), ctypes.c_void_p(self.status.data_ptr()),
            ctypes.byref(p))
        _check(ctx.ptr, st)
        self.ptr = p
        _register(self, 0)

    def set_inputs(self, theta=None, f=None, A=None, t=None):
        """Overwrite bound inputs in place (stream-ordered copies)."""
        if theta is not None:
            sho = theta if isinstance(theta, SHO) else SHO.from_dict(theta)
            self.theta.copy_(torch.tensor([sho.amp, sho.omega, sho.q, sho.sigma_w], dtype=torch.float64))
        if f is not None:
            self.f.copy_(_dev_tensor(f, torch.float64, self.f.device))
        if A is not None:
            m1, Ac = _trend_colmajor(A, self.t.numel(), self.t.device)
            if m1 != self.m1:
                raise ValueError("A must keep its shape")
            self.A.copy_(Ac)
        if t is not None:
            self.t.copy_(_dev_tensor(t, torch.float64, self.t.device))

    def launch(self) -> dict:
        _check(self.ctx.ptr, lib().nu_graph_launch(self.ctx.ptr, self.ptr))
        return self.out

    def close(self):
        if getattr(self, "ptr", None):
            lib().nu_graph_destroy(self.ptr)
            self.ptr = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


# ---------------------------------------------------------------------------
# The hyperparameter fit and its learned warm start (entry point 7)

PRIOR = {"amp": (0.005, 0.03), "prot": (0.3, 2.0), "q": (1.0, 100.0), "sigma_w": (3e-4, 3e-3)}


def _sho_rows(thetas, dev) -> torch.Tensor:
    """(k, 4) float64 device rows (amp, omega, q, sigma_w) = k nu_sho structs."""
    if isinstance(thetas, torch.Tensor):
        return thetas.to(device=dev, dtype=torch.float64).reshape(-1, 4).contiguous()
    rows = []
    for th in thetas:
        sho = th if isinstance(th, SHO) else SHO.from_dict(th)
        rows.append([sho.amp, sho.omega, sho.q, sho.sigma_w])
    return torch.tensor(rows, dtype=torch.float64, device=dev)


def gp_sample(ctx: Context, t, n_curves: int, theta=None, seed: int = 0, curve_base: int = 0, n_bins: int = 512,
              flux: bool = False, inputs: bool = True) -> dict:
    """Curves from the SHO process + white noise (7a): theta None draws from the training prior."""
    dev = ctx.device
    t_d = _dev_tensor(t, torch.float64, dev)
    n = t_d.numel()
    th = None if theta is None else _sho_rows(theta, dev)
    out = {"theta": torch.empty((n_curves, 4), dtype=torch.float64, device=dev),
           "target": torch.empty((n_curves, 4), dtype=torch.float32, device=dev)}
    if flux:
        out["flux"] = torch.empty((n_curves, n), dtype=torch.float64, device=dev)
    if inputs:
        out["input"] = torch.empty((n_curves, n_bins), dtype=torch.float32, device=dev)

    def ptr(k):
        return ctypes.c_void_p(out[k].data_ptr()) if k in out else ctypes.c_void_p(0)

    st = lib().nu_gp_sample(ctx.ptr, ctypes.c_void_p(t_d.data_ptr()), n, int(n_curves),
                            ctypes.c_void_p(th.data_ptr() if th is not None else 0), int(seed), int(curve_base),
                            int(n_bins), ptr("flux"), ptr("input"), ptr("target"), ptr("theta"))
    _check(ctx.ptr, st)
    out["_keep"] = (t_d, th)
    return out


def gp_nll(ctx: Context, batch: dict, thetas, n_eval: int = 1) -> torch.Tensor:
    """-ln L_0 (7b) of curve c at thetas[c * n_eval + e]; batch from ``prepare_batch``."""
    dev = ctx.device
    th = _sho_rows(thetas, dev)
    nc = batch["n_curves"]
    if th.shape[0] != nc * n_eval:
        raise ValueError("need n_curves * n_eval thetas")
    off = torch.as_tensor(batch["sample_off"], device=dev)
    nll = torch.empty((nc, n_eval), dtype=torch.float64, device=dev)
    A = batch["A"]
    st = lib().nu_gp_nll(ctx.ptr, nc, ctypes.c_void_p(off.data_ptr()), ctypes.c_void_p(batch["t"].data_ptr()),
                         ctypes.c_void_p(batch["f"].data_ptr()), ctypes.c_void_p(A.data_ptr() if A is not None else 0),
                         batch["m1"], ctypes.c_void_p(th.data_ptr()), int(n_eval), ctypes.c_void_p(nll.data_ptr()))
    _check(ctx.ptr, st)
    torch.cuda.synchronize(dev)
    return nll


def plain_init(ctx: Context, batch: dict, prot_grid) -> torch.Tensor:
    """The plain start (7c): (n_curves, 4) fit coordinates ln(amp, P_rot, Q, sigma_w)."""
    dev = ctx.device
    grid = _dev_tensor(prot_grid, torch.float64, dev)
    off = torch.as_tensor(batch["sample_off"], device=dev)
    x0 = torch.empty((batch["n_curves"], 4), dtype=torch.float64, device=dev)
    st = lib().nu_plain_init(ctx.ptr, batch["n_curves"], ctypes.c_void_p(off.data_ptr()),
                             ctypes.c_void_p(batch["t"].data_ptr()), ctypes.c_void_p(batch["f"].data_ptr()),
                             ctypes.c_void_p(grid.data_ptr()), grid.numel(), ctypes.c_void_p(x0.data_ptr()))
    _check(ctx.ptr, st)
    torch.cuda.synchronize(dev)
    return x0


def fit_hyper(ctx: Context, batch: dict, x0, max_iter: int = 100, gtol: float = 1e-2) -> dict:
    """BFGS maximum-likelihood fit (7d) from x0 (n_curves, 4) in fit coordinates."""
    nc = batch["n_curves"]
    x0h = np.ascontiguousarray(x0.cpu().numpy() if isinstance(x0, torch.Tensor) else np.asarray(x0),
                               dtype=np.float64).reshape(nc, 4)
    x = np.zeros((nc, 4))
    nll = np.zeros(nc)
    nev = np.zeros(nc, dtype=np.int32)
    its = np.zeros(nc, dtype=np.int32)
    A = batch["A"]
    PD = ctypes.POINTER(ctypes.c_double)
    PI = ctypes.POINTER(ctypes.c_int32)
    st = lib().nu_fit_hyper(ctx.ptr, nc, batch["sample_off"].ctypes.data_as(ctypes.POINTER(ctypes.c_int64)),
                            ctypes.c_void_p(batch["t"].data_ptr()), ctypes.c_void_p(batch["f"].data_ptr()),
                            ctypes.c_void_p(A.data_ptr() if A is not None else 0), batch["m1"],
                            x0h.ctypes.data_as(PD), int(max_iter), float(gtol), x.ctypes.data_as(PD),
                            nll.ctypes.data_as(PD), nev.ctypes.data_as(PI), its.ctypes.data_as(PI))
    _check(ctx.ptr, st)
    return {"x": x, "nll": nll, "n_eval": nev, "iters": its}


class CNN:
    """The warm-start network (7e) with its parameters, Adam state and activations on the device."""

    def __init__(self, ctx: Context, half: bool = True, max_batch: int = 256, params=None, seed: int = 0):
        self.ctx = ctx
        self.max_batch = max_batch
        p = ctypes.c_void_p()
        _check(ctx.ptr, lib().nu_cnn_create(ctx.ptr, int(half), int(max_batch), ctypes.byref(p)))
        self.ptr = p
        _register(self, 0)
        self.n_params = int(lib().nu_cnn_param_count())
        if params is not None:
            self.set_params(params)
        else:
            _check(ctx.ptr, lib().nu_cnn_init(ctx.ptr, self.ptr, int(seed)))

    def set_params(self, params):
        a = np.ascontiguousarray(np.asarray(params, dtype=np.float32))
        if a.size != self.n_params:
            raise ValueError(f"need {self.n_params} parameters")
        _check(self.ctx.ptr, lib().nu_cnn_set_params(self.ctx.ptr, self.ptr,
                                                     a.ctypes.data_as(ctypes.POINTER(ctypes.c_float))))

    def get_params(self) -> np.ndarray:
        a = np.empty(self.n_params, dtype=np.float32)
        _check(self.ctx.ptr, lib().nu_cnn_get_params(self.ctx.ptr, self.ptr,
                                                     a.ctypes.data_as(ctypes.POINTER(ctypes.c_float))))
        return a

    def forward(self, inputs: torch.Tensor):
        """Outputs (batch, 4) standardised, and the same in fit coordinates (float64)."""
        b = inputs.shape[0]
        out = torch.empty((b, 4), dtype=torch.float32, device=self.ctx.device)
        xlog = torch.empty((b, 4), dtype=torch.float64, device=self.ctx.device)
        _check(self.ctx.ptr, lib().nu_cnn_forward(self.ctx.ptr, self.ptr, ctypes.c_void_p(inputs.data_ptr()), b,
                                                  ctypes.c_void_p(out.data_ptr()), ctypes.c_void_p(xlog.data_ptr())))
        return out, xlog

    def warm_start(self, inputs: torch.Tensor, x_plain: torch.Tensor) -> torch.Tensor:
        """Fit coordinates (batch, 4): the network's amp, P_rot, Q and the plain start's sigma_w (7f)."""
        b = inputs.shape[0]
        x = torch.empty((b, 4), dtype=torch.float64, device=self.ctx.device)
        xp = x_plain.to(device=self.ctx.device, dtype=torch.float64).contiguous()
        _check(self.ctx.ptr, lib().nu_warm_start(self.ctx.ptr, self.ptr, ctypes.c_void_p(inputs.data_ptr()), b,
                                                 ctypes.c_void_p(xp.data_ptr()), ctypes.c_void_p(x.data_ptr())))
        return x

    def gradient(self, inputs: torch.Tensor, targets: torch.Tensor):
        b = inputs.shape[0]
        g = torch.empty(self.n_params, dtype=torch.float32, device=self.ctx.device)
        loss = torch.empty(1, dtype=torch.float32, device=self.ctx.device)
        _check(self.ctx.ptr, lib().nu_cnn_gradient(self.ctx.ptr, self.ptr, ctypes.c_void_p(inputs.data_ptr()),
                                                   ctypes.c_void_p(targets.data_ptr()), b,
                                                   ctypes.c_void_p(g.data_ptr()), ctypes.c_void_p(loss.data_ptr())))
        return g, loss

    def train_step(self, inputs: torch.Tensor, targets: torch.Tensor, lr: float = 1e-3, loss=None):
        b = inputs.shape[0]
        _check(self.ctx.ptr, lib().nu_cnn_train_step(self.ctx.ptr, self.ptr, ctypes.c_void_p(inputs.data_ptr()),
                                                     ctypes.c_void_p(targets.data_ptr()), b, float(lr),
                                                     ctypes.c_void_p(loss.data_ptr() if loss is not None else 0)))

    def close(self):
        if getattr(self, "ptr", None):
            lib().nu_cnn_destroy(self.ptr)
            self.ptr = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


# ---------------------------------------------------------------------------
class SearchResult:
    """Periodogram and best candidate of a periodic search (host arrays)."""

    def __init__(self, periods, raw: dict, t_first: float, dt: float, durations_slots):
        self.periods = np.asarray(periods, dtype=np.float64)
        self.Q_snr = raw["q_snr"].cpu().numpy()
        self.best_phase = raw["best_phase"].cpu().numpy()
        self.best_dur = raw["best_dur"].cpu().numpy()
        self.depth = raw["best_depth"].cpu().numpy()
        self.sigma = raw["best_sigma"].cpu().numpy()
        self.lnp = raw["best_lnp"].cpu().numpy()
        i = int(raw["best_index"].cpu().item())
        self.best_index = i
        if i >= 0:
            j = int(self.best_dur[i])
            self.best = (float(self.periods[i]), t_first + float(self.best_phase[i]) * dt,
                         float(durations_slots[j]) * dt, float(self.depth[i]), float(self.sigma[i]))
        else:
            self.best = None


class Nuance:
    """The paper's search object: ``Nuance(time, flux, gp=SHO(...), X=X)``.

    ``time`` must sit on a regular lattice of cadence ``dt`` (gaps allowed);
    epochs are all lattice slots from the first to the last sample. ``gp`` is
    an SHO (or its dict) or a sum-of-terms Kernel. ``solver="statespace"``
    runs the linear search from the state-space form of the covariance (no
    dense factor is formed); ``"dense"`` factors K.
    """

    def __init__(self, time, flux, gp, X=None, dt: Optional[float] = None, device: int = 0,
                 solver: str = "dense"):
        if solver not in ("dense", "statespace"):
            raise ValueError("solver must be 'dense' or 'statespace'")
        t = np.asarray(time, dtype=np.float64)
        if t.ndim != 1 or t.size < 2 or not np.all(np.diff(t) > 0):
            raise ValueError("time must be strictly increasing with at least two samples")
        self.dt = float(np.min(np.diff(t))) if dt is None else float(dt)
        lat = np.rint((t - t[0]) / self.dt).astype(np.int64)
        if np.max(np.abs(t - t[0] - lat * self.dt)) > 1e-6 * self.dt or np.any(np.diff(lat) <= 0):
            raise ValueError("time is not on a regular lattice of cadence dt")
        self.t_first = float(t[0])
        self.lattice = lat
        self.n_epochs = int(lat[-1]) + 1
        self.flux = np.asarray(flux, dtype=np.float64)
        self.X = None if X is None else np.asarray(X, dtype=np.float64)
        self.ctx = Context(device)
        self.solver = solver
        self.gp = gp
        self.time = t
        self.factor = gp_factor(self.ctx, t, gp) if solver == "dense" else None
        self._ls = None
        self._dur_slots = None

    def linear_search(self, t0s=None, Ds=(0.04,), precision: str = "fp64", template=None) -> dict:
        """Single-event fits on every epoch slot for the durations ``Ds`` (time units). ``template``: None for
        boxes, or a function of the window length in slots returning the shape (one value per slot)."""
        if t0s is not None and np.asarray(t0s).size not in (self.lattice.size, self.n_epochs):
            raise ValueError("epochs are the lattice slots of the time array")
        slots = np.rint(np.asarray(Ds, dtype=np.float64) / self.dt).astype(np.int32)
        if np.any(slots < 1):
            raise ValueError("durations must be at least one cadence")
        self._dur_slots = slots
        shapes = None if template is None else [np.asarray(template(int(d)), dtype=np.float64) for d in slots]
        if self.solver == "statespace":
            self._ls = linear_search_ss(self.ctx, self.time, self.gp, self.flux, self.X, self.lattice,
                                        self.n_epochs, slots, shapes=shapes)
        else:
            self._ls = linear_search(self.ctx, self.factor, self.flux, self.X, self.lattice, self.n_epochs, slots,
                                     precision, shapes=shapes)
        return self._ls

    def periodic_search(self, periods, sign: int = 1) -> SearchResult:
        if self._ls is None:
            raise RuntimeError("run linear_search first")
        periods = np.asarray(periods, dtype=np.float64)
        if np.any(~np.isfinite(periods)) or np.any(periods < self.dt):
            raise ValueError("periods must be finite and at least one cadence")
        ls = self._ls
        raw = periodic_search(self.ctx, ls["depth"], ls["var"], ls["dll"], ls["valid"], self.dt, periods, sign)
        return SearchResult(periods, raw, self.t_first, self.dt, self._dur_slots)

    def search_planets(self, periods, n_planets: int = 2, sign: int = 1) -> list:
        """Several candidates from the one linear search (Section 3.3): each periodic search is followed by
        masking the found transits (windows of width 2 D) in copies of the linear-search products.
        Returns (period, t0, duration, depth, snr) per candidate."""
        if self._ls is None:
            raise RuntimeError("run linear_search first")
        periods = np.asarray(periods, dtype=np.float64)
        if np.any(~np.isfinite(periods)) or np.any(periods < self.dt):
            raise ValueError("periods must be finite and at least one cadence")
        found = search_planets(self.ctx, self._ls, self.dt, periods, self._dur_slots, n_planets, sign)
        return [(c["period"], self.t_first + c["phase"] * self.dt, float(self._dur_slots[c["dur_index"]]) * self.dt,
                 c["depth"], c["snr"]) for c in found]
