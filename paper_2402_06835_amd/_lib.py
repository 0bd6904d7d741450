"""ctypes declarations of the C ABI in include/nuance_mi355x.h.

The shared library is built in-tree by ``paper_2402_06835_amd.build``. There
is no fallback: if the library is missing or fails to load, every call
raises.
"""
from __future__ import annotations

import ctypes
import os

LIB_PATH = os.path.join(os.path.dirname(os.path.abspath(__file__)), "libnuance_mi355x.so")

c_int, c_int32, c_int64, c_double, c_void_p, c_char_p, c_size_t = (
    ctypes.c_int, ctypes.c_int32, ctypes.c_int64, ctypes.c_double, ctypes.c_void_p, ctypes.c_char_p,
    ctypes.c_size_t)
P = ctypes.POINTER

NU_OK, NU_ERR_ARG, NU_ERR_NOT_PD, NU_ERR_OOM, NU_ERR_DEVICE, NU_ERR_UNSUPPORTED = range(6)
STATUS_NAMES = {0: "NU_OK", 1: "NU_ERR_ARG", 2: "NU_ERR_NOT_PD", 3: "NU_ERR_OOM", 4: "NU_ERR_DEVICE",
                5: "NU_ERR_UNSUPPORTED"}
PRECISIONS = {"fp64": 0, "fp32_refine": 1, "bf16x3_refine": 2}


class NuSho(ctypes.Structure):
    _fields_ = [("amp", c_double), ("omega", c_double), ("q", c_double), ("sigma_w", c_double)]


class NuKernel(ctypes.Structure):
    _fields_ = [("n_sho", c_int32), ("n_exp", c_int32), ("sho_amp", c_double * 4), ("sho_omega", c_double * 4),
                ("sho_q", c_double * 4), ("exp_sigma", c_double * 4), ("exp_ell", c_double * 4),
                ("sigma_w", c_double)]


# name -> (restype, argtypes)
SIGNATURES = {
    "nu_rotation_kernel": (c_int, [c_double] * 10 + [P(NuKernel)]),
    "nu_ctx_create": (c_int, [c_int, c_void_p, c_size_t, P(c_void_p)]),
    "nu_ctx_device_bytes": (c_size_t, [c_void_p]),
    "nu_ctx_destroy": (None, [c_void_p]),
    "nu_ctx_set_stream": (c_int, [c_void_p, c_void_p]),
    "nu_ctx_release_memory": (c_int, [c_void_p]),
    "nu_ctx_set_inverse_prefetch": (c_int, [c_void_p, c_int, c_int]),
    "nu_ctx_last_error": (c_char_p, [c_void_p]),
    "nu_ctx_enable_timing": (c_int, [c_void_p, c_int]),
    "nu_ctx_set_timing_filter": (c_int, [c_void_p, c_char_p]),
    "nu_ctx_timing_reset": (c_int, [c_void_p]),
    "nu_ctx_timing_count": (c_int, [c_void_p]),
    "nu_ctx_timing_entry": (c_int, [c_void_p, c_int, P(c_char_p), P(c_int64), P(c_double), P(c_double)]),
    "nu_gp_factor": (c_int, [c_void_p, c_void_p, c_int64, P(NuSho), P(c_void_p), P(c_double), P(c_int64)]),
    "nu_gp_factor_kernel": (c_int, [c_void_p, c_void_p, c_int64, P(NuKernel), P(c_void_p), P(c_double), P(c_int64)]),
    "nu_gp_factor_into": (c_int, [c_void_p, c_void_p, c_void_p, c_int64, P(NuSho), P(c_double), P(c_int64)]),
    "nu_factor_destroy": (None, [c_void_p]),
    "nu_factor_n": (c_int64, [c_void_p]),
    "nu_linear_search": (c_int, [c_void_p, c_void_p, c_void_p, c_void_p, c_int, c_void_p, c_int64, P(c_int32), c_int,
                                 c_int, c_void_p, c_void_p, c_void_p, c_void_p, c_void_p]),
    "nu_linear_search_ss": (c_int, [c_void_p, c_void_p, c_int64, P(NuKernel), c_void_p, c_void_p, c_int, c_void_p,
                                    c_int64, P(c_int32), c_int, P(c_double), c_void_p, c_void_p, c_void_p, c_void_p,
                                    c_void_p, P(c_int64)]),
    "nu_linear_search_template": (c_int, [c_void_p, c_void_p, c_void_p, c_void_p, c_int, c_void_p, c_int64,
                                          P(c_int32), c_int, P(c_double), c_int, c_void_p, c_void_p, c_void_p,
                                          c_void_p, c_void_p]),
    "nu_periodic_search": (c_int, [c_void_p, c_void_p, c_void_p, c_void_p, c_void_p, c_int, c_int64, c_double,
                                   c_void_p, c_int64, c_int, c_void_p, c_void_p, c_void_p, c_void_p, c_void_p,
                                   c_void_p, c_void_p]),
    "nu_periodic_search_noalloc": (c_int, [c_void_p, c_void_p, c_void_p, c_void_p, c_void_p, c_int, c_int64,
                                           c_double, c_void_p, c_int64, c_int, c_void_p, c_void_p, c_void_p,
                                           c_void_p, c_void_p, c_void_p, c_void_p]),
    "nu_periodic_search_segments": (c_int, [c_void_p, c_void_p, c_void_p, c_void_p, c_void_p, c_int, c_int,
                                            P(c_int64), P(c_int64), c_double, c_void_p, c_int64, c_int, c_void_p,
                                            c_void_p, c_void_p, c_void_p, c_void_p, c_void_p, c_void_p]),
    "nu_mask_transit": (c_int, [c_void_p, c_void_p, c_void_p, c_void_p, c_void_p, c_int, c_int64, c_double,
                                c_double, c_int64, c_int]),
    "nu_search_batch": (c_int, [c_void_p, c_int, P(c_int64), P(c_int64), c_void_p, c_void_p, c_void_p, c_int,
                                c_void_p, P(NuSho), P(c_double), P(c_int32), c_int, c_void_p, c_int64, c_int, c_int,
                                ctypes.c_size_t, c_void_p, c_void_p, c_void_p, c_void_p, c_void_p, c_void_p,
                                c_void_p, c_void_p, c_void_p, c_void_p, c_void_p, c_void_p, P(c_double),
                                P(c_int64)]),
    "nu_batch_graph_create": (c_int, [c_void_p, c_int, P(c_int64), P(c_int64), c_void_p, c_void_p, c_void_p, c_int,
                                      c_void_p, c_void_p, P(c_double), P(c_int32), c_int, c_void_p, c_int64, c_int,
                                      c_int, ctypes.c_size_t, c_void_p, c_void_p, c_void_p, c_void_p, c_void_p,
                                      c_void_p, c_void_p, c_void_p, c_void_p, c_void_p, c_void_p, c_void_p, c_void_p,
                                      c_void_p, P(c_void_p)]),
    "nu_batch_graph_launch": (c_int, [c_void_p, c_void_p]),
    "nu_batch_graph_destroy": (None, [c_void_p]),
    "nu_graph_create": (c_int, [c_void_p, c_void_p, c_int64, c_void_p, c_void_p, c_void_p, c_int, c_void_p,
                                c_int64, P(c_int32), c_int, c_int, c_double, c_void_p, c_int64, c_int, c_void_p,
                                c_void_p, c_void_p, c_void_p, c_void_p, c_void_p, c_void_p, c_void_p, c_void_p,
                                c_void_p, c_void_p, c_void_p, c_void_p, P(c_void_p)]),
    "nu_graph_launch": (c_int, [c_void_p, c_void_p]),
    "nu_graph_destroy": (None, [c_void_p]),
    "nu_ctx_autotune": (c_int, [c_void_p, c_int64, c_int]),
    "nu_ctx_get_tuning": (c_int, [c_void_p, c_int, P(c_int)]),
    "nu_ctx_set_tuning": (c_int, [c_void_p, c_int, c_int]),
    "nu_gp_sample": (c_int, [c_void_p, c_void_p, c_int64, c_int, c_void_p, ctypes.c_uint64, ctypes.c_uint64, c_int,
                             c_void_p, c_void_p, c_void_p, c_void_p]),
    "nu_gp_nll": (c_int, [c_void_p, c_int, c_void_p, c_void_p, c_void_p, c_void_p, c_int, c_void_p, c_int, c_void_p]),
    "nu_plain_init": (c_int, [c_void_p, c_int, c_void_p, c_void_p, c_void_p, c_void_p, c_int, c_void_p]),
    "nu_fit_hyper": (c_int, [c_void_p, c_int, P(c_int64), c_void_p, c_void_p, c_void_p, c_int, P(c_double), c_int,
                             c_double, P(c_double), P(c_double), P(c_int32), P(c_int32)]),
    "nu_cnn_param_count": (c_int64, []),
    "nu_cnn_create": (c_int, [c_void_p, c_int, c_int, P(c_void_p)]),
    "nu_cnn_destroy": (None, [c_void_p]),
    "nu_cnn_set_params": (c_int, [c_void_p, c_void_p, P(ctypes.c_float)]),
    "nu_cnn_get_params": (c_int, [c_void_p, c_void_p, P(ctypes.c_float)]),
    "nu_cnn_init": (c_int, [c_void_p, c_void_p, ctypes.c_uint64]),
    "nu_cnn_forward": (c_int, [c_void_p, c_void_p, c_void_p, c_int, c_void_p, c_void_p]),
    "nu_warm_start": (c_int, [c_void_p, c_void_p, c_void_p, c_int, c_void_p, c_void_p]),
    "nu_cnn_gradient": (c_int, [c_void_p, c_void_p, c_void_p, c_void_p, c_int, c_void_p, c_void_p]),
    "nu_cnn_train_step": (c_int, [c_void_p, c_void_p, c_void_p, c_void_p, c_int, ctypes.c_float, c_void_p]),
}

# launch classes of the tile policy (include/nuance_mi355x.h, entry point 6)
TUNE_CLASSES = ("panel", "panel_update", "trailing", "inverse_fp64", "inverse_fp32", "band", "inverse_bf16x3")

_LIB = None


class NuanceError(RuntimeError):
    def __init__(self, status: int, message: str):
        super().__init__(f"{STATUS_NAMES.get(status, status)}: {message}")
        self.status = status


def lib() -> ctypes.CDLL:
    """Load the HIP library (once). Raises if it is not built."""
    global _LIB
    if _LIB is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"HIP library not built: {LIB_PATH} is missing "
                               "(run python -m paper_2402_06835_amd.build)")
        L = ctypes.CDLL(LIB_PATH)
        for name, (res, args) in SIGNATURES.items():
            fn = getattr(L, name)
            fn.restype = res
            fn.argtypes = args
        _LIB = L
    return _LIB
