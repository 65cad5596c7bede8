"""ctypes binding of ``libsfseg.so`` (declared in include/sfseg.h).

Argument marshalling only: every step of the power iteration runs in the
library's gfx950 kernels.  PyTorch supplies device memory and streams.  The
binding fails loudly when the library is missing -- there is no fallback.
"""
from __future__ import annotations

import ctypes
import os
from typing import Optional

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libsfseg.so")

SFSEG_OK = 0
SFSEG_ERR_INVALID_ARG = -1
SFSEG_ERR_OOM = -2
SFSEG_ERR_HIP = -3
SFSEG_ERR_ZERO_NORM = -4
SFSEG_ERR_NONFINITE = -5
SFSEG_ERR_STATE = -6
SFSEG_ERR_UNSUPPORTED = -7

SFSEG_F32, SFSEG_BF16, SFSEG_F16 = 0, 1, 2
DTYPES = {"f32": SFSEG_F32, "bf16": SFSEG_BF16, "f16": SFSEG_F16}
MAX_RS, MAX_RT, MAX_FEATURES = 8, 4, 2


class Config(ctypes.Structure):
    _fields_ = [("T", ctypes.c_int32), ("H", ctypes.c_int32), ("W", ctypes.c_int32),
                ("r_t", ctypes.c_int32), ("r_s", ctypes.c_int32), ("storage", ctypes.c_int32),
                ("sigma_t", ctypes.c_double), ("sigma_s", ctypes.c_double),
                ("alpha", ctypes.c_double), ("p", ctypes.c_double)]


class Result(ctypes.Structure):
    _fields_ = [("iters", ctypes.c_int32), ("converged", ctypes.c_int32),
                ("delta", ctypes.c_double), ("lam", ctypes.c_double)]


class Timing(ctypes.Structure):
    _fields_ = [("total_ms", ctypes.c_double), ("init_ms", ctypes.c_double),
                ("loop_ms", ctypes.c_double), ("iters", ctypes.c_int32),
                ("launches", ctypes.c_int32)]


class Binarize(ctypes.Structure):
    _fields_ = [("iters", ctypes.c_int32), ("project_from", ctypes.c_int32),
                ("slope", ctypes.c_float), ("threshold", ctypes.c_float)]


class Plan(ctypes.Structure):
    _fields_ = [("shape", ctypes.c_int32), ("chunks", ctypes.c_int32),
                ("blocks", ctypes.c_int32), ("threads", ctypes.c_int32)]


class SfsegError(RuntimeError):
    """A libsfseg entry point returned a negative status."""

    def __init__(self, status: int, fn: str, msg: str):
        super().__init__(f"{fn}: {msg} (status {status})")
        self.status = status


_lib = None


def lib():
    """Load libsfseg.so (raises if it has not been built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is missing: build it with "
                          "`python -m paper_1907_02731_amd.build` (hipcc, gfx950)")
    L = ctypes.CDLL(LIB_PATH)
    P = ctypes.c_void_p
    pcfg = ctypes.POINTER(Config)
    L.sfseg_config_default.argtypes = [pcfg]
    L.sfseg_config_default.restype = None
    L.sfseg_config_validate.argtypes = [pcfg]
    L.sfseg_config_validate.restype = ctypes.c_int
    L.sfseg_create.argtypes = [pcfg, P, P, P, ctypes.POINTER(P)]
    L.sfseg_create.restype = ctypes.c_int
    L.sfseg_create_mc.argtypes = [pcfg, P, P, ctypes.c_int32, P, ctypes.POINTER(P)]
    L.sfseg_create_mc.restype = ctypes.c_int
    L.sfseg_set_features.argtypes = [P, P, P]
    L.sfseg_set_features.restype = ctypes.c_int
    L.sfseg_power_iterate.argtypes = [P, P, ctypes.c_int32, ctypes.c_double,
                                      ctypes.POINTER(Result)]
    L.sfseg_power_iterate.restype = ctypes.c_int
    L.sfseg_eigvec.argtypes = [P, P]
    L.sfseg_eigvec.restype = ctypes.c_int
    L.sfseg_apply.argtypes = [P, P, P]
    L.sfseg_apply.restype = ctypes.c_int
    L.sfseg_spectral_grad.argtypes = [P, P, P, ctypes.c_int32, P, ctypes.POINTER(ctypes.c_double)]
    L.sfseg_spectral_grad.restype = ctypes.c_int
    L.sfseg_refine_frames.argtypes = [P, P, ctypes.POINTER(ctypes.c_double)]
    L.sfseg_refine_frames.restype = ctypes.c_int
    L.sfseg_apply_noalloc.argtypes = [P, P, P]
    L.sfseg_apply_noalloc.restype = ctypes.c_int
    L.sfseg_apply_noalloc_bytes.argtypes = [P]
    L.sfseg_apply_noalloc_bytes.restype = ctypes.c_size_t
    pbin = ctypes.POINTER(Binarize)
    L.sfseg_binarize_default.argtypes = [pbin]
    L.sfseg_binarize_default.restype = None
    L.sfseg_project.argtypes = [P, ctypes.c_float, ctypes.c_float]
    L.sfseg_project.restype = ctypes.c_int
    L.sfseg_threshold.argtypes = [P, ctypes.c_float, P]
    L.sfseg_threshold.restype = ctypes.c_int
    L.sfseg_segment.argtypes = [P, P, pbin, P, ctypes.POINTER(Result)]
    L.sfseg_segment.restype = ctypes.c_int
    L.sfseg_get_plan.argtypes = [P, ctypes.POINTER(Plan)]
    L.sfseg_get_plan.restype = ctypes.c_int
    L.sfseg_set_plan.argtypes = [P, ctypes.c_int32, ctypes.c_int32]
    L.sfseg_set_plan.restype = ctypes.c_int
    L.sfseg_autotune.argtypes = [P, ctypes.c_int32, ctypes.POINTER(Plan)]
    L.sfseg_autotune.restype = ctypes.c_int
    L.sfseg_batch_create.argtypes = [pcfg, ctypes.c_int32, ctypes.POINTER(P), ctypes.POINTER(P), P,
                                     ctypes.POINTER(P)]
    L.sfseg_batch_create.restype = ctypes.c_int
    L.sfseg_batch_size.argtypes = [P, ctypes.POINTER(ctypes.c_int32)]
    L.sfseg_batch_size.restype = ctypes.c_int
    L.sfseg_batch_iterate.argtypes = [P, ctypes.POINTER(P), ctypes.c_int32, ctypes.c_double,
                                      ctypes.POINTER(Result)]
    L.sfseg_batch_iterate.restype = ctypes.c_int
    L.sfseg_batch_eigvec.argtypes = [P, ctypes.POINTER(P)]
    L.sfseg_batch_eigvec.restype = ctypes.c_int
    L.sfseg_last_timing.argtypes = [P, ctypes.POINTER(Timing)]
    L.sfseg_last_timing.restype = ctypes.c_int
    L.sfseg_destroy.argtypes = [P]
    L.sfseg_destroy.restype = None
    L.sfseg_status_string.argtypes = [ctypes.c_int]
    L.sfseg_status_string.restype = ctypes.c_char_p
    L.sfseg_last_error.argtypes = []
    L.sfseg_last_error.restype = ctypes.c_char_p
    i32, i64, dbl = ctypes.c_int32, ctypes.c_int64, ctypes.c_double
    pf = ctypes.POINTER(ctypes.c_float)
    L.sfseg_unet_param_count.argtypes = []
    L.sfseg_unet_param_count.restype = i64
    L.sfseg_unet_create.argtypes = [i32, i32, i32, i32, P, ctypes.POINTER(P)]
    L.sfseg_unet_create.restype = ctypes.c_int
    L.sfseg_unet_set_params.argtypes = [P, pf, i64]
    L.sfseg_unet_set_params.restype = ctypes.c_int
    L.sfseg_unet_get_params.argtypes = [P, pf, i64]
    L.sfseg_unet_get_params.restype = ctypes.c_int
    L.sfseg_unet_get_grads.argtypes = [P, pf, i64]
    L.sfseg_unet_get_grads.restype = ctypes.c_int
    L.sfseg_unet_forward.argtypes = [P, P, i32, i32, i32, P]
    L.sfseg_unet_forward.restype = ctypes.c_int
    L.sfseg_unet_backward.argtypes = [P, P, ctypes.POINTER(dbl)]
    L.sfseg_unet_backward.restype = ctypes.c_int
    L.sfseg_unet_backward_from.argtypes = [P, P]
    L.sfseg_unet_backward_from.restype = ctypes.c_int
    L.sfseg_unet_adam_step.argtypes = [P, dbl, dbl, dbl, dbl, i32]
    L.sfseg_unet_adam_step.restype = ctypes.c_int
    L.sfseg_unet_sync.argtypes = [P]
    L.sfseg_unet_sync.restype = ctypes.c_int
    L.sfseg_unet_destroy.argtypes = [P]
    L.sfseg_unet_destroy.restype = None
    _lib = L
    return L


def check(status: int, fn: str) -> None:
    if status != SFSEG_OK:
        raise SfsegError(status, fn, lib().sfseg_last_error().decode(errors="replace"))


def make_config(T: int, H: int, W: int, *, r_t: int = 1, r_s: int = 2,
                sigma_t: float = 1.0, sigma_s: float = 1.0, alpha: float = 1.0,
                p: float = 0.2, storage: str = "f32") -> Config:
    if storage not in DTYPES:
        raise ValueError(f"storage must be one of {sorted(DTYPES)}")
    c = Config()
    lib().sfseg_config_default(ctypes.byref(c))
    c.T, c.H, c.W = int(T), int(H), int(W)
    c.r_t, c.r_s = int(r_t), int(r_s)
    c.sigma_t, c.sigma_s = float(sigma_t), float(sigma_s)
    c.alpha, c.p = float(alpha), float(p)
    c.storage = DTYPES[storage]
    return c


def validate(cfg: Config) -> int:
    return int(lib().sfseg_config_validate(ctypes.byref(cfg)))
