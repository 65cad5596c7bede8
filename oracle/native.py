"""ctypes front end of the oracle's C part (test infrastructure only).

``apply`` evaluates y = M x over a whole volume and ``apply_rows`` evaluates
selected rows of M x, both in float64 with the entries of Eq. (2), for
volumes too large for the explicit CSR matrix of ``sfseg_oracle``.
"""
from __future__ import annotations

import ctypes
import os
from typing import Optional

import numpy as np

from .sfseg_oracle import OracleConfig, unary_weights

_LIB = None
_HERE = os.path.dirname(os.path.abspath(__file__))


def _lib():
    global _LIB
    if _LIB is None:
        path = os.path.join(_HERE, "libsfseg_oracle.so")
        if not os.path.exists(path):
            from .build_oracle import build
            build()
        lib = ctypes.CDLL(path)
        d, i64, i32 = ctypes.c_double, ctypes.c_int64, ctypes.c_int
        pd = ctypes.POINTER(ctypes.c_double)
        pi64 = ctypes.POINTER(ctypes.c_int64)
        lib.oracle_apply.argtypes = [i64, i64, i64, i32, i32, d, d, d, pd, pd, pd, pd]
        lib.oracle_apply.restype = i32
        lib.oracle_apply_rows.argtypes = [i64, i64, i64, i32, i32, d, d, d, pd, pd, pd,
                                          pi64, i64, pd]
        lib.oracle_apply_rows.restype = i32
        lib.oracle_num_threads.argtypes = []
        lib.oracle_num_threads.restype = i32
        _LIB = lib
    return _LIB


def _p(a: np.ndarray):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


class MatrixFree:
    """Matrix-free FP64 operator for one clip: w = S^p and F are fixed."""

    def __init__(self, S: np.ndarray, F: Optional[np.ndarray], cfg: OracleConfig):
        S = np.asarray(S)
        if S.ndim != 3:
            raise ValueError("S must be a (T, H, W) volume")
        self.shape = S.shape
        self.cfg = cfg
        self.w = np.ascontiguousarray(unary_weights(S, cfg.p), dtype=np.float64)
        Fv = S if F is None else F
        self.f = np.ascontiguousarray(Fv, dtype=np.float64)
        if self.f.shape != self.shape:
            raise ValueError("F must have the shape of S")

    @property
    def n(self) -> int:
        return int(np.prod(self.shape))

    def apply(self, x: np.ndarray) -> np.ndarray:
        x = np.ascontiguousarray(x, dtype=np.float64).ravel()
        if x.size != self.n:
            raise ValueError("x has the wrong size")
        y = np.empty_like(x)
        T, H, W = self.shape
        c = self.cfg
        rc = _lib().oracle_apply(T, H, W, c.r_t, c.r_s, c.sigma_t, c.sigma_s, c.alpha,
                                 _p(self.w), _p(self.f), _p(x), _p(y))
        if rc != 0:
            raise RuntimeError("oracle_apply rejected its arguments")
        return y

    def apply_rows(self, x: np.ndarray, rows: np.ndarray) -> np.ndarray:
        x = np.ascontiguousarray(x, dtype=np.float64).ravel()
        rows = np.ascontiguousarray(rows, dtype=np.int64).ravel()
        if x.size != self.n:
            raise ValueError("x has the wrong size")
        out = np.empty(rows.size, dtype=np.float64)
        T, H, W = self.shape
        c = self.cfg
        rc = _lib().oracle_apply_rows(
            T, H, W, c.r_t, c.r_s, c.sigma_t, c.sigma_s, c.alpha, _p(self.w), _p(self.f),
            _p(x), rows.ctypes.data_as(ctypes.POINTER(ctypes.c_int64)), rows.size, _p(out))
        if rc != 0:
            raise RuntimeError("oracle_apply_rows rejected its arguments")
        return out


def num_threads() -> int:
    return int(_lib().oracle_num_threads())
