"""FP64 CPU oracle for SFSeg's power iteration -- TEST INFRASTRUCTURE ONLY.

Burceanu & Leordeanu, "A 3D Convolutional Approach to Spectral Object
Segmentation in Space and Time" (IJCAI 2020, arXiv 1907.02731).

Only ``tests/``, the smoke check and the benchmark's CPU-baseline leg may
import this module.  It shares no code with the HIP path: it builds the
adjacency matrix M of the space-time pixel graph *explicitly* (a scipy CSR
matrix in float64, entry by entry from Eq. (2)) and runs classical power
iteration on it (Eq. (4) followed by the normalisation of Eq. (8)).  The
GPU path never builds M; it applies it as three 3D Gaussian filterings
(Eq. (7)).  The two meet only on the seeded inputs.

What is computed (Sec. 3, Eqs. (1), (2), (4), (8)); node i = (t, y, x):

    w_i  = S_i ** p                        (0 ** p := 0 for p > 0; p = 0 gives w = 1)
    G(d) = exp(-dt^2/(2 sigma_t^2) - (dy^2 + dx^2)/(2 sigma_s^2))
           on the box |dt| <= r_t, |dy| <= r_s, |dx| <= r_s, 0 elsewhere
    M_ij = w_i w_j [1 - alpha (F_i - F_j)^2] G(j - i)          (Eq. (2))
           for j inside the volume (no wrap-around, no padding), j = i included
    x <- x0 / ||x0||;  repeat  y = M x,  lambda = x^T y,  x' = y / ||y||,
                               delta = ||x' - x||_2,  x = x'
                       until delta < tol or max_iters steps.

Readings of points the paper leaves open (each also listed in the design
notes): beta of Eq. (1) is 1/(2 sigma^2) per axis with sigma_t for frames and
sigma_s for rows/columns; G is unnormalised (G(0) = 1); the neighbourhood is a
box (needed for separability, Sec. 4.2); j = i is a neighbour; the volume
boundary truncates the neighbourhood (any padding other than zeros would make
M non-symmetric); the leading alpha of Eq. (5) is kept, so lambda is the
Rayleigh quotient of Eq. (2)'s M itself; x0 is normalised first; the
convergence measure is the L2 distance between successive unit iterates;
S = F when only one feature map is given; no optical-flow window transform and
no binarisation (Alg. 1, step 3) on this path.

Parity pins for every function here live in ``tests/test_oracle_pins.py``.
"""
from __future__ import annotations

import dataclasses
import math
from typing import Callable, Optional

import numpy as np
import scipy.sparse as sp

__all__ = [
    "OracleConfig", "unary_weights", "gaussian_taps", "spacetime_kernel",
    "build_adjacency", "build_adjacency_exact", "build_adjacency_multi", "power_iteration",
    "ZeroNormError",
]


@dataclasses.dataclass(frozen=True)
class OracleConfig:
    """Graph parameters (Sec. 3; defaults alpha = 1, p = 0.2 from Sec. 5)."""
    r_t: int = 1
    r_s: int = 2
    sigma_t: float = 1.0
    sigma_s: float = 1.0
    alpha: float = 1.0
    p: float = 0.2


class ZeroNormError(ArithmeticError):
    """The iterate (or the start vector) has zero L2 norm."""


def unary_weights(S: np.ndarray, p: float) -> np.ndarray:
    """Unary term s_i^p of Eq. (2), in float64.

    0^p is 0 for p > 0; p = 0 turns the unary term off (w = 1 everywhere).
    """
    S = np.asarray(S, dtype=np.float64)
    if p == 0.0:
        return np.ones_like(S)
    w = np.zeros_like(S)
    pos = S > 0
    w[pos] = np.power(S[pos], p)
    return w


def gaussian_taps(r: int, sigma: float) -> np.ndarray:
    """1D factor of G along one axis: exp(-d^2 / (2 sigma^2)) for d = -r..r.

    The product of the three axis factors is G of Eq. (1); separability is the
    point made in Sec. 4.2 (complexity paragraph).
    """
    d = np.arange(-r, r + 1, dtype=np.float64)
    return np.exp(-(d * d) / (2.0 * sigma * sigma))


def spacetime_kernel(cfg: OracleConfig) -> np.ndarray:
    """Dense (2r_t+1, 2r_s+1, 2r_s+1) array of G(dt, dy, dx), Eq. (1)."""
    gt = gaussian_taps(cfg.r_t, cfg.sigma_t)
    gs = gaussian_taps(cfg.r_s, cfg.sigma_s)
    return gt[:, None, None] * gs[None, :, None] * gs[None, None, :]


def _pair_slices(n: int, d: int):
    """Index ranges (src, dst) of all a with 0 <= a < n and 0 <= a + d < n."""
    if abs(d) >= n:
        return slice(0, 0), slice(0, 0)
    if d >= 0:
        return slice(0, n - d), slice(d, n)
    return slice(-d, n), slice(0, n + d)


def _build(S: np.ndarray, F: Optional[np.ndarray], cfg: OracleConfig,
           pairwise: Callable[[np.ndarray], np.ndarray]) -> sp.csr_matrix:
    S = np.asarray(S, dtype=np.float64)
    if S.ndim != 3:
        raise ValueError("S must be a (T, H, W) volume")
    F = S if F is None else np.asarray(F, dtype=np.float64)
    if F.shape != S.shape:
        raise ValueError("F must have the shape of S")
    T, H, W = S.shape
    N = T * H * W
    w = unary_weights(S, cfg.p)
    idx = np.arange(N, dtype=np.int64).reshape(T, H, W)
    G = spacetime_kernel(cfg)
    rows, cols, vals = [], [], []
    # One pass per neighbour offset (dt, dy, dx): every pair (i, j) with
    # j = i + offset and both inside the volume.
    for a, dt in enumerate(range(-cfg.r_t, cfg.r_t + 1)):
        st_i, st_j = _pair_slices(T, dt)
        for b, dy in enumerate(range(-cfg.r_s, cfg.r_s + 1)):
            sy_i, sy_j = _pair_slices(H, dy)
            for c, dx in enumerate(range(-cfg.r_s, cfg.r_s + 1)):
                sx_i, sx_j = _pair_slices(W, dx)
                I = idx[st_i, sy_i, sx_i]
                J = idx[st_j, sy_j, sx_j]
                if I.size == 0:
                    continue
                dF = F[st_i, sy_i, sx_i] - F[st_j, sy_j, sx_j]
                v = (w[st_i, sy_i, sx_i] * w[st_j, sy_j, sx_j]
                     * pairwise(dF) * G[a, b, c])
                rows.append(I.ravel())
                cols.append(J.ravel())
                vals.append(v.ravel())
    M = sp.csr_matrix((np.concatenate(vals), (np.concatenate(rows), np.concatenate(cols))),
                      shape=(N, N))
    M.sum_duplicates()
    return M


def build_adjacency(S: np.ndarray, F: Optional[np.ndarray], cfg: OracleConfig) -> sp.csr_matrix:
    """Explicit sparse M of Eq. (2): first-order Taylor pairwise term.

    Row/column index of voxel (t, y, x) is (t * H + y) * W + x (row-major,
    W fastest).  ``F=None`` means F = S.
    """
    alpha = float(cfg.alpha)
    return _build(S, F, cfg, lambda dF: 1.0 - alpha * dF * dF)


def build_adjacency_multi(S: np.ndarray, Fs: np.ndarray, cfg: OracleConfig) -> sp.csr_matrix:
    """Multi-channel adjacency (Sec. 3.3, Eq. (9)): one step with several
    pairwise feature channels F_1..F_C is the sum of the single-channel steps,
    so the matrix is the sum over channels of Eq. (2)'s M built with F_c:

        M_ij = w_i w_j [C - alpha sum_c (F_c,i - F_c,j)^2] G(j - i).

    ``Fs`` has shape (C, T, H, W)."""
    Fs = np.asarray(Fs, dtype=np.float64)
    if Fs.ndim != 4 or Fs.shape[1:] != np.shape(S):
        raise ValueError("Fs must be (C, T, H, W) with (T, H, W) the shape of S")
    M = build_adjacency(S, Fs[0], cfg)
    for c in range(1, Fs.shape[0]):
        M = M + build_adjacency(S, Fs[c], cfg)
    return M.tocsr()


def build_adjacency_exact(S: np.ndarray, F: Optional[np.ndarray], cfg: OracleConfig) -> sp.csr_matrix:
    """Explicit sparse M of Eq. (1): the Gaussian pairwise term before the
    Taylor approximation (used to study the approximation gap, Sec. 4.2)."""
    alpha = float(cfg.alpha)
    return _build(S, F, cfg, lambda dF: np.exp(-alpha * dF * dF))


def power_iteration(apply: Callable[[np.ndarray], np.ndarray], x0: np.ndarray,
                    max_iters: int, tol: float, keep_history: bool = False) -> dict:
    """Classical power iteration (Eq. (4), then Eq. (8) after every step).

    ``apply(x)`` must return M x for a flat float64 vector.  Returns a dict
    with the unit iterate ``x`` after ``iters`` steps, ``lam`` = x_prev^T M
    x_prev (the Rayleigh quotient of Eq. (3) at the last input iterate),
    ``delta`` = ||x_k - x_{k-1}||_2 of the last step, ``converged`` (delta <
    tol) and optionally the list of iterates.
    """
    x = np.asarray(x0, dtype=np.float64).ravel().copy()
    n0 = float(np.linalg.norm(x))
    if not (n0 > 0.0) or not math.isfinite(n0):
        raise ZeroNormError("start vector has zero (or non-finite) norm")
    x /= n0
    hist = [x.copy()] if keep_history else None
    lam = float("nan")
    delta = float("inf")
    k = 0
    while k < max_iters:
        y = apply(x)
        lam = float(x @ y)
        n = float(np.linalg.norm(y))
        if not (n > 0.0):
            raise ZeroNormError(f"M x has zero norm at step {k + 1}")
        x_new = y / n
        delta = float(np.linalg.norm(x_new - x))
        x = x_new
        k += 1
        if keep_history:
            hist.append(x.copy())
        if delta < tol:
            break
    out = {"x": x, "lam": lam, "delta": delta, "iters": k, "converged": bool(delta < tol)}
    if keep_history:
        out["history"] = hist
    return out
