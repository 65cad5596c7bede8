"""FP64 oracle of the frame-wise Rayleigh-Ritz refinement of a start vector --
TEST INFRASTRUCTURE ONLY.

Only ``tests/``, the smoke check and the benchmark's CPU-baseline leg may
import this module.  It shares no code with the HIP path.

This refinement is not part of the paper; it serves the warm-started form
(a better start vector for the unchanged power iteration).  Eq. (3) makes the
principal eigenvector the maximiser of the Rayleigh quotient x^T M x / x^T x.
The Rayleigh-Ritz principle maximises the same quotient over a subspace: for
a basis q_1 .. q_m, the maximiser is sum_t a_t q_t with a the top eigenvector
of the pencil (Q^T M Q, Q^T Q), and the maximum is the largest Ritz value.

Here the subspace is spanned by the frames of a vector x: q_t is x restricted
to frame t (zero on every other frame), t = 0 .. T-1, so the Ritz vector is x
with each frame rescaled by its own factor a_t.  The q_t have disjoint
supports, so Q^T Q = G = diag(||x_t||^2); M couples frames at most r_t apart
(Eq. (1) with the temporal box of radius r_t), so B = Q^T M Q is a band
matrix with B[i][j] = 0 for |i - j| > r_t.

Definitions (computed plainly, one product of M per frame):

* B[i][j] = q_i^T (M q_j), G[t] = q_t^T q_t;
* frames with x_t = 0 span nothing and get a_t = 0;
* over the other frames, mu = the largest eigenvalue of B a = mu G a, a its
  eigenvector, signed so that sum_t a_t G[t] > 0 (positive overlap with x);
* the refined vector x' = sum_t a_t q_t.

Pins: ``tests/test_ritz_oracle.py``.
"""
from __future__ import annotations

from typing import Callable, Tuple

import numpy as np
import scipy.linalg


def frame_basis_vector(x: np.ndarray, shape: Tuple[int, int, int], t: int) -> np.ndarray:
    """q_t: x (flat, T*H*W, W fastest) restricted to frame t."""
    T, H, W = shape
    q = np.zeros(T * H * W, dtype=np.float64)
    lo = t * H * W
    q[lo:lo + H * W] = np.asarray(x, dtype=np.float64).ravel()[lo:lo + H * W]
    return q


def frame_band(apply: Callable[[np.ndarray], np.ndarray], x: np.ndarray,
               shape: Tuple[int, int, int]) -> Tuple[np.ndarray, np.ndarray]:
    """B = Q^T M Q (T x T, dense) and G = diag(Q^T Q) (T,) for the frame
    basis of x; ``apply(v)`` returns M v for a flat float64 vector."""
    T = shape[0]
    qs = [frame_basis_vector(x, shape, t) for t in range(T)]
    B = np.zeros((T, T), dtype=np.float64)
    for j in range(T):
        mq = apply(qs[j])
        for i in range(T):
            B[i, j] = float(qs[i] @ mq)
    G = np.array([float(q @ q) for q in qs], dtype=np.float64)
    return B, G


def frame_ritz(apply: Callable[[np.ndarray], np.ndarray], x: np.ndarray,
               shape: Tuple[int, int, int]) -> dict:
    """The frame-wise Rayleigh-Ritz refinement of x: a dict with the refined
    vector ``x`` (flat float64), the frame factors ``a`` (T,), the largest
    Ritz value ``mu`` and the matrices ``B``, ``G``."""
    B, G = frame_band(apply, x, shape)
    keep = G > 0.0
    if not np.any(keep):
        raise ValueError("x is zero on every frame")
    Bk = B[np.ix_(keep, keep)]
    Bk = 0.5 * (Bk + Bk.T)  # Q^T M Q is symmetric; remove rounding asymmetry
    w, V = scipy.linalg.eigh(Bk, np.diag(G[keep]))
    a = np.zeros(shape[0], dtype=np.float64)
    a[keep] = V[:, -1]
    if float(a @ G) < 0.0:
        a = -a
    T, H, W = shape
    xr = (a[:, None] * np.asarray(x, dtype=np.float64).reshape(T, H * W)).ravel()
    return {"x": xr, "a": a, "mu": float(w[-1]), "B": B, "G": G}
