"""FP64 oracle of the binarisation of Sec. 4.1 -- TEST INFRASTRUCTURE ONLY.

Only ``tests/``, the smoke check and the benchmark's CPU-baseline leg may
import this module.  It shares no code with the HIP path.

Algorithm 1 ends every outer iteration with a projection of the normalised
solution towards a discrete one (its Step 3), and Sec. 4.1 describes it: once
the iterate has had some unconstrained steps it is mapped through a sigmoid,
a smooth stand-in for a step function, and that mapped vector starts the
following iteration; a hard threshold after the final iteration yields the
segmentation.  The paper gives neither the sigmoid's slope, nor its
centre, nor the iteration it starts at, nor the scale it acts on.  The
readings taken here:

* scale: the iterate divided by its largest entry, z = x / max_j x_j, so that
  the sigmoid acts on a soft segmentation in [0, 1] (for x >= 0) whatever the
  norm used by the power step; a start vector S in [0, 1] is on that scale;
* projection: P(x)_i = sigma(kappa (z_i - theta)), sigma(u) = 1 / (1 + e^-u),
  slope kappa > 0, centre theta;
* schedule: outer iterations k = 1 .. N_i; after iteration k the projection
  is applied when k_0 <= k < N_i (k_0 = first projected iteration); the
  projected vector, normalised, is the next iteration's input;
* hard threshold after the last iteration: mask_i = [x_i > theta max_j x_j]
  (strict), on the last power iterate.  With x_i and theta float32 values
  the product theta * max_j x_j is exact in float64 (24 + 24 significand
  bits), so the decision is exact;
* defaults (not in the paper): N_i = 5 (the paper's experiments), k_0 = 3,
  kappa = 10, theta = 0.5.

The fixed point of this iteration is no longer an eigenvector of M, so
parity is on the sequence: the same steps in float64.

Pins: ``tests/test_binarize_oracle.py``.
"""
from __future__ import annotations

import math
from typing import Callable

import numpy as np

from .sfseg_oracle import ZeroNormError


def logistic(u: np.ndarray) -> np.ndarray:
    """sigma(u) = 1 / (1 + exp(-u)) in float64, evaluated as
    exp(u) / (1 + exp(u)) for u < 0 so that no exp overflows."""
    u = np.asarray(u, dtype=np.float64)
    out = np.empty_like(u)
    pos = u >= 0
    out[pos] = 1.0 / (1.0 + np.exp(-u[pos]))
    e = np.exp(u[~pos])
    out[~pos] = e / (1.0 + e)
    return out


def max_scale(x: np.ndarray) -> float:
    """The largest entry of x: the scale of the projection and of the hard
    threshold.  Raises ZeroNormError when no entry is positive."""
    m = float(np.max(x))
    if not math.isfinite(m):
        raise ArithmeticError("non-finite iterate")
    if not (m > 0.0):
        raise ZeroNormError("the iterate has no positive entry to scale by")
    return m


def project_binary(x: np.ndarray, slope: float, threshold: float) -> np.ndarray:
    """Sec. 4.1 sigmoid projection: sigma(slope * (x / max(x) - threshold))."""
    x = np.asarray(x, dtype=np.float64)
    z = x / max_scale(x)
    return logistic(slope * (z - threshold))


def hard_threshold(x: np.ndarray, threshold: float) -> np.ndarray:
    """Sec. 4.1 final hard threshold: x_i > threshold * max(x), as bool.
    No positive entry (max <= 0) gives the comparison against threshold *
    max all the same; it is exact for float32 x and threshold."""
    x = np.asarray(x, dtype=np.float64)
    m = float(np.max(x))
    return x > float(threshold) * m


def segment(apply: Callable[[np.ndarray], np.ndarray], x0: np.ndarray, iters: int,
            project_from: int, slope: float, threshold: float,
            keep_history: bool = False) -> dict:
    """Algorithm 1 with the Sec. 4.1 binarisation.

    Outer iteration k = 1 .. iters: y = M x (Eq. (4) via ``apply``),
    x = y / ||y|| (Eq. (8)); then, when project_from <= k < iters,
    x = P(x) / ||P(x)|| with P the sigmoid projection.  After the last
    iteration the hard threshold gives ``mask``.  Returns the last unit power
    iterate ``x`` (before the threshold), ``mask``, ``lam`` = x_in^T M x_in
    and ``delta`` = ||x - x_in|| of the last step (x_in the unit input of that
    step, a projected vector when the step before was projected), and
    optionally the history of (power iterate, projected vector or None).
    """
    if iters < 1:
        raise ValueError("iters must be >= 1")
    x = np.asarray(x0, dtype=np.float64).ravel().copy()
    n0 = float(np.linalg.norm(x))
    if not (n0 > 0.0) or not math.isfinite(n0):
        raise ZeroNormError("start vector has zero (or non-finite) norm")
    x /= n0
    hist = [] if keep_history else None
    lam = delta = float("nan")
    for k in range(1, iters + 1):
        y = apply(x)
        lam = float(x @ y)
        n = float(np.linalg.norm(y))
        if not (n > 0.0):
            raise ZeroNormError(f"M x has zero norm at iteration {k}")
        x_new = y / n
        delta = float(np.linalg.norm(x_new - x))
        x = x_new
        proj = None
        if project_from <= k < iters:
            p = project_binary(x, slope, threshold)
            proj = p / np.linalg.norm(p)
        if keep_history:
            hist.append((x.copy(), None if proj is None else proj.copy()))
        if proj is not None:
            x = proj
    out = {"x": x, "mask": hard_threshold(x, threshold), "lam": lam, "delta": delta,
           "iters": iters}
    if keep_history:
        out["history"] = hist
    return out
