"""Approximation-gap study (Sec. 4.2, quantitative analysis) -- test
infrastructure on the FP64 CPU oracle only.

Eq. (2) replaces the Gaussian pairwise term exp(-alpha dF^2) of Eq. (1) by
its first-order expansion 1 - alpha dF^2, which is what turns M into a sum of
filterings.  On synthetic clips small enough for the exact matrix, this
measures how far the principal eigenvector of the approximate matrix (the
vector SFSeg converges to) lies from the exact one, and how SFSeg's iterates
approach the exact eigenvector from a start 70 degrees away from it: the
angle in degrees, and the IoU of the hard-thresholded masks (x > 0.5 max x),
over the iterations.

The start vector is the exact eigenvector plus non-negative noise orthogonal
to it, scaled by bisection until the angle is 70 degrees: a noisy soft
segmentation, as in the paper's toy examples, and non-negative like every
input the method sees.

    python tests/gap_study.py      # prints the tables
"""
from __future__ import annotations

import math
import os
import sys

import numpy as np
from scipy.sparse.linalg import eigsh

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

from oracle import OracleConfig, build_adjacency, build_adjacency_exact, power_iteration  # noqa: E402
from oracle.binarize_oracle import hard_threshold  # noqa: E402
from paper_1907_02731_amd.synth import make_clip  # noqa: E402

START_ANGLE = 70.0
THRESHOLD = 0.5
REPORT_AT = (0, 1, 2, 3, 5, 10, 20, 50, 100, 200, 400)

# (name, (T, H, W), graph parameters, generator seed, iterations)
CASES = [
    ("4000 nodes (10 x 20 x 20)", (10, 20, 20),
     OracleConfig(r_t=1, r_s=3, sigma_t=1.0, sigma_s=2.0, alpha=1.0, p=0.2), 5, 400),
    ("six frames (6 x 24 x 32)", (6, 24, 32),
     OracleConfig(r_t=1, r_s=3, sigma_t=1.0, sigma_s=2.0, alpha=1.0, p=0.2), 6, 400),
]


def clip(shape, seed):
    """Noisy soft segmentation in [0, 1]: one drifting object, one distractor."""
    T, H, W = shape
    return make_clip(T, H, W, seed=seed, n_blobs=1, noise_sigma=0.15, motion="drift",
                     dtype=np.float64)


def principal(M):
    """Principal eigenpair of a symmetric non-negative matrix (Lanczos),
    with the eigenvector's sign made non-negative."""
    lam, vec = eigsh(M, k=1, which="LA", tol=1e-13, maxiter=20000)
    v = vec[:, 0]
    if v.sum() < 0:
        v = -v
    return float(lam[0]), v / np.linalg.norm(v)


def angle_deg(a, b):
    """Angle between the lines through a and b, in degrees (2 atan2 of the
    half-difference and half-sum of the unit vectors, accurate near 0)."""
    a = a / np.linalg.norm(a)
    b = b / np.linalg.norm(b)
    if float(a @ b) < 0.0:
        b = -b
    return math.degrees(2.0 * math.atan2(np.linalg.norm(a - b), np.linalg.norm(a + b)))


def iou(a, b, thr=THRESHOLD):
    A, B = hard_threshold(a, thr), hard_threshold(b, thr)
    union = np.count_nonzero(A | B)
    return 1.0 if union == 0 else np.count_nonzero(A & B) / union


def start_at(v, degrees, seed):
    """v + beta u with u >= 0 noise orthogonalised against v (negative part
    dropped), beta found by bisection so that the angle to v is `degrees`."""
    rng = np.random.Generator(np.random.PCG64(seed))
    r = rng.random(v.size)
    u = np.maximum(r - (r @ v) * v, 0.0)
    u /= np.linalg.norm(u)
    if angle_deg(u, v) <= degrees:
        raise ValueError("noise direction too close to the eigenvector")
    lo, hi = 0.0, 1.0
    while angle_deg(v + hi * u, v) < degrees:
        hi *= 2.0
    for _ in range(200):
        mid = 0.5 * (lo + hi)
        if angle_deg(v + mid * u, v) < degrees:
            lo = mid
        else:
            hi = mid
    x0 = v + 0.5 * (lo + hi) * u
    return x0 / np.linalg.norm(x0)


def study(shape, cfg, seed, iters):
    S = clip(shape, seed)
    M1 = build_adjacency_exact(S, None, cfg)  # Eq. (1)
    M2 = build_adjacency(S, None, cfg)        # Eq. (2)
    lam1, v1 = principal(M1)
    lam2, v2 = principal(M2)
    x0 = start_at(v1, START_ANGLE, seed)
    res = power_iteration(lambda x: M2 @ x, x0, iters, 0.0, keep_history=True)
    hist = res["history"]
    rows = [(k, angle_deg(x, v1), iou(x, v1), angle_deg(x, v2)) for k, x in enumerate(hist)]
    return {"S": S, "cfg": cfg, "x0": x0, "v_exact": v1, "v_approx": v2, "lam_exact": lam1,
            "lam_approx": lam2, "history": hist, "rows": rows,
            "floor_angle": angle_deg(v2, v1), "floor_iou": iou(v2, v1)}


def table(name, out):
    lines = [f"{name}: lambda exact {out['lam_exact']:.6f}, approximate {out['lam_approx']:.6f}; "
             f"angle between the two eigenvectors {out['floor_angle']:.4f} deg, "
             f"mask IoU {out['floor_iou']:.4f}",
             "| iteration | angle to exact (deg) | IoU with exact | angle to Eq. (2) eigenvector (deg) |",
             "|---|---|---|---|"]
    for k, a1, j, a2 in out["rows"]:
        if k in REPORT_AT:
            lines.append(f"| {k} | {a1:.4f} | {j:.4f} | {a2:.4f} |")
    return "\n".join(lines)


def main():
    for name, shape, cfg, seed, iters in CASES:
        print(table(name, study(shape, cfg, seed, iters)), flush=True)
        print(flush=True)


if __name__ == "__main__":
    main()
