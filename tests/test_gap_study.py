"""Approximation-gap study (Sec. 4.2) on the FP64 oracle: the structure of
the experiment and the facts it rests on (the numbers themselves are
printed; run with -s, or run tests/gap_study.py)."""
import numpy as np
import pytest
from scipy.linalg import eigh

from gap_study import (CASES, START_ANGLE, angle_deg, clip, principal, start_at, study,
                       table)
from oracle import OracleConfig, build_adjacency, build_adjacency_exact


def test_lanczos_principal_matches_dense_eigh():
    cfg = OracleConfig(r_t=1, r_s=2, sigma_t=1.0, sigma_s=1.5, alpha=1.0, p=0.2)
    S = clip((4, 10, 12), 3)
    for build in (build_adjacency, build_adjacency_exact):
        M = build(S, None, cfg)
        lam, v = principal(M)
        w, V = eigh(M.toarray())
        assert abs(lam - w[-1]) <= 1e-11 * w[-1]
        assert angle_deg(v, V[:, -1]) <= 1e-6


def test_equal_features_make_the_two_matrices_equal():
    # dF = 0 on every edge: exp(-alpha 0) = 1 - alpha 0, so Eq. (1) = Eq. (2)
    cfg = OracleConfig(r_t=1, r_s=2, sigma_t=1.0, sigma_s=1.5, alpha=1.0, p=0.5)
    S = clip((3, 8, 9), 4)
    F = np.full(S.shape, 0.3)
    d = build_adjacency_exact(S, F, cfg) - build_adjacency(S, F, cfg)
    assert abs(d).max() == 0.0


@pytest.mark.parametrize("name,shape,cfg,seed,iters", CASES)
def test_gap_study(name, shape, cfg, seed, iters):
    out = study(shape, cfg, seed, iters)
    print("\n" + table(name, out), flush=True)
    x0, v1, v2 = out["x0"], out["v_exact"], out["v_approx"]
    assert np.all(x0 >= 0.0) and np.all(v1 >= -1e-12)
    assert abs(angle_deg(x0, v1) - START_ANGLE) <= 1e-9
    a2 = [r[3] for r in out["rows"]]
    # power iteration on a symmetric non-negative matrix: the angle to its
    # principal eigenvector never grows, and here it reaches it
    assert all(b <= a + 1e-9 for a, b in zip(a2, a2[1:]))
    assert a2[-1] <= 1e-3
    # so the angle to the exact eigenvector ends at the gap between the two
    assert abs(out["rows"][-1][1] - out["floor_angle"]) <= 1e-3
    assert 0.0 < out["floor_angle"] < START_ANGLE


def test_start_vector_bisection():
    v = np.zeros(50)
    v[:10] = 1.0
    v /= np.linalg.norm(v)
    for deg in (10.0, 45.0, 70.0):
        x = start_at(v, deg, seed=1)
        assert np.all(x >= 0) and abs(angle_deg(x, v) - deg) <= 1e-9
