"""Pins of the binarisation oracle (Sec. 4.1, Algorithm 1 step 3) against
values fixed outside it: scipy's logistic function, textbook logistic values,
exact float32 ties, and special cases that reduce the algorithm to something
known (no projection = plain power iteration; M = I = the iterated logistic
map)."""
import math

import numpy as np
import pytest
from scipy.special import expit

from oracle import OracleConfig, ZeroNormError, build_adjacency, power_iteration
from oracle.binarize_oracle import (hard_threshold, logistic, max_scale, project_binary,
                                    segment)

# sigma(5), sigma(1), sigma(-1), sigma(-3) of the logistic function
SIG5, SIG1, SIGM1, SIGM3 = 0.9933071490757153, 0.7310585786300049, 0.2689414213699951, \
    0.04742587317756678
SIGM5 = 0.0066928509242848554  # sigma(-5)


def test_logistic_matches_scipy_and_its_identities():
    r = np.random.Generator(np.random.PCG64(0))
    u = np.concatenate([r.uniform(-60, 60, 1000), [-800.0, -40.0, 0.0, 40.0, 800.0]])
    np.testing.assert_allclose(logistic(u), expit(u), rtol=1e-15, atol=0)
    np.testing.assert_allclose(logistic(u) + logistic(-u), 1.0, rtol=0, atol=4.5e-16)
    assert logistic(np.array([0.0]))[0] == 0.5
    h = 1e-5
    d = (logistic(np.array([h])) - logistic(np.array([-h])))[0] / (2 * h)
    assert abs(d - 0.25) < 1e-10
    np.testing.assert_allclose(logistic(np.array([5.0, 1.0, -1.0, -3.0])),
                               [SIG5, SIG1, SIGM1, SIGM3], rtol=1e-15)


def test_projection_values_and_scale_invariance():
    x = np.array([2.0, 1.0, 0.5, 0.0])
    p = project_binary(x, 10.0, 0.5)
    np.testing.assert_allclose(p, [SIG5, 0.5, expit(-2.5), SIGM5], rtol=1e-14)
    np.testing.assert_array_equal(project_binary(3.0 * x, 10.0, 0.5), p)
    assert max_scale(x) == 2.0
    with pytest.raises(ZeroNormError):
        project_binary(np.array([0.0, -1.0]), 10.0, 0.5)
    with pytest.raises(ArithmeticError):
        project_binary(np.array([1.0, np.inf]), 10.0, 0.5)


def test_hard_threshold_is_strict_and_exact_at_float32_ties():
    half_up = float(np.nextafter(np.float32(0.5), np.float32(1)))
    half_dn = float(np.nextafter(np.float32(0.5), np.float32(0)))
    x = np.array([1.0, half_up, 0.5, half_dn, 0.0])
    np.testing.assert_array_equal(hard_threshold(x, 0.5), [True, True, False, False, False])
    # theta * max is exact for float32 operands: max = 3 * 2^-3, theta = 1/3 in float32
    th = float(np.float32(1.0 / 3.0))
    m = np.float32(0.375)
    at = float(np.float64(th) * np.float64(m))
    above = float(np.nextafter(np.float32(at), np.float32(1)))
    x = np.array([m, above], dtype=np.float64)
    np.testing.assert_array_equal(hard_threshold(x, th), [True, True])
    x = np.array([m, float(np.float32(at))])  # float32(at) <= at (rounded down or exact)
    assert hard_threshold(x, th)[1] == (float(np.float32(at)) > at)


def _clip(seed, shape=(3, 6, 7)):
    r = np.random.Generator(np.random.PCG64(seed))
    return r.random(shape)


def test_no_projection_is_plain_power_iteration():
    S = _clip(1)
    cfg = OracleConfig(r_t=1, r_s=2, sigma_t=1.0, sigma_s=1.5, alpha=1.0, p=0.5)
    M = build_adjacency(S, None, cfg)
    ref = power_iteration(lambda v: M @ v, S.ravel(), 7, 0.0)
    out = segment(lambda v: M @ v, S.ravel(), 7, 7, 10.0, 0.5)
    np.testing.assert_array_equal(out["x"], ref["x"])
    assert out["lam"] == ref["lam"] and out["delta"] == ref["delta"]
    np.testing.assert_array_equal(out["mask"], ref["x"] > 0.5 * ref["x"].max())


def test_identity_operator_gives_the_iterated_logistic_map():
    # r_t = r_s = 0 and S = 1 make Eq. (2)'s M the identity, so Algorithm 1
    # with projection after every iteration but the last is the logistic map
    # z -> sigma(kappa (z / max z - theta)) iterated on the start vector.
    x0 = np.array([1.0, 0.6, 0.4, 0.2])
    cfg = OracleConfig(r_t=0, r_s=0, sigma_t=1.0, sigma_s=1.0, alpha=1.0, p=0.3)
    M = build_adjacency(np.ones((1, 1, 4)), x0.reshape(1, 1, 4), cfg)
    np.testing.assert_array_equal(M.toarray(), np.eye(4))
    out = segment(lambda v: M @ v, x0, 4, 1, 10.0, 0.5, keep_history=True)
    first = out["history"][0][1]
    e = np.array([SIG5, SIG1, SIGM1, SIGM3])
    np.testing.assert_allclose(first, e / np.linalg.norm(e), rtol=1e-14)
    v = x0.copy()
    for _ in range(3):
        v = expit(10.0 * (v / v.max() - 0.5))
    np.testing.assert_allclose(out["x"], v / np.linalg.norm(v), rtol=1e-13)
    np.testing.assert_array_equal(out["mask"], [True, True, False, False])
    assert out["history"][3][1] is None  # the last iteration is not projected
    assert abs(out["lam"] - 1.0) < 1e-15 and out["delta"] < 1e-15


def test_schedule_and_scale_invariance():
    S = _clip(2)
    cfg = OracleConfig(r_t=1, r_s=1, sigma_t=1.0, sigma_s=1.0, alpha=0.8, p=0.4)
    M = build_adjacency(S, None, cfg)
    out = segment(lambda v: M @ v, S.ravel(), 4, 2, 8.0, 0.4, keep_history=True)
    assert [h[1] is not None for h in out["history"]] == [False, True, True, False]
    # the projected vector is the projection of that iteration's power iterate
    x2, p2 = out["history"][1]
    q = project_binary(x2, 8.0, 0.4)
    np.testing.assert_allclose(p2, q / np.linalg.norm(q), rtol=1e-14)
    # the next power step starts from it
    y = M @ p2
    np.testing.assert_allclose(out["history"][2][0], y / np.linalg.norm(y), rtol=1e-13)
    # S scaled by 4: M scales by 4^(2p), the unit iterates and the mask do not change
    M4 = build_adjacency(4.0 * S, S, cfg)
    out4 = segment(lambda v: M4 @ v, S.ravel(), 4, 2, 8.0, 0.4)
    np.testing.assert_allclose(out4["x"], out["x"], rtol=1e-12, atol=1e-15)
    np.testing.assert_array_equal(out4["mask"], out["mask"])


def test_errors():
    with pytest.raises(ValueError):
        segment(lambda v: v, np.ones(3), 0, 1, 10.0, 0.5)
    with pytest.raises(ZeroNormError):
        segment(lambda v: v, np.zeros(3), 2, 1, 10.0, 0.5)
    with pytest.raises(ZeroNormError):
        segment(lambda v: -np.abs(v), np.ones(3), 3, 1, 10.0, 0.5)
    assert math.isclose(float(logistic(np.array([-1e4]))[0]), 0.0, abs_tol=0)
