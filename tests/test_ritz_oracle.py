"""Pins of the frame-wise Rayleigh-Ritz oracle (``oracle/ritz_oracle.py``)
against what the mathematics fixes independently of it: the projected matrix
Q^T M Q written out with an explicit basis matrix and the dense M of Eq. (2);
exact recovery of the principal eigenvector (from a dense symmetric
eigensolver) when the start vector is that eigenvector with every frame
rescaled; the Courant-Fischer bounds rho(x) <= mu <= lambda_1; zero frames;
and planted mistakes that those pins catch."""
import numpy as np
import pytest

from oracle import OracleConfig, build_adjacency, power_iteration
from oracle.ritz_oracle import frame_band, frame_ritz
from paper_1907_02731_amd.synth import make_clip

CFG = OracleConfig(r_t=2, r_s=2, sigma_t=1.0, sigma_s=1.5, alpha=1.0, p=0.2)


def _clip(seed, T=9, H=7, W=8):
    return make_clip(T, H, W, seed=seed, n_blobs=1, noise_sigma=0.1, motion="drift",
                     dtype=np.float64)


def _dense(S, cfg=CFG):
    M = build_adjacency(S, None, cfg).toarray()
    assert np.allclose(M, M.T)
    lam, V = np.linalg.eigh(M)
    v1 = V[:, -1] * np.sign(V[:, -1].sum())
    return M, lam, v1


def _scaled_frames(v, shape, seed):
    T = shape[0]
    s = np.random.Generator(np.random.PCG64(seed)).uniform(0.2, 3.0, T)
    return (s[:, None] * v.reshape(T, -1)).ravel()


def test_band_equals_the_projected_matrix():
    S = _clip(1)
    M, _, _ = _dense(S)
    x = np.random.Generator(np.random.PCG64(5)).random(S.size)
    T, H, W = S.shape
    Q = np.zeros((S.size, T))
    for t in range(T):
        Q[t * H * W:(t + 1) * H * W, t] = x[t * H * W:(t + 1) * H * W]
    B, G = frame_band(lambda v: M @ v, x, S.shape)
    np.testing.assert_allclose(B, Q.T @ M @ Q, rtol=1e-12, atol=1e-12)
    np.testing.assert_allclose(np.diag(G), Q.T @ Q, rtol=1e-13, atol=0)
    # M couples frames at most r_t apart
    i, j = np.indices(B.shape)
    assert np.all(B[np.abs(i - j) > CFG.r_t] == 0.0)
    assert np.any(B[np.abs(i - j) == CFG.r_t] != 0.0)


@pytest.mark.parametrize("seed", [2, 3])
def test_recovers_the_eigenvector_from_frame_scaled_copies(seed):
    S = _clip(seed)
    M, lam, v1 = _dense(S)
    x = _scaled_frames(v1, S.shape, seed + 10)
    r = frame_ritz(lambda v: M @ v, x, S.shape)
    xr = r["x"] / np.linalg.norm(r["x"])
    assert float(xr @ v1) > 1.0 - 1e-12
    assert abs(r["mu"] - lam[-1]) <= 1e-12 * lam[-1]
    # positive overlap with the input
    assert float(r["x"] @ x) > 0.0


@pytest.mark.parametrize("seed", [4, 5, 6])
def test_ritz_value_lies_between_the_rayleigh_quotient_and_lambda_1(seed):
    S = _clip(seed, T=7, H=6, W=9)
    M, lam, v1 = _dense(S)
    rng = np.random.Generator(np.random.PCG64(seed))
    for x in (S.ravel().copy(), rng.random(S.size), v1 + 0.3 * rng.random(S.size)):
        rho = float(x @ M @ x) / float(x @ x)
        r = frame_ritz(lambda v: M @ v, x, S.shape)
        xr = r["x"]
        assert rho - 1e-12 * lam[-1] <= r["mu"] <= lam[-1] * (1 + 1e-12)
        # mu is the Rayleigh quotient of the refined vector
        assert abs(float(xr @ M @ xr) / float(xr @ xr) - r["mu"]) <= 1e-12 * lam[-1]


def test_zero_frames_get_zero_factors():
    S = _clip(7)
    M, _, v1 = _dense(S)
    T, H, W = S.shape
    x = v1.copy().reshape(T, -1)
    x[0] = 0.0
    x[3] = 0.0
    r = frame_ritz(lambda v: M @ v, x.ravel(), S.shape)
    assert r["a"][0] == 0.0 and r["a"][3] == 0.0
    assert np.all(np.isfinite(r["x"])) and np.count_nonzero(r["a"]) == T - 2


def test_refined_start_reaches_the_same_eigenvector_in_fewer_steps():
    """A longer clip (slowly converging temporal modes): a few plain steps,
    then the refinement, then plain steps to the tolerance, against plain
    steps from S."""
    cfg = OracleConfig(r_t=2, r_s=3, sigma_t=1.0, sigma_s=2.0, alpha=1.0, p=0.2)
    S = make_clip(40, 12, 16, seed=8, n_blobs=2, noise_sigma=0.15, motion="affine",
                  dtype=np.float64)
    M = build_adjacency(S, None, cfg)
    ap = lambda v: M @ v  # noqa: E731
    cold = power_iteration(ap, S.ravel(), 20000, 1e-7)
    x5 = power_iteration(ap, S.ravel(), 5, 0.0)["x"]
    r = frame_ritz(ap, x5, S.shape)
    warm = power_iteration(ap, r["x"], 20000, 1e-7)
    assert cold["converged"] and warm["converged"]
    assert 5 + warm["iters"] < cold["iters"]
    assert abs(warm["lam"] - cold["lam"]) <= 1e-10 * cold["lam"]


def test_planted_mistakes_fail_the_pins():
    S = _clip(2)
    M, lam, v1 = _dense(S)
    x = _scaled_frames(v1, S.shape, 12)
    B, G = frame_band(lambda v: M @ v, x, S.shape)
    T = S.shape[0]

    def refined(Bm, Gm):
        w, V = np.linalg.eigh(np.diag(Gm ** -0.5) @ Bm @ np.diag(Gm ** -0.5))
        a = V[:, -1] * Gm ** -0.5
        xr = (a[:, None] * x.reshape(T, -1)).ravel()
        return abs(float(xr @ v1)) / np.linalg.norm(xr)

    assert refined(B, G) > 1.0 - 1e-12  # the correct pencil
    assert refined(B, np.ones(T)) < 1.0 - 1e-4  # G dropped
    Bs = np.zeros_like(B)
    Bs[:, 1:] = B[:, :-1]  # band shifted by one frame
    Bs = 0.5 * (Bs + Bs.T)
    assert refined(Bs, G) < 1.0 - 1e-4
