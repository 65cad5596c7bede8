"""GPU parity: the HIP path (through the C ABI) against the FP64 oracle.

Bars (float32 storage):
  * one operator application y = M x: ||y_gpu - y_oracle||_2 <= 1e-6 ||y_oracle||_2
    and max |y_gpu - y_oracle| <= 1e-5 max |y_oracle| (float32 sums of up to
    605 non-negative terms carry ~1e-7 relative rounding);
  * trajectories: the unit iterate after the same number of steps from the
    same start, ||x_gpu - x_oracle||_2 <= 1e-5;
  * invariants at any size: ||x|| = 1, x = 0 exactly where S = 0, and x >= 0
    up to float32 cancellation (x >= -1e-6 max x).
"""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

from oracle import OracleConfig, build_adjacency, power_iteration  # noqa: E402
from oracle.native import MatrixFree  # noqa: E402
from paper_1907_02731_amd import _lib  # noqa: E402
from paper_1907_02731_amd.solver import Solver  # noqa: E402
from paper_1907_02731_amd.synth import full_clip, make_clip, random_vector, tiny_clip  # noqa: E402

pytestmark = pytest.mark.gpu

DEV = "cuda:0"
TINY = OracleConfig(r_t=1, r_s=2, sigma_t=1.0, sigma_s=1.0, alpha=1.0, p=0.2)
FULL = OracleConfig(r_t=2, r_s=5, sigma_t=1.0, sigma_s=2.0, alpha=1.0, p=0.2)


def _t(a):
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.float32)).to(DEV)


def _solver(S, F=None, cfg=TINY, storage="f32"):
    return Solver(_t(S), None if F is None else _t(F), r_t=cfg.r_t, r_s=cfg.r_s,
                  sigma_t=cfg.sigma_t, sigma_s=cfg.sigma_s, alpha=cfg.alpha, p=cfg.p,
                  storage=storage)


def _f64(t):
    return t.detach().cpu().numpy().astype(np.float64)


def _check_apply(y_gpu, y_ref):
    y_gpu = y_gpu.ravel()
    y_ref = y_ref.ravel()
    nref = np.linalg.norm(y_ref)
    assert np.linalg.norm(y_gpu - y_ref) <= 1e-6 * max(nref, 1e-30)
    assert np.max(np.abs(y_gpu - y_ref)) <= 1e-5 * max(np.max(np.abs(y_ref)), 1e-30)


# ---------------------------------------------------------------------------
# Small volumes: explicit CSR oracle
# ---------------------------------------------------------------------------

@pytest.fixture(scope="module")
def tiny():
    S = tiny_clip(0).astype(np.float32)
    M = build_adjacency(S.astype(np.float64), None, TINY)
    return S, M


@pytest.mark.parametrize("which", ["S", "uniform", "signed"])
def test_apply_tiny_clip(tiny, which):
    S, M = tiny
    x = {"S": S, "uniform": random_vector(S.shape, seed=101, dtype=np.float32),
         "signed": random_vector(S.shape, seed=102, signed=True, dtype=np.float32)}[which]
    with _solver(S) as sol:
        y = _f64(sol.apply(_t(x)))
    _check_apply(y, M @ x.astype(np.float64).ravel())


CASES = [
    # shape, cfg: ragged tiles in x and y, radii larger than the volume, no
    # spatial / temporal neighbours, the largest compiled radii, single voxel.
    ((5, 37, 101), OracleConfig(r_t=2, r_s=3, sigma_t=0.8, sigma_s=1.5, alpha=1.0, p=0.2)),
    ((3, 17, 65), OracleConfig(r_t=1, r_s=5, sigma_t=1.0, sigma_s=2.0, alpha=0.7, p=0.5)),
    ((2, 3, 200), OracleConfig(r_t=4, r_s=8, sigma_t=2.0, sigma_s=3.0, alpha=1.0, p=0.1)),
    ((9, 16, 64), OracleConfig(r_t=3, r_s=0, sigma_t=1.2, sigma_s=1.0, alpha=1.0, p=0.2)),
    ((4, 33, 7), OracleConfig(r_t=0, r_s=1, sigma_t=1.0, sigma_s=0.7, alpha=2.0, p=1.0)),
    ((1, 1, 1), OracleConfig(r_t=0, r_s=0, sigma_t=1.0, sigma_s=1.0, alpha=1.0, p=0.2)),
    ((11, 20, 30), OracleConfig(r_t=2, r_s=2, sigma_t=1.0, sigma_s=1.0, alpha=0.0, p=0.0)),
]


@pytest.mark.parametrize("shape,cfg", CASES, ids=[str(c[0]) for c in CASES])
def test_apply_ragged_and_edge_shapes(shape, cfg):
    S = make_clip(*shape, seed=sum(shape), n_blobs=1, noise_sigma=0.15, dtype=np.float32) \
        if shape != (1, 1, 1) else np.full(shape, 0.6, np.float32)
    F = random_vector(shape, seed=7, dtype=np.float32)
    x = random_vector(shape, seed=8, signed=True, dtype=np.float32)
    M = build_adjacency(S.astype(np.float64), F.astype(np.float64), cfg)
    with _solver(S, F, cfg) as sol:
        y = _f64(sol.apply(_t(x)))
    _check_apply(y, M @ x.astype(np.float64).ravel())


def test_trajectory_tiny_clip(tiny):
    S, M = tiny
    with _solver(S) as sol:
        res = sol.iterate(max_iters=50, tol=1e-8)
        x = _f64(sol.eigvec()).ravel()
    ref = power_iteration(lambda v: M @ v, S.astype(np.float64).ravel(), res.iters, 0.0)
    assert res.iters == ref["iters"]
    assert np.linalg.norm(x - ref["x"]) <= 1e-5
    assert abs(res.lam - ref["lam"]) <= 1e-6 * ref["lam"]
    assert abs(res.delta - ref["delta"]) <= 1e-6
    # invariants
    assert abs(np.linalg.norm(x) - 1.0) <= 1e-6
    assert x.min() >= -1e-6 * x.max()   # Perron vector; float32 cancellation near zero
    assert np.all(x[S.ravel() == 0] == 0.0)


def test_separate_F_and_start_vector():
    shape = (6, 30, 70)
    S = make_clip(*shape, seed=201, n_blobs=2, noise_sigma=0.1, dtype=np.float32)
    F = random_vector(shape, seed=202, dtype=np.float32)
    x0 = random_vector(shape, seed=203, dtype=np.float32)
    cfg = OracleConfig(r_t=1, r_s=3, sigma_t=1.0, sigma_s=1.5, alpha=0.8, p=0.3)
    M = build_adjacency(S.astype(np.float64), F.astype(np.float64), cfg)
    with _solver(S, F, cfg) as sol:
        res = sol.iterate(_t(x0), max_iters=25, tol=0.0)
        x = _f64(sol.eigvec()).ravel()
    ref = power_iteration(lambda v: M @ v, x0.astype(np.float64).ravel(), 25, 0.0)
    assert res.iters == 25 and not res.converged
    assert np.linalg.norm(x - ref["x"]) <= 1e-5


def test_resume_from_eigvec_continues_the_trajectory(tiny):
    S, _ = tiny
    with _solver(S) as sol:
        sol.iterate(max_iters=20, tol=0.0)
        x20 = sol.eigvec().clone()
        sol.iterate(max_iters=10, tol=0.0)
        x10 = sol.eigvec().clone()
        sol.iterate(x10, max_iters=10, tol=0.0)
        x10_10 = _f64(sol.eigvec())
    assert np.linalg.norm(x10_10 - _f64(x20)) <= 1e-6


def test_converges_and_reports_delta(tiny):
    S, M = tiny
    with _solver(S) as sol:
        res = sol.iterate(max_iters=5000, tol=1e-5)
        x = _f64(sol.eigvec()).ravel()
        t = sol.timing()
    assert res.converged and res.delta < 1e-5
    assert t["iters"] == res.iters and t["launches"] >= res.iters
    # the oracle stops at the same step (same start, same rule)
    ref = power_iteration(lambda v: M @ v, S.astype(np.float64).ravel(), 5000, 1e-5)
    assert abs(ref["iters"] - res.iters) <= 1
    # Rayleigh quotient and residual of the returned vector, in float64
    y = M @ x
    lam = x @ y
    assert abs(res.lam - lam) <= 1e-5 * lam
    assert np.linalg.norm(y - lam * x) / lam <= 10 * res.delta + 1e-6


def test_max_iters_zero_returns_normalised_start(tiny):
    S, _ = tiny
    with _solver(S) as sol:
        res = sol.iterate(max_iters=0, tol=1e-5)
        x = _f64(sol.eigvec()).ravel()
    assert res.iters == 0
    s = S.astype(np.float64).ravel()
    assert np.linalg.norm(x - s / np.linalg.norm(s)) <= 1e-7


def test_bitwise_deterministic(tiny):
    S, _ = tiny
    outs = []
    for _ in range(2):
        with _solver(S) as sol:
            sol.iterate(max_iters=30, tol=0.0)
            outs.append(sol.eigvec().cpu().numpy())
    assert np.array_equal(outs[0], outs[1])


def test_error_paths():
    shape = (3, 8, 9)
    with _solver(np.zeros(shape, np.float32)) as sol:
        with pytest.raises(_lib.SfsegError) as e:
            sol.iterate(max_iters=5)
        assert e.value.status == _lib.SFSEG_ERR_ZERO_NORM
        with pytest.raises(_lib.SfsegError) as e:
            sol.eigvec()
        assert e.value.status == _lib.SFSEG_ERR_STATE
    S = np.full(shape, 0.5, np.float32)
    with _solver(S) as sol:
        with pytest.raises(_lib.SfsegError) as e:
            sol.iterate(_t(np.zeros(shape)), max_iters=5)
        assert e.value.status == _lib.SFSEG_ERR_ZERO_NORM
    bad = S.copy()
    bad[1, 2, 3] = np.nan
    with pytest.raises(_lib.SfsegError) as e:
        _solver(bad)
    assert e.value.status == _lib.SFSEG_ERR_NONFINITE
    neg = S.copy()
    neg[0, 0, 0] = -0.1
    with pytest.raises(_lib.SfsegError) as e:
        _solver(neg)
    assert e.value.status == _lib.SFSEG_ERR_NONFINITE


# ---------------------------------------------------------------------------
# Full-resolution clip, 70 x 480 x 854, r_s = 5, r_t = 2, sigma_s = 2, sigma_t = 1
# ---------------------------------------------------------------------------

@pytest.fixture(scope="module")
def full():
    S = full_clip(1)
    return S, MatrixFree(S, None, FULL)


def _sample_rows(shape, n, seed):
    T, H, W = shape
    rng = np.random.Generator(np.random.PCG64(seed))
    idx = rng.integers(0, T * H * W, size=n)
    # faces, edges and corners of the volume
    faces = []
    for t in (0, 1, T // 2, T - 2, T - 1):
        for y in (0, 1, 4, 5, H // 2, H - 6, H - 1):
            for x in (0, 3, 5, 63, 64, 69, W // 2, W - 7, W - 1):
                faces.append((t * H + y) * W + x)
    return np.concatenate([idx, np.array(faces, dtype=np.int64)])


def test_full_apply_sampled_rows(full):
    S, mf = full
    rows = _sample_rows(S.shape, 20000, seed=5)
    for x in (S, random_vector(S.shape, seed=301, signed=True, dtype=np.float32)):
        with _solver(S, cfg=FULL) as sol:
            y = _f64(sol.apply(_t(x))).ravel()
        ref = mf.apply_rows(x.astype(np.float64), rows)
        scale = np.max(np.abs(ref))
        assert np.max(np.abs(y[rows] - ref)) <= 1e-5 * scale


def test_full_trajectory_three_steps(full):
    S, mf = full
    with _solver(S, cfg=FULL) as sol:
        res = sol.iterate(max_iters=3, tol=0.0)
        x = _f64(sol.eigvec()).ravel()
    ref = power_iteration(mf.apply, S.astype(np.float64).ravel(), 3, 0.0)
    assert res.iters == 3
    assert np.linalg.norm(x - ref["x"]) <= 1e-5
    assert abs(res.lam - ref["lam"]) <= 1e-6 * ref["lam"]


def _toeplitz_power_ones(n, r, sigma, K):
    import scipy.linalg as sla
    col = np.zeros(n)
    m = min(n, r + 1)
    col[:m] = np.exp(-np.arange(m) ** 2 / (2.0 * sigma * sigma))
    A = sla.toeplitz(col)
    v = np.ones(n)
    for _ in range(K):
        v = A @ v
        v /= np.linalg.norm(v)
    return v


def test_full_separable_closed_form_trajectory():
    T, H, W, K = 70, 480, 854, 25
    S = np.ones((T, H, W), np.float32)
    F = np.full((T, H, W), 0.5, np.float32)
    with _solver(S, F, cfg=FULL) as sol:
        res = sol.iterate(max_iters=K, tol=0.0)
        x = _f64(sol.eigvec())
    at = _toeplitz_power_ones(T, FULL.r_t, FULL.sigma_t, K)
    ay = _toeplitz_power_ones(H, FULL.r_s, FULL.sigma_s, K)
    ax = _toeplitz_power_ones(W, FULL.r_s, FULL.sigma_s, K)
    v = at[:, None, None] * ay[None, :, None] * ax[None, None, :]
    v /= np.linalg.norm(v)
    assert res.iters == K
    assert np.linalg.norm(x - v) <= 1e-5


def test_full_converged_invariants(full):
    S, mf = full
    with _solver(S, cfg=FULL) as sol:
        res = sol.iterate(max_iters=3000, tol=1e-5)
        x = _f64(sol.eigvec()).ravel()
    print(f"full clip: iters={res.iters} converged={res.converged} delta={res.delta:.3e} "
          f"lambda={res.lam:.8f}", flush=True)
    assert res.converged
    assert abs(np.linalg.norm(x) - 1.0) <= 1e-6
    assert x.min() >= -1e-6 * x.max()   # Perron vector; float32 cancellation near zero
    assert np.all(x[S.ravel() == 0] == 0.0)
    y = mf.apply(x)
    lam = x @ y
    assert abs(res.lam - lam) <= 1e-5 * lam
    assert np.linalg.norm(y - lam * x) / lam <= 10 * res.delta + 1e-6


@pytest.fixture(scope="module")
def long_clip():
    # 24 frames: up to 3 runs of frames per tile with r_t = 1
    S = make_clip(24, 40, 70, seed=24, n_blobs=2, noise_sigma=0.1, motion="drift",
                  dtype=np.float32)
    return S, build_adjacency(S.astype(np.float64), None, TINY)


@pytest.mark.parametrize("shape,chunks", [(0, 1), (1, 1), (0, 2), (1, 3)])
def test_every_plan_gives_the_same_trajectory(long_clip, shape, chunks):
    S, M = long_clip
    with _solver(S) as sol:
        sol.set_plan(shape, chunks)
        pl = sol.plan()
        assert (pl["shape"], pl["chunks"]) == (shape, chunks)
        assert pl["blocks"] % 8 == 0 and pl["threads"] == (256 if shape == 0 else 512)
        y = _f64(sol.apply(_t(S)))
        sol.iterate(max_iters=30, tol=0.0)
        x = _f64(sol.eigvec()).ravel()
    _check_apply(y, M @ S.astype(np.float64).ravel())
    ref = power_iteration(lambda v: M @ v, S.astype(np.float64).ravel(), 30, 0.0)
    assert np.linalg.norm(x - ref["x"]) <= 1e-5


def test_plan_rejects_bad_values(tiny):
    S, _ = tiny
    with _solver(S) as sol:
        for shape, chunks in ((4, 1), (-1, 1), (0, 0), (0, 10_000)):
            with pytest.raises(_lib.SfsegError) as e:
                sol.set_plan(shape, chunks)
            assert e.value.status == _lib.SFSEG_ERR_INVALID_ARG
