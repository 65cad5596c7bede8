"""The matrix-core step (plan shape 2): the y and x filter passes of Eq. (7)
as 16x16x32 float16 matrix products with float32 accumulation, every operand
split into float16 parts (data in two, the taps in three), against the FP64
oracle.

Bars are those of the float32 vector-ALU shapes: one application
||y - M x|| <= 1e-6 ||M x|| and max-abs <= 1e-5 max |M x| (ragged tiles,
every spatial radius 0..8 and temporal radius 0..2 the shape supports,
signed and non-negative x); trajectories ||x_gpu - x_oracle|| <= 1e-5 after
the same steps (tiny clip 50 steps, every frame-run plan, the full clip 100
steps); plans the shape does not support are rejected.
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
MFMA = 2
TINY = OracleConfig(r_t=1, r_s=2, sigma_t=1.0, sigma_s=1.0, alpha=1.0, p=0.2)
FULL = OracleConfig(r_t=2, r_s=5, sigma_t=1.0, sigma_s=2.0, alpha=1.0, p=0.2)


def _t(a):
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.float32)).to(DEV)


def _solver(S, cfg, F=None, storage="f32", chunks=1):
    sol = Solver(_t(S), None if F is None else _t(F), r_t=cfg.r_t, r_s=cfg.r_s,
                 sigma_t=cfg.sigma_t, sigma_s=cfg.sigma_s, alpha=cfg.alpha, p=cfg.p,
                 storage=storage)
    sol.set_plan(MFMA, chunks)
    return sol


def _check_apply(y, ref):
    y, ref = y.ravel(), ref.ravel()
    assert np.linalg.norm(y - ref) <= 1e-6 * np.linalg.norm(ref)
    assert np.max(np.abs(y - ref)) <= 1e-5 * np.max(np.abs(ref))


CASES = [
    # shape, graph: ragged tiles in x and y, every supported radius pair kind
    ((5, 37, 101), OracleConfig(r_t=2, r_s=3, sigma_t=0.8, sigma_s=1.5, alpha=1.0, p=0.2)),
    ((3, 17, 65), OracleConfig(r_t=1, r_s=5, sigma_t=1.0, sigma_s=2.0, alpha=0.7, p=0.5)),
    ((4, 40, 130), OracleConfig(r_t=2, r_s=8, sigma_t=1.0, sigma_s=3.0, alpha=1.0, p=0.1)),
    ((6, 16, 64), OracleConfig(r_t=0, r_s=0, sigma_t=1.0, sigma_s=1.0, alpha=1.0, p=0.2)),
    ((4, 33, 7), OracleConfig(r_t=0, r_s=1, sigma_t=1.0, sigma_s=0.7, alpha=2.0, p=1.0)),
    ((7, 20, 70), OracleConfig(r_t=2, r_s=6, sigma_t=1.5, sigma_s=2.5, alpha=1.0, p=0.2)),
    ((2, 3, 5), OracleConfig(r_t=1, r_s=4, sigma_t=1.0, sigma_s=2.0, alpha=1.0, p=0.2)),
    ((1, 1, 1), OracleConfig(r_t=0, r_s=0, sigma_t=1.0, sigma_s=1.0, alpha=1.0, p=0.2)),
]


@pytest.mark.parametrize("case", range(len(CASES)))
def test_mfma_apply_matches_the_oracle(case):
    shape, cfg = CASES[case]
    S = make_clip(*shape, seed=1200 + case, n_blobs=2, noise_sigma=0.1, motion="drift",
                  dtype=np.float32)
    F = random_vector(shape, seed=1300 + case, dtype=np.float32)
    M = build_adjacency(S.astype(np.float64), F.astype(np.float64), cfg)
    for x in (random_vector(shape, seed=1400 + case, signed=True, dtype=np.float32), S):
        with _solver(S, cfg, F) as sol:
            y = sol.apply(_t(x)).cpu().numpy().astype(np.float64)
        _check_apply(y, M @ x.astype(np.float64).ravel())


def test_mfma_trajectory_tiny_clip():
    S = tiny_clip(0).astype(np.float32)
    M = build_adjacency(S.astype(np.float64), None, TINY)
    K = 50
    with _solver(S, TINY) as sol:
        res = sol.iterate(max_iters=K, tol=0.0)
        x = sol.eigvec().cpu().numpy().astype(np.float64).ravel()
    ref = power_iteration(lambda v: M @ v, S.astype(np.float64).ravel(), K, 0.0)
    err = np.linalg.norm(x - ref["x"])
    print(f"mfma tiny clip K={K}: ||x - x_oracle|| = {err:.3e}", flush=True)
    assert res.iters == K
    assert err <= 1e-5
    assert abs(res.lam - ref["lam"]) <= 1e-6 * ref["lam"]


@pytest.mark.parametrize("chunks", [1, 2, 3])
def test_mfma_frame_runs_agree(chunks):
    S = make_clip(24, 40, 70, seed=24, n_blobs=2, noise_sigma=0.1, motion="drift",
                  dtype=np.float32)
    M = build_adjacency(S.astype(np.float64), None, TINY)
    with _solver(S, TINY, chunks=chunks) as sol:
        pl = sol.plan()
        assert (pl["shape"], pl["chunks"], pl["threads"]) == (MFMA, chunks, 256)
        y = sol.apply(_t(S)).cpu().numpy().astype(np.float64)
        sol.iterate(max_iters=30, tol=0.0)
        x = sol.eigvec().cpu().numpy().astype(np.float64).ravel()
    _check_apply(y, M @ S.astype(np.float64).ravel())
    ref = power_iteration(lambda v: M @ v, S.astype(np.float64).ravel(), 30, 0.0)
    assert np.linalg.norm(x - ref["x"]) <= 1e-5


def test_mfma_start_vector_far_outside_float16_range():
    # The step's scale enters the fields before they are split, so a start
    # vector of any magnitude gives the same trajectory.
    S = tiny_clip(0).astype(np.float32)
    M = build_adjacency(S.astype(np.float64), None, TINY)
    x0 = random_vector(S.shape, seed=77, dtype=np.float32)
    K = 20
    for scale in (1e-12, 1e12):
        with _solver(S, TINY) as sol:
            sol.iterate(_t(x0 * scale), max_iters=K, tol=0.0)
            x = sol.eigvec().cpu().numpy().astype(np.float64).ravel()
        ref = power_iteration(lambda v: M @ v, x0.astype(np.float64).ravel(), K, 0.0)
        assert np.linalg.norm(x - ref["x"]) <= 1e-5


def test_mfma_full_clip_100_steps():
    S = full_clip(1)
    mf = MatrixFree(S, None, FULL)
    rows = np.random.Generator(np.random.PCG64(5)).integers(0, S.size, size=20000)
    with _solver(S, FULL, chunks=3) as sol:
        y = sol.apply(_t(S)).cpu().numpy().astype(np.float64).ravel()
        res = sol.iterate(max_iters=100, tol=0.0)
        x = sol.eigvec().cpu().numpy().astype(np.float64).ravel()
    ref_rows = mf.apply_rows(S.astype(np.float64), rows)
    assert np.max(np.abs(y[rows] - ref_rows)) <= 1e-5 * np.max(np.abs(ref_rows))
    ref = power_iteration(mf.apply, S.astype(np.float64).ravel(), 100, 0.0)
    err = float(np.linalg.norm(x - ref["x"]))
    print(f"mfma full clip K=100: ||x - x_oracle|| = {err:.3e}, lambda rel "
          f"{abs(res.lam - ref['lam']) / ref['lam']:.3e}", flush=True)
    assert err <= 1e-5
    assert abs(res.lam - ref["lam"]) <= 1e-6 * ref["lam"]


def test_mfma_shape_rejected_where_it_does_not_exist():
    S = tiny_clip(0).astype(np.float32)
    kw = dict(r_s=2, sigma_t=1.0, sigma_s=1.0, alpha=1.0, p=0.2)
    for storage, r_t in (("bf16", 1), ("f16", 1), ("f32", 3)):
        with Solver(_t(S), r_t=r_t, storage=storage, **kw) as sol:
            with pytest.raises(_lib.SfsegError) as e:
                sol.set_plan(MFMA, 1)
            assert e.value.status == _lib.SFSEG_ERR_UNSUPPORTED
