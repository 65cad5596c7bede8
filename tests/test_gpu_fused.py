"""Two power-iteration steps per pass over HBM (plan shape 3, temporal
blocking): each launch computes Y2 = c M (c M Y0) on a 32 x 8 tile, with the
intermediate iterate and its r_s halo recomputed in LDS, and leaves both
steps' float64 sums for the next fold.

Against the FP64 oracle: one application (the one-step mode) within the
apply bar on ragged shapes and every supported radius pair; trajectories of
even and odd step counts (an odd count ends with a one-step launch) within
1e-5, with the Rayleigh quotient and the change of the last step; a
tolerance between two oracle steps stops the fused plan on a whole pair;
frame runs; the full clip after 100 steps; Algorithm 1's binarised run on
the fused plan; unsupported storage types and radii are rejected.
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
FUSED = 3
TINY = OracleConfig(r_t=1, r_s=2, sigma_t=1.0, sigma_s=1.0, alpha=1.0, p=0.2)
FULL = OracleConfig(r_t=2, r_s=5, sigma_t=1.0, sigma_s=2.0, alpha=1.0, p=0.2)


def _t(a):
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.float32)).to(DEV)


def _solver(S, cfg, F=None, chunks=1, shape=FUSED):
    sol = Solver(_t(S), None if F is None else _t(F), r_t=cfg.r_t, r_s=cfg.r_s,
                 sigma_t=cfg.sigma_t, sigma_s=cfg.sigma_s, alpha=cfg.alpha, p=cfg.p)
    sol.set_plan(shape, chunks)
    return sol


CASES = [
    ((5, 37, 101), OracleConfig(r_t=2, r_s=3, sigma_t=0.8, sigma_s=1.5, alpha=1.0, p=0.2)),
    ((3, 17, 65), OracleConfig(r_t=1, r_s=5, sigma_t=1.0, sigma_s=2.0, alpha=0.7, p=0.5)),
    ((9, 24, 40), OracleConfig(r_t=2, r_s=5, sigma_t=1.0, sigma_s=2.0, alpha=1.0, p=0.2)),
    ((6, 16, 64), OracleConfig(r_t=0, r_s=0, sigma_t=1.0, sigma_s=1.0, alpha=1.0, p=0.2)),
    ((4, 33, 7), OracleConfig(r_t=0, r_s=1, sigma_t=1.0, sigma_s=0.7, alpha=2.0, p=1.0)),
    ((2, 3, 5), OracleConfig(r_t=1, r_s=4, sigma_t=1.0, sigma_s=2.0, alpha=1.0, p=0.2)),
    ((1, 1, 1), OracleConfig(r_t=0, r_s=0, sigma_t=1.0, sigma_s=1.0, alpha=1.0, p=0.2)),
]


@pytest.mark.parametrize("case", range(len(CASES)))
def test_fused_apply_matches_the_oracle(case):
    shape, cfg = CASES[case]
    S = make_clip(*shape, seed=1800 + case, n_blobs=2, noise_sigma=0.1, motion="drift",
                  dtype=np.float32)
    F = random_vector(shape, seed=1900 + case, dtype=np.float32)
    M = build_adjacency(S.astype(np.float64), F.astype(np.float64), cfg)
    for x in (random_vector(shape, seed=2000 + case, signed=True, dtype=np.float32), S):
        with _solver(S, cfg, F) as sol:
            y = sol.apply(_t(x)).cpu().numpy().astype(np.float64).ravel()
        ref = M @ x.astype(np.float64).ravel()
        assert np.linalg.norm(y - ref) <= 1e-6 * np.linalg.norm(ref)
        assert np.max(np.abs(y - ref)) <= 1e-5 * np.max(np.abs(ref))


@pytest.mark.parametrize("case,K", [(0, 1), (0, 2), (0, 30), (0, 31), (2, 17), (2, 40)])
def test_fused_trajectories_match_the_oracle(case, K):
    shape, cfg = CASES[case]
    S = make_clip(*shape, seed=2100 + case, n_blobs=2, noise_sigma=0.1, motion="affine",
                  dtype=np.float32)
    M = build_adjacency(S.astype(np.float64), None, cfg)
    with _solver(S, cfg) as sol:
        res = sol.iterate(max_iters=K, tol=0.0)
        x = sol.eigvec().cpu().numpy().astype(np.float64).ravel()
    ref = power_iteration(lambda v: M @ v, S.astype(np.float64).ravel(), K, 0.0)
    err = np.linalg.norm(x - ref["x"])
    print(f"fused {shape} K={K}: ||x - x_oracle|| = {err:.3e}", flush=True)
    assert res.iters == K
    assert err <= 1e-5
    assert abs(res.lam - ref["lam"]) <= 1e-6 * abs(ref["lam"])
    assert abs(res.delta - ref["delta"]) <= 1e-4 * ref["delta"] + 1e-7


def test_fused_tolerance_stops_on_a_whole_pair():
    S = tiny_clip(0).astype(np.float32)
    M = build_adjacency(S.astype(np.float64), None, TINY)
    ref = power_iteration(lambda v: M @ v, S.astype(np.float64).ravel(), 60, 0.0,
                          keep_history=True)
    hist = ref["history"]
    deltas = [np.linalg.norm(hist[k] - hist[k - 1]) for k in range(1, len(hist))]
    for k in (20, 21):  # the tolerance first met after an odd and after an even step
        tol = 0.5 * (deltas[k - 1] + deltas[k - 2])  # delta_k < tol <= delta_{k-1}
        with _solver(S, TINY) as sol:
            res = sol.iterate(max_iters=1000, tol=tol)
            x = sol.eigvec().cpu().numpy().astype(np.float64).ravel()
        want = k if k % 2 == 0 else k + 1  # launches take two steps
        assert res.converged and res.iters == want
        assert np.linalg.norm(x - hist[want]) <= 1e-5


@pytest.mark.parametrize("chunks", [1, 2, 3])
def test_fused_frame_runs_agree(chunks):
    S = make_clip(24, 40, 70, seed=24, n_blobs=2, noise_sigma=0.1, motion="drift",
                  dtype=np.float32)
    M = build_adjacency(S.astype(np.float64), None, TINY)
    with _solver(S, TINY, chunks=chunks) as sol:
        pl = sol.plan()
        assert (pl["shape"], pl["chunks"], pl["threads"]) == (FUSED, chunks, 256)
        sol.iterate(max_iters=30, tol=0.0)
        x = sol.eigvec().cpu().numpy().astype(np.float64).ravel()
    ref = power_iteration(lambda v: M @ v, S.astype(np.float64).ravel(), 30, 0.0)
    assert np.linalg.norm(x - ref["x"]) <= 1e-5


def test_fused_binarised_run_matches_the_default_plan():
    S = tiny_clip(0).astype(np.float32)
    outs = []
    for shape in (0, FUSED):
        with _solver(S, TINY, shape=shape) as sol:
            mask = torch.empty(S.shape, dtype=torch.uint8, device=DEV)
            res = sol.segment(iters=5, project_from=3, slope=10.0, threshold=0.5, out=mask)[0]
            outs.append((res.lam, sol.eigvec().cpu().numpy().astype(np.float64).ravel()))
    assert abs(outs[0][0] - outs[1][0]) <= 1e-6 * abs(outs[0][0])
    assert np.linalg.norm(outs[0][1] - outs[1][1]) <= 1e-5


def test_fused_full_clip_100_steps():
    S = full_clip(1)
    mf = MatrixFree(S, None, FULL)
    with _solver(S, FULL, chunks=1) as sol:
        res = sol.iterate(max_iters=100, tol=0.0)
        x = sol.eigvec().cpu().numpy().astype(np.float64).ravel()
        t = sol.timing()
    ref = power_iteration(mf.apply, S.astype(np.float64).ravel(), 100, 0.0)
    err = float(np.linalg.norm(x - ref["x"]))
    print(f"fused full clip K=100: ||x - x_oracle|| = {err:.3e}, {t['loop_ms'] * 10:.1f} us "
          f"per step", flush=True)
    assert err <= 1e-5
    assert abs(res.lam - ref["lam"]) <= 1e-6 * ref["lam"]


def test_fused_shape_rejected_where_it_does_not_exist():
    S = tiny_clip(0).astype(np.float32)
    for storage, r_s, r_t in (("bf16", 2, 1), ("f32", 6, 1), ("f32", 2, 3)):
        with Solver(_t(S), r_t=r_t, r_s=r_s, storage=storage) as sol:
            with pytest.raises(_lib.SfsegError) as e:
                sol.set_plan(FUSED, 1)
            assert e.value.status == _lib.SFSEG_ERR_UNSUPPORTED
