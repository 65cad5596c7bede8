"""The frame-wise Rayleigh-Ritz refinement (sfseg_refine_frames) against the
FP64 oracle (``oracle/ritz_oracle.py``), and the refined warm start against
the plain method.

The GPU forms the band matrix B[i][j] = q_i^T M q_j with 2 r_t + 1 products
(one per residue class of frames) and solves the small pencil on the host;
the oracle applies M to every frame separately and calls a dense generalized
symmetric eigensolver.  Both refine the same vector: the GPU's iterate after a
few steps, as read back through sfseg_eigvec.  Bars: the refined unit vector
within 1e-5 (relative L2, float32 storage) of the oracle's, the Ritz value
within 1e-6; bfloat16 storage (products rounded to 8 bits) within 3e-2.
"""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

from oracle import OracleConfig  # noqa: E402
from oracle.native import MatrixFree  # noqa: E402
from oracle.ritz_oracle import frame_ritz  # noqa: E402
from paper_1907_02731_amd import _lib  # noqa: E402
from paper_1907_02731_amd.solver import BatchSolver, Solver  # noqa: E402
from paper_1907_02731_amd.synth import make_clip, tiny_clip  # noqa: E402

pytestmark = pytest.mark.gpu

DEV = "cuda:0"

CASES = [
    # shape, graph: ragged tiles, every temporal radius kind, a single frame
    ((8, 64, 96), OracleConfig(r_t=1, r_s=2, sigma_t=1.0, sigma_s=1.0, alpha=1.0, p=0.2)),
    ((11, 37, 101), OracleConfig(r_t=2, r_s=3, sigma_t=1.0, sigma_s=1.5, alpha=1.0, p=0.2)),
    ((20, 24, 40), OracleConfig(r_t=2, r_s=5, sigma_t=1.0, sigma_s=2.0, alpha=1.0, p=0.2)),
    ((13, 17, 33), OracleConfig(r_t=4, r_s=2, sigma_t=2.0, sigma_s=1.0, alpha=0.7, p=0.5)),
    ((6, 16, 20), OracleConfig(r_t=0, r_s=1, sigma_t=1.0, sigma_s=1.0, alpha=1.0, p=0.2)),
    ((1, 30, 50), OracleConfig(r_t=2, r_s=2, sigma_t=1.0, sigma_s=1.0, alpha=1.0, p=0.2)),
]


def _t(a):
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.float32)).to(DEV)


def _kw(cfg):
    return dict(r_t=cfg.r_t, r_s=cfg.r_s, sigma_t=cfg.sigma_t, sigma_s=cfg.sigma_s,
                alpha=cfg.alpha, p=cfg.p)


def _clip(shape, seed):
    T, H, W = shape
    return make_clip(T, H, W, seed=seed, n_blobs=2, noise_sigma=0.15, motion="affine",
                     dtype=np.float32)


def _refine_both(S, cfg, storage="f32", pre=3):
    with Solver(_t(S), storage=storage, **_kw(cfg)) as sol:
        sol.iterate(max_iters=pre, tol=0.0)
        xk = sol.eigvec().cpu().numpy().astype(np.float64).ravel()
        xg, mu = sol.refine_frames()
        xg = xg.cpu().numpy().astype(np.float64).ravel()
        xg2, mu2 = sol.refine_frames()
        assert np.array_equal(xg, xg2.cpu().numpy().astype(np.float64).ravel()) and mu == mu2
    ref = frame_ritz(MatrixFree(S, None, cfg).apply, xk, S.shape)
    xr = ref["x"] / np.linalg.norm(ref["x"])
    return xk, xg, mu, xr, ref


@pytest.mark.parametrize("case", range(len(CASES)))
def test_refinement_matches_the_oracle(case):
    shape, cfg = CASES[case]
    S = _clip(shape, 40 + case)
    xk, xg, mu, xr, ref = _refine_both(S, cfg)
    err = float(np.linalg.norm(xg - xr))
    print(f"\n{shape} r_t={cfg.r_t}: |x_gpu - x_oracle| = {err:.2e}, mu {mu:.10f} oracle "
          f"{ref['mu']:.10f}", flush=True)
    assert abs(np.linalg.norm(xg) - 1.0) <= 1e-6
    assert err <= 1e-5
    assert abs(mu - ref["mu"]) <= 1e-6 * abs(ref["mu"])
    # the refined vector's Rayleigh quotient is mu, not below the input's
    y = MatrixFree(S, None, cfg).apply(xk / np.linalg.norm(xk))
    assert mu >= float(xk @ y) / float(xk @ xk) * (1 - 1e-6)


@pytest.mark.parametrize("plan", [(1, 1), (2, 1), (3, 1)])
def test_refinement_on_every_plan_shape(plan):
    """The products go through the context's step kernel in its one-
    application mode: the 512-thread shape, the matrix-core shape and the
    two-step shape give the same refinement to float32 rounding."""
    shape, cfg = CASES[2]
    S = _clip(shape, 50)
    with Solver(_t(S), **_kw(cfg)) as sol:
        sol.set_plan(*plan)
        sol.iterate(max_iters=2, tol=0.0)
        xk = sol.eigvec().cpu().numpy().astype(np.float64).ravel()
        xg, mu = sol.refine_frames()
        xg = xg.cpu().numpy().astype(np.float64).ravel()
    ref = frame_ritz(MatrixFree(S, None, cfg).apply, xk, S.shape)
    xr = ref["x"] / np.linalg.norm(ref["x"])
    err = float(np.linalg.norm(xg - xr))
    print(f"\nplan {plan}: |x_gpu - x_oracle| = {err:.2e}", flush=True)
    assert err <= 1e-5 and abs(mu - ref["mu"]) <= 1e-6 * ref["mu"]


def test_refinement_bf16_storage_within_budget():
    shape, cfg = CASES[2]
    S = _clip(shape, 7)
    _, xg, mu, xr, ref = _refine_both(S, cfg, storage="bf16")
    err = float(np.linalg.norm(xg - xr))
    print(f"\nbf16: |x_gpu - x_oracle| = {err:.2e}, mu rel {abs(mu - ref['mu']) / ref['mu']:.2e}",
          flush=True)
    assert err <= 3e-2 and abs(mu - ref["mu"]) <= 1e-2 * ref["mu"]


def test_zero_frames_stay_zero():
    shape, cfg = CASES[1]
    S = _clip(shape, 9)
    S[0] = 0.0
    S[4] = 0.0
    with Solver(_t(S), **_kw(cfg)) as sol:
        sol.iterate(max_iters=1, tol=0.0)
        x, mu = sol.refine_frames()
        x = x.cpu().numpy()
    # w = S^p is zero on those frames, so is every iterate, and so is the refinement
    assert np.all(x[0] == 0.0) and np.all(x[4] == 0.0)
    assert np.all(np.isfinite(x)) and abs(float(np.linalg.norm(x)) - 1.0) <= 1e-6


def test_refined_warm_start_reaches_the_same_eigenvector_in_fewer_steps():
    """A 40-frame clip: plain steps from S against pre-steps + refinement +
    plain steps, both to delta < 1e-6.  Same Rayleigh quotient; the two
    vectors within the error that stopping at delta leaves, delta r / (1 - r)
    for each, r the contraction over the cold run's last 20 steps, with a
    factor 3 for steps before the asymptotic rate."""
    cfg = OracleConfig(r_t=2, r_s=5, sigma_t=1.0, sigma_s=2.0, alpha=1.0, p=0.2)
    S = make_clip(40, 96, 160, seed=11, n_blobs=3, noise_sigma=0.15, motion="affine",
                  dtype=np.float32)
    tol = 1e-6
    with Solver(_t(S), **_kw(cfg)) as sol:
        rc = sol.iterate(max_iters=20000, tol=tol)
        xc = sol.eigvec().cpu().numpy().astype(np.float64).ravel()
        r20 = sol.iterate(max_iters=rc.iters - 20, tol=0.0)
        rw, steps, mus = sol.iterate_refined(pre_steps=5, max_iters=20000, tol=tol)
        xw = sol.eigvec().cpu().numpy().astype(np.float64).ravel()
    rate = (rc.delta / r20.delta) ** (1.0 / 20)
    bound = 3.0 * (rc.delta + rw.delta) * rate / (1.0 - rate)
    d = float(np.linalg.norm(xw - xc))
    print(f"\ncold {rc.iters} steps, refined {steps} steps (Ritz value {mus[0]:.8f}, lambda "
          f"{rc.lam:.8f}); contraction {rate:.5f}, |x_w - x_c| {d:.2e} <= {bound:.2e}", flush=True)
    assert rc.converged and rw.converged
    assert steps < rc.iters
    assert abs(rw.lam - rc.lam) <= 1e-6 * rc.lam
    assert mus[0] <= rc.lam * (1 + 1e-6)
    assert d <= bound


def test_refinement_state_errors():
    S = tiny_clip(1).astype(np.float32)
    cfg = CASES[0][1]
    with Solver(_t(S), **_kw(cfg)) as sol:
        with pytest.raises(_lib.SfsegError) as e:
            sol.refine_frames()
        assert e.value.status == _lib.SFSEG_ERR_STATE
    with BatchSolver([_t(S)], **_kw(cfg)) as bs:
        L = _lib.lib()
        out = torch.empty(S.shape, dtype=torch.float32, device=DEV)
        assert L.sfseg_refine_frames(bs._ctx, out.data_ptr(), None) == _lib.SFSEG_ERR_STATE
