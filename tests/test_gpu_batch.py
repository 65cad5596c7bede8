"""Batched form: clips of uneven size iterated by one persistent launch per
step, each with its own convergence test.

Every clip of a batch must follow exactly the trajectory it follows alone
(same per-voxel arithmetic; only the grouping of the float64 norm sums
differs), match the FP64 oracle after the same number of steps, and stop at
its own step count.
"""
import json

import numpy as np
import pytest

torch = pytest.importorskip("torch")

from oracle import OracleConfig, build_adjacency, power_iteration  # noqa: E402
from paper_1907_02731_amd import _lib  # noqa: E402
from paper_1907_02731_amd.solver import BatchSolver, Solver  # noqa: E402
from paper_1907_02731_amd.synth import make_clip  # noqa: E402

pytestmark = pytest.mark.gpu
DEV = "cuda:0"
CFG = OracleConfig(r_t=1, r_s=2, sigma_t=1.0, sigma_s=1.0, alpha=1.0, p=0.2)
KW = dict(r_t=CFG.r_t, r_s=CFG.r_s, sigma_t=CFG.sigma_t, sigma_s=CFG.sigma_s, alpha=CFG.alpha,
          p=CFG.p)
SHAPES = [(8, 40, 70), (12, 33, 90), (5, 64, 64), (20, 20, 37), (3, 17, 130)]


def _t(a):
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.float32)).to(DEV)


@pytest.fixture(scope="module")
def clips():
    out = []
    for i, sh in enumerate(SHAPES):
        S = make_clip(*sh, seed=500 + i, n_blobs=2, noise_sigma=0.1, motion="drift",
                      dtype=np.float32)
        out.append((S, build_adjacency(S.astype(np.float64), None, CFG)))
    return out


def test_batch_trajectories_match_single_and_oracle(clips):
    K = 30
    with BatchSolver([_t(S) for S, _ in clips], **KW) as bs:
        assert len(bs) == len(clips)
        res = bs.iterate(max_iters=K, tol=0.0)
        xs = [x.cpu().numpy().astype(np.float64).ravel() for x in bs.eigvecs()]
    for (S, M), r, x in zip(clips, res, xs):
        assert r.iters == K
        with Solver(_t(S), **KW) as sol:
            r1 = sol.iterate(max_iters=K, tol=0.0)
            x1 = sol.eigvec().cpu().numpy().astype(np.float64).ravel()
        ref = power_iteration(lambda v: M @ v, S.astype(np.float64).ravel(), K, 0.0)
        assert np.linalg.norm(x - x1) <= 1e-6
        assert abs(r.lam - r1.lam) <= 1e-9 * r1.lam
        assert np.linalg.norm(x - ref["x"]) <= 1e-5


# Error budgets of the 16-bit storage forms against the FP64 oracle after 30
# steps (relative L2): one rounding of w, F and every iterate to 8 (bfloat16)
# or 11 (float16) significant bits.  The same bars as the single-clip form.
BUDGET16 = {"bf16": 5e-2, "f16": 1e-2}


@pytest.mark.parametrize("storage", ["bf16", "f16"])
def test_batch_16bit_storage_matches_single_and_budget(clips, storage):
    """The batched kernels with bfloat16 / float16 storage (own values of
    the tile in the register ring, as in the float32 form): every clip
    follows its single-clip trajectory, and stays within the storage error
    budget of the FP64 oracle."""
    K = 30
    with BatchSolver([_t(S) for S, _ in clips], storage=storage, **KW) as bs:
        res = bs.iterate(max_iters=K, tol=0.0)
        xs = [x.cpu().numpy().astype(np.float64).ravel() for x in bs.eigvecs()]
    for (S, M), r, x in zip(clips, res, xs):
        assert r.iters == K
        with Solver(_t(S), storage=storage, **KW) as sol:
            r1 = sol.iterate(max_iters=K, tol=0.0)
            x1 = sol.eigvec().cpu().numpy().astype(np.float64).ravel()
        ref = power_iteration(lambda v: M @ v, S.astype(np.float64).ravel(), K, 0.0)
        rel = np.linalg.norm(x - ref["x"]) / np.linalg.norm(ref["x"])
        print(f"{storage} {S.shape}: ||x_batch - x_single|| = {np.linalg.norm(x - x1):.3e}, "
              f"rel L2 vs oracle {rel:.3e}", flush=True)
        assert np.linalg.norm(x - x1) <= 1e-6
        assert abs(r.lam - r1.lam) <= 1e-9 * r1.lam
        assert rel <= BUDGET16[storage]
        assert np.all(x[S.ravel() == 0] == 0.0)


def test_each_clip_stops_on_its_own(clips):
    tol = 1e-5
    with BatchSolver([_t(S) for S, _ in clips], **KW) as bs:
        res = bs.iterate(max_iters=3000, tol=tol)
        xs = [x.cpu().numpy().astype(np.float64).ravel() for x in bs.eigvecs()]
        t = bs.timing()
    counts = [r.iters for r in res]
    print("iterations per clip:", counts, flush=True)
    assert all(r.converged and r.delta < tol for r in res)
    assert t["iters"] == max(counts)
    for (S, M), r, x in zip(clips, res, xs):
        ref = power_iteration(lambda v: M @ v, S.astype(np.float64).ravel(), 3000, tol)
        assert abs(ref["iters"] - r.iters) <= 1
        with Solver(_t(S), **KW) as sol:
            r1 = sol.iterate(max_iters=3000, tol=tol)
            x1 = sol.eigvec().cpu().numpy().astype(np.float64).ravel()
        assert abs(r1.iters - r.iters) <= 1
        if r1.iters == r.iters:
            assert np.linalg.norm(x - x1) <= 1e-6


@pytest.mark.parametrize("shape,chunks", [(0, 1), (1, 1), (0, 2), (1, 2)])
def test_batch_plans_agree(clips, shape, chunks):
    K = 20
    with BatchSolver([_t(S) for S, _ in clips], **KW) as bs:
        bs.set_plan(shape, chunks)
        pl = bs.plan()
        assert (pl["shape"], pl["chunks"]) == (shape, chunks)
        bs.iterate(max_iters=K, tol=0.0)
        xs = [x.cpu().numpy().astype(np.float64).ravel() for x in bs.eigvecs()]
    for (S, M), x in zip(clips, xs):
        ref = power_iteration(lambda v: M @ v, S.astype(np.float64).ravel(), K, 0.0)
        assert np.linalg.norm(x - ref["x"]) <= 1e-5


def test_batch_start_vectors_and_errors(clips):
    S0, M0 = clips[0]
    S1, _ = clips[1]
    x0 = np.random.Generator(np.random.PCG64(9)).random(S0.shape).astype(np.float32)
    with BatchSolver([_t(S0), _t(np.zeros(S1.shape, np.float32))], **KW) as bs:
        with pytest.raises(_lib.SfsegError) as e:
            bs.iterate([_t(x0), None], max_iters=10, tol=0.0)
        assert e.value.status == _lib.SFSEG_ERR_ZERO_NORM
        assert "clip 1" in str(e.value)
        # the healthy clip still has its result
        assert bs.last_results[0].iters == 10
    with BatchSolver([_t(S0)], **KW) as bs:
        bs.iterate([_t(x0)], max_iters=10, tol=0.0)
        x = bs.eigvecs()[0].cpu().numpy().astype(np.float64).ravel()
    ref = power_iteration(lambda v: M0 @ v, x0.astype(np.float64).ravel(), 10, 0.0)
    assert np.linalg.norm(x - ref["x"]) <= 1e-5


def test_batch_rejects_mixed_parameters_and_single_calls(clips):
    S0, _ = clips[0]
    with pytest.raises(_lib.SfsegError) as e:
        # second clip built with a different radius through the raw ABI
        cfgs = (_lib.Config * 2)(_lib.make_config(*S0.shape, **KW),
                                 _lib.make_config(*S0.shape, **dict(KW, r_s=3)))
        a, b = _t(S0), _t(S0)
        import ctypes
        ps = (ctypes.c_void_p * 2)(a.data_ptr(), b.data_ptr())
        out = ctypes.c_void_p()
        _lib.check(_lib.lib().sfseg_batch_create(cfgs, 2, ps, None, None, ctypes.byref(out)),
                   "sfseg_batch_create")
    assert e.value.status == _lib.SFSEG_ERR_INVALID_ARG
    with BatchSolver([_t(S0)], **KW) as bs:
        import ctypes
        res = _lib.Result()
        assert _lib.lib().sfseg_power_iterate(bs._handle(), None, 5, 0.0, ctypes.byref(res)) == \
            _lib.SFSEG_ERR_STATE


def test_autotune_single_and_batch_with_cache(clips, tmp_path):
    cache = str(tmp_path / "plans.json")
    S0, M0 = clips[0]
    with Solver(_t(S0), **KW) as sol:
        pl = sol.autotune(steps=4, cache=cache)
        assert not pl["cached"]
        sol.iterate(max_iters=15, tol=0.0)
        x = sol.eigvec().cpu().numpy().astype(np.float64).ravel()
    ref = power_iteration(lambda v: M0 @ v, S0.astype(np.float64).ravel(), 15, 0.0)
    assert np.linalg.norm(x - ref["x"]) <= 1e-5
    with Solver(_t(S0), **KW) as sol:
        pl2 = sol.autotune(steps=4, cache=cache)
        assert pl2["cached"] and (pl2["shape"], pl2["chunks"]) == (pl["shape"], pl["chunks"])
    with BatchSolver([_t(S) for S, _ in clips], **KW) as bs:
        pb = bs.autotune(steps=3, cache=cache)
        assert pb["threads"] in (256, 512)
    assert len(json.load(open(cache))) == 2


def test_batch_at_real_resolutions_matches_the_oracle():
    """Three clips at the batch workload's resolutions (240x427, 360x640,
    480x854) with the full-size graph (r_s = 5, r_t = 2, sigma_s = 2,
    sigma_t = 1): each clip's iterate after 3 batched steps against the
    matrix-free FP64 oracle."""
    from oracle.native import MatrixFree
    full = OracleConfig(r_t=2, r_s=5, sigma_t=1.0, sigma_s=2.0, alpha=1.0, p=0.2)
    shapes = [(20, 240, 427), (12, 360, 640), (8, 480, 854)]
    Ss = [make_clip(*sh, seed=700 + i, dtype=np.float32) for i, sh in enumerate(shapes)]
    K = 3
    with BatchSolver([_t(S) for S in Ss], r_t=2, r_s=5, sigma_t=1.0, sigma_s=2.0, alpha=1.0,
                     p=0.2) as bs:
        res = bs.iterate(max_iters=K, tol=0.0)
        xs = [x.cpu().numpy().astype(np.float64).ravel() for x in bs.eigvecs()]
    for S, r, x in zip(Ss, res, xs):
        mf = MatrixFree(S, None, full)
        ref = power_iteration(mf.apply, S.astype(np.float64).ravel(), K, 0.0)
        assert r.iters == K
        assert np.linalg.norm(x - ref["x"]) <= 1e-5
        assert abs(r.lam - ref["lam"]) <= 1e-6 * ref["lam"]


def test_batched_warm_start_reaches_the_same_eigenvectors():
    """The batched form started from the warm-start network's estimates (the
    shipped weights) on ragged clips of the benchmark's kind: per clip the
    same Rayleigh quotient as the plain method from S (to 1e-6), and the two
    vectors within the error that stopping at delta leaves, delta r / (1 - r)
    for each, r the contraction over the plain run's last 20 steps, with a
    factor 3 for steps before the asymptotic rate."""
    from paper_1907_02731_amd.synth import full_clip
    from paper_1907_02731_amd.warmstart import GRAPH, WEIGHTS, UNet, load_params
    shapes = [(24, 96, 160), (40, 120, 214), (33, 80, 150)]
    clips = [torch.from_numpy(full_clip(5000 + i, T=T, H=H, W=W)).to(DEV)
             for i, (T, H, W) in enumerate(shapes)]
    tol = 1e-5
    with UNet(tuple(max(s[d] for s in shapes) for d in range(3))) as net:
        net.set_params(load_params(WEIGHTS))
        x0s = [net.forward(S) for S in clips]
    with BatchSolver(clips, **GRAPH) as bs:
        rw = bs.iterate(x0s, max_iters=20000, tol=tol)
        xw = [x.cpu().numpy().astype(np.float64).ravel() for x in bs.eigvecs()]
    for i, S in enumerate(clips):
        with Solver(S, **GRAPH) as sol:
            rc = sol.iterate(max_iters=20000, tol=tol)
            xc = sol.eigvec().cpu().numpy().astype(np.float64).ravel()
            r20 = sol.iterate(max_iters=rc.iters - 20, tol=0.0)
        rate = (rc.delta / r20.delta) ** (1.0 / 20)
        bound = 3.0 * (rc.delta + rw[i].delta) * rate / (1.0 - rate)
        d = float(np.linalg.norm(xw[i] - xc))
        print(f"\nclip {shapes[i]}: plain {rc.iters} steps, batched warm {rw[i].iters}; "
              f"contraction {rate:.5f}, |x_w - x_c| {d:.2e} <= {bound:.2e}", flush=True)
        assert rc.converged and rw[i].converged
        assert abs(rw[i].lam - rc.lam) <= 1e-6 * rc.lam
        assert 0.0 < rate < 1.0 and d <= bound
