"""Binarisation (Sec. 4.1; Algorithm 1, step 3) on the GPU, through the C-ABI,
against the FP64 oracle of ``oracle.binarize_oracle``.

Bars (float32 storage):
  * one projection of the same iterate: unit vectors within 1e-6 (L2); each
    P_i carries a few float32 roundings, amplified at most slope / 4 = 2.5 by
    the sigmoid;
  * Algorithm 1 (5 iterations, projection after 3 and 4): last unit power
    iterate within 1e-5 of the oracle's, lambda within 1e-6 relative;
  * hard threshold of a stored iterate the test controls (x0 with zero steps):
    bit-exact, ties included.  After Algorithm 1 the GPU thresholds its stored
    values while the test sees them scaled to unit norm (one more rounding), so
    mask and oracle may differ only within 4 float32 ulps of threshold * max;
    against the oracle's own FP64 run, only within the trajectory bar.
"""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

from oracle import OracleConfig, build_adjacency, power_iteration  # noqa: E402
from oracle.binarize_oracle import hard_threshold, project_binary, segment  # noqa: E402
from oracle.native import MatrixFree  # noqa: E402
from paper_1907_02731_amd import _lib  # noqa: E402
from paper_1907_02731_amd.solver import Solver  # noqa: E402
from paper_1907_02731_amd.synth import full_clip, random_vector, tiny_clip  # noqa: E402

pytestmark = pytest.mark.gpu
DEV = "cuda:0"
TINY = OracleConfig(r_t=1, r_s=2, sigma_t=1.0, sigma_s=1.0, alpha=1.0, p=0.2)
FULL = OracleConfig(r_t=2, r_s=5, sigma_t=1.0, sigma_s=2.0, alpha=1.0, p=0.2)


def _t(a, dtype=np.float32):
    return torch.from_numpy(np.ascontiguousarray(a, dtype=dtype)).to(DEV)


def _f64(t):
    return t.detach().cpu().numpy().astype(np.float64)


def _solver(S, cfg=TINY, storage="f32"):
    return Solver(_t(S), None, r_t=cfg.r_t, r_s=cfg.r_s, sigma_t=cfg.sigma_t,
                  sigma_s=cfg.sigma_s, alpha=cfg.alpha, p=cfg.p, storage=storage)


def _unit(v):
    v = np.asarray(v, dtype=np.float64).ravel()
    return v / np.linalg.norm(v)


@pytest.fixture(scope="module")
def tiny():
    S = tiny_clip(0).astype(np.float32)
    return S, build_adjacency(S.astype(np.float64), None, TINY)


@pytest.mark.parametrize("slope,thr", [(10.0, 0.5), (25.0, 0.3), (3.0, 0.8)])
def test_projection_of_the_same_iterate(tiny, slope, thr):
    S, _ = tiny
    with _solver(S) as sol:
        sol.iterate(max_iters=10, tol=0.0)
        x = _f64(sol.eigvec())
        sol.project(slope, thr)
        p = _f64(sol.eigvec()).ravel()
    ref = _unit(project_binary(x.ravel(), slope, thr))
    assert abs(np.linalg.norm(p) - 1.0) <= 1e-6
    assert np.linalg.norm(p - ref) <= 1e-6
    assert np.max(np.abs(p - ref)) <= 1e-6 * np.max(ref)


def test_algorithm_1_matches_oracle(tiny):
    S, M = tiny
    with _solver(S) as sol:
        res, mask = sol.segment()
        x = _f64(sol.eigvec()).ravel()
        m = mask.cpu().numpy().ravel().astype(bool)
    ref = segment(lambda v: M @ v, S.astype(np.float64).ravel(), 5, 3, 10.0, 0.5)
    assert res.iters == 5 and not res.converged
    assert np.linalg.norm(x - ref["x"]) <= 1e-5
    assert abs(res.lam - ref["lam"]) <= 1e-6 * ref["lam"]
    assert abs(res.delta - ref["delta"]) <= 1e-5
    _check_mask(m, x, ref, 0.5)


def _check_mask(m, x, ref, thr):
    xmax = x.max()
    band = np.abs(x - thr * xmax) <= 4 * np.finfo(np.float32).eps * xmax
    own = hard_threshold(x, thr)
    assert np.all((m == own) | band), int(np.sum((m != own) & ~band))
    z = ref["x"] / ref["x"].max()
    near = np.abs(z - thr) <= 2e-5
    assert np.all((m == ref["mask"]) | near)
    assert m.any() and not m.all()


@pytest.mark.parametrize("iters", [6, 20, 37])
def test_without_projection_is_the_plain_iteration(tiny, iters):
    # Algorithm 1 folds every step's sums inside the next step launch;
    # power iteration runs captured chunks of 16 steps and folds the last
    # step of each chunk in a one-block launch.  The fold is the same fixed
    # order wherever it runs, so the two agree bit for bit.
    S, _ = tiny
    with _solver(S) as sol:
        ra, _ = sol.segment(iters=iters, project_from=iters, mask=False)
        a = _f64(sol.eigvec())
        rb = sol.iterate(max_iters=iters, tol=0.0)
        b = _f64(sol.eigvec())
    np.testing.assert_array_equal(a, b)
    assert ra.iters == rb.iters == iters
    assert ra.lam == rb.lam and ra.delta == rb.delta


def test_threshold_is_exact_on_a_stored_iterate():
    # zero steps leave x0 itself (float32 storage) as the stored iterate
    shape = (3, 20, 77)
    r = np.random.Generator(np.random.PCG64(7))
    x0 = r.random(shape).astype(np.float32)
    x0.flat[5] = np.float32(4.0)  # the maximum
    thr = np.float32(0.3)
    at = np.float32(np.float64(thr) * 4.0)  # 1.2 rounded to float32
    x0.flat[10] = at
    x0.flat[11] = np.nextafter(at, np.float32(2))
    x0.flat[12] = np.nextafter(at, np.float32(0))
    S = np.ones(shape, dtype=np.float32)
    with _solver(S) as sol:
        sol.iterate(x0=_t(x0), max_iters=0, tol=0.0)
        for th in (float(thr), 0.0, 0.999, 1.0, -0.5):
            m = sol.threshold(th).cpu().numpy().astype(bool)
            np.testing.assert_array_equal(m, hard_threshold(x0.astype(np.float64),
                                                            float(np.float32(th))))


@pytest.mark.parametrize("shape,cfg", [
    ((5, 37, 101), OracleConfig(r_t=2, r_s=3, sigma_t=0.8, sigma_s=1.5, alpha=1.0, p=0.2)),
    ((2, 3, 200), OracleConfig(r_t=4, r_s=8, sigma_t=2.0, sigma_s=3.0, alpha=1.0, p=0.1)),
    ((1, 1, 1), OracleConfig(r_t=1, r_s=1, sigma_t=1.0, sigma_s=1.0, alpha=1.0, p=0.5)),
])
def test_ragged_and_edge_shapes(shape, cfg):
    r = np.random.Generator(np.random.PCG64(sum(shape)))
    S = r.random(shape).astype(np.float32)
    M = build_adjacency(S.astype(np.float64), None, cfg)
    with _solver(S, cfg) as sol:
        res, mask = sol.segment(iters=4, project_from=1, slope=8.0, threshold=0.4)
        x = _f64(sol.eigvec()).ravel()
        m = mask.cpu().numpy().ravel().astype(bool)
    ref = segment(lambda v: M @ v, S.astype(np.float64).ravel(), 4, 1, 8.0, 0.4)
    assert np.linalg.norm(x - ref["x"]) <= 1e-5
    xmax = x.max()
    band = np.abs(x - 0.4 * xmax) <= 4 * np.finfo(np.float32).eps * xmax
    assert np.all((m == hard_threshold(x, 0.4)) | band)


@pytest.mark.parametrize("storage,tol", [("bf16", 2e-2), ("f16", 4e-3)])
def test_sixteen_bit_storage(tiny, storage, tol):
    S, M = tiny
    with _solver(S, storage=storage) as sol:
        sol.segment(mask=False)
        x = _f64(sol.eigvec()).ravel()
    ref = segment(lambda v: M @ v, S.astype(np.float64).ravel(), 5, 3, 10.0, 0.5)
    assert np.linalg.norm(x - ref["x"]) <= tol


def test_errors(tiny):
    S, _ = tiny
    L = _lib.lib()
    with _solver(S) as sol:
        h = sol._handle()
        assert L.sfseg_project(h, 10.0, 0.5) == _lib.SFSEG_ERR_STATE  # no iterate yet
        sol.iterate(max_iters=2, tol=0.0)
        assert L.sfseg_project(h, 0.0, 0.5) == _lib.SFSEG_ERR_INVALID_ARG
        assert L.sfseg_project(h, float("inf"), 0.5) == _lib.SFSEG_ERR_INVALID_ARG
        assert L.sfseg_project(h, 10.0, float("nan")) == _lib.SFSEG_ERR_INVALID_ARG
        assert L.sfseg_threshold(h, 0.5, None) == _lib.SFSEG_ERR_INVALID_ARG
        b = _lib.Binarize(0, 1, 10.0, 0.5)
        assert L.sfseg_segment(h, None, b, None, None) == _lib.SFSEG_ERR_INVALID_ARG
        b = _lib.Binarize(5, 0, 10.0, 0.5)
        assert L.sfseg_segment(h, None, b, None, None) == _lib.SFSEG_ERR_INVALID_ARG
        # no positive entry: the projection refuses and leaves the iterate alone
        neg = -random_vector(S.shape, seed=3, dtype=np.float32)
        sol.iterate(x0=_t(neg), max_iters=0, tol=0.0)
        before = _f64(sol.eigvec())
        with pytest.raises(_lib.SfsegError) as e:
            sol.project()
        assert e.value.status == _lib.SFSEG_ERR_ZERO_NORM
        np.testing.assert_array_equal(_f64(sol.eigvec()), before)
        # and the context still works afterwards
        res, _ = sol.segment()
        assert res.iters == 5


def test_full_size_algorithm_1():
    S = full_clip(1)
    mf = MatrixFree(S, None, FULL)
    with _solver(S, FULL) as sol:
        res, mask = sol.segment()
        x = _f64(sol.eigvec()).ravel()
        m = mask.cpu().numpy().ravel().astype(bool)
    ref = segment(mf.apply, S.astype(np.float64).ravel(), 5, 3, 10.0, 0.5)
    assert np.linalg.norm(x - ref["x"]) <= 1e-5
    assert abs(res.lam - ref["lam"]) <= 1e-6 * ref["lam"]
    _check_mask(m, x, ref, 0.5)
