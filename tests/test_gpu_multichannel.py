"""Several pairwise feature channels (Sec. 3.3, Eq. (9)) on the GPU, through
the C-ABI, against the FP64 oracle: the multi-channel matrix is the sum of
the single-channel matrices of Eq. (2)."""
import ctypes

import numpy as np
import pytest

torch = pytest.importorskip("torch")

from oracle import OracleConfig, build_adjacency_multi, power_iteration  # noqa: E402
from paper_1907_02731_amd import _lib  # noqa: E402
from paper_1907_02731_amd.solver import Solver  # noqa: E402
from paper_1907_02731_amd.synth import feature_channels  # noqa: E402

pytestmark = pytest.mark.gpu
DEV = "cuda:0"
CFG = OracleConfig(r_t=1, r_s=2, sigma_t=1.0, sigma_s=1.0, alpha=1.0, p=0.2)
KW = dict(r_t=CFG.r_t, r_s=CFG.r_s, sigma_t=CFG.sigma_t, sigma_s=CFG.sigma_s, alpha=CFG.alpha,
          p=CFG.p)


def _t(a):
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.float32)).to(DEV)


def _f64(t):
    return t.cpu().numpy().astype(np.float64)


@pytest.fixture(scope="module")
def clip():
    Fs = feature_channels(8, 64, 96, seed=11, n_blobs=2, noise_sigma=0.1, motion="drift")
    S = Fs[0]
    return S, Fs, build_adjacency_multi(S.astype(np.float64), Fs.astype(np.float64), CFG)


@pytest.mark.parametrize("shape", [0, 1])
def test_apply_matches_oracle(clip, shape):
    S, Fs, M = clip
    r = np.random.Generator(np.random.PCG64(3))
    x = r.random(S.shape).astype(np.float32)
    with Solver(_t(S), _t(Fs), **KW) as sol:
        assert sol.n_features == 2
        sol.set_plan(shape, 1)
        y = _f64(sol.apply(_t(x))).ravel()
    ref = M @ x.astype(np.float64).ravel()
    err = np.linalg.norm(y - ref) / np.linalg.norm(ref)
    print(f"shape {shape}: rel L2 {err:.3e}", flush=True)
    assert err <= 1e-6


def test_trajectory_matches_oracle(clip):
    S, Fs, M = clip
    K = 50
    with Solver(_t(S), _t(Fs), **KW) as sol:
        res = sol.iterate(max_iters=K, tol=0.0)
        x = _f64(sol.eigvec()).ravel()
    ref = power_iteration(lambda v: M @ v, S.astype(np.float64).ravel(), K, 0.0)
    assert res.iters == K
    assert np.linalg.norm(x - ref["x"]) <= 1e-5
    assert abs(res.lam - ref["lam"]) <= 1e-6 * ref["lam"]


@pytest.mark.parametrize("shape,rs,rt", [((3, 17, 130), 2, 1), ((2, 3, 200), 8, 4),
                                         ((1, 1, 1), 1, 0)])
def test_ragged_and_edge_shapes(shape, rs, rt):
    cfg = OracleConfig(r_t=rt, r_s=rs, sigma_t=1.3, sigma_s=2.1, alpha=0.7, p=0.5)
    r = np.random.Generator(np.random.PCG64(sum(shape) + rs))
    S = r.random(shape).astype(np.float32)
    Fs = r.random((2,) + shape).astype(np.float32)
    x = (2 * r.random(shape) - 1).astype(np.float32)
    M = build_adjacency_multi(S.astype(np.float64), Fs.astype(np.float64), cfg)
    with Solver(_t(S), _t(Fs), r_t=rt, r_s=rs, sigma_t=1.3, sigma_s=2.1, alpha=0.7, p=0.5) as sol:
        y = _f64(sol.apply(_t(x))).ravel()
    ref = M @ x.astype(np.float64).ravel()
    assert np.linalg.norm(y - ref) <= 1e-6 * max(np.linalg.norm(ref), 1e-30)


def test_equal_channels_double_lambda_and_keep_the_vector(clip):
    S, Fs, _ = clip
    F = Fs[1]
    with Solver(_t(S), _t(F), **KW) as one:
        r1 = one.iterate(max_iters=40, tol=0.0)
        x1 = _f64(one.eigvec())
    with Solver(_t(S), _t(np.stack([F, F])), **KW) as two:
        r2 = two.iterate(max_iters=40, tol=0.0)
        x2 = _f64(two.eigvec())
    assert abs(r2.lam - 2.0 * r1.lam) <= 1e-6 * r2.lam
    assert np.linalg.norm(x2 - x1) <= 1e-6


def test_errors(clip):
    S, Fs, _ = clip
    L = _lib.lib()
    cfg = _lib.make_config(*S.shape, **KW)
    out = ctypes.c_void_p()
    s_, f_ = _t(S), _t(Fs)
    assert L.sfseg_create_mc(ctypes.byref(cfg), s_.data_ptr(), f_.data_ptr(), 3, None,
                             ctypes.byref(out)) == _lib.SFSEG_ERR_INVALID_ARG
    assert L.sfseg_create_mc(ctypes.byref(cfg), s_.data_ptr(), None, 2, None,
                             ctypes.byref(out)) == _lib.SFSEG_ERR_INVALID_ARG
    cfg16 = _lib.make_config(*S.shape, storage="bf16", **KW)
    assert L.sfseg_create_mc(ctypes.byref(cfg16), s_.data_ptr(), f_.data_ptr(), 2, None,
                             ctypes.byref(out)) == _lib.SFSEG_ERR_UNSUPPORTED
    assert not out.value


def test_full_size_sampled_rows():
    """70 x 480 x 854, r_s = 5, r_t = 2, two channels: 20,000 sampled rows of
    M x against the matrix-free FP64 oracle summed over channels."""
    from oracle.native import MatrixFree
    cfg = OracleConfig(r_t=2, r_s=5, sigma_t=1.0, sigma_s=2.0, alpha=1.0, p=0.2)
    Fs = feature_channels(70, 480, 854, seed=1)
    S = Fs[0]
    r = np.random.Generator(np.random.PCG64(12))
    x = r.random(S.shape).astype(np.float32)
    rows = np.sort(r.choice(S.size, size=20000, replace=False))
    with Solver(_t(S), _t(Fs), r_t=2, r_s=5, sigma_t=1.0, sigma_s=2.0, alpha=1.0, p=0.2) as sol:
        y = _f64(sol.apply(_t(x))).ravel()
    ref = sum(MatrixFree(S, F, cfg).apply_rows(x.astype(np.float64), rows) for F in Fs)
    assert np.max(np.abs(y[rows] - ref)) <= 1e-5 * np.max(np.abs(ref))
