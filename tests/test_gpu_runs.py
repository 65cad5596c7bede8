"""Work plans that cut each tile's frames into several runs, against the FP64
matrix-free oracle (Eq. (7)) and against each other.

A run of output frames [ta, tb) filters the input frames ta - r_t .. tb + r_t - 1;
frames outside the clip are zeros (the zero padding of the t filter) and are
not filtered at all, and the frame loop, which advances in whole turns of the
(2 r_t + 1)-frame register ring, stops at the run's last input frame.  One
application y = M x computes every output voxel with the same operations in
the same order whatever the plan, so the outputs of all plans must agree bit
for bit; the plan only changes which block computes a voxel.  Cases: runs
shorter than a ring turn, runs that start or end inside the clip's zero
padding, r_t from 1 to 4, both block shapes, float32 and bfloat16 storage
(every storage type keeps the tile's own x, w, F in a register shift ring).
"""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

from oracle import OracleConfig  # noqa: E402
from oracle.native import MatrixFree  # noqa: E402
from paper_1907_02731_amd.solver import Solver  # noqa: E402
from paper_1907_02731_amd.synth import make_clip, random_vector  # noqa: E402

pytestmark = pytest.mark.gpu
DEV = "cuda:0"

# (T, H, W, r_t, r_s): the largest plan has T // (4 r_t + 4) runs
CASES = [
    (36, 20, 70, 2, 3),   # 3 runs of 12 frames with r_t = 2
    (40, 18, 70, 1, 2),   # 5 runs of 8 frames with r_t = 1
    (41, 20, 70, 4, 2),   # 2 runs of 20/21 frames with r_t = 4
    (13, 17, 33, 2, 2),   # one run only: frames past the clip on both sides
]


def _cfg(r_t, r_s):
    return OracleConfig(r_t=r_t, r_s=r_s, sigma_t=1.3, sigma_s=1.7, alpha=1.0, p=0.2)


def _t(a):
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.float32)).to(DEV)


def _apply_all_plans(S, x, cfg, storage):
    out = {}
    with Solver(_t(S), None, r_t=cfg.r_t, r_s=cfg.r_s, sigma_t=cfg.sigma_t,
                sigma_s=cfg.sigma_s, alpha=cfg.alpha, p=cfg.p, storage=storage) as sol:
        top = max(1, S.shape[0] // (4 * cfg.r_t + 4))
        for shape in (0, 1):
            for chunks in range(1, top + 1):
                sol.set_plan(shape, chunks)
                pl = sol.plan()
                assert (pl["shape"], pl["chunks"]) == (shape, chunks)
                out[(shape, chunks)] = sol.apply(_t(x)).cpu().numpy()
    return out


@pytest.mark.parametrize("T,H,W,r_t,r_s", CASES)
def test_every_plan_applies_the_same_matrix(T, H, W, r_t, r_s):
    cfg = _cfg(r_t, r_s)
    S = make_clip(T, H, W, seed=T + r_t, n_blobs=2, noise_sigma=0.1, motion="drift",
                  dtype=np.float32)
    x = random_vector(S.shape, seed=r_s, dtype=np.float32)
    ys = _apply_all_plans(S, x, cfg, "f32")
    base = ys[(0, 1)]
    for plan, y in ys.items():
        np.testing.assert_array_equal(y, base, err_msg=f"plan {plan}")
    ref = MatrixFree(S, None, cfg).apply(x.astype(np.float64).ravel())
    y = base.astype(np.float64).ravel()
    nref = np.linalg.norm(ref)
    assert np.linalg.norm(y - ref) <= 1e-6 * nref
    assert np.max(np.abs(y - ref)) <= 1e-5 * np.max(np.abs(ref))
    # the first and last frames see the zero padding: check them on their own
    for t in (0, T - 1):
        sl = slice(t * H * W, (t + 1) * H * W)
        assert np.linalg.norm(y[sl] - ref[sl]) <= 1e-6 * max(np.linalg.norm(ref[sl]), 1e-30)


@pytest.mark.parametrize("T,H,W,r_t,r_s", CASES[:2])
def test_every_plan_applies_the_same_matrix_bf16(T, H, W, r_t, r_s):
    cfg = _cfg(r_t, r_s)
    S = make_clip(T, H, W, seed=T + r_t, n_blobs=2, noise_sigma=0.1, motion="drift",
                  dtype=np.float32)
    x = random_vector(S.shape, seed=r_s, dtype=np.float32)
    ys = _apply_all_plans(S, x, cfg, "bf16")
    base = ys[(0, 1)]
    for plan, y in ys.items():
        np.testing.assert_array_equal(y, base, err_msg=f"plan {plan}")
    # bfloat16 storage of x, w, F and y: 8 significant bits each
    ref = MatrixFree(S, None, cfg).apply(x.astype(np.float64).ravel())
    assert np.linalg.norm(base.astype(np.float64).ravel() - ref) <= 2e-2 * np.linalg.norm(ref)
