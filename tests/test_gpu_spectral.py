"""sfseg_spectral_grad: the warm start's training loss on the error that
survives k power-iteration steps, L = 1 - cos(M^k x^, x*), and its gradient
dL/dx^ = M^k dL/dv, computed by the library (2k products through the step
kernel, float64 norms and loss sums) against the FP64 oracle
(``oracle.unet_oracle.spectral_cosine_loss`` over the explicit CSR matrix of
Eq. (2)).

Bars: |L_gpu - L_oracle| <= 1e-6 and relative L2 of the gradient <= 1e-5
(float32 products, about 1e-7 relative each, over 2k of them).
"""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

from oracle import OracleConfig, build_adjacency  # noqa: E402
from oracle import unet_oracle as U  # noqa: E402
from paper_1907_02731_amd import _lib  # noqa: E402
from paper_1907_02731_amd.solver import Solver  # noqa: E402
from paper_1907_02731_amd.synth import make_clip, random_vector  # noqa: E402

pytestmark = pytest.mark.gpu
DEV = "cuda:0"


def _t(a):
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.float32)).to(DEV)


CASES = [
    ((6, 24, 32), OracleConfig(r_t=1, r_s=2, sigma_t=1.0, sigma_s=1.0, alpha=1.0, p=0.2), 0),
    ((6, 24, 32), OracleConfig(r_t=1, r_s=2, sigma_t=1.0, sigma_s=1.0, alpha=1.0, p=0.2), 1),
    ((6, 24, 32), OracleConfig(r_t=1, r_s=2, sigma_t=1.0, sigma_s=1.0, alpha=1.0, p=0.2), 6),
    ((8, 64, 96), OracleConfig(r_t=2, r_s=5, sigma_t=1.0, sigma_s=2.0, alpha=1.0, p=0.2), 3),
]


@pytest.mark.parametrize("case", range(len(CASES)))
def test_spectral_grad_matches_the_oracle(case):
    shape, cfg, k = CASES[case]
    S = make_clip(*shape, seed=1500 + case, n_blobs=2, noise_sigma=0.12, motion="affine",
                  dtype=np.float32)
    xh = random_vector(shape, seed=1600 + case, dtype=np.float32) + 0.05
    target = make_clip(*shape, seed=1700 + case, n_blobs=1, noise_sigma=0.05, motion="drift",
                       dtype=np.float32) + 0.01
    M = build_adjacency(S.astype(np.float64), None, cfg)
    ref_loss, ref_g = U.spectral_cosine_loss(lambda v: M @ v, xh.astype(np.float64),
                                             target.astype(np.float64), k)
    with Solver(_t(S), r_t=cfg.r_t, r_s=cfg.r_s, sigma_t=cfg.sigma_t, sigma_s=cfg.sigma_s,
                alpha=cfg.alpha, p=cfg.p) as sol:
        g, loss = sol.spectral_grad(_t(xh), _t(target), k)
        g = g.cpu().numpy().astype(np.float64)
        # a second call reuses the work buffers and gives the same bits
        g2, loss2 = sol.spectral_grad(_t(xh), _t(target), k)
        assert np.array_equal(g2.cpu().numpy().astype(np.float64), g) and loss2 == loss
    rel = np.linalg.norm(g - ref_g) / np.linalg.norm(ref_g)
    print(f"k={k} {shape}: loss {loss:.6e} (oracle {ref_loss:.6e}), gradient rel L2 {rel:.2e}",
          flush=True)
    assert abs(loss - ref_loss) <= 1e-6
    assert rel <= 1e-5


def test_spectral_grad_rejects_bad_arguments():
    S = make_clip(4, 16, 16, seed=3, dtype=np.float32)
    with Solver(_t(S)) as sol:
        x = _t(S)
        with pytest.raises(_lib.SfsegError) as e:
            sol.spectral_grad(x, x, -1)
        assert e.value.status == _lib.SFSEG_ERR_INVALID_ARG
        with pytest.raises(_lib.SfsegError) as e:
            sol.spectral_grad(x, torch.zeros_like(x), 2)
        assert e.value.status == _lib.SFSEG_ERR_ZERO_NORM
        with pytest.raises(_lib.SfsegError) as e:
            sol.spectral_grad(x, x, 2, out=x)
        assert e.value.status == _lib.SFSEG_ERR_INVALID_ARG
