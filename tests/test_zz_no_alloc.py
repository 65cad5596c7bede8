"""sfseg_apply_noalloc: one application y = M x whose staging volumes, state
slots and partial sums live in the library's static per-GPU array instead of
memory allocated by the call.

Checked through the C ABI against sfseg_apply (the same kernels: equal bit
for bit) and against the FP64 oracle (the apply bar of the parity tests), on
two calls in a row where the second context's volume is smaller than the
first's, so stale contents the first call left in the array must not leak
into the second; float32 and bfloat16 storage; and the host-side rejection
of a volume larger than the array.
"""
import ctypes

import numpy as np
import pytest

torch = pytest.importorskip("torch")

from oracle import OracleConfig, build_adjacency  # noqa: E402
from paper_1907_02731_amd import _lib  # noqa: E402
from paper_1907_02731_amd.solver import Solver  # noqa: E402
from paper_1907_02731_amd.synth import make_clip, random_vector  # noqa: E402

pytestmark = pytest.mark.gpu
DEV = "cuda:0"

CASES = [
    # (shape, graph): the larger first, then a smaller, ragged one
    ((6, 37, 101), OracleConfig(r_t=2, r_s=3, sigma_t=0.8, sigma_s=1.5, alpha=1.0, p=0.2)),
    ((3, 17, 65), OracleConfig(r_t=1, r_s=5, sigma_t=1.0, sigma_s=2.0, alpha=0.7, p=0.5)),
]


def _t(a):
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.float32)).to(DEV)


def _noalloc(sol, x):
    y = torch.full(sol.shape, float("nan"), dtype=torch.float32, device=DEV)
    torch.cuda.synchronize()
    L = _lib.lib()
    assert L.sfseg_apply_noalloc_bytes(sol._handle()) <= (64 << 20)
    _lib.check(L.sfseg_apply_noalloc(sol._handle(), ctypes.c_void_p(x.data_ptr()),
                                     ctypes.c_void_p(y.data_ptr())), "sfseg_apply_noalloc")
    sol.stream.synchronize()
    return y


@pytest.mark.parametrize("storage", ["f32", "bf16"])
def test_noalloc_apply_equals_apply_on_two_calls(storage):
    for i, (shape, cfg) in enumerate(CASES):
        S = make_clip(*shape, seed=900 + i, n_blobs=2, noise_sigma=0.1, motion="drift",
                      dtype=np.float32)
        x = random_vector(shape, seed=910 + i, signed=True, dtype=np.float32)
        print(f"no-alloc apply: case {i} shape {shape} storage {storage}", flush=True)
        with Solver(_t(S), r_t=cfg.r_t, r_s=cfg.r_s, sigma_t=cfg.sigma_t, sigma_s=cfg.sigma_s,
                    alpha=cfg.alpha, p=cfg.p, storage=storage) as sol:
            xt = _t(x)
            y_ref = sol.apply(xt).cpu().numpy()
            y = _noalloc(sol, xt).cpu().numpy()
            # a second call on the same context gives the same bits again
            y2 = _noalloc(sol, xt).cpu().numpy()
        assert np.array_equal(y, y_ref)
        assert np.array_equal(y2, y_ref)
        if storage == "f32":
            M = build_adjacency(S.astype(np.float64), None, cfg)
            ref = M @ x.astype(np.float64).ravel()
            yy = y.astype(np.float64).ravel()
            assert np.linalg.norm(yy - ref) <= 1e-6 * np.linalg.norm(ref)
            assert np.max(np.abs(yy - ref)) <= 1e-5 * np.max(np.abs(ref))


def test_noalloc_rejects_a_volume_beyond_the_array():
    # 6 x 1000 x 1500 float32: two padded staging volumes of ~37 MB each
    S = torch.zeros((6, 1000, 1500), dtype=torch.float32, device=DEV)
    S[:, 100:200, 100:200] = 0.5
    with Solver(S, r_t=1, r_s=2) as sol:
        need = _lib.lib().sfseg_apply_noalloc_bytes(sol._handle())
        assert need > (64 << 20)
        y = torch.empty_like(S)
        rc = _lib.lib().sfseg_apply_noalloc(sol._handle(), ctypes.c_void_p(S.data_ptr()),
                                            ctypes.c_void_p(y.data_ptr()))
        assert rc == _lib.SFSEG_ERR_INVALID_ARG
        assert b"too large" in _lib.lib().sfseg_last_error()
