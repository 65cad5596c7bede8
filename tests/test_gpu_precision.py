"""16-bit storage forms (bfloat16, float16): w, F and the iterate are stored in
16 bits, filtering runs in float32, norms and Rayleigh sums in float64.

Two kinds of checks:
  * bit-level: with inputs that are exact in the storage type and p = 1 (so
    w = S exactly), one application must equal the float64 product M x
    rounded once to the storage type, to within one unit in the last place
    (the float32 filtering can move a value across a rounding boundary);
  * error budget: the iterate after K steps is compared with the FP64 oracle
    (inputs not pre-rounded); the relative L2 and max-abs errors are printed
    and bounded by what the storage precision allows.
"""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

from oracle import OracleConfig, build_adjacency, power_iteration  # noqa: E402
from paper_1907_02731_amd.solver import Solver  # noqa: E402
from paper_1907_02731_amd.synth import make_clip, random_vector, tiny_clip  # noqa: E402

pytestmark = pytest.mark.gpu
DEV = "cuda:0"


def round_bf16(a):
    """Round float32 values to the nearest bfloat16 (ties to even), as float32."""
    b = np.ascontiguousarray(a, dtype=np.float32).view(np.uint32).astype(np.uint64)
    b = (b + 0x7FFF + ((b >> 16) & 1)) & 0xFFFF0000
    return b.astype(np.uint32).view(np.float32)


def round_f16(a):
    return np.asarray(a, dtype=np.float32).astype(np.float16).astype(np.float32)


ROUND = {"bf16": round_bf16, "f16": round_f16}
ULP_REL = {"bf16": 2.0 ** -8, "f16": 2.0 ** -11}
# spacing of the subnormal range (float16 rounds to multiples of 2^-24 below 2^-14)
ULP_ABS = {"bf16": 0.0, "f16": 2.0 ** -24}


def _t(a):
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.float32)).to(DEV)


@pytest.mark.parametrize("storage", ["bf16", "f16"])
def test_apply_equals_rounded_product(storage):
    rnd = ROUND[storage]
    shape = (5, 40, 70)
    S = rnd(make_clip(*shape, seed=401, n_blobs=2, noise_sigma=0.1, dtype=np.float32))
    F = rnd(random_vector(shape, seed=402, dtype=np.float32))
    x = rnd(random_vector(shape, seed=403, signed=True, dtype=np.float32))
    cfg = OracleConfig(r_t=1, r_s=3, sigma_t=1.0, sigma_s=1.5, alpha=0.8, p=1.0)
    M = build_adjacency(S.astype(np.float64), F.astype(np.float64), cfg)
    ref = M @ x.astype(np.float64).ravel()
    with Solver(_t(S), _t(F), r_t=cfg.r_t, r_s=cfg.r_s, sigma_t=cfg.sigma_t,
                sigma_s=cfg.sigma_s, alpha=cfg.alpha, p=cfg.p, storage=storage) as sol:
        y = sol.apply(_t(x)).cpu().numpy().astype(np.float64).ravel()
    # every output is a storage-type value ...
    assert np.array_equal(rnd(y.astype(np.float32)), y.astype(np.float32))
    # ... within one unit in the last place of the exact product
    ulp = np.maximum(ULP_REL[storage] * np.abs(ref), ULP_ABS[storage])
    tol = 1.01 * ulp + 1e-6 * np.max(np.abs(ref)) * ULP_REL[storage]
    assert np.all(np.abs(y - ref) <= tol)


@pytest.mark.parametrize("storage,bound", [("bf16", 5e-2), ("f16", 1e-2)])
def test_trajectory_error_budget(storage, bound):
    S = tiny_clip(0).astype(np.float32)
    cfg = OracleConfig(r_t=1, r_s=2, sigma_t=1.0, sigma_s=1.0, alpha=1.0, p=0.2)
    M = build_adjacency(S.astype(np.float64), None, cfg)
    K = 50
    with Solver(_t(S), r_t=cfg.r_t, r_s=cfg.r_s, sigma_t=cfg.sigma_t, sigma_s=cfg.sigma_s,
                alpha=cfg.alpha, p=cfg.p, storage=storage) as sol:
        res = sol.iterate(max_iters=K, tol=0.0)
        x = sol.eigvec().cpu().numpy().astype(np.float64).ravel()
    ref = power_iteration(lambda v: M @ v, S.astype(np.float64).ravel(), K, 0.0)
    rel_l2 = np.linalg.norm(x - ref["x"]) / np.linalg.norm(ref["x"])
    max_abs = np.max(np.abs(x - ref["x"]))
    lam_rel = abs(res.lam - ref["lam"]) / ref["lam"]
    print(f"{storage}: K={K} rel_l2={rel_l2:.3e} max_abs={max_abs:.3e} "
          f"lambda_rel={lam_rel:.3e} delta={res.delta:.3e}", flush=True)
    assert res.iters == K
    assert abs(np.linalg.norm(x) - 1.0) <= 1e-6
    assert rel_l2 <= bound
    assert lam_rel <= bound
    assert np.all(x[S.ravel() == 0] == 0.0)


@pytest.mark.parametrize("storage", ["bf16", "f16"])
def test_16bit_runs_converge_to_the_rounded_fixed_point(storage):
    # Rounding is deterministic, so the 16-bit iteration settles on a fixed
    # point of the rounded map; the change still falls below 1e-5, and the
    # vector it settles on stays within the storage error budget of the
    # float32 result.
    S = tiny_clip(0).astype(np.float32)
    kw = dict(r_t=1, r_s=2, sigma_t=1.0, sigma_s=1.0, alpha=1.0, p=0.2)
    with Solver(_t(S), storage=storage, **kw) as sol:
        res = sol.iterate(max_iters=2000, tol=1e-5)
        x = sol.eigvec().cpu().numpy().astype(np.float64).ravel()
    with Solver(_t(S), storage="f32", **kw) as sol:
        ref = sol.iterate(max_iters=2000, tol=1e-5)
        x32 = sol.eigvec().cpu().numpy().astype(np.float64).ravel()
    err = np.linalg.norm(x - x32)
    print(f"{storage}: converged={res.converged} iters={res.iters} (f32 {ref.iters}) "
          f"delta={res.delta:.3e} ||x - x_f32||={err:.3e}", flush=True)
    assert res.converged
    assert err <= (5e-2 if storage == "bf16" else 1e-2)
