"""The deferred fold of the step's partial sums (each launch folds the
previous step's block sums; a one-block finish launch folds the last step of
every captured 16-step chunk) against the FP64 oracle at the step counts
around the chunk boundaries: iterate, Rayleigh quotient and change after K
steps, and the step at which a tolerance stops the iteration."""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

from oracle import OracleConfig, build_adjacency, power_iteration  # noqa: E402
from paper_1907_02731_amd.solver import Solver  # noqa: E402
from paper_1907_02731_amd.synth import tiny_clip  # noqa: E402

pytestmark = pytest.mark.gpu
CFG = OracleConfig(r_t=1, r_s=2, sigma_t=1.0, sigma_s=1.0, alpha=1.0, p=0.2)
KW = dict(r_t=1, r_s=2, sigma_t=1.0, sigma_s=1.0, alpha=1.0, p=0.2)


@pytest.fixture(scope="module")
def case():
    S = tiny_clip(0).astype(np.float32)
    M = build_adjacency(S.astype(np.float64), None, CFG)
    ref = power_iteration(lambda v: M @ v, S.astype(np.float64).ravel(), 80, 0.0,
                          keep_history=True)
    deltas = [float(np.linalg.norm(b - a)) for a, b in zip(ref["history"], ref["history"][1:])]
    return S, M, ref, deltas


@pytest.mark.parametrize("K", [1, 2, 15, 16, 17, 31, 32, 33, 48])
def test_state_after_k_steps(case, K):
    S, M, ref, deltas = case
    with Solver(torch.from_numpy(S).cuda(), **KW) as sol:
        res = sol.iterate(max_iters=K, tol=0.0)
        x = sol.eigvec().cpu().numpy().astype(np.float64).ravel()
    xk = ref["history"][K]
    x_prev = ref["history"][K - 1]
    lam = float(x_prev @ (M @ x_prev))
    assert res.iters == K and not res.converged
    assert np.linalg.norm(x - xk) <= 1e-5
    assert abs(res.lam - lam) <= 1e-6 * lam
    assert abs(res.delta - deltas[K - 1]) <= 1e-6 + 1e-4 * deltas[K - 1]


@pytest.mark.parametrize("K", [3, 16, 17, 32, 33])
def test_tolerance_stops_at_the_oracle_step(case, K):
    S, M, ref, deltas = case
    # a tolerance between the changes of steps K-1 and K (geometric mean):
    # the oracle stops after exactly K steps
    d_prev, d_k = deltas[K - 2], deltas[K - 1]
    assert d_k < d_prev
    tol = float(np.sqrt(d_prev * d_k))
    with Solver(torch.from_numpy(S).cuda(), **KW) as sol:
        res = sol.iterate(max_iters=1000, tol=tol)
        x = sol.eigvec().cpu().numpy().astype(np.float64).ravel()
    assert res.converged and res.iters == K
    assert np.linalg.norm(x - ref["history"][K]) <= 1e-5
