"""Eigenvector error of converged results on the full-resolution clip, bounded
with the spectrum from Lanczos (the eigensolver Sec. 4.2 compares SFSeg with).

``tests/golden/lanczos_full_clip.json`` holds lambda_1 >= lambda_2 >= lambda_3
of Eq. (2)'s M for the seeded 70 x 480 x 854 clip (spatial radius 5,
temporal radius 2, sigma_s 2, sigma_t 1, alpha 1, p 0.2), computed by
``tests/golden/make_lanczos_full_clip.py`` with scipy's ``eigsh`` over the
FP64 matrix-free oracle.  For a unit vector x with Rayleigh quotient
rho = x^T M x and residual r = ||M x - rho x|| (one oracle product), and
lambda_2 < rho <= lambda_1, two bounds of symmetric eigenvalue theory hold:

    Kato-Temple:   0 <= lambda_1 - rho <= r^2 / (rho - lambda_2)
    Davis-Kahan:   sin angle(x, v_1) <= r / (rho - lambda_2)

The plain, batched, warm-started and frame-refined results (each iterated to
delta < 1e-5 on the GPU) are checked against the first -- the GPU's Rayleigh quotient
pinned to Lanczos' lambda_1 -- and the second gives each vector's distance to
the true eigenvector v_1; warm and cold results must lie within the sum of
their two bounds of each other (the same eigenvector, judged by the
spectrum rather than by a fixed tolerance).  The measured values are printed.
"""
import json
import os

import numpy as np
import pytest

torch = pytest.importorskip("torch")

from oracle import OracleConfig  # noqa: E402
from oracle.native import MatrixFree  # noqa: E402
from paper_1907_02731_amd.solver import BatchSolver, Solver  # noqa: E402
from paper_1907_02731_amd.synth import full_clip  # noqa: E402

pytestmark = pytest.mark.gpu

HERE = os.path.dirname(os.path.abspath(__file__))
GOLDEN = os.path.join(HERE, "golden", "lanczos_full_clip.json")
FULL = OracleConfig(r_t=2, r_s=5, sigma_t=1.0, sigma_s=2.0, alpha=1.0, p=0.2)
KW = dict(r_t=2, r_s=5, sigma_t=1.0, sigma_s=2.0, alpha=1.0, p=0.2)
TOL = 1e-5


@pytest.fixture(scope="module")
def spectrum():
    with open(GOLDEN) as fh:
        g = json.load(fh)
    assert g["clip"]["shape"] == [70, 480, 854] and g["clip"]["seed"] == 1
    assert g["config"] == {"r_t": 2, "r_s": 5, "sigma_t": 1.0, "sigma_s": 2.0, "alpha": 1.0,
                           "p": 0.2}
    lam = g["lambda"]
    # each Ritz value is within its residual of an eigenvalue (symmetric M)
    return lam[0], lam[1], g["residual_norm"][0]


@pytest.fixture(scope="module")
def clip():
    S = full_clip(1)
    return S, MatrixFree(S, None, FULL)


def _bounds(x, mf, lam1, lam2):
    x = x / np.linalg.norm(x)
    y = mf.apply(x)
    rho = float(x @ y)
    r = float(np.linalg.norm(y - rho * x))
    assert rho > lam2, "the vector is not in the principal eigenvector's basin"
    return rho, r, r * r / (rho - lam2), r / (rho - lam2)


def _check(name, x, res, mf, spectrum):
    lam1, lam2, ritz_res = spectrum
    rho, r, kt, dk = _bounds(x, mf, lam1, lam2)
    slack = 1e-12 * lam1 + ritz_res
    print(f"\n{name}: steps {res.iters}, delta {res.delta:.3e}, rho {rho:.12f}, lambda_1 "
          f"{lam1:.12f}, lambda_1 - rho {lam1 - rho:.3e} (Kato-Temple bound {kt:.3e}), "
          f"gpu lambda rel {abs(res.lam - lam1) / lam1:.3e}, residual {r:.3e}, "
          f"sin angle to v_1 <= {dk:.3e}", flush=True)
    assert res.converged and res.delta < TOL
    assert -slack <= lam1 - rho <= kt + slack
    # the GPU's own Rayleigh quotient (at the step's input) agrees to the same order
    assert abs(res.lam - rho) <= 1e-7 * lam1
    return dk


def _plan(sol):
    from test_gpu_fullsize import tuned_plan
    pl = tuned_plan([(70, 480, 854)])
    if pl is not None:
        sol.set_plan(*pl)


def test_plain_batched_and_warm_results_are_within_the_spectral_bounds(spectrum, clip):
    S, mf = clip
    lam1, lam2, _ = spectrum
    print(f"\nlambda_1 {lam1:.12f}, lambda_2 {lam2:.12f}, lambda_2 / lambda_1 "
          f"{lam2 / lam1:.6f}", flush=True)
    St = torch.from_numpy(S).cuda()
    with Solver(St, **KW) as sol:
        _plan(sol)
        rc = sol.iterate(max_iters=5000, tol=TOL)
        xc = sol.eigvec().cpu().numpy().astype(np.float64).ravel()
    dk_c = _check("plain", xc, rc, mf, spectrum)

    with BatchSolver([St], **KW) as bs:
        rb = bs.iterate(max_iters=5000, tol=TOL)[0]
        xb = bs.eigvecs()[0].cpu().numpy().astype(np.float64).ravel()
    dk_b = _check("batched", xb, rb, mf, spectrum)

    from paper_1907_02731_amd.warmstart import WEIGHTS, UNet, load_params
    with UNet(S.shape) as net:
        net.set_params(load_params(WEIGHTS))
        x0 = net.forward(St)
        with Solver(St, **KW) as sol:
            _plan(sol)
            rw = sol.iterate(x0, max_iters=5000, tol=TOL)
            xw = sol.eigvec().cpu().numpy().astype(np.float64).ravel()
    dk_w = _check("warm start", xw, rw, mf, spectrum)

    # frame-wise Rayleigh-Ritz refined start: 5 plain steps, the refinement, plain steps
    with Solver(St, **KW) as sol:
        _plan(sol)
        rr, steps, mus = sol.iterate_refined(pre_steps=5, max_iters=5000, tol=TOL)
        xr = sol.eigvec().cpu().numpy().astype(np.float64).ravel()
    dk_r = _check("refined start", xr, rr, mf, spectrum)
    print(f"refined start: {steps} steps in all against {rc.iters} plain; Ritz value "
          f"{mus[0]:.10f} <= lambda_1 {lam1:.10f}", flush=True)
    assert steps < rc.iters
    assert mus[0] <= lam1 * (1 + 1e-12) + spectrum[2]

    # both ends of each pair lie within their bounds of v_1
    for (na, xa, da), (nb, xb_, db) in (((("plain", xc, dk_c)), ("warm start", xw, dk_w)),
                                        ((("plain", xc, dk_c)), ("batched", xb, dk_b)),
                                        ((("plain", xc, dk_c)), ("refined start", xr, dk_r))):
        d = float(np.linalg.norm(xa - xb_))
        print(f"||x_{nb} - x_{na}|| = {d:.3e} <= {1.01 * (da + db):.3e}", flush=True)
        assert d <= 1.01 * (da + db) + 1e-7
