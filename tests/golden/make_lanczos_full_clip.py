"""Write the leading eigenvalues of the full-resolution clip's adjacency.

Test infrastructure.  Lanczos (scipy's ``eigsh``, implicitly restarted) on
the FP64 matrix-free oracle of Eq. (2) -- the eigensolver the paper compares
SFSeg's filtering form against in Sec. 4.2 -- applied to the seeded
70 x 480 x 854 clip (spatial radius 5, temporal radius 2, sigma_s 2,
sigma_t 1, alpha 1, p 0.2).  The three largest eigenvalues and the residual
norm of each Ritz pair, measured by one more oracle product, go to
``lanczos_full_clip.json`` beside this file; GPU tests read lambda_1 and
lambda_2 from there to bound the error of converged iterates.

Only ``oracle/`` and the seeded input generator are used.  Run from the
repository root:

    python tests/golden/make_lanczos_full_clip.py
"""
from __future__ import annotations

import hashlib
import json
import os
import platform
import sys
import time

import numpy as np
from scipy.sparse.linalg import LinearOperator, eigsh

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

from oracle import OracleConfig  # noqa: E402
from oracle.native import MatrixFree, num_threads  # noqa: E402
from paper_1907_02731_amd.synth import full_clip  # noqa: E402

SEED = 1
CFG = OracleConfig(r_t=2, r_s=5, sigma_t=1.0, sigma_s=2.0, alpha=1.0, p=0.2)
K_EIG = 3
NCV = 40
TOL = 1e-10


def oracle_hash() -> str:
    h = hashlib.sha256()
    for name in ("dia_oracle.c", "native.py", "sfseg_oracle.py"):
        with open(os.path.join(ROOT, "oracle", name), "rb") as f:
            h.update(f.read())
    return h.hexdigest()[:16]


def cpu_model() -> str:
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return platform.processor() or "unknown"


def main() -> None:
    S = full_clip(SEED)
    mf = MatrixFree(S, None, CFG)
    n = mf.n
    count = [0]
    t0 = time.time()

    def mv(v):
        count[0] += 1
        if count[0] % 20 == 0:
            print(f"  {count[0]} products, {time.time() - t0:.0f} s", flush=True)
        return mf.apply(np.asarray(v, dtype=np.float64).ravel())

    op = LinearOperator((n, n), matvec=mv, dtype=np.float64)
    v0 = S.astype(np.float64).ravel()
    v0 /= np.linalg.norm(v0)
    vals, vecs = eigsh(op, k=K_EIG, which="LA", tol=TOL, ncv=NCV, v0=v0)
    order = np.argsort(vals)[::-1]
    vals, vecs = vals[order], vecs[:, order]
    n_products = count[0]
    elapsed = time.time() - t0
    resid = []
    for i in range(K_EIG):
        v = vecs[:, i] / np.linalg.norm(vecs[:, i])
        resid.append(float(np.linalg.norm(mf.apply(v) - vals[i] * v)))
    out = {
        "what": "three largest eigenvalues of M (Eq. (2)) for the seeded full-resolution clip, "
                "by Lanczos on the FP64 matrix-free oracle (Sec. 4.2 compares SFSeg against "
                "Lanczos)",
        "clip": {"generator": "paper_1907_02731_amd.synth.full_clip", "seed": SEED,
                 "shape": list(S.shape)},
        "config": {"r_t": CFG.r_t, "r_s": CFG.r_s, "sigma_t": CFG.sigma_t,
                   "sigma_s": CFG.sigma_s, "alpha": CFG.alpha, "p": CFG.p},
        "eigsh": {"k": K_EIG, "which": "LA", "tol": TOL, "ncv": NCV, "v0": "S / ||S||",
                  "products": n_products, "seconds": round(elapsed, 1)},
        "lambda": [float(v) for v in vals],
        "residual_norm": resid,
        "lambda2_over_lambda1": float(vals[1] / vals[0]),
        "oracle_sha256_16": oracle_hash(),
        "command": "python tests/golden/make_lanczos_full_clip.py",
        "host": {"cpu": cpu_model(), "threads": num_threads()},
    }
    path = os.path.join(HERE, "lanczos_full_clip.json")
    with open(path, "w") as f:
        json.dump(out, f, indent=1)
        f.write("\n")
    print(json.dumps(out, indent=1), flush=True)


if __name__ == "__main__":
    main()
