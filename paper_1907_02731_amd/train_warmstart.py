"""Train the warm-start network and compare warm and cold starts.

    python -m paper_1907_02731_amd.train_warmstart [--n 2000] [--epochs 4] [--out PATH]

1. draws ``n`` seeded synthetic clips of 32 x 128 x 224 (``--shape``; seeds
   40000 + i),
2. computes each clip's principal eigenvector with the plain method (batched
   power iteration to delta < 1e-6) as the training target,
3. trains the network with Adam on 1 - cos(x^, x*) or, with --loss spectral,
   on 1 - cos(M^k x^, x*) (the error left after k power steps), one clip per
   step,
4. saves the float32 parameters (numpy .npy, exchange layout of sfseg.h),
5. on held-out full-resolution clips (70 x 480 x 854, seeds 1001 ...) runs the
   plain method from S (cold) and from the network's estimate (warm) to
   delta < 1e-5 and prints steps and wall time of both.

Every step of the network and of the power iteration runs in libsfseg's
kernels; this script only draws the synthetic data and keeps the books.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np
import torch

from .synth import full_clip
from .warmstart import (GRAPH, TRAIN_SHAPE, WEIGHTS, UNet, eigenvector_targets, he_init,
                        load_params, save_params, solve_cold, solve_warm, train, train_spectral,
                        training_clips)


def log(msg: str) -> None:
    print(msg, flush=True)


def evaluate(net: UNet, seeds, tol: float = 1e-5):
    rows = []
    for sd in seeds:
        S = torch.from_numpy(full_clip(sd)).cuda()
        solve_cold(S, tol=tol)          # warm caches and kernels once
        rc, xc, tc = solve_cold(S, tol=tol)
        rw, xw, tw, ti = solve_warm(S, net, tol=tol)
        row = {"seed": sd, "cold_steps": rc.iters, "warm_steps": rw.iters,
               "cold_s": tc, "warm_s": tw, "inference_s": ti,
               "lambda_rel_diff": abs(rw.lam - rc.lam) / rc.lam,
               "x_diff": float(np.linalg.norm(xw.cpu().numpy().astype(np.float64) -
                                              xc.cpu().numpy().astype(np.float64)))}
        log(json.dumps(row))
        rows.append(row)
        del S
    return rows


def main(argv=None):
    ap = argparse.ArgumentParser(description=__doc__.splitlines()[0])
    ap.add_argument("--n", default="2000",
                    help="training clips (one count, or one per --shape entry)")
    ap.add_argument("--epochs", type=int, default=4)
    ap.add_argument("--lr", type=float, default=1e-3)
    ap.add_argument("--lr-final", type=float, default=5e-5)
    ap.add_argument("--seed", type=int, default=0)
    ap.add_argument("--out", default=WEIGHTS)
    ap.add_argument("--eval-seeds", default="1001,1002")
    ap.add_argument("--log-every", type=int, default=200)
    ap.add_argument("--loss", choices=["cos", "spectral"], default="cos",
                    help="cos: 1 - cos(x^, x*); spectral: 1 - cos(M^k x^, x*)")
    ap.add_argument("--k", type=int, default=32, help="power steps inside the spectral loss")
    ap.add_argument("--init", default="", help="start from these parameters (.npy)")
    ap.add_argument("--shape", default=",".join(str(v) for v in TRAIN_SHAPE),
                    help="training clip shape T,H,W (several: T,H,W;T,H,W)")
    args = ap.parse_args(argv)

    shapes = [tuple(int(v) for v in sh.split(",")) for sh in args.shape.split(";")]
    counts = [int(v) for v in args.n.split(",")]
    if len(counts) == 1:
        counts = counts * len(shapes)
    if len(counts) != len(shapes):
        ap.error("--n needs one count or one per shape")
    t0 = time.time()
    clips = []
    seed = 40000
    for shape, n in zip(shapes, counts):
        for i in range(0, n, 100):
            clips += training_clips(min(100, n - i), seed0=seed + i, shape=shape)
            log(f"clips {len(clips)}/{sum(counts)} ({time.time() - t0:.0f}s)")
        seed += n
    targets = eigenvector_targets(clips, tol=1e-6, log=log)
    inputs = [torch.from_numpy(c).cuda() for c in clips]
    del clips
    log(f"data ready ({time.time() - t0:.0f}s)")

    with UNet(tuple(max(sh[d] for sh in shapes) for d in range(3)), training=True) as net:
        net.set_params(load_params(args.init) if args.init else he_init(args.seed))
        if args.loss == "cos":
            losses = train(net, inputs, targets, epochs=args.epochs, lr=args.lr,
                           lr_final=args.lr_final, seed=args.seed, log=log,
                           log_every=args.log_every)
        else:
            losses = train_spectral(net, inputs, targets, k=args.k, epochs=args.epochs,
                                    lr=args.lr, lr_final=args.lr_final, seed=args.seed, log=log,
                                    log_every=args.log_every)
        params = net.get_params()
    save_params(params, args.out)
    log(f"saved {args.out}; final mean loss {np.mean(losses[-200:]):.5f} ({time.time() - t0:.0f}s)")
    del inputs, targets
    torch.cuda.empty_cache()

    with UNet((70, 480, 854)) as net:
        net.set_params(params)
        rows = evaluate(net, [int(s) for s in args.eval_seeds.split(",") if s])
    log(json.dumps({"mean_cold_steps": float(np.mean([r["cold_steps"] for r in rows])),
                    "mean_warm_steps": float(np.mean([r["warm_steps"] for r in rows])),
                    "mean_cold_s": float(np.mean([r["cold_s"] for r in rows])),
                    "mean_warm_s": float(np.mean([r["warm_s"] for r in rows]))}))
    return 0


if __name__ == "__main__":
    sys.exit(main())
