#!/usr/bin/env python3
"""Benchmark of the SFSeg power iteration on one MI355X.

One step = one whole solve of the hot path for one synthetic clip resident in
HBM: prep (w = S^p, storage copies of F and S), start-vector normalisation,
power iterations until the change between successive unit iterates drops
below the tolerance, and the float32 eigenvector output.  The metric is
voxel-iterations per second over the timed steps; the per-step time is the
time to converge.

Prints one JSON line.  ``roofline`` describes the dominant kernel (the fused
step kernel): algorithmic bytes per launch (16 B per voxel in float32: read
x, w, F; write y) over its average launch duration from the library's HIP
events on its own stream.  ``cpu_baseline`` times the FP64 matrix-free oracle
on this host for a bounded sample of the same workload.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0  # MI355X HBM3E, vendor figure
# FP32 vector peak without packed-FP32 instructions (the library is built with
# them disabled): 256 CUs x 4 SIMDs x 16 lanes x 2 flop (FMA) x 2.4 GHz.
ALU_PEAK_TFLOPS = 256 * 4 * 16 * 2 * 2.4e9 / 1e12
ALU_PEAK_PACKED_TFLOPS = 157.3  # vendor figure, packed FP32


def flops_per_voxel(r_s: int, r_t: int, nf: int = 1) -> int:
    """Algorithmic FLOPs of one step per voxel: 1 + 2 nf fields (nf feature
    channels), each filtered along y, x (2 r_s + 1 taps) and t (2 r_t + 1
    taps) at 2 flop per tap; 1 + 2 nf to form the fields, 1 + 6 nf for the
    combine of Eq. (7) (summed over channels, Eq. (9)), 4 for the two float64
    reduction FMAs.  176 for one channel at r_s = 5, r_t = 2."""
    nfld = 1 + 2 * nf
    return nfld * 2 * (2 * (2 * r_s + 1) + (2 * r_t + 1)) + nfld + (1 + 6 * nf) + 4


def roofline(kernel: str, voxels: float, seconds: float, storage: str, r_s: int, r_t: int,
             traffic, nf: int = 1):
    """Roofline entry of the step kernel against HBM bandwidth: algorithmic
    bytes per launch (16 B per voxel in float32: read x, w, F, write y; 8 B in
    16-bit storage; 4 B more per extra feature channel) over the average
    launch duration, as a fraction of the 8 TB/s peak.  The VALU view sits
    beside it: 176 flop per voxel (one channel, r_s = 5, r_t = 2) against the
    FP32 vector peak without packed-FP32 instructions, which the library is
    built without."""
    fl = flops_per_voxel(r_s, r_t, nf) * voxels
    by = (BYTES_PER_VOXEL[storage] + (nf - 1) * BYTES_PER_VOXEL[storage] // 4) * voxels
    tf = fl / seconds / 1e12
    gbs = by / seconds / 1e9
    return {"bound": "hbm", "kernel": kernel, "achieved": gbs, "peak": HBM_PEAK_GBS,
            "unit": "GB/s", "frac": gbs / HBM_PEAK_GBS, "traffic": traffic,
            "bytes_per_launch": by, "avg_launch_us": seconds * 1e6,
            "traffic_GBps": None if traffic is None else traffic / seconds / 1e9,
            "alu": {"achieved": tf, "peak": ALU_PEAK_TFLOPS, "unit": "TFLOP/s",
                    "frac": tf / ALU_PEAK_TFLOPS, "flops_per_launch": fl,
                    "frac_of_packed_peak": tf / ALU_PEAK_PACKED_TFLOPS}}


def host_info() -> dict:
    model = "unknown"
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    return {"cpu_model": model, "logical_cpus": os.cpu_count()}


def copy_bandwidth(nbytes: int = 1 << 30, reps: int = 10) -> dict:
    """Device-to-device copy of nbytes on the GPU (read + write counted),
    timed with events, median of reps: the reachable HBM bandwidth beside
    the vendor peak."""
    import torch

    a = torch.empty(nbytes // 4, dtype=torch.float32, device="cuda:0").fill_(1.0)
    b = torch.empty_like(a)
    for _ in range(3):
        b.copy_(a)
    ts = []
    for _ in range(reps):
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        b.copy_(a)
        e1.record()
        e1.synchronize()
        ts.append(e0.elapsed_time(e1) / 1e3)
    t = float(np.median(ts))
    del a, b
    return {"bytes": 2 * nbytes, "seconds": t, "GBps": 2 * nbytes / t / 1e9,
            "frac_of_peak": 2 * nbytes / t / 1e9 / HBM_PEAK_GBS,
            "what": f"torch copy of {nbytes >> 20} MiB on the device, read + write bytes, "
                    f"median of {reps}"}


TRAFFIC_FILE = os.path.join(ROOT, "profiles", "step_kernel_full_traffic.json")
# Work plans the autotuner chose on this GPU, keyed by clip shape, radii,
# storage and feature channels; reused so that repeated runs time the same plan.
PLAN_CACHE = os.path.join(ROOT, "paper_1907_02731_amd", "tuned_plans.json")
KERNEL_SOURCES = ["paper_1907_02731_amd/csrc/step_kernel.h", "paper_1907_02731_amd/csrc/step_f32.hip",
                  "paper_1907_02731_amd/csrc/sfseg_internal.h"]


def kernel_source_hash() -> str:
    import hashlib
    h = hashlib.sha256()
    for rel in KERNEL_SOURCES:
        with open(os.path.join(ROOT, rel), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def measured_traffic(workload: str, storage: str, nf: int = 1, plan=None):
    """HBM bytes per step-kernel launch from the committed counter summary,
    if it was taken on the kernel sources as they are now and with the same
    work plan (else None)."""
    try:
        with open(TRAFFIC_FILE) as fh:
            t = json.load(fh)
    except (OSError, ValueError):
        return None
    if t.get("kernel_source_hash") != kernel_source_hash():
        return None
    key = f"{workload}/{storage}" + ("" if nf == 1 else f"/nf{nf}")
    entry = t.get("workloads", {}).get(key)
    if entry is None:
        return None
    if plan is not None and entry.get("plan") != [plan["shape"], plan["chunks"]]:
        return None
    return entry.get("hbm_bytes_per_launch")
BYTES_PER_VOXEL = {"f32": 16, "bf16": 8, "f16": 8}

WORKLOADS = {
    # name: (T, H, W, r_t, r_s, sigma_t, sigma_s, generator seed)
    "full": (70, 480, 854, 2, 5, 1.0, 2.0, 1),
    "tiny": (8, 64, 96, 1, 2, 1.0, 1.0, 0),
}


def parse():
    ap = argparse.ArgumentParser(description=__doc__.splitlines()[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", choices=sorted(WORKLOADS) + ["batch", "warmstart", "segment"],
                    default="full",
                    help="full: one 70x480x854 clip; tiny: 8x64x96; batch: 24 ragged clips "
                         "(frames 20-100, 240x427 / 360x640 / 480x854) in one batched solve, "
                         "timed against solving them one by one")
    ap.add_argument("--clips", type=int, default=24, help="clips in the batch workload")
    ap.add_argument("--no-autotune", dest="autotune", action="store_false",
                    help="keep the library's default work plan instead of the autotuner's "
                         "(which runs outside the timed region, or comes from the plan cache)")
    ap.add_argument("--plan-cache", default=PLAN_CACHE,
                    help="JSON file of tuned plans ('' to always time the plans afresh)")
    ap.add_argument("--storage", choices=["f32", "bf16", "f16"], default="f32")
    ap.add_argument("--tol", type=float, default=1e-5)
    ap.add_argument("--max-iters", type=int, default=5000)
    ap.add_argument("--alpha", type=float, default=1.0)
    ap.add_argument("--p", type=float, default=0.2)
    ap.add_argument("--iters", type=int, default=0,
                    help="run exactly this many steps per solve (tol = 0); for profiling")
    ap.add_argument("--shape", type=int, default=-1, help="step-kernel block shape (0/1)")
    ap.add_argument("--chunks", type=int, default=-1,
                    help="frame runs per tile (0: the balanced work list)")
    ap.add_argument("--precision-report", action="store_true",
                    help="for 16-bit storage: error of the final iterate against the float32 "
                         "result after the same number of steps, and the FP64 oracle's residual "
                         "||Mx - lambda x|| / lambda for both")
    ap.add_argument("--precision-oracle-steps", type=int, default=100,
                    help="with --precision-report: steps after which the 16-bit and float32 "
                         "iterates are compared with the FP64 oracle's (0 to skip)")
    ap.add_argument("--calibration-copy", action="store_true",
                    help="run plain torch copies of 4*T*H*W bytes first (to scale the HBM "
                         "byte counters of a profiling run)")
    ap.add_argument("--features", type=int, default=1, choices=[1, 2],
                    help="pairwise feature channels (2: the clip and a motion-like map, Eq. (9))")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--refine-pre-steps", type=int, default=5,
                    help="plain steps before the frame-wise Rayleigh-Ritz refinement")
    ap.add_argument("--no-forms", action="store_true",
                    help="full workload: skip the batched and warm-start time-to-converge "
                         "measurements that the default line carries beside the plain one")
    ap.add_argument("--cpu-steps", type=int, default=20,
                    help="oracle power-iteration steps timed for the CPU baseline")
    return ap.parse_args()


def cpu_baseline(S, cfg_o, steps, Fs=None):
    from oracle import power_iteration
    from oracle.native import MatrixFree, num_threads

    # several feature channels: the matrix is the sum of the per-channel ones
    mfs = [MatrixFree(S, None, cfg_o)] if Fs is None else [MatrixFree(S, F, cfg_o) for F in Fs]
    x0 = S.astype(np.float64).ravel()
    t0 = time.perf_counter()
    power_iteration(lambda v: sum(m.apply(v) for m in mfs), x0, steps, 0.0)
    dt = time.perf_counter() - t0
    return {"value": S.size * steps / dt, "unit": "voxel-iterations/s", "cores": num_threads(),
            "kind": "oracle", "cpu_model": host_info()["cpu_model"],
            "sample": f"{steps} FP64 power-iteration steps of the matrix-free oracle on the "
                      f"whole {'x'.join(map(str, S.shape))} clip ({dt:.1f} s)"}


def precision_report(S, St, kw, K, x_lo, oracle_steps: int = 100):
    """Error of a 16-bit-storage iterate: against float32 storage after the same
    K steps, the FP64 oracle's relative residual of each vector, and -- after
    ``oracle_steps`` steps from S -- the relative L2 and max-abs errors of the
    16-bit and float32 iterates against the FP64 oracle's iterate (power
    iteration over the matrix-free operator on the host's cores)."""
    import torch

    from oracle import OracleConfig, power_iteration
    from oracle.native import MatrixFree
    from paper_1907_02731_amd.solver import Solver

    def run(storage, k):
        with Solver(St, **dict(kw, storage=storage)) as ref:
            ref.autotune(steps=16, cache=PLAN_CACHE)
            ref.iterate(max_iters=k, tol=0.0)
            return ref.eigvec().cpu().numpy().astype(np.float64).ravel(), ref.plan()

    x32, _ = run("f32", K)
    xl = x_lo.cpu().numpy().astype(np.float64).ravel()
    cfg = OracleConfig(r_t=kw["r_t"], r_s=kw["r_s"], sigma_t=kw["sigma_t"],
                       sigma_s=kw["sigma_s"], alpha=kw["alpha"], p=kw["p"])
    mf = MatrixFree(S, None, cfg)

    def residual(x):
        y = mf.apply(x)
        lam = float(x @ y)
        return float(np.linalg.norm(y - lam * x) / lam), lam

    r32, l32 = residual(x32)
    rlo, llo = residual(xl)
    out = {"storage": kw["storage"], "steps": K,
           "rel_l2_vs_f32": float(np.linalg.norm(xl - x32) / np.linalg.norm(x32)),
           "max_abs_vs_f32": float(np.max(np.abs(xl - x32))),
           "oracle_residual_f32": r32, "oracle_residual": rlo,
           "oracle_rayleigh_f32": l32, "oracle_rayleigh": llo}
    if oracle_steps > 0:
        t0 = time.perf_counter()
        ref = power_iteration(mf.apply, S.astype(np.float64).ravel(), oracle_steps, 0.0)
        t_or = time.perf_counter() - t0
        xo = ref["x"]
        cmp = {"steps": oracle_steps, "oracle_seconds": t_or}
        for name in (kw["storage"], "f32"):
            xg, plan = run(name, oracle_steps)
            cmp[name] = {"rel_l2": float(np.linalg.norm(xg - xo) / np.linalg.norm(xo)),
                         "max_abs": float(np.max(np.abs(xg - xo))), "plan": plan}
        cmp["max_abs_x"] = float(np.max(np.abs(xo)))
        out["vs_fp64_oracle"] = cmp
    return out


def batch_measure(args, storage: str = "f32", reps: int = None, warmup: int = None,
                  warm: bool = False) -> dict:
    """The batched form on the 24-clip ragged workload: every clip iterated
    to the tolerance by one persistent launch per step, against the same
    clips solved one after another by the plain method (contexts made outside
    the timed regions).  Inputs resident in HBM.  With `warm`, also the
    batched form started from the warm-start network's estimates (inference
    on every clip inside the timed region)."""
    import torch

    from paper_1907_02731_amd.solver import BatchSolver, Solver
    from paper_1907_02731_amd.synth import full_clip, ragged_shapes

    reps = args.steps if reps is None else reps
    warmup = args.warmup if warmup is None else warmup
    T1, H1, W1, r_t, r_s, s_t, s_s, _ = WORKLOADS["full"]
    shapes = ragged_shapes(args.clips, seed=3)
    dev = torch.device("cuda:0")
    clips = [torch.from_numpy(full_clip(3000 + i, T=T, H=H, W=W)).to(dev)
             for i, (T, H, W) in enumerate(shapes)]
    torch.cuda.synchronize()
    N = sum(T * H * W for T, H, W in shapes)
    kw = dict(r_t=r_t, r_s=r_s, sigma_t=s_t, sigma_s=s_s, alpha=args.alpha, p=args.p,
              storage=storage)
    max_iters, tol = (args.iters, 0.0) if args.iters > 0 else (args.max_iters, args.tol)
    bs = BatchSolver(clips, **kw)
    plan_info = bs.autotune(steps=16, cache=args.plan_cache or None) if args.autotune else None
    if args.shape >= 0 or args.chunks >= 0:
        pl = bs.plan()
        bs.set_plan(args.shape if args.shape >= 0 else pl["shape"],
                    args.chunks if args.chunks >= 0 else pl["chunks"])

    def batched():
        r = bs.iterate(max_iters=max_iters, tol=tol)
        bs.eigvecs()
        return r

    for _ in range(warmup):
        batched()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(reps):
        res = batched()
    torch.cuda.synchronize()
    t_batch = (time.perf_counter() - t0) / reps
    iters = [r.iters for r in res]
    vi = sum(T * H * W * k for (T, H, W), k in zip(shapes, iters))
    tm = bs.timing()
    plan = bs.plan()
    t_warm, warm_iters = None, None
    if warm:
        from paper_1907_02731_amd.warmstart import WEIGHTS, UNet, load_params
        net = UNet(tuple(max(sh[d] for sh in shapes) for d in range(3)))
        net.set_params(load_params(WEIGHTS))
        outs = [torch.empty_like(S) for S in clips]

        def batched_warm():
            for S, o in zip(clips, outs):
                net.forward(S, o)
            r = bs.iterate(outs, max_iters=max_iters, tol=tol)
            bs.eigvecs()
            return r

        for _ in range(warmup):
            batched_warm()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(reps):
            resw = batched_warm()
        torch.cuda.synchronize()
        t_warm = (time.perf_counter() - t0) / reps
        warm_iters = [r.iters for r in resw]
        net.close()
        del outs
    bs.close()

    singles = [Solver(S, **kw) for S in clips]
    for s_ in singles:
        if args.autotune:
            s_.autotune(steps=16, cache=args.plan_cache or None)
        s_.iterate(max_iters=2, tol=0.0)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    plain_iters = []
    for s_ in singles:
        r = s_.iterate(max_iters=max_iters, tol=tol)
        s_.eigvec()
        plain_iters.append(r.iters)
    torch.cuda.synchronize()
    t_plain = time.perf_counter() - t0
    for s_ in singles:
        s_.close()
    del clips
    torch.cuda.empty_cache()
    return {"shapes": shapes, "voxels": N, "iters": iters, "plain_iters": plain_iters,
            "voxel_iters": vi, "t_batch": t_batch, "t_plain": t_plain, "timing": tm,
            "plan": plan, "autotune": plan_info, "r_s": r_s, "r_t": r_t, "s_s": s_s, "s_t": s_t,
            "t_warm": t_warm, "warm_iters": warm_iters}


def bench_batch(args):
    m = batch_measure(args, args.storage)
    shapes, tm = m["shapes"], m["timing"]
    line = {
        "metric": "voxel-iterations/s (time to converge to 1e-5)",
        "value": m["voxel_iters"] / m["t_batch"],
        "unit": "voxel-iterations/s",
        "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": m["t_batch"] * 1e3,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": args.storage, "data": "synthetic",
        "config": {"workload": f"batch: {len(shapes)} clips, {m['voxels']} voxels, frames "
                               f"20-100, resolutions 240x427/360x640/480x854, r_s={m['r_s']}, "
                               f"r_t={m['r_t']}, sigma_s={m['s_s']}, sigma_t={m['s_t']}, to "
                               f"delta<{args.tol:g}",
                   "clips": [list(s) for s in shapes]},
        "plan": m["plan"], "autotune": m["autotune"],
        "iters_per_clip": m["iters"],
        "time_to_converge_ms": {"batched": m["t_batch"] * 1e3,
                                "plain_sequential": m["t_plain"] * 1e3,
                                "speedup": m["t_plain"] / m["t_batch"]},
        "plain_iters_per_clip": m["plain_iters"],
        "batched_avg_launch_us": tm["loop_ms"] * 1e3 / max(tm["launches"], 1),
        "roofline": roofline("batch_step_kernel (persistent, all clips)",
                             m["voxel_iters"] / max(tm["iters"], 1),
                             tm["loop_ms"] / 1e3 / max(tm["iters"], 1), args.storage, m["r_s"],
                             m["r_t"], None),
    }
    print(json.dumps(line), flush=True)


def warmstart_measure(args, reps: int = None, warmup: int = None, S_np=None) -> dict:
    """Learned warm start on the full-resolution clip: network inference, then
    the plain method from its estimate to the same tolerance, against the plain
    method from S (cold start); both end to end with the inputs in HBM."""
    import torch

    from paper_1907_02731_amd.synth import full_clip
    from paper_1907_02731_amd.warmstart import (GRAPH, WEIGHTS, UNet, load_params, solve_cold,
                                                solve_refined, solve_warm)

    if not os.path.exists(WEIGHTS):
        raise FileNotFoundError(f"no trained weights at {WEIGHTS} (train them with "
                                "python -m paper_1907_02731_amd.train_warmstart)")
    reps = args.steps if reps is None else reps
    warmup = args.warmup if warmup is None else warmup
    T, H, W = 70, 480, 854
    S = torch.from_numpy(full_clip(1) if S_np is None else S_np).cuda()
    net = UNet((T, H, W))
    net.set_params(load_params(WEIGHTS))
    plan, plan_info = None, None
    if args.autotune:  # both solves use the plan the full workload is tuned to
        from paper_1907_02731_amd.solver import Solver
        with Solver(S, **GRAPH) as sol:
            plan_info = sol.autotune(steps=32, cache=args.plan_cache or None)
        plan = (plan_info["shape"], plan_info["chunks"])
    def refined(use_net):
        return solve_refined(S, tol=args.tol, graph=GRAPH, plan=plan,
                             pre_steps=args.refine_pre_steps, net=net if use_net else None)

    for _ in range(warmup):
        solve_cold(S, tol=args.tol, graph=GRAPH, plan=plan)
        solve_warm(S, net, tol=args.tol, graph=GRAPH, plan=plan)
        refined(False)
        refined(True)
    cold, warm, ref, wref = [], [], [], []
    for _ in range(reps):
        cold.append(solve_cold(S, tol=args.tol, graph=GRAPH, plan=plan))
        warm.append(solve_warm(S, net, tol=args.tol, graph=GRAPH, plan=plan))
        ref.append(refined(False))
        wref.append(refined(True))
    net.close()
    tc = float(np.median([c[2] for c in cold]))
    tw = float(np.median([w[2] for w in warm]))
    ti = float(np.median([w[3] for w in warm]))
    rc, rw = cold[-1][0], warm[-1][0]
    xc = cold[-1][1].cpu().numpy().astype(np.float64)

    def same(r, x):
        return {"lambda_rel_diff": abs(r.lam - rc.lam) / rc.lam,
                "x_l2_diff": float(np.linalg.norm(x.cpu().numpy().astype(np.float64) - xc))}

    def refined_entry(runs, label):
        r = runs[-1]
        t = float(np.median([v[2] for v in runs]))
        return {"start": label, "pre_steps": args.refine_pre_steps, "steps": r[3],
                "seconds": t, "speedup": tc / t, "ritz_value": r[4][0], "lambda": r[0].lam,
                "same_eigenvector": same(r[0], r[1])}

    return {"shape": (T, H, W), "cold": {"steps": rc.iters, "seconds": tc, "lambda": rc.lam},
            "warm": {"steps": rw.iters, "seconds": tw, "inference_seconds": ti,
                     "lambda": rw.lam},
            "speedup": tc / tw, "steps_saved": rc.iters - rw.iters, "autotune": plan_info,
            "same_eigenvector": same(rw, warm[-1][1]),
            "refined": refined_entry(ref, "S"),
            "warm_refined": refined_entry(wref, "network estimate")}


def bench_warmstart(args):
    try:
        m = warmstart_measure(args)
    except FileNotFoundError as e:
        print(f"bench.py: {e}", file=sys.stderr)
        sys.exit(2)
    T, H, W = m["shape"]
    N = T * H * W
    line = {
        "metric": "time to converge to 1e-5, warm start (network + plain iterations) vs cold start",
        "value": N * m["cold"]["steps"] / m["warm"]["seconds"],
        "unit": "voxel-iterations/s (cold-start iterations per warm-start second)",
        "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": m["warm"]["seconds"] * 1e3, "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "f32 (network bf16)", "data": "synthetic",
        "config": {"workload": "warmstart: one 70x480x854 clip (seed 1, held out from training), "
                               "r_s=5, r_t=2, sigma_s=2.0, sigma_t=1.0, alpha=1.0, p=0.2, tol 1e-5",
                   "T": T, "H": H, "W": W, "tol": args.tol},
        "cold": m["cold"], "warm": m["warm"], "speedup": m["speedup"],
        "steps_saved": m["steps_saved"], "autotune": m["autotune"],
        "same_eigenvector": m["same_eigenvector"],
        "refined_start": m["refined"], "warm_start_refined": m["warm_refined"],
    }
    print(json.dumps(line), flush=True)


def bench_segment(args):
    """Algorithm 1 with the binarisation of Sec. 4.1 on the full-resolution
    clip: 5 power iterations from S, sigmoid projection after iterations 3 and
    4 (slope 10, threshold 0.5), hard threshold into a uint8 mask.  A step is
    set features + the whole run, inputs in HBM.  The cost of one projection
    and of the threshold is taken live from the library's HIP events by
    running the same solve without them."""
    import torch

    from paper_1907_02731_amd.solver import Solver
    from paper_1907_02731_amd.synth import full_clip

    T, H, W, r_t, r_s, s_t, s_s, seed = WORKLOADS["full"]
    iters, k0, slope, thr = 5, 3, 10.0, 0.5
    S = full_clip(seed)
    dev = torch.device("cuda:0")
    St = torch.from_numpy(S).to(dev)
    mask = torch.empty((T, H, W), dtype=torch.uint8, device=dev)
    if args.calibration_copy:
        cp = torch.empty_like(St)
        for _ in range(3):
            cp.copy_(St)
        del cp
    kw = dict(r_t=r_t, r_s=r_s, sigma_t=s_t, sigma_s=s_s, alpha=args.alpha, p=args.p,
              storage=args.storage)
    sol = Solver(St, **kw)
    plan_info = sol.autotune(steps=32, cache=args.plan_cache or None) if args.autotune else None

    def one_step():
        sol.set_features(St)
        return sol.segment(iters=iters, project_from=k0, slope=slope, threshold=thr, out=mask)[0]

    for _ in range(args.warmup):
        one_step()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    recs = [one_step() for _ in range(args.steps)]
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0

    def lib_ms(**kw_seg):
        out = []
        for _ in range(5):
            sol.segment(iters=iters, slope=slope, threshold=thr, **kw_seg)
            out.append(sol.timing())
        return (float(np.median([t["total_ms"] for t in out])),
                float(np.median([t["loop_ms"] for t in out])))

    _, plain_loop = lib_ms(project_from=iters, mask=False)
    proj_total, _ = lib_ms(project_from=k0, mask=False)
    plain_total, _ = lib_ms(project_from=iters, mask=False)
    full_total, _ = lib_ms(project_from=k0, out=mask)
    n_proj = iters - k0
    step_s = plain_loop / 1e3 / iters
    proj_s = (proj_total - plain_total) / 1e3 / n_proj
    thr_s = (full_total - proj_total) / 1e3
    N = T * H * W
    # algorithmic bytes: the projection reads Y and writes P, the threshold
    # reads Y and writes the uint8 mask; the max pass that each needs first
    # (one more read of Y) is an implementation cost and counts against them
    es = BYTES_PER_VOXEL[args.storage] // 4
    proj_bytes = 2 * es * N
    thr_bytes = (es + 1) * N
    last = recs[-1]
    line = {
        "metric": "voxel-iterations/s (Algorithm 1 with binarisation, 5 iterations)",
        "value": N * iters * args.steps / elapsed,
        "unit": "voxel-iterations/s",
        "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": elapsed * 1e3 / args.steps,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": args.storage, "data": "synthetic",
        "config": {"workload": f"segment: one {T}x{H}x{W} clip, r_s={r_s}, r_t={r_t}, "
                               f"sigma_s={s_s}, sigma_t={s_t}, alpha={args.alpha}, p={args.p}, "
                               f"{iters} power iterations from S, sigmoid projection after "
                               f"iterations {k0}..{iters - 1} (slope {slope:g}, threshold "
                               f"{thr:g}), hard threshold into a uint8 mask",
                   "T": T, "H": H, "W": W, "iters": iters, "project_from": k0,
                   "slope": slope, "threshold": thr},
        "lambda": last.lam, "delta": last.delta,
        "plan": sol.plan(), "autotune": plan_info,
        "mask_fraction": float(mask.float().mean().item()),
        "roofline": roofline("step_kernel (fused stencil + reductions)", N, step_s,
                             args.storage, r_s, r_t,
                             measured_traffic("full", args.storage, 1, sol.plan())),
        "binarize": {
            "project_us": proj_s * 1e6, "project_bytes": proj_bytes,
            "project_GBps": proj_bytes / proj_s / 1e9,
            "project_frac_hbm": proj_bytes / proj_s / 1e9 / HBM_PEAK_GBS,
            "threshold_us": thr_s * 1e6, "threshold_bytes": thr_bytes,
            "threshold_GBps": thr_bytes / thr_s / 1e9,
            "threshold_frac_hbm": thr_bytes / thr_s / 1e9 / HBM_PEAK_GBS,
            "note": "max + projection + finish launches and max + threshold launches, each "
                    "the difference of library-timed solves with and without them (medians "
                    "of 5); bytes are algorithmic (Y read once, P or the mask written)",
        },
    }
    if not args.no_cpu_baseline:
        from oracle import OracleConfig
        from oracle.binarize_oracle import segment
        from oracle.native import MatrixFree, num_threads
        cfg_o = OracleConfig(r_t=r_t, r_s=r_s, sigma_t=s_t, sigma_s=s_s, alpha=args.alpha, p=args.p)
        mf = MatrixFree(S, None, cfg_o)
        c0 = time.perf_counter()
        segment(mf.apply, S.astype(np.float64).ravel(), iters, k0, slope, thr)
        dt = time.perf_counter() - c0
        line["cpu_baseline"] = {
            "value": N * iters / dt, "unit": "voxel-iterations/s", "cores": num_threads(),
            "kind": "oracle",
            "sample": f"the whole FP64 Algorithm 1 ({iters} iterations, projections, threshold) "
                      f"of the matrix-free oracle on the {T}x{H}x{W} clip ({dt:.1f} s)"}
    sol.close()
    print(json.dumps(line), flush=True)


def main():
    args = parse()
    if args.gpus != 1:
        print(f"bench.py: the library and this benchmark run on one GPU (asked for --gpus "
              f"{args.gpus}); sharding a clip or a batch across GPUs is not implemented.",
              file=sys.stderr)
        sys.exit(2)
    if args.workload == "batch":
        bench_batch(args)
        return
    if args.workload == "warmstart":
        bench_warmstart(args)
        return
    if args.workload == "segment":
        bench_segment(args)
        return

    import torch

    from paper_1907_02731_amd.solver import Solver
    from paper_1907_02731_amd.synth import feature_channels, full_clip, tiny_clip

    T, H, W, r_t, r_s, s_t, s_s, seed = WORKLOADS[args.workload]
    S = full_clip(seed) if args.workload == "full" else tiny_clip(seed).astype(np.float32)
    assert S.shape == (T, H, W)
    nf = args.features
    Fs = None
    if nf > 1:
        if args.workload == "full":
            Fs = feature_channels(T, H, W, seed=seed)
        else:
            Fs = feature_channels(T, H, W, seed=seed, n_blobs=2, noise_sigma=0.1, motion="drift")
        S = Fs[0].copy()
    dev = torch.device("cuda:0")
    St = torch.from_numpy(S).to(dev)
    Ft = None if Fs is None else torch.from_numpy(Fs).to(dev)
    out = torch.empty_like(St)
    if args.calibration_copy:
        for _ in range(3):
            out.copy_(St)
    torch.cuda.synchronize()

    kw = dict(r_t=r_t, r_s=r_s, sigma_t=s_t, sigma_s=s_s, alpha=args.alpha, p=args.p,
              storage=args.storage)
    sol = Solver(St, Ft, **kw)
    plan_info = sol.autotune(steps=32, cache=args.plan_cache or None) if args.autotune else None
    if args.shape >= 0 or args.chunks >= 0:
        pl = sol.plan()
        sol.set_plan(args.shape if args.shape >= 0 else pl["shape"],
                     args.chunks if args.chunks >= 0 else pl["chunks"])

    max_iters, tol = (args.iters, 0.0) if args.iters > 0 else (args.max_iters, args.tol)

    def one_step():
        sol.set_features(St, Ft)
        r = sol.iterate(max_iters=max_iters, tol=tol)
        sol.eigvec(out)
        return r, sol.timing()

    for _ in range(args.warmup):
        one_step()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    recs = [one_step() for _ in range(args.steps)]
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0

    N = T * H * W
    iters = [r.iters for r, _ in recs]
    total_iters = sum(iters)
    value = N * total_iters / elapsed
    loop_ms = sum(t["loop_ms"] for _, t in recs)
    avg_kernel_s = loop_ms / 1e3 / max(total_iters, 1)
    last = recs[-1][0]

    line = {
        "metric": "voxel-iterations/s (time to converge to 1e-5)",
        "value": value,
        "unit": "voxel-iterations/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": elapsed * 1e3 / args.steps,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": args.storage,
        "data": "synthetic",
        "config": {
            "workload": f"{args.workload}: one {T}x{H}x{W} clip, r_s={r_s}, r_t={r_t}, "
                        f"sigma_s={s_s}, sigma_t={s_t}, alpha={args.alpha}, p={args.p}, "
                        f"power iteration from S to delta<{args.tol:g}"
                        + (f", {nf} pairwise feature channels" if nf > 1 else ""),
            "T": T, "H": H, "W": W, "tol": args.tol, "features": nf,
        },
        "iters_per_step": iters,
        "plan": sol.plan(),
        "autotune": plan_info,
        "converged": bool(last.converged),
        "delta": last.delta,
        "lambda": last.lam,
        "time_to_converge_ms": {"plain": elapsed * 1e3 / args.steps},
        "roofline": roofline("step_kernel (fused stencil + reductions)", N, avg_kernel_s,
                             args.storage, r_s, r_t,
                             measured_traffic(args.workload, args.storage, nf, sol.plan()),
                             nf=nf),
        "host": host_info(),
    }
    sol.close()
    line["copy_bandwidth"] = copy_bandwidth()
    if args.workload == "full" and args.storage == "f32" and nf == 1 and not args.no_forms \
            and args.iters == 0:
        # the other two forms of the metric, on the same GPU at the same tolerance
        w = warmstart_measure(args, reps=3, warmup=1, S_np=S)
        b = batch_measure(args, "f32", reps=2, warmup=1, warm=True)
        ttc = line["time_to_converge_ms"]
        ttc["warm_start"] = w["warm"]["seconds"] * 1e3
        ttc["warm_start_inference"] = w["warm"]["inference_seconds"] * 1e3
        ttc["cold_start_same_run"] = w["cold"]["seconds"] * 1e3
        ttc["warm_start_speedup"] = w["speedup"]
        ttc["refined_start"] = w["refined"]["seconds"] * 1e3
        ttc["refined_start_speedup"] = w["refined"]["speedup"]
        ttc["warm_start_refined"] = w["warm_refined"]["seconds"] * 1e3
        ttc["warm_start_refined_speedup"] = w["warm_refined"]["speedup"]
        ttc["batched_24_clips"] = b["t_batch"] * 1e3
        ttc["plain_24_clips_one_by_one"] = b["t_plain"] * 1e3
        ttc["batched_speedup"] = b["t_plain"] / b["t_batch"]
        ttc["batched_24_clips_warm_start"] = b["t_warm"] * 1e3
        ttc["batched_warm_start_speedup"] = b["t_plain"] / b["t_warm"]
        line["forms"] = {
            "warm_start": {"cold": w["cold"], "warm": w["warm"], "steps_saved": w["steps_saved"],
                           "same_eigenvector": w["same_eigenvector"]},
            "refined_start": w["refined"],
            "warm_start_refined": w["warm_refined"],
            "batched": {"clips": len(b["shapes"]), "voxels": b["voxels"],
                        "iters_per_clip": b["iters"], "plain_iters_per_clip": b["plain_iters"],
                        "warm_start_iters_per_clip": b["warm_iters"],
                        "plan": b["plan"],
                        "voxel_iterations_per_s": b["voxel_iters"] / b["t_batch"],
                        "avg_launch_us": b["timing"]["loop_ms"] * 1e3 /
                        max(b["timing"]["launches"], 1)},
        }
    if args.precision_report:
        line["precision"] = precision_report(S, St, kw, max(iters), out,
                                              args.precision_oracle_steps)
    if not args.no_cpu_baseline:
        from oracle import OracleConfig
        cfg_o = OracleConfig(r_t=r_t, r_s=r_s, sigma_t=s_t, sigma_s=s_s, alpha=args.alpha,
                             p=args.p)
        line["cpu_baseline"] = cpu_baseline(S, cfg_o, args.cpu_steps if nf == 1 else
                                            max(1, args.cpu_steps // nf), Fs)
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
