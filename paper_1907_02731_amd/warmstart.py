"""Learned warm start of the power iteration.

Algorithm 1 starts from the input soft segmentation S.  ``UNet`` (the
library's sfseg_unet_* kernels) maps S to an estimate of the principal
eigenvector; ``solve_warm`` passes that estimate as the start vector and lets
the plain power iteration run to the same tolerance as a cold start, so the
method itself still decides the result and the network can only change how
many steps it takes.

Everything here is argument marshalling and the training loop's bookkeeping:
forward and backward passes, the loss and the Adam update run in the
library's gfx950 kernels.
"""
from __future__ import annotations

import ctypes
import math
import os
import time
from typing import Dict, Iterable, List, Optional, Sequence, Tuple

import numpy as np
import torch

from . import _lib
from .solver import BatchSolver, Solver
from .synth import make_clip

# (Cin, Cout, kernel) in the library's exchange order.
LAYERS: List[Tuple[int, int, int]] = [
    (1, 16, 3), (16, 16, 3), (16, 32, 3), (32, 32, 3), (32, 64, 3), (64, 64, 3),
    (96, 32, 3), (32, 32, 3), (48, 16, 3), (16, 16, 3), (16, 1, 1),
]

# Graph parameters of the full-resolution configuration the network serves.
GRAPH = dict(r_t=2, r_s=5, sigma_t=1.0, sigma_s=2.0, alpha=1.0, p=0.2)
TRAIN_SHAPE = (32, 128, 224)
WEIGHTS = os.path.join(os.path.dirname(os.path.abspath(__file__)), "weights",
                       "unet_r5t2.npy")


def he_init(seed: int) -> np.ndarray:
    """Flat float32 parameters: He-normal weights (fan-in), zero biases."""
    rng = np.random.Generator(np.random.PCG64(seed))
    parts = []
    for cin, cout, k in LAYERS:
        fan = cin * (27 if k == 3 else 1)
        parts.append(rng.normal(0.0, math.sqrt(2.0 / fan), size=cout * fan))
        parts.append(np.zeros(cout))
    return np.concatenate(parts).astype(np.float32)


class UNet:
    """A network object of the library sized for volumes up to ``max_shape``."""

    def __init__(self, max_shape: Sequence[int], training: bool = False,
                 device: str = "cuda:0", stream: Optional[torch.cuda.Stream] = None):
        L = _lib.lib()
        self.max_shape = tuple(int(v) for v in max_shape)
        self.device = torch.device(device)
        self.stream = stream if stream is not None else torch.cuda.Stream(device=self.device)
        self.n_params = int(L.sfseg_unet_param_count())
        self._net = ctypes.c_void_p()
        with torch.cuda.device(self.device):
            _lib.check(L.sfseg_unet_create(*self.max_shape, int(bool(training)),
                                           ctypes.c_void_p(self.stream.cuda_stream),
                                           ctypes.byref(self._net)), "sfseg_unet_create")

    def close(self) -> None:
        if getattr(self, "_net", None) is not None and self._net.value:
            with torch.cuda.device(self.device):
                _lib.lib().sfseg_unet_destroy(self._net)
            self._net = ctypes.c_void_p()

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def _h(self):
        if not self._net.value:
            raise RuntimeError("network is closed")
        return self._net

    def _host(self, fn, name):
        buf = np.empty(self.n_params, dtype=np.float32)
        with torch.cuda.device(self.device):
            _lib.check(fn(self._h(), buf.ctypes.data_as(ctypes.POINTER(ctypes.c_float)),
                          self.n_params), name)
        return buf

    def set_params(self, flat: np.ndarray) -> None:
        buf = np.ascontiguousarray(flat, dtype=np.float32)
        if buf.size != self.n_params:
            raise ValueError(f"expected {self.n_params} parameters, got {buf.size}")
        with torch.cuda.device(self.device):
            _lib.check(_lib.lib().sfseg_unet_set_params(
                self._h(), buf.ctypes.data_as(ctypes.POINTER(ctypes.c_float)), self.n_params),
                "sfseg_unet_set_params")

    def get_params(self) -> np.ndarray:
        return self._host(_lib.lib().sfseg_unet_get_params, "sfseg_unet_get_params")

    def get_grads(self) -> np.ndarray:
        return self._host(_lib.lib().sfseg_unet_get_grads, "sfseg_unet_get_grads")

    def forward(self, S: torch.Tensor, out: Optional[torch.Tensor] = None) -> torch.Tensor:
        if S.dim() != 3 or S.dtype != torch.float32 or S.device.type != "cuda":
            raise TypeError("S must be a float32 CUDA tensor of shape (T, H, W)")
        S = S.contiguous()
        T, H, W = (int(v) for v in S.shape)
        with torch.cuda.device(self.device):
            if out is None:
                out = torch.empty_like(S)
            self.stream.wait_stream(torch.cuda.current_stream())
            _lib.check(_lib.lib().sfseg_unet_forward(self._h(), S.data_ptr(), T, H, W,
                                                     out.data_ptr()), "sfseg_unet_forward")
            torch.cuda.current_stream().wait_stream(self.stream)
        return out

    def backward(self, target: torch.Tensor) -> float:
        loss = ctypes.c_double()
        target = target.contiguous()
        with torch.cuda.device(self.device):
            self.stream.wait_stream(torch.cuda.current_stream())
            _lib.check(_lib.lib().sfseg_unet_backward(self._h(), target.data_ptr(),
                                                      ctypes.byref(loss)), "sfseg_unet_backward")
        return float(loss.value)

    def backward_from(self, grad_out: torch.Tensor) -> None:
        """Gradients of an arbitrary loss given dL/dx^ of the last forward pass."""
        grad_out = grad_out.contiguous()
        with torch.cuda.device(self.device):
            self.stream.wait_stream(torch.cuda.current_stream())
            _lib.check(_lib.lib().sfseg_unet_backward_from(self._h(), grad_out.data_ptr()),
                       "sfseg_unet_backward_from")

    def adam_step(self, lr: float, step: int, beta1: float = 0.9, beta2: float = 0.999,
                  eps: float = 1e-8) -> None:
        with torch.cuda.device(self.device):
            _lib.check(_lib.lib().sfseg_unet_adam_step(self._h(), float(lr), float(beta1),
                                                       float(beta2), float(eps), int(step)),
                       "sfseg_unet_adam_step")

    def sync(self) -> None:
        with torch.cuda.device(self.device):
            _lib.check(_lib.lib().sfseg_unet_sync(self._h()), "sfseg_unet_sync")


# ---------------------------------------------------------------------------
# training data, training, warm-started solves
# ---------------------------------------------------------------------------
def eigenvector_targets(clips: Sequence[np.ndarray], tol: float = 1e-6, max_iters: int = 20000,
                        graph: Dict = GRAPH, group: int = 24, device: str = "cuda:0",
                        log=None) -> List[torch.Tensor]:
    """Principal eigenvectors of each clip's graph by the plain method (batched
    power iteration from S), as float32 CUDA tensors of unit norm."""
    out: List[torch.Tensor] = []
    for g0 in range(0, len(clips), group):
        part = [torch.from_numpy(np.ascontiguousarray(c, dtype=np.float32)).to(device)
                for c in clips[g0:g0 + group]]
        with BatchSolver(part, **graph) as bs:
            res = bs.iterate(max_iters=max_iters, tol=tol)
            out += [v.clone() for v in bs.eigvecs()]
        if log:
            log(f"targets {g0 + len(part)}/{len(clips)}: steps {min(r.iters for r in res)}-"
                f"{max(r.iters for r in res)}")
    return out


def training_clips(n: int, seed0: int = 40000, shape: Sequence[int] = TRAIN_SHAPE) -> List[np.ndarray]:
    """Seeded synthetic clips drawn like the full-resolution configuration."""
    return [make_clip(*shape, seed=seed0 + i, n_blobs=3, noise_sigma=0.15, motion="affine",
                      dtype=np.float32) for i in range(n)]


def train(net: UNet, inputs: Sequence[torch.Tensor], targets: Sequence[torch.Tensor], *,
          epochs: int = 1, lr: float = 1e-3, lr_final: float = 1e-4, seed: int = 0, log=None,
          log_every: int = 100) -> List[float]:
    """Adam on the cosine loss, one clip per step, cosine-decayed rate."""
    rng = np.random.Generator(np.random.PCG64(seed))
    total = epochs * len(inputs)
    losses: List[float] = []
    step = 0
    t0 = time.time()
    for _ in range(epochs):
        for i in rng.permutation(len(inputs)):
            step += 1
            rate = lr_final + 0.5 * (lr - lr_final) * (1 + math.cos(math.pi * (step - 1) / total))
            net.forward(inputs[i])
            losses.append(net.backward(targets[i]))
            net.adam_step(rate, step)
            if log and (step % log_every == 0 or step == total):
                log(f"step {step}/{total} loss(mean of last {log_every}) "
                    f"{np.mean(losses[-log_every:]):.5f} rate {rate:.2e} {time.time() - t0:.1f}s")
    return losses


def train_spectral(net: UNet, inputs: Sequence[torch.Tensor], targets: Sequence[torch.Tensor], *,
                   k: int = 32, graph: Dict = GRAPH, epochs: int = 1, lr: float = 1e-3,
                   lr_final: float = 1e-4, seed: int = 0, log=None, log_every: int = 100,
                   params0: Optional[np.ndarray] = None) -> List[float]:
    """Adam on the error that survives k power-iteration steps:

        L = 1 - cos(M^k x^, x*),   dL/dx^ = M^k dL/dy   (M is symmetric),

    with M the clip's graph; the loss and dL/dx^ come from the library
    (sfseg_spectral_grad).  Components of x^ along fast-decaying eigenvectors
    are damped by (lambda_i / lambda_1)^k before the loss sees them, so the
    network is trained on the slow components, the ones that set the number
    of steps."""
    rng = np.random.Generator(np.random.PCG64(seed))
    total = epochs * len(inputs)
    losses: List[float] = []
    step = 0
    t0 = time.time()
    sols: Dict[Tuple[int, ...], Solver] = {}   # one context per clip shape
    g_bufs: Dict[Tuple[int, ...], torch.Tensor] = {}
    try:
        for _ in range(epochs):
            for i in rng.permutation(len(inputs)):
                step += 1
                rate = lr_final + 0.5 * (lr - lr_final) * (1 + math.cos(math.pi * (step - 1) / total))
                shape = tuple(int(v) for v in inputs[i].shape)
                if shape not in sols:
                    sols[shape] = Solver(inputs[i], **graph)
                sol = sols[shape]
                sol.set_features(inputs[i])
                xhat = net.forward(inputs[i])
                g, loss = sol.spectral_grad(xhat, targets[i], k, out=g_bufs.get(shape))
                g_bufs[shape] = g
                net.backward_from(g)
                net.adam_step(rate, step)
                losses.append(loss)
                if log and (step % log_every == 0 or step == total):
                    log(f"step {step}/{total} loss after {k} steps (mean of last {log_every}) "
                        f"{np.mean(losses[-log_every:]):.6f} rate {rate:.2e} {time.time() - t0:.1f}s")
    finally:
        for sol in sols.values():
            sol.close()
    return losses


def save_params(flat: np.ndarray, path: str = WEIGHTS) -> None:
    os.makedirs(os.path.dirname(path), exist_ok=True)
    np.save(path, np.ascontiguousarray(flat, dtype=np.float32))


def load_params(path: str = WEIGHTS) -> np.ndarray:
    return np.load(path, allow_pickle=False)


def solve_cold(S: torch.Tensor, tol: float = 1e-5, graph: Dict = GRAPH, max_iters: int = 20000,
               plan: Optional[Tuple[int, int]] = None):
    """Plain method from S: (result, eigenvector, seconds).  `plan` = (block
    shape, frame runs per tile) for the step kernel, else the default."""
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    with Solver(S, **graph) as sol:
        if plan is not None:
            sol.set_plan(*plan)
        r = sol.iterate(max_iters=max_iters, tol=tol)
        x = sol.eigvec()
    torch.cuda.synchronize()
    return r, x, time.perf_counter() - t0


def solve_refined(S: torch.Tensor, tol: float = 1e-5, graph: Dict = GRAPH,
                  max_iters: int = 20000, plan: Optional[Tuple[int, int]] = None,
                  pre_steps: int = 5, refinements: int = 1, between: int = 20,
                  net: Optional[UNet] = None):
    """Plain steps from S (or from the network's estimate, `net`), the
    frame-wise Rayleigh-Ritz refinement (sfseg_refine_frames), then the plain
    method to the same tolerance: (result, eigenvector, seconds, steps in all,
    Ritz values); the seconds include the network's inference."""
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    x0 = net.forward(S) if net is not None else None
    with Solver(S, **graph) as sol:
        if plan is not None:
            sol.set_plan(*plan)
        r, steps, mus = sol.iterate_refined(x0, pre_steps=pre_steps, refinements=refinements,
                                            between=between, max_iters=max_iters, tol=tol)
        x = sol.eigvec()
    torch.cuda.synchronize()
    return r, x, time.perf_counter() - t0, steps, mus


def solve_warm(S: torch.Tensor, net: UNet, tol: float = 1e-5, graph: Dict = GRAPH,
               max_iters: int = 20000, plan: Optional[Tuple[int, int]] = None):
    """Network estimate as the start vector, then the plain method to the same
    tolerance: (result, eigenvector, seconds, seconds of inference)."""
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    x0 = net.forward(S)
    torch.cuda.synchronize()
    t_inf = time.perf_counter() - t0
    with Solver(S, **graph) as sol:
        if plan is not None:
            sol.set_plan(*plan)
        r = sol.iterate(x0, max_iters=max_iters, tol=tol)
        x = sol.eigvec()
    torch.cuda.synchronize()
    return r, x, time.perf_counter() - t0, t_inf
