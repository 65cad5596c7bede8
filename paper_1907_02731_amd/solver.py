"""PyTorch-facing wrapper of the libsfseg C ABI.

``Solver`` owns one library context for one clip, ``BatchSolver`` one for a
batch of clips of uneven size.  Each runs on a stream of its own (default
priority) and orders itself after / before the caller's current stream with
stream waits, so tensors produced or consumed on the caller's stream need no
extra synchronisation.  ``autotune`` picks the fastest work plan and can keep
it in a JSON cache keyed by the clip shapes, the graph parameters and the GPU.
"""
from __future__ import annotations

import ctypes
import json
import os
from dataclasses import dataclass
from typing import List, Optional, Sequence

import torch

from . import _lib


@dataclass
class IterResult:
    iters: int
    converged: bool
    delta: float
    lam: float


def _dev_ptr(t: Optional[torch.Tensor], name: str, shape) -> Optional[int]:
    if t is None:
        return None
    if not isinstance(t, torch.Tensor) or t.device.type != "cuda":
        raise TypeError(f"{name} must be a CUDA (HIP) tensor")
    if t.dtype != torch.float32:
        raise TypeError(f"{name} must be float32")
    if not t.is_contiguous():
        raise ValueError(f"{name} must be contiguous")
    if tuple(t.shape) != tuple(shape):
        raise ValueError(f"{name} must have shape {tuple(shape)}, got {tuple(t.shape)}")
    return t.data_ptr()


class Solver:
    """Power iteration for the principal eigenvector of one clip's graph.

    Parameters follow the graph definition (w = S^p, Gaussian box of radii
    r_t / r_s and widths sigma_t / sigma_s, Taylor pairwise term with alpha).
    ``S`` and ``F`` are float32 CUDA tensors of shape (T, H, W); F=None uses S.
    """

    def __init__(self, S: torch.Tensor, F: Optional[torch.Tensor] = None, *, r_t: int = 1,
                 r_s: int = 2, sigma_t: float = 1.0, sigma_s: float = 1.0,
                 alpha: float = 1.0, p: float = 0.2, storage: str = "f32",
                 stream: Optional[torch.cuda.Stream] = None):
        L = _lib.lib()
        if S.dim() != 3:
            raise ValueError("S must be (T, H, W)")
        self.shape = tuple(int(v) for v in S.shape)
        self.device = S.device
        self.cfg = _lib.make_config(*self.shape, r_t=r_t, r_s=r_s, sigma_t=sigma_t,
                                    sigma_s=sigma_s, alpha=alpha, p=p, storage=storage)
        # F: (T, H, W) for one feature channel, (C, T, H, W) for C channels (Eq. (9))
        self.n_features = 1 if F is None or F.dim() == 3 else int(F.shape[0])
        self.f_shape = self.shape if self.n_features == 1 and (F is None or F.dim() == 3) \
            else (self.n_features,) + self.shape
        ps = _dev_ptr(S, "S", self.shape)
        pf = _dev_ptr(F, "F", self.f_shape)
        self.stream = stream if stream is not None else torch.cuda.Stream(device=S.device)
        self._ctx = ctypes.c_void_p()
        with torch.cuda.device(self.device):
            self.stream.wait_stream(torch.cuda.current_stream())
            _lib.check(L.sfseg_create_mc(ctypes.byref(self.cfg), ps, pf, self.n_features,
                                         ctypes.c_void_p(self.stream.cuda_stream),
                                         ctypes.byref(self._ctx)), "sfseg_create_mc")

    # -- context management ------------------------------------------------
    def close(self) -> None:
        if getattr(self, "_ctx", None) is not None and self._ctx.value:
            with torch.cuda.device(self.device):
                _lib.lib().sfseg_destroy(self._ctx)
            self._ctx = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    def _handle(self):
        if not self._ctx.value:
            raise RuntimeError("solver is closed")
        return self._ctx

    # -- entry points --------------------------------------------------------
    def set_features(self, S: torch.Tensor, F: Optional[torch.Tensor] = None) -> None:
        ps = _dev_ptr(S, "S", self.shape)
        pf = _dev_ptr(F, "F", self.f_shape)
        with torch.cuda.device(self.device):
            self.stream.wait_stream(torch.cuda.current_stream())
            _lib.check(_lib.lib().sfseg_set_features(self._handle(), ps, pf),
                       "sfseg_set_features")

    def iterate(self, x0: Optional[torch.Tensor] = None, max_iters: int = 100,
                tol: float = 1e-5) -> IterResult:
        px = _dev_ptr(x0, "x0", self.shape)
        res = _lib.Result()
        with torch.cuda.device(self.device):
            self.stream.wait_stream(torch.cuda.current_stream())
            _lib.check(_lib.lib().sfseg_power_iterate(self._handle(), px, int(max_iters),
                                                      float(tol), ctypes.byref(res)),
                       "sfseg_power_iterate")
        return IterResult(int(res.iters), bool(res.converged), float(res.delta), float(res.lam))

    def eigvec(self, out: Optional[torch.Tensor] = None) -> torch.Tensor:
        with torch.cuda.device(self.device):
            if out is None:
                with torch.cuda.stream(self.stream):
                    out = torch.empty(self.shape, dtype=torch.float32, device=self.device)
            else:
                self.stream.wait_stream(torch.cuda.current_stream())
            po = _dev_ptr(out, "out", self.shape)
            _lib.check(_lib.lib().sfseg_eigvec(self._handle(), po), "sfseg_eigvec")
            torch.cuda.current_stream().wait_stream(self.stream)
        return out

    def apply(self, x: torch.Tensor, out: Optional[torch.Tensor] = None) -> torch.Tensor:
        px = _dev_ptr(x, "x", self.shape)
        with torch.cuda.device(self.device):
            if out is None:
                with torch.cuda.stream(self.stream):
                    out = torch.empty(self.shape, dtype=torch.float32, device=self.device)
            po = _dev_ptr(out, "out", self.shape)
            self.stream.wait_stream(torch.cuda.current_stream())
            _lib.check(_lib.lib().sfseg_apply(self._handle(), px, po), "sfseg_apply")
            torch.cuda.current_stream().wait_stream(self.stream)
        return out

    def spectral_grad(self, xhat: torch.Tensor, target: torch.Tensor, k: int,
                      out: Optional[torch.Tensor] = None):
        """Loss 1 - cos(M^k xhat, target) and its gradient with respect to
        xhat (sfseg_spectral_grad): (grad, loss)."""
        px = _dev_ptr(xhat, "xhat", self.shape)
        pt = _dev_ptr(target, "target", self.shape)
        with torch.cuda.device(self.device):
            if out is None:
                with torch.cuda.stream(self.stream):
                    out = torch.empty(self.shape, dtype=torch.float32, device=self.device)
            po = _dev_ptr(out, "out", self.shape)
            self.stream.wait_stream(torch.cuda.current_stream())
            loss = ctypes.c_double()
            _lib.check(_lib.lib().sfseg_spectral_grad(self._handle(), px, pt, int(k), po,
                                                      ctypes.byref(loss)), "sfseg_spectral_grad")
            torch.cuda.current_stream().wait_stream(self.stream)
        return out, float(loss.value)

    def refine_frames(self, out: Optional[torch.Tensor] = None):
        """Frame-wise Rayleigh-Ritz refinement of the current iterate
        (sfseg_refine_frames): (unit start vector, largest Ritz value)."""
        with torch.cuda.device(self.device):
            if out is None:
                with torch.cuda.stream(self.stream):
                    out = torch.empty(self.shape, dtype=torch.float32, device=self.device)
            po = _dev_ptr(out, "out", self.shape)
            self.stream.wait_stream(torch.cuda.current_stream())
            mu = ctypes.c_double()
            _lib.check(_lib.lib().sfseg_refine_frames(self._handle(), po, ctypes.byref(mu)),
                       "sfseg_refine_frames")
            torch.cuda.current_stream().wait_stream(self.stream)
        return out, float(mu.value)

    def iterate_refined(self, x0: Optional[torch.Tensor] = None, pre_steps: int = 5,
                        refinements: int = 1, between: int = 20, max_iters: int = 20000,
                        tol: float = 1e-5):
        """Warm-started solve: `pre_steps` plain steps from x0 (S by
        default), the frame-wise refinement, then -- `refinements` - 1 more
        times -- `between` plain steps and another refinement, then plain
        steps to `tol`.  Returns (final IterResult, steps in all, Ritz values).
        Every step and refinement runs in the library."""
        r = self.iterate(x0, max_iters=pre_steps, tol=0.0)
        steps = r.iters
        mus = []
        for i in range(refinements):
            if i:
                r = self.iterate(x, max_iters=between, tol=0.0)
                steps += r.iters
            x, mu = self.refine_frames()
            mus.append(mu)
        r = self.iterate(x, max_iters=max_iters, tol=tol)
        return r, steps + r.iters, mus

    # -- binarisation (Sec. 4.1) ----------------------------------------------
    def _mask_out(self, out: Optional[torch.Tensor]) -> torch.Tensor:
        if out is None:
            with torch.cuda.stream(self.stream):
                return torch.empty(self.shape, dtype=torch.uint8, device=self.device)
        if (not isinstance(out, torch.Tensor) or out.device.type != "cuda"
                or out.dtype != torch.uint8 or not out.is_contiguous()
                or tuple(out.shape) != tuple(self.shape)):
            raise TypeError(f"mask must be a contiguous uint8 CUDA tensor of shape {self.shape}")
        self.stream.wait_stream(torch.cuda.current_stream())
        return out

    def project(self, slope: float = 10.0, threshold: float = 0.5) -> None:
        """Replace the current iterate by its sigmoid projection (sfseg_project)."""
        with torch.cuda.device(self.device):
            self.stream.wait_stream(torch.cuda.current_stream())
            _lib.check(_lib.lib().sfseg_project(self._handle(), float(slope), float(threshold)),
                       "sfseg_project")

    def threshold(self, threshold: float = 0.5,
                  out: Optional[torch.Tensor] = None) -> torch.Tensor:
        """Hard threshold of the current iterate as a uint8 (T, H, W) mask."""
        with torch.cuda.device(self.device):
            out = self._mask_out(out)
            _lib.check(_lib.lib().sfseg_threshold(self._handle(), float(threshold),
                                                  out.data_ptr()), "sfseg_threshold")
            torch.cuda.current_stream().wait_stream(self.stream)
        return out

    def segment(self, x0: Optional[torch.Tensor] = None, iters: int = 5, project_from: int = 3,
                slope: float = 10.0, threshold: float = 0.5, mask: bool = True,
                out: Optional[torch.Tensor] = None):
        """Algorithm 1 with the Sec. 4.1 binarisation (sfseg_segment).
        Returns (IterResult, uint8 mask or None)."""
        px = _dev_ptr(x0, "x0", self.shape)
        b = _lib.Binarize(int(iters), int(project_from), float(slope), float(threshold))
        res = _lib.Result()
        with torch.cuda.device(self.device):
            m = self._mask_out(out) if mask else None
            self.stream.wait_stream(torch.cuda.current_stream())
            _lib.check(_lib.lib().sfseg_segment(self._handle(), px, ctypes.byref(b),
                                                None if m is None else m.data_ptr(),
                                                ctypes.byref(res)), "sfseg_segment")
            torch.cuda.current_stream().wait_stream(self.stream)
        return IterResult(int(res.iters), bool(res.converged), float(res.delta), float(res.lam)), m

    def plan(self) -> dict:
        pl = _lib.Plan()
        _lib.check(_lib.lib().sfseg_get_plan(self._handle(), ctypes.byref(pl)), "sfseg_get_plan")
        return {"shape": int(pl.shape), "chunks": int(pl.chunks), "blocks": int(pl.blocks),
                "threads": int(pl.threads)}

    def set_plan(self, shape: int, chunks: int) -> None:
        with torch.cuda.device(self.device):
            _lib.check(_lib.lib().sfseg_set_plan(self._handle(), int(shape), int(chunks)),
                       "sfseg_set_plan")

    def timing(self) -> dict:
        t = _lib.Timing()
        _lib.check(_lib.lib().sfseg_last_timing(self._handle(), ctypes.byref(t)),
                   "sfseg_last_timing")
        return {"total_ms": t.total_ms, "init_ms": t.init_ms, "loop_ms": t.loop_ms,
                "iters": int(t.iters), "launches": int(t.launches)}

    def autotune(self, steps: int = 8, cache: Optional[str] = None) -> dict:
        return _autotune(self, steps, cache, [self.shape])


def _arch(device) -> str:
    return torch.cuda.get_device_properties(device).gcnArchName


def _autotune(solver, steps: int, cache: Optional[str], shapes) -> dict:
    """Pick the fastest work plan (timed by the library) and optionally
    remember it in `cache`, a JSON file of {key: [shape, chunks]}."""
    c = solver.cfg
    key = json.dumps({"shapes": [list(s) for s in shapes], "r_t": c.r_t, "r_s": c.r_s,
                      "storage": c.storage, "features": int(getattr(solver, "n_features", 1)),
                      "arch": _arch(solver.device)}, sort_keys=True)
    table = {}
    if cache and os.path.exists(cache):
        with open(cache) as fh:
            table = json.load(fh)
    if key in table:
        solver.set_plan(*table[key])
        return dict(solver.plan(), cached=True)
    pl = _lib.Plan()
    with torch.cuda.device(solver.device):
        solver.stream.wait_stream(torch.cuda.current_stream())
        _lib.check(_lib.lib().sfseg_autotune(solver._handle(), int(steps), ctypes.byref(pl)),
                   "sfseg_autotune")
    if cache:
        table[key] = [int(pl.shape), int(pl.chunks)]
        tmp = cache + ".tmp"
        with open(tmp, "w") as fh:
            json.dump(table, fh, indent=1, sort_keys=True)
        os.replace(tmp, cache)
    return dict(solver.plan(), cached=False)


class BatchSolver:
    """Power iteration of many clips at once (one persistent launch per step).

    ``S`` is a sequence of float32 CUDA tensors (T_i, H_i, W_i); ``F`` is None
    or a sequence of the same shapes (None entries mean F = S).  All clips
    share the graph parameters.
    """

    def __init__(self, S: Sequence[torch.Tensor], F: Optional[Sequence] = None, *, r_t: int = 1,
                 r_s: int = 2, sigma_t: float = 1.0, sigma_s: float = 1.0, alpha: float = 1.0,
                 p: float = 0.2, storage: str = "f32",
                 stream: Optional[torch.cuda.Stream] = None):
        L = _lib.lib()
        n = len(S)
        if n < 1:
            raise ValueError("need at least one clip")
        self.shapes = [tuple(int(v) for v in t.shape) for t in S]
        self.device = S[0].device
        cfgs = (_lib.Config * n)()
        for i, sh in enumerate(self.shapes):
            if len(sh) != 3:
                raise ValueError("each clip must be (T, H, W)")
            cfgs[i] = _lib.make_config(*sh, r_t=r_t, r_s=r_s, sigma_t=sigma_t, sigma_s=sigma_s,
                                       alpha=alpha, p=p, storage=storage)
        self.cfg = cfgs[0]
        self._cfgs = cfgs
        ps = (ctypes.c_void_p * n)(*[_dev_ptr(t, f"S[{i}]", self.shapes[i]) for i, t in enumerate(S)])
        pf = None
        if F is not None:
            pf = (ctypes.c_void_p * n)(*[_dev_ptr(t, f"F[{i}]", self.shapes[i])
                                         for i, t in enumerate(F)])
        self.stream = stream if stream is not None else torch.cuda.Stream(device=self.device)
        self._ctx = ctypes.c_void_p()
        with torch.cuda.device(self.device):
            self.stream.wait_stream(torch.cuda.current_stream())
            _lib.check(L.sfseg_batch_create(cfgs, n, ps, pf, ctypes.c_void_p(self.stream.cuda_stream),
                                            ctypes.byref(self._ctx)), "sfseg_batch_create")

    def __len__(self):
        return len(self.shapes)

    def close(self) -> None:
        if getattr(self, "_ctx", None) is not None and self._ctx.value:
            with torch.cuda.device(self.device):
                _lib.lib().sfseg_destroy(self._ctx)
            self._ctx = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    def _handle(self):
        if not self._ctx.value:
            raise RuntimeError("solver is closed")
        return self._ctx

    def iterate(self, x0: Optional[Sequence] = None, max_iters: int = 100,
                tol: float = 1e-5) -> List[IterResult]:
        n = len(self)
        px = None
        if x0 is not None:
            px = (ctypes.c_void_p * n)(*[_dev_ptr(t, f"x0[{i}]", self.shapes[i])
                                         for i, t in enumerate(x0)])
        res = (_lib.Result * n)()
        with torch.cuda.device(self.device):
            self.stream.wait_stream(torch.cuda.current_stream())
            st = _lib.lib().sfseg_batch_iterate(self._handle(), px, int(max_iters), float(tol), res)
        out = [IterResult(int(r.iters), bool(r.converged), float(r.delta), float(r.lam))
               for r in res]
        self.last_results = out
        _lib.check(st, "sfseg_batch_iterate")
        return out

    def eigvecs(self) -> List[torch.Tensor]:
        with torch.cuda.device(self.device):
            with torch.cuda.stream(self.stream):
                outs = [torch.empty(sh, dtype=torch.float32, device=self.device)
                        for sh in self.shapes]
            po = (ctypes.c_void_p * len(outs))(*[t.data_ptr() for t in outs])
            _lib.check(_lib.lib().sfseg_batch_eigvec(self._handle(), po), "sfseg_batch_eigvec")
            torch.cuda.current_stream().wait_stream(self.stream)
        return outs

    def plan(self) -> dict:
        return Solver.plan(self)

    def set_plan(self, shape: int, chunks: int) -> None:
        Solver.set_plan(self, shape, chunks)

    def timing(self) -> dict:
        return Solver.timing(self)

    def autotune(self, steps: int = 4, cache: Optional[str] = None) -> dict:
        return _autotune(self, steps, cache, self.shapes)
