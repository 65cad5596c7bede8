"""FP64 CPU oracle of the warm-start network -- TEST INFRASTRUCTURE ONLY.

The method starts its power iteration from a soft segmentation that another
method provides (Sec. 4, Algorithm 1 initialises x with the input map), and
the paper's conclusion proposes learning the whole pipeline end to end.  The
warm start here is a small 3D convolutional network that maps the input map
S to an estimate of the principal eigenvector; its output only replaces the
start vector, and plain power iteration then runs to the same tolerance, so
the method itself still decides the result.

This module is the plain, slow, float64 definition that the GPU kernels are
checked against.  It shares no code with them.  Arrays are channels-first:
an activation is (C, T, H, W), a 3x3x3 weight is (Cout, Cin, 3, 3, 3) with
tap [dt + 1, dy + 1, dx + 1] multiplying the input at offset (dt, dy, dx).

Network (3 levels, widths 16 / 32 / 64; every conv is 3x3x3 with zero padding
and a bias, followed by ReLU; "pool" is a 2x2x2 average over a zero-padded
window, output size ceil(n / 2); "up" repeats each voxel 2x2x2 and crops to
the size of the skip connection it is concatenated with):

    e1 = relu(conv(relu(conv(S, enc1a)), enc1b))              16 ch, full size
    e2 = relu(conv(relu(conv(pool(e1), enc2a)), enc2b))       32 ch, 1/2
    b  = relu(conv(relu(conv(pool(e2), bota)), botb))         64 ch, 1/4
    d2 = relu(conv(relu(conv([up(b), e2], dec2a)), dec2b))    32 ch, 1/2 (96 in)
    d1 = relu(conv(relu(conv([up(d2), e1], dec1a)), dec1b))   16 ch, full (48 in)
    x^ = softplus(head . d1 + head_b)                          1 ch (1x1x1 conv)

Loss (scale invariant, the eigenvector is defined up to scale):
    L = 1 - <x^, x*> / (||x^|| ||x*||)

Flat parameter order (the exchange format with the library): for each layer
in LAYERS, W in row-major (Cout, Cin, 3, 3, 3) order ((1, 16) for the head),
then b (Cout).
"""
from __future__ import annotations

from typing import Dict, List, Tuple

import numpy as np

__all__ = ["LAYERS", "param_count", "init_params", "pack", "unpack", "conv3", "conv3_backward",
           "pool2", "pool2_backward", "up2", "up2_backward", "forward", "backward",
           "cosine_loss", "spectral_cosine_loss"]

# (name, Cin, Cout, kernel size)
LAYERS: List[Tuple[str, int, int, int]] = [
    ("enc1a", 1, 16, 3), ("enc1b", 16, 16, 3),
    ("enc2a", 16, 32, 3), ("enc2b", 32, 32, 3),
    ("bota", 32, 64, 3), ("botb", 64, 64, 3),
    ("dec2a", 96, 32, 3), ("dec2b", 32, 32, 3),
    ("dec1a", 48, 16, 3), ("dec1b", 16, 16, 3),
    ("head", 16, 1, 1),
]


def _wshape(cin: int, cout: int, k: int):
    return (cout, cin, 3, 3, 3) if k == 3 else (cout, cin)


def param_count() -> int:
    return sum(int(np.prod(_wshape(ci, co, k))) + co for _, ci, co, k in LAYERS)


def init_params(seed: int) -> Dict[str, Tuple[np.ndarray, np.ndarray]]:
    """He-normal weights (fan-in), small random biases."""
    rng = np.random.Generator(np.random.PCG64(seed))
    out = {}
    for name, ci, co, k in LAYERS:
        fan_in = ci * (27 if k == 3 else 1)
        W = rng.normal(0.0, np.sqrt(2.0 / fan_in), size=_wshape(ci, co, k))
        b = rng.normal(0.0, 0.01, size=co)
        out[name] = (W, b)
    return out


def pack(params) -> np.ndarray:
    return np.concatenate([np.concatenate([params[n][0].ravel(), params[n][1].ravel()])
                           for n, _, _, _ in LAYERS])


def unpack(flat: np.ndarray):
    flat = np.asarray(flat, dtype=np.float64)
    if flat.size != param_count():
        raise ValueError(f"expected {param_count()} parameters, got {flat.size}")
    out, o = {}, 0
    for name, ci, co, k in LAYERS:
        shp = _wshape(ci, co, k)
        n = int(np.prod(shp))
        out[name] = (flat[o:o + n].reshape(shp), flat[o + n:o + n + co].copy())
        o += n + co
    return out


# ---------------------------------------------------------------------------
# layers (float64, channels-first)
# ---------------------------------------------------------------------------
def _shifted(x: np.ndarray, dt: int, dy: int, dx: int) -> np.ndarray:
    """x at offset (dt, dy, dx): out[..., t, y, x] = x[..., t+dt, y+dy, x+dx], 0 outside."""
    p = np.pad(x, [(0, 0), (1, 1), (1, 1), (1, 1)])
    T, H, W = x.shape[1:]
    return p[:, 1 + dt:1 + dt + T, 1 + dy:1 + dy + H, 1 + dx:1 + dx + W]


def conv3(x: np.ndarray, W: np.ndarray, b: np.ndarray) -> np.ndarray:
    """3x3x3 convolution (cross-correlation), zero padding 1, bias."""
    y = np.zeros((W.shape[0],) + x.shape[1:])
    for dt in (-1, 0, 1):
        for dy in (-1, 0, 1):
            for dx in (-1, 0, 1):
                xs = _shifted(x, dt, dy, dx)
                y += np.tensordot(W[:, :, dt + 1, dy + 1, dx + 1], xs, axes=(1, 0))
    return y + b[:, None, None, None]


def conv3_backward(x: np.ndarray, W: np.ndarray, gy: np.ndarray):
    """Gradients of conv3 with respect to x, W and b given dL/dy."""
    gx = np.zeros_like(x)
    gW = np.zeros_like(W)
    for dt in (-1, 0, 1):
        for dy in (-1, 0, 1):
            for dx in (-1, 0, 1):
                xs = _shifted(x, dt, dy, dx)
                gW[:, :, dt + 1, dy + 1, dx + 1] = np.tensordot(gy, xs, axes=([1, 2, 3], [1, 2, 3]))
                # y[t] gets W x[t + d]  =>  x[s] receives W^T gy[s - d]
                gx += np.tensordot(W[:, :, dt + 1, dy + 1, dx + 1], _shifted(gy, -dt, -dy, -dx),
                                   axes=(0, 0))
    gb = gy.sum(axis=(1, 2, 3))
    return gx, gW, gb


def pool2(x: np.ndarray) -> np.ndarray:
    """2x2x2 average over a zero-padded window; output size ceil(n / 2)."""
    C, T, H, W = x.shape
    To, Ho, Wo = (T + 1) // 2, (H + 1) // 2, (W + 1) // 2
    p = np.zeros((C, 2 * To, 2 * Ho, 2 * Wo))
    p[:, :T, :H, :W] = x
    return p.reshape(C, To, 2, Ho, 2, Wo, 2).sum(axis=(2, 4, 6)) / 8.0


def pool2_backward(g: np.ndarray, shape) -> np.ndarray:
    C, To, Ho, Wo = g.shape
    full = np.repeat(np.repeat(np.repeat(g, 2, axis=1), 2, axis=2), 2, axis=3) / 8.0
    return full[:, :shape[1], :shape[2], :shape[3]].copy()


def up2(x: np.ndarray, shape) -> np.ndarray:
    """Nearest-neighbour 2x upsampling cropped to spatial shape (T, H, W)."""
    full = np.repeat(np.repeat(np.repeat(x, 2, axis=1), 2, axis=2), 2, axis=3)
    return full[:, :shape[0], :shape[1], :shape[2]].copy()


def up2_backward(g: np.ndarray, src_shape) -> np.ndarray:
    C = g.shape[0]
    To, Ho, Wo = src_shape
    p = np.zeros((C, 2 * To, 2 * Ho, 2 * Wo))
    p[:, :g.shape[1], :g.shape[2], :g.shape[3]] = g
    return p.reshape(C, To, 2, Ho, 2, Wo, 2).sum(axis=(2, 4, 6))


def cosine_loss(xh: np.ndarray, target: np.ndarray):
    """L = 1 - cos(xh, target) and dL/dxh."""
    a = xh.ravel()
    t = target.ravel()
    na, nt = np.linalg.norm(a), np.linalg.norm(t)
    c = float(a @ t) / (na * nt)
    g = -(t / (na * nt) - c * a / (na * na))
    return 1.0 - c, g.reshape(xh.shape)


def spectral_cosine_loss(apply, xh: np.ndarray, target: np.ndarray, k: int):
    """Loss on the error that survives k power-iteration steps, and its
    gradient with respect to the start vector xh:

        v = M^k xh,   L = 1 - cos(v, target),
        dL/dxh = (M^k)^T dL/dv = M^k dL/dv          (M of Eq. (2) is symmetric)

    ``apply(x)`` returns M x for a flat float64 vector.  Power iteration
    (Eq. (4), Eq. (8)) from xh reaches the direction of v after k steps, so L
    measures what k steps leave of the start vector's error.  v is formed by
    k products and normalised once at the end (the loss does not depend on its
    scale); the gradient is dL/dv pushed back through the k products."""
    x = np.asarray(xh, dtype=np.float64).ravel()
    v = x.copy()
    for _ in range(k):
        v = apply(v)
    loss, gv = cosine_loss(v, target)
    g = gv.ravel()
    for _ in range(k):
        g = apply(g)
    return loss, g.reshape(np.shape(xh))


def _relu(v):
    return np.maximum(v, 0.0)


def forward(params, S: np.ndarray):
    """x^ for input S of shape (T, H, W); returns (x^, cache)."""
    c = {}
    x = S[None].astype(np.float64)
    c["in"] = x
    c["e1a"] = _relu(conv3(x, *params["enc1a"]))
    c["e1"] = _relu(conv3(c["e1a"], *params["enc1b"]))
    c["p1"] = pool2(c["e1"])
    c["e2a"] = _relu(conv3(c["p1"], *params["enc2a"]))
    c["e2"] = _relu(conv3(c["e2a"], *params["enc2b"]))
    c["p2"] = pool2(c["e2"])
    c["ba"] = _relu(conv3(c["p2"], *params["bota"]))
    c["b"] = _relu(conv3(c["ba"], *params["botb"]))
    c["cat2"] = np.concatenate([up2(c["b"], c["e2"].shape[1:]), c["e2"]])
    c["d2a"] = _relu(conv3(c["cat2"], *params["dec2a"]))
    c["d2"] = _relu(conv3(c["d2a"], *params["dec2b"]))
    c["cat1"] = np.concatenate([up2(c["d2"], c["e1"].shape[1:]), c["e1"]])
    c["d1a"] = _relu(conv3(c["cat1"], *params["dec1a"]))
    c["d1"] = _relu(conv3(c["d1a"], *params["dec1b"]))
    Wh, bh = params["head"]
    c["z"] = np.tensordot(Wh, c["d1"], axes=(1, 0))[0] + bh[0]
    xh = np.logaddexp(0.0, c["z"])
    return xh, c


def backward(params, cache, target: np.ndarray):
    """Loss and gradients {layer: (gW, gb)} of the cosine loss."""
    c = cache
    loss, gxh = cosine_loss(np.logaddexp(0.0, c["z"]), target)
    gz = gxh / (1.0 + np.exp(-c["z"]))                  # softplus' = sigmoid
    grads = {}
    Wh, _ = params["head"]
    grads["head"] = (np.tensordot(gz, c["d1"], axes=([0, 1, 2], [1, 2, 3]))[None, :],
                     np.array([gz.sum()]))
    g = Wh[0][:, None, None, None] * gz[None]            # dL/dd1

    def conv_relu_back(name, x_in, y_out, g_out):
        gpre = g_out * (y_out > 0)
        gx, gW, gb = conv3_backward(x_in, params[name][0], gpre)
        grads[name] = (gW, gb)
        return gx

    g = conv_relu_back("dec1b", c["d1a"], c["d1"], g)
    g = conv_relu_back("dec1a", c["cat1"], c["d1a"], g)
    n_up = c["d2"].shape[0]
    g_e1_skip = g[n_up:]
    g = up2_backward(g[:n_up], c["d2"].shape[1:])
    g = conv_relu_back("dec2b", c["d2a"], c["d2"], g)
    g = conv_relu_back("dec2a", c["cat2"], c["d2a"], g)
    n_up = c["b"].shape[0]
    g_e2_skip = g[n_up:]
    g = up2_backward(g[:n_up], c["b"].shape[1:])
    g = conv_relu_back("botb", c["ba"], c["b"], g)
    g = conv_relu_back("bota", c["p2"], c["ba"], g)
    g = pool2_backward(g, c["e2"].shape) + g_e2_skip
    g = conv_relu_back("enc2b", c["e2a"], c["e2"], g)
    g = conv_relu_back("enc2a", c["p1"], c["e2a"], g)
    g = pool2_backward(g, c["e1"].shape) + g_e1_skip
    g = conv_relu_back("enc1b", c["e1a"], c["e1"], g)
    conv_relu_back("enc1a", c["in"], c["e1a"], g)
    return loss, grads
