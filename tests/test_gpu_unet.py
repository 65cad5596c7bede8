"""Warm-start network on the GPU: forward, gradients and Adam against the
FP64 oracle (``oracle/unet_oracle.py``), and a short training run showing
what the network gains over a cold start.

The network computes in bfloat16 (activations, weight copies, gradients
between layers) with FP32 accumulation, so its results are compared with the
FP64 oracle under tolerances scaled to bfloat16 (8 significant bits through
ten layers); every measured error is printed.
"""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

from oracle import unet_oracle as U  # noqa: E402
from paper_1907_02731_amd.synth import make_clip  # noqa: E402
from paper_1907_02731_amd.warmstart import (UNet, eigenvector_targets, he_init,  # noqa: E402
                                            solve_cold, solve_warm, train)

pytestmark = pytest.mark.gpu
DEV = "cuda:0"


def _t(a):
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.float32)).to(DEV)


def _rel(a, b):
    return float(np.linalg.norm(np.ravel(a) - np.ravel(b)) / max(np.linalg.norm(np.ravel(b)), 1e-30))


SHAPES = [(4, 8, 8), (5, 13, 37), (3, 20, 70)]


@pytest.mark.parametrize("shape", SHAPES)
def test_forward_matches_oracle(shape):
    params = U.init_params(21)
    r = np.random.Generator(np.random.PCG64(22))
    S = r.random(shape)
    ref, _ = U.forward(params, S)
    with UNet(shape) as net:
        net.set_params(U.pack(params))
        got = net.forward(_t(S)).cpu().numpy().astype(np.float64)
    err = _rel(got, ref)
    print(f"forward {shape}: rel L2 {err:.3e}", flush=True)
    assert got.shape == ref.shape and np.all(got > 0)
    assert err <= 3e-2


@pytest.mark.parametrize("shape", [(1, 1, 1), (2, 3, 5), (5, 13, 37), (3, 20, 70), (7, 9, 130),
                                   (9, 70, 200)])
def test_inference_forward_equals_the_training_forward(shape):
    """The inference network fuses what training keeps apart (the upsampled
    half of the last concatenation read at the parent voxels, the head in the
    last convolution's epilogue, the first layer reading S without a copy,
    the skip tensor on its own); on the same weights and input it gives the
    training network's output bit for bit.  Shapes with ragged row and voxel
    tiles, several tiles of the first layer, and odd sizes at every level."""
    params = U.init_params(23)
    r = np.random.Generator(np.random.PCG64(24))
    S = _t(r.random(shape))
    with UNet(shape) as a, UNet(shape, training=True) as b:
        a.set_params(U.pack(params))
        b.set_params(U.pack(params))
        x_inf = a.forward(S).cpu().numpy()
        x_tr = b.forward(S).cpu().numpy()
    d = float(np.max(np.abs(x_inf - x_tr)))
    print(f"inference vs training {shape}: max |diff| {d:.3e}", flush=True)
    assert np.all(np.isfinite(x_inf)) and np.all(x_inf > 0)
    assert np.array_equal(x_inf, x_tr)


@pytest.mark.parametrize("training", [False, True])
def test_forward_in_place_and_in_a_larger_network(training):
    """S and out may be the same buffer (the first kernel reads S, the last
    writes out), and a network sized for a larger volume gives the same
    output, bit for bit, on a smaller one."""
    shape = (5, 13, 37)
    params = U.pack(U.init_params(25))
    S = np.random.Generator(np.random.PCG64(26)).random(shape)
    with UNet(shape, training=training) as a, UNet((9, 40, 96), training=training) as b:
        a.set_params(params)
        b.set_params(params)
        ref = a.forward(_t(S)).cpu().numpy()
        buf = _t(S)
        a.forward(buf, out=buf)
        big = b.forward(_t(S)).cpu().numpy()
        inplace = buf.cpu().numpy()
    assert np.array_equal(inplace, ref)
    assert np.array_equal(big, ref)


@pytest.mark.parametrize("shape", [(5, 13, 37), (6, 24, 40)])
def test_gradients_match_oracle(shape):
    params = U.init_params(31)
    r = np.random.Generator(np.random.PCG64(32))
    S = r.random(shape)
    target = r.random(shape) + 0.05
    xh, cache = U.forward(params, S)
    loss_ref, grads = U.backward(params, cache, target)
    with UNet(shape, training=True) as net:
        net.set_params(U.pack(params))
        net.forward(_t(S))
        loss = net.backward(_t(target))
        g = U.unpack(net.get_grads())
    print(f"loss gpu {loss:.6f} oracle {loss_ref:.6f}", flush=True)
    assert abs(loss - loss_ref) <= 2e-2 * abs(loss_ref) + 1e-4
    # The cosine loss's gradient is orthogonal to the prediction, so the weight
    # gradients are sums with heavy cancellation; with bfloat16 gradients
    # between layers the relative error of a layer's gradient is a few
    # percent.  A wrong tap, sign or channel would give errors of order one.
    worst = 0.0
    for name, _, _, _ in U.LAYERS:
        ew = _rel(g[name][0], grads[name][0])
        eb = _rel(g[name][1], grads[name][1])
        print(f"  {name:6s} gW rel {ew:.3e}  gb rel {eb:.3e}", flush=True)
        worst = max(worst, ew, eb)
    assert worst <= 0.08
    a, b = U.pack(g), U.pack(grads)
    assert float(a @ b) / (np.linalg.norm(a) * np.linalg.norm(b)) >= 0.999


def test_adam_step_matches_the_update_rule():
    shape = (4, 8, 8)
    params = U.init_params(41)
    flat = U.pack(params).astype(np.float32)
    r = np.random.Generator(np.random.PCG64(42))
    S, target = r.random(shape), r.random(shape) + 0.05
    with UNet(shape, training=True) as net:
        net.set_params(flat)
        m = np.zeros_like(flat)
        v = np.zeros_like(flat)
        w = flat.astype(np.float64)
        for step in (1, 2):
            net.forward(_t(S))
            net.backward(_t(target))
            g = net.get_grads().astype(np.float64)
            net.adam_step(1e-3, step)
            m = 0.9 * m + 0.1 * g
            v = 0.999 * v + 0.001 * g * g
            w = w - 1e-3 * (m / (1 - 0.9 ** step)) / (np.sqrt(v / (1 - 0.999 ** step)) + 1e-8)
            got = net.get_params().astype(np.float64)
            assert np.max(np.abs(got - w)) <= 1e-6 * max(1.0, np.max(np.abs(w)))
            w = got


def test_param_layout_and_errors():
    with UNet((2, 4, 4)) as net:
        assert net.n_params == U.param_count() == he_init(0).size
        with pytest.raises(ValueError):
            net.set_params(np.zeros(3, np.float32))
        from paper_1907_02731_amd import _lib
        with pytest.raises(_lib.SfsegError) as e:
            net.forward(_t(np.zeros((3, 4, 4))))       # larger than the network's maximum
        assert e.value.status == _lib.SFSEG_ERR_INVALID_ARG
        with pytest.raises(_lib.SfsegError) as e:
            net.backward(_t(np.ones((2, 4, 4))))        # created without training buffers
        assert e.value.status == _lib.SFSEG_ERR_STATE


def test_training_gains_over_cold_start():
    """A short training run on small clips.  The loss falls; on held-out clips
    the network's estimate is much closer to the principal eigenvector than
    the input map S is; started from it, the plain method reaches the same
    eigenvector in fewer steps on average (strictly).  Same eigenvector: the
    Rayleigh quotients agree to 1e-6, and the two vectors lie within the sum
    of their distances to v_1 as the convergence rate bounds them: after a
    stop at change delta the error left is about delta r / (1 - r), r the
    measured per-step contraction (lambda_2 / lambda_1, taken from the change
    over the last 20 steps of the cold run), with a factor 3 for the
    pre-asymptotic steps.  Wall time including inference is printed; the
    full-resolution comparison is the benchmark's warm-start workload."""
    shape = (16, 64, 96)
    graph = dict(r_t=2, r_s=5, sigma_t=1.0, sigma_s=2.0, alpha=1.0, p=0.2)
    clips = [make_clip(*shape, seed=70000 + i, n_blobs=3, noise_sigma=0.15, motion="affine",
                       dtype=np.float32) for i in range(56)]
    tg = eigenvector_targets(clips, tol=1e-6, graph=graph)
    inputs = [_t(c) for c in clips]

    def cos_err(a, b):
        a = a.double().ravel()
        b = b.double().ravel()
        return 1.0 - float(a @ b / (torch.linalg.norm(a) * torch.linalg.norm(b)))

    with UNet(shape, training=True) as net:
        net.set_params(he_init(5))
        losses = train(net, inputs[:48], tg[:48], epochs=4, lr=2e-3, lr_final=2e-4, seed=1)
        first, last = np.mean(losses[:24]), np.mean(losses[-24:])
        print(f"loss: first 24 steps {first:.4f}, last 24 steps {last:.4f}", flush=True)
        assert last < 0.2 * first
        cold_it, warm_it, e_s, e_net, t_cold, t_warm = [], [], [], [], [], []
        for S, t in zip(inputs[48:], tg[48:]):
            e_s.append(cos_err(S, t))
            e_net.append(cos_err(net.forward(S), t))
            rc, xc, tc = solve_cold(S, tol=1e-5, graph=graph)
            rw, xw, tw, _ = solve_warm(S, net, tol=1e-5, graph=graph)
            assert rc.converged and rw.converged
            assert abs(rw.lam - rc.lam) <= 1e-6 * rc.lam
            # per-step contraction from the cold run's change over its last 20 steps
            r20 = solve_cold(S, tol=0.0, graph=graph, max_iters=rc.iters - 20)[0]
            rate = (rc.delta / r20.delta) ** (1.0 / 20)
            assert 0.0 < rate < 1.0
            bound = 3.0 * (rc.delta + rw.delta) * rate / (1.0 - rate)
            d = float(np.linalg.norm(xw.cpu().numpy().astype(np.float64) -
                                     xc.cpu().numpy().astype(np.float64)))
            print(f"  contraction {rate:.4f}: ||x_warm - x_cold|| = {d:.2e} <= {bound:.2e}",
                  flush=True)
            assert d <= bound
            cold_it.append(rc.iters)
            warm_it.append(rw.iters)
            t_cold.append(tc)
            t_warm.append(tw)
    print(f"held-out 1 - cos to the eigenvector: S {np.mean(e_s):.4f}, network {np.mean(e_net):.4f}",
          flush=True)
    print(f"held-out steps to 1e-5: cold {cold_it} warm {warm_it}", flush=True)
    print(f"held-out time to 1e-5 (warm includes inference): cold {1e3 * np.mean(t_cold):.2f} ms, "
          f"warm {1e3 * np.mean(t_warm):.2f} ms", flush=True)
    assert np.mean(e_net) <= 0.25 * np.mean(e_s)
    assert np.mean(warm_it) < np.mean(cold_it)
