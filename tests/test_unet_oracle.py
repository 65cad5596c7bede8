"""Pins of the warm-start network's FP64 oracle (CPU only).

The forward layers are checked against brute-force loops and exact identities;
the hand-written backward pass against central finite differences of the loss
and against adjoint identities, so that a dropped term, a wrong sign or a
flipped tap anywhere in it fails a test.
"""
import numpy as np
import pytest

from oracle import unet_oracle as U


def _rng(seed):
    return np.random.Generator(np.random.PCG64(seed))


def _conv3_loops(x, W, b):
    Cin, T, H, Wd = x.shape
    Cout = W.shape[0]
    y = np.zeros((Cout, T, H, Wd))
    for co in range(Cout):
        for t in range(T):
            for i in range(H):
                for j in range(Wd):
                    acc = b[co]
                    for ci in range(Cin):
                        for a in range(3):
                            for bb in range(3):
                                for cc in range(3):
                                    tt, ii, jj = t + a - 1, i + bb - 1, j + cc - 1
                                    if 0 <= tt < T and 0 <= ii < H and 0 <= jj < Wd:
                                        acc += W[co, ci, a, bb, cc] * x[ci, tt, ii, jj]
                    y[co, t, i, j] = acc
    return y


def test_conv3_matches_brute_force_loops():
    r = _rng(1)
    x = r.normal(size=(2, 3, 4, 5))
    W = r.normal(size=(3, 2, 3, 3, 3))
    b = r.normal(size=3)
    np.testing.assert_allclose(U.conv3(x, W, b), _conv3_loops(x, W, b), rtol=1e-12, atol=1e-12)


def test_conv3_delta_kernels_are_shifts():
    r = _rng(2)
    x = r.normal(size=(1, 4, 5, 6))
    W = np.zeros((1, 1, 3, 3, 3))
    W[0, 0, 1, 1, 1] = 1.0
    np.testing.assert_array_equal(U.conv3(x, W, np.zeros(1)), x)
    W[:] = 0.0
    W[0, 0, 2, 1, 0] = 1.0          # reads x[t + 1, y, x - 1]
    y = U.conv3(x, W, np.zeros(1))
    np.testing.assert_array_equal(y[0, :-1, :, 1:], x[0, 1:, :, :-1])
    assert np.all(y[0, -1] == 0.0) and np.all(y[0, :, :, 0] == 0.0)


def test_conv3_backward_is_the_adjoint():
    r = _rng(3)
    x = r.normal(size=(3, 3, 5, 4))
    W = r.normal(size=(2, 3, 3, 3, 3))
    gy = r.normal(size=(2, 3, 5, 4))
    gx, gW, gb = U.conv3_backward(x, W, gy)
    # <conv(x), gy> is linear in x and in W: its gradients are gx and gW
    lhs = np.sum(U.conv3(x, W, np.zeros(2)) * gy)
    assert abs(lhs - np.sum(gx * x)) <= 1e-10 * abs(lhs)
    assert abs(lhs - np.sum(gW * W)) <= 1e-10 * abs(lhs)
    np.testing.assert_allclose(gb, gy.sum(axis=(1, 2, 3)))


@pytest.mark.parametrize("shape", [(2, 4, 6), (3, 5, 7), (1, 1, 1)])
def test_pool_and_up_adjoints_and_values(shape):
    r = _rng(4)
    x = r.normal(size=(2,) + shape)
    p = U.pool2(x)
    assert p.shape[1:] == tuple((n + 1) // 2 for n in shape)
    g = r.normal(size=p.shape)
    assert abs(np.sum(p * g) - np.sum(x * U.pool2_backward(g, x.shape))) <= 1e-12
    u = U.up2(g, shape)
    assert u.shape[1:] == shape
    assert abs(np.sum(u * x) - np.sum(g * U.up2_backward(x, g.shape[1:]))) <= 1e-12
    # constant input: interior windows average to the constant; a corner
    # window of an odd size holds the zero padding
    c = U.pool2(np.ones((1,) + shape))
    assert c[0, 0, 0, 0] == (1.0 if min(shape) >= 2 else 1.0 / 8.0)
    if min(shape) >= 2:
        # up then pool returns the input (each output averages 8 equal values)
        even = tuple(2 * ((n + 1) // 2) for n in shape)
        np.testing.assert_allclose(U.pool2(U.up2(p, even)), p, rtol=1e-15)


def test_cosine_loss_values_and_scale_invariance():
    r = _rng(5)
    a = r.random(50) + 0.1
    assert abs(U.cosine_loss(a, a)[0]) <= 1e-15
    assert abs(U.cosine_loss(3.0 * a, a)[0]) <= 1e-15
    b = r.random(50)
    l1, g1 = U.cosine_loss(a, b)
    l2, g2 = U.cosine_loss(2.0 * a, b)
    assert abs(l1 - l2) <= 1e-14
    np.testing.assert_allclose(g2, g1 / 2.0, rtol=1e-12)
    assert abs(g1 @ a) <= 1e-12          # no gradient along the prediction itself


def test_param_pack_roundtrip_and_count():
    p = U.init_params(7)
    flat = U.pack(p)
    assert flat.size == U.param_count() == sum(
        co * ci * (27 if k == 3 else 1) + co for _, ci, co, k in U.LAYERS)
    q = U.unpack(flat)
    for n, _, _, _ in U.LAYERS:
        np.testing.assert_array_equal(p[n][0], q[n][0])
        np.testing.assert_array_equal(p[n][1], q[n][1])


@pytest.mark.parametrize("shape", [(4, 8, 8), (3, 5, 7)])
def test_network_gradient_matches_finite_differences(shape):
    r = _rng(6)
    params = U.init_params(11)
    S = r.random(shape)
    target = r.random(shape) + 0.05
    xh, cache = U.forward(params, S)
    assert xh.shape == shape and np.all(xh > 0)
    loss, grads = U.backward(params, cache, target)

    def loss_at(p):
        return U.cosine_loss(U.forward(p, S)[0], target)[0]

    flat = U.pack(params)
    gflat = U.pack(grads)
    # every layer's weights and biases: a few coordinates each
    idx, o = [], 0
    for name, ci, co, k in U.LAYERS:
        nw = co * ci * (27 if k == 3 else 1)
        idx += list(o + r.choice(nw, size=3, replace=False)) + [o + nw + int(r.integers(co))]
        o += nw + co
    h = 1e-6
    for i in idx:
        fp, fm = flat.copy(), flat.copy()
        fp[i] += h
        fm[i] -= h
        fd = (loss_at(U.unpack(fp)) - loss_at(U.unpack(fm))) / (2 * h)
        # central differences: O(h^2) truncation, ~1e-16 / h rounding
        assert abs(fd - gflat[i]) <= 1e-5 * abs(fd) + 2e-9, (i, fd, gflat[i])


def test_planted_backward_mistake_is_caught():
    # a transposed tap in the data gradient must break the finite-difference pin
    r = _rng(8)
    x = r.normal(size=(2, 3, 4, 4))
    W = r.normal(size=(2, 2, 3, 3, 3))
    gy = r.normal(size=(2, 3, 4, 4))
    gx, _, _ = U.conv3_backward(x, W, gy)
    Wbad = W.copy()
    Wbad[:, :, 0], Wbad[:, :, 2] = W[:, :, 2].copy(), W[:, :, 0].copy()
    gx_bad, _, _ = U.conv3_backward(x, Wbad, gy)
    lhs = np.sum(U.conv3(x, W, np.zeros(2)) * gy)
    assert abs(lhs - np.sum(gx * x)) <= 1e-10 * abs(lhs)
    assert abs(lhs - np.sum(gx_bad * x)) > 1e-3 * abs(lhs)


# ---------------------------------------------------------------------------
# Spectral training loss: L = 1 - cos(M^k x^, x*)
# ---------------------------------------------------------------------------

def _small_graph():
    from oracle import OracleConfig, build_adjacency
    r = _rng(21)
    S = r.random((3, 6, 7))
    S[S < 0.2] = 0.0
    cfg = OracleConfig(r_t=1, r_s=2, sigma_t=1.0, sigma_s=1.5, alpha=1.0, p=0.2)
    return S, build_adjacency(S, None, cfg)


@pytest.mark.parametrize("k", [1, 3])
def test_spectral_loss_gradient_matches_finite_differences(k):
    S, M = _small_graph()
    r = _rng(22)
    xh = r.random(S.shape) + 0.1
    target = r.random(S.shape)
    loss, g = U.spectral_cosine_loss(lambda v: M @ v, xh, target, k)
    for _ in range(5):
        d = r.normal(size=S.shape)
        h = 1e-6
        lp = U.spectral_cosine_loss(lambda v: M @ v, xh + h * d, target, k)[0]
        lm = U.spectral_cosine_loss(lambda v: M @ v, xh - h * d, target, k)[0]
        fd = (lp - lm) / (2 * h)
        assert abs(fd - np.sum(g * d)) <= 1e-6 * abs(fd) + 1e-9


def test_spectral_loss_of_a_diagonal_operator_is_a_weighted_cosine():
    # r_s = r_t = 0: M = diag(w^2) (Eq. (2) with only the self-loop), so
    # M^k x = w^(2k) x element by element and the gradient is w^(2k) times the
    # cosine-loss gradient at that vector -- written out by hand.
    from oracle import OracleConfig, build_adjacency
    r = _rng(23)
    S = r.random((2, 4, 5)) + 0.1
    cfg = OracleConfig(r_t=0, r_s=0, sigma_t=1.0, sigma_s=1.0, alpha=1.0, p=0.5)
    M = build_adjacency(S, None, cfg)
    d = (S ** 0.5).ravel() ** 2
    xh, t = r.random(S.shape), r.random(S.shape)
    k = 4
    v = d ** k * xh.ravel()
    nv, nt = np.linalg.norm(v), np.linalg.norm(t)
    c = v @ t.ravel() / (nv * nt)
    g = d ** k * -(t.ravel() / (nv * nt) - c * v / nv ** 2)
    loss, gg = U.spectral_cosine_loss(lambda u: M @ u, xh, t, k)
    assert abs(loss - (1.0 - c)) <= 1e-14
    assert np.allclose(gg.ravel(), g, rtol=1e-12, atol=1e-15)


def test_spectral_loss_at_the_eigenvector_is_zero_and_flat():
    S, M = _small_graph()
    lam, V = np.linalg.eigh(M.toarray())
    v1 = np.abs(V[:, -1]).reshape(S.shape)
    loss, g = U.spectral_cosine_loss(lambda v: M @ v, 2.0 * v1, v1, 5)
    assert abs(loss) <= 1e-12
    assert np.linalg.norm(g) <= 1e-9


def test_planted_spectral_mistake_is_caught():
    # one product too few on the way back breaks the finite-difference pin
    S, M = _small_graph()
    r = _rng(24)
    xh, target = r.random(S.shape) + 0.1, r.random(S.shape)
    k = 3
    v = xh.ravel()
    for _ in range(k):
        v = M @ v
    _, gv = U.cosine_loss(v, target.ravel())
    g_bad = gv
    for _ in range(k - 1):
        g_bad = M @ g_bad
    d = r.normal(size=S.shape)
    h = 1e-6
    fd = (U.spectral_cosine_loss(lambda u: M @ u, xh + h * d, target, k)[0]
          - U.spectral_cosine_loss(lambda u: M @ u, xh - h * d, target, k)[0]) / (2 * h)
    assert abs(fd - np.sum(g_bad * d.ravel())) > 1e-3 * abs(fd)
