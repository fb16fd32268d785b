"""Pins of the FP64 surrogate-network oracle: finite differences of the loss
(independent of the analytic backward), the convolution's impulse response
and shift equivariance, and Adam's closed form for a constant gradient."""
import numpy as np

from oracle import cnn


def small(seed=0, n=2, cin=4, hidden=5, cout=3, h=6, w=8):
    r = np.random.default_rng(seed)
    x = r.normal(size=(n, cin, h, w))
    t = r.normal(size=(n, cout, h, w))
    p = list(cnn.init_params(cin, hidden, cout, r))
    p[1] = r.normal(size=hidden) * 0.1
    p[3] = r.normal(size=hidden) * 0.1
    p[5] = r.normal(size=cout) * 0.1
    p[4] = p[4] * 10
    return x, t, tuple(p)


def test_conv_impulse_response():
    """A unit impulse at (i0, j0) of input channel c gives, at (i, j), the
    bias plus w[:, c, i0 - i + 1, j0 - j + 1] (circularly), else the bias."""
    r = np.random.default_rng(1)
    w = r.normal(size=(3, 2, 3, 3))
    b = r.normal(size=3)
    x = np.zeros((1, 2, 5, 7))
    i0, j0, c = 0, 6, 1
    x[0, c, i0, j0] = 1.0
    y = cnn.conv3x3(x, w, b)
    for i in range(5):
        for j in range(7):
            di = (i0 - i + 1) % 5
            dj = (j0 - j + 1) % 7
            exp = b + (w[:, c, di, dj] if di < 3 and dj < 3 else 0.0)
            assert np.allclose(y[0, :, i, j], exp, atol=1e-15)


def test_conv_shift_equivariance():
    r = np.random.default_rng(2)
    x = r.normal(size=(2, 3, 6, 5))
    w = r.normal(size=(4, 3, 3, 3))
    b = r.normal(size=4)
    y = cnn.conv3x3(x, w, b)
    ys = cnn.conv3x3(np.roll(x, (2, -1), axis=(2, 3)), w, b)
    assert np.allclose(np.roll(y, (2, -1), axis=(2, 3)), ys, atol=1e-13)


def test_gradients_match_finite_differences():
    x, t, p = small()
    l0, grads = cnn.backward(x, p, t)
    r = np.random.default_rng(3)
    h = 1e-6
    for k, (theta, g) in enumerate(zip(p, grads)):
        for _ in range(6):
            idx = tuple(r.integers(0, s) for s in theta.shape)
            pp = [a.copy() for a in p]
            pm = [a.copy() for a in p]
            pp[k][idx] += h
            pm[k][idx] -= h
            fd = (cnn.loss(cnn.forward(x, pp)[2], t) - cnn.loss(cnn.forward(x, pm)[2], t)) / (2 * h)
            assert abs(fd - g[idx]) <= 1e-6 * max(1.0, abs(fd)), (k, idx, fd, g[idx])


def test_input_gradient_matches_finite_differences():
    """The transposed convolution used for the input gradient."""
    r = np.random.default_rng(4)
    x = r.normal(size=(2, 3, 5, 6))
    w = r.normal(size=(4, 3, 3, 3))
    dy = r.normal(size=(2, 4, 5, 6))
    dx = cnn.conv3x3_grad_input(dy, w)
    h = 1e-6
    for _ in range(10):
        idx = tuple(r.integers(0, s) for s in x.shape)
        xp, xm = x.copy(), x.copy()
        xp[idx] += h
        xm[idx] -= h
        fd = ((dy * cnn.conv3x3(xp, w, np.zeros(4))).sum() - (dy * cnn.conv3x3(xm, w, np.zeros(4))).sum()) / (2 * h)
        assert abs(fd - dx[idx]) < 1e-7 * max(1, abs(fd))


def test_residual_identity_and_zero_loss():
    """With the last layer zero the network is the identity on the first
    cout channels, and the loss against that target is exactly zero."""
    x, _, p = small()
    p = list(p)
    p[4] = np.zeros_like(p[4])
    p[5] = np.zeros_like(p[5])
    _, _, y = cnn.forward(x, p)
    assert (y == x[:, :3]).all()
    l, g = cnn.backward(x, p, x[:, :3])
    assert l == 0.0 and all(not a.any() for a in g)


def test_adam_constant_gradient():
    """For a constant gradient g the bias-corrected moments are exactly g and
    g^2, so every step moves theta by lr g / (|g| + eps)."""
    theta = np.array([1.0, -2.0, 0.5])
    g = np.array([0.3, -4.0, 1e-3])
    m = np.zeros(3)
    v = np.zeros(3)
    for t in range(1, 6):
        new, m, v = cnn.adam_step(theta, g, m, v, t, lr=0.01)
        assert np.allclose(theta - new, 0.01 * g / (np.abs(g) + 1e-8), rtol=1e-12)
        theta = new
