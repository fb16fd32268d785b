"""FP64 reference of the surrogate network: a three-layer convolutional net on
periodic coarse fields, its mean-squared-error loss, gradients and Adam update.

TEST INFRASTRUCTURE ONLY (see the package docstring).  Plain numpy in float64,
written from the definitions: a 3x3 convolution with circular padding,
ReLU, a residual connection on the first cout input channels, the chain rule
for the gradients, and Adam (Kingma & Ba, "Adam: a method for stochastic
optimization", ICLR 2015, algorithm 1).

Shapes: x [N, cin, H, W]; w0 [hidden, cin, 3, 3], w1 [hidden, hidden, 3, 3],
w2 [cout, hidden, 3, 3]; biases b0 [hidden], b1 [hidden], b2 [cout].
"""
import numpy as np


def conv3x3(x, w, b):
    """y[n, o, i, j] = b[o] + sum_c sum_{ky,kx} w[o, c, ky, kx] x[n, c, i+ky-1, j+kx-1]
    with indices taken modulo H and W."""
    y = np.zeros((x.shape[0], w.shape[0], x.shape[2], x.shape[3])) + b[None, :, None, None]
    for ky in range(3):
        for kx in range(3):
            xs = np.roll(x, shift=(-(ky - 1), -(kx - 1)), axis=(2, 3))  # xs[.., i, j] = x[.., i+ky-1, j+kx-1]
            y += np.einsum("oc,nchw->nohw", w[:, :, ky, kx], xs)
    return y


def conv3x3_grad_input(dy, w):
    """Gradient of sum(dy * conv3x3(x, w, b)) with respect to x."""
    dx = np.zeros((dy.shape[0], w.shape[1], dy.shape[2], dy.shape[3]))
    for ky in range(3):
        for kx in range(3):
            t = np.einsum("oc,nohw->nchw", w[:, :, ky, kx], dy)
            dx += np.roll(t, shift=(ky - 1, kx - 1), axis=(2, 3))  # moves the term back to i+ky-1, j+kx-1
    return dx


def conv3x3_grad_weight(dy, x):
    """Gradients of sum(dy * conv3x3(x, w, b)) with respect to w and b."""
    dw = np.zeros((dy.shape[1], x.shape[1], 3, 3))
    for ky in range(3):
        for kx in range(3):
            xs = np.roll(x, shift=(-(ky - 1), -(kx - 1)), axis=(2, 3))
            dw[:, :, ky, kx] = np.einsum("nohw,nchw->oc", dy, xs)
    return dw, dy.sum(axis=(0, 2, 3))


def forward(x, params):
    w0, b0, w1, b1, w2, b2 = params
    a1 = np.maximum(conv3x3(x, w0, b0), 0.0)
    a2 = np.maximum(conv3x3(a1, w1, b1), 0.0)
    cout = w2.shape[0]
    y = x[:, :cout] + conv3x3(a2, w2, b2)
    return a1, a2, y


def loss(y, target):
    return float(np.mean((y - target) ** 2))


def backward(x, params, target):
    """Loss and gradients (dw0, db0, dw1, db1, dw2, db2) by the chain rule."""
    w0, b0, w1, b1, w2, b2 = params
    a1, a2, y = forward(x, params)
    dy = 2.0 * (y - target) / y.size
    dw2, db2 = conv3x3_grad_weight(dy, a2)
    dz2 = conv3x3_grad_input(dy, w2) * (a2 > 0)
    dw1, db1 = conv3x3_grad_weight(dz2, a1)
    dz1 = conv3x3_grad_input(dz2, w1) * (a1 > 0)
    dw0, db0 = conv3x3_grad_weight(dz1, x)
    return loss(y, target), (dw0, db0, dw1, db1, dw2, db2)


def adam_step(theta, grad, m, v, t, lr, beta1=0.9, beta2=0.999, eps=1e-8):
    """One Adam update at step t >= 1; returns new (theta, m, v)."""
    m = beta1 * m + (1 - beta1) * grad
    v = beta2 * v + (1 - beta2) * grad * grad
    mhat = m / (1 - beta1 ** t)
    vhat = v / (1 - beta2 ** t)
    return theta - lr * mhat / (np.sqrt(vhat) + eps), m, v


def init_params(cin, hidden, cout, rng, scale=1.0):
    """He-style uniform initialisation (weights), zero biases."""
    def u(shape, fan_in):
        lim = scale * np.sqrt(6.0 / fan_in)
        return rng.uniform(-lim, lim, size=shape)
    return (u((hidden, cin, 3, 3), 9 * cin), np.zeros(hidden),
            u((hidden, hidden, 3, 3), 9 * hidden), np.zeros(hidden),
            u((cout, hidden, 3, 3), 9 * hidden) * 0.1, np.zeros(cout))
