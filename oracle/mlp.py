"""Plain FP64 reference of the learned form's network (TEST INFRASTRUCTURE
ONLY): inputs standardised (x - in_shift)/in_scale, then
n_in -> h (tanh) -> h (tanh) -> n_out (linear), mean-squared error on
standardised targets (t - shift)/scale, Adam with decoupled weight decay.
Parameter layout: W1 [n_in][h], b1 [h], W2 [h][h], b2 [h], W3 [h][n_out],
b3 [n_out], flattened in that order; y = x W + b.

Pins: the gradient is checked against central finite differences of the
loss (tests/test_oracle_mlp.py).
"""
import numpy as np


def unpack(p, n_in, h, n_out):
    p = np.asarray(p, np.float64)
    shapes = [(n_in, h), (h,), (h, h), (h,), (h, n_out), (n_out,)]
    out, o = [], 0
    for s in shapes:
        k = int(np.prod(s))
        out.append(p[o:o + k].reshape(s))
        o += k
    assert o == p.size
    return out


def forward(p, X, n_in, h, n_out, in_shift=None, in_scale=None):
    W1, b1, W2, b2, W3, b3 = unpack(p, n_in, h, n_out)
    X = np.asarray(X, np.float64)
    if in_shift is not None:
        X = (X - in_shift) / in_scale
    a1 = np.tanh(X @ W1 + b1)
    a2 = np.tanh(a1 @ W2 + b2)
    return a2 @ W3 + b3, (a1, a2)


def loss_grad(p, X, T, shift, scale, n_in, h, n_out, in_shift=None, in_scale=None):
    W1, b1, W2, b2, W3, b3 = unpack(p, n_in, h, n_out)
    X = np.asarray(X, np.float64)
    if in_shift is not None:
        X = (X - in_shift) / in_scale
    y, (a1, a2) = forward(p, X, n_in, h, n_out)
    ts = (np.asarray(T, np.float64) - shift) / scale
    r = y - ts
    B = X.shape[0]
    loss = float((r * r).mean())
    dy = 2.0 * r / (B * n_out)
    gW3 = a2.T @ dy
    gb3 = dy.sum(0)
    dz2 = (dy @ W3.T) * (1.0 - a2 * a2)
    gW2 = a1.T @ dz2
    gb2 = dz2.sum(0)
    dz1 = (dz2 @ W2.T) * (1.0 - a1 * a1)
    gW1 = X.T @ dz1
    gb1 = dz1.sum(0)
    g = np.concatenate([gW1.ravel(), gb1, gW2.ravel(), gb2, gW3.ravel(), gb3])
    return loss, g


def adam_step(p, g, m, v, step, lr, wd, b1=0.9, b2=0.999, eps=1e-8):
    """One Adam update (step counts from 1); returns new (p, m, v)."""
    m = b1 * m + (1 - b1) * g
    v = b2 * v + (1 - b2) * g * g
    mh = m / (1 - b1 ** step)
    vh = v / (1 - b2 ** step)
    p = p - lr * (mh / (np.sqrt(vh) + eps) + wd * p)
    return p, m, v
