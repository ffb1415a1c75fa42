"""Pins of the reference network: gradient vs central finite differences,
and the Adam update vs its closed form on a scalar."""
import numpy as np
import pytest

from oracle import mlp


def test_gradient_matches_finite_differences():
    rng = np.random.default_rng(0)
    n_in, h, n_out, B = 7, 5, 3, 4
    n = n_in * h + h + h * h + h + h * n_out + n_out
    p = rng.normal(size=n) * 0.5
    X = rng.normal(size=(B, n_in))
    T = rng.normal(size=(B, n_out))
    shift = rng.normal(size=n_out)
    scale = rng.uniform(0.5, 2.0, n_out)
    loss, g = mlp.loss_grad(p, X, T, shift, scale, n_in, h, n_out)
    eps = 1e-6
    fd = np.empty(n)
    for i in range(n):
        e = np.zeros(n)
        e[i] = eps
        lp, _ = mlp.loss_grad(p + e, X, T, shift, scale, n_in, h, n_out)
        lm, _ = mlp.loss_grad(p - e, X, T, shift, scale, n_in, h, n_out)
        fd[i] = (lp - lm) / (2 * eps)
    assert np.abs(fd - g).max() < 1e-8 * max(1.0, np.abs(g).max())


def test_adam_first_step_is_signed_lr():
    """With zero moments the first Adam step moves each parameter by
    lr * g / (|g| + eps) (bias correction cancels), i.e. lr * sign(g)."""
    p = np.array([1.0, -2.0, 0.5])
    g = np.array([0.3, -4.0, 1e-3])
    p1, m, v = mlp.adam_step(p, g, np.zeros(3), np.zeros(3), 1, 0.01, 0.0)
    assert np.allclose(p1, p - 0.01 * np.sign(g), atol=1e-7)


def test_adam_decoupled_weight_decay_closed_form():
    """Decoupled weight decay (AdamW): the step is
    p <- p - lr (m_hat / (sqrt(v_hat) + eps) + wd p).  A parameter with zero
    gradient only decays, by the factor 1 - lr wd per step; on the first
    step a nonzero gradient adds lr g / (|g| + eps)."""
    lr, wd, eps = 0.01, 0.1, 1e-8
    p = np.array([1.0, -2.0, 0.5])
    g = np.array([0.0, 0.3, 0.0])
    p1, m, v = mlp.adam_step(p, g, np.zeros(3), np.zeros(3), 1, lr, wd, eps=eps)
    assert p1[0] == 1.0 * (1 - lr * wd) and p1[2] == 0.5 * (1 - lr * wd)
    assert p1[1] == pytest.approx(-2.0 - lr * (0.3 / (0.3 + eps) + wd * (-2.0)), abs=1e-15)
    # ten steps at zero gradient: (1 - lr wd)^10
    q = p.copy()
    mm, vv = np.zeros(3), np.zeros(3)
    for k in range(1, 11):
        q, mm, vv = mlp.adam_step(q, np.zeros(3), mm, vv, k, lr, wd)
    assert np.allclose(q, p * (1 - lr * wd) ** 10, rtol=1e-14, atol=0)
