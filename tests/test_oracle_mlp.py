"""Pins of the float64 reference of the b_n network: closed-form GELU values,
bfloat16 rounding, finite-difference gradients, one Adam step.  CPU only."""
import math

import numpy as np

from oracle import mlp


def test_gelu_closed_forms():
    assert mlp.gelu(np.array(0.0)) == 0.0
    # GELU(1) = Phi(1) = (1 + erf(1/sqrt 2))/2
    assert abs(mlp.gelu(np.array(1.0)) - 0.5 * (1 + math.erf(1 / math.sqrt(2)))) < 1e-16
    x = np.linspace(-6, 6, 101)
    assert np.allclose(mlp.gelu(x) - mlp.gelu(-x), x, atol=1e-14)  # x Phi(x) - (-x) Phi(-x) = x
    h = 1e-6
    fd = (mlp.gelu(x + h) - mlp.gelu(x - h)) / (2 * h)
    assert np.allclose(mlp.gelu_grad(x), fd, atol=1e-8)


def test_bf16_rounding():
    vals = np.array([1.0, 1.0 + 2.0 ** -8, 1.0 + 3 * 2.0 ** -8, -2.5, 3.140625, 1.0 + 2.0 ** -9],
                    dtype=np.float32)
    want = np.array([1.0, 1.0, 1.0 + 2 * 2.0 ** -7, -2.5, 3.140625, 1.0])
    assert np.array_equal(mlp.bf16(vals), want)
    r = np.random.default_rng(0).standard_normal(1000).astype(np.float32)
    b = mlp.bf16(r)
    assert np.all(np.abs(b - r) <= np.abs(r) * 2.0 ** -8)
    assert np.array_equal(mlp.bf16(b), b)


def test_gradient_matches_finite_differences():
    rng = np.random.default_rng(1)
    n = sum(int(np.prod(s)) for _, s in mlp.SHAPES)
    p = rng.standard_normal(n) * 0.1
    x = rng.standard_normal((24, 16))
    t = rng.standard_normal((24, 16))
    mask = (rng.random((24, 16)) < 0.7).astype(float)
    loss, g = mlp.loss_and_grad(p, x, t, mask)
    idx = np.concatenate([rng.choice(n, 60, replace=False),
                          [0, 4095, 4096, 4351, n - 16, n - 1]])
    h = 1e-6
    for i in idx:
        pp, pm = p.copy(), p.copy()
        pp[i] += h
        pm[i] -= h
        fd = (mlp.loss_and_grad(pp, x, t, mask)[0] - mlp.loss_and_grad(pm, x, t, mask)[0]) / (2 * h)
        assert abs(fd - g[i]) <= 1e-6 * max(1.0, abs(fd)), (i, fd, g[i])


def test_adam_first_step():
    g = np.array([0.5, -2.0, 1e-3])
    p = np.zeros(3)
    p1, m, v = mlp.adam_step(p, g, np.zeros(3), np.zeros(3), 1, lr=0.1)
    # bias-corrected first step: m_hat = g, v_hat = g^2, step = lr g / (|g| + eps)
    assert np.allclose(p1, -0.1 * g / (np.abs(g) + 1e-8), rtol=1e-12)
