"""Pins of the CNN reference: gradients against central finite
differences, convolution against an explicit loop, GELU against its
closed form and Adam against a hand-computed first step."""
import math

import numpy as np

from oracle import cnn


def _setup(seed=0, B=2, H=5, W=6):
    rng = np.random.default_rng(seed)
    p = rng.normal(size=cnn.param_count()) * 0.2
    x = rng.normal(size=(B, 7, H, W))
    t = rng.normal(size=(B, 3, H, W))
    return p, x, t


def test_conv_matches_explicit_loops():
    rng = np.random.default_rng(1)
    x = rng.normal(size=(1, 2, 4, 3))
    W = rng.normal(size=(3, 2, 3, 3))
    b = rng.normal(size=3)
    y = cnn.conv3x3(x, W, b)
    for o in range(3):
        for i in range(4):
            for j in range(3):
                s = b[o]
                for c in range(2):
                    for di in range(3):
                        for dj in range(3):
                            ii, jj = i + di - 1, j + dj - 1
                            if 0 <= ii < 4 and 0 <= jj < 3:
                                s += W[o, c, di, dj] * x[0, c, ii, jj]
                assert abs(y[0, o, i, j] - s) < 1e-12


def test_gelu_closed_form_and_derivative():
    for z in [-5.0, -1.3, 0.0, 0.7, 3.0]:
        want = 0.5 * z * (1 + math.erf(z / math.sqrt(2)))
        assert abs(cnn.gelu(np.array(z)) - want) < 1e-15
        h = 1e-6
        fd = (cnn.gelu(np.array(z + h)) - cnn.gelu(np.array(z - h))) / (2 * h)
        assert abs(cnn.gelu_grad(np.array(z)) - fd) < 1e-8


def test_gradient_matches_finite_differences():
    p, x, t = _setup()
    loss, g = cnn.loss_and_grad(p, x, t)
    rng = np.random.default_rng(3)
    idx = rng.choice(p.size, 60, replace=False)
    for k in idx:
        h = 1e-6
        pp, pm = p.copy(), p.copy()
        pp[k] += h
        pm[k] -= h
        lp, _ = cnn.loss_and_grad(pp, x, t)
        lm, _ = cnn.loss_and_grad(pm, x, t)
        fd = (lp - lm) / (2 * h)
        assert abs(fd - g[k]) <= 1e-6 * max(1e-3, abs(g[k])) + 1e-9, (k, fd, g[k])


def test_bf16_rounding():
    v = np.array([1.0, 1.00390625, 1.005859375, -3.14159, 1e-30, 65504.0])
    r = cnn.to_bf16(v)
    assert r[0] == 1.0 and r[1] == 1.0  # halfway 1 + 2^-8 ties to even (1.0)
    assert r[2] == 1.0078125            # 1 + 1.5*2^-8 rounds up
    assert abs(r[3] + 3.140625) < 1e-12
    assert np.all(np.abs(r - v) <= np.abs(v) * 2.0 ** -8)


def test_adam_first_step_moves_by_lr():
    p = np.array([1.0, -2.0, 0.5])
    g = np.array([0.3, -4.0, 1e-9])
    m, v = np.zeros(3), np.zeros(3)
    q = p.copy()
    cnn.adam(q, g, m, v, 1, lr=1e-3)
    # first bias-corrected Adam step is lr * g / (|g| + eps) ~ lr * sign(g)
    assert np.allclose(q[:2], p[:2] - 1e-3 * np.sign(g[:2]), atol=1e-9)
