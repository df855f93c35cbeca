"""Pins of the MLP oracle: BF16 rounding against known bit patterns, GELU
against values of the error function, gradients against central finite
differences of the FP64 network, Adam against a hand-computed step, the
cosine schedule at its end points."""
import math

import numpy as np

from oracle import mlp
import workloads.synth as ws


def test_bf16_rounding_bit_patterns():
    # BF16 keeps 8 significant bits: spacing 2^-7 in [1, 2)
    cases = {
        1.0: 1.0,
        1.0 + 2.0 ** -8: 1.0,                       # tie -> even (mantissa 0)
        1.0 + 3 * 2.0 ** -8: 1.0 + 2.0 ** -6,       # tie -> even (mantissa 2)
        1.0 + 2.0 ** -8 + 2.0 ** -12: 1.0 + 2.0 ** -7,
        -3.0: -3.0,
        0.1: 0.10009765625,                          # 0x3DCD
        65504.0: 65536.0,
        1e-3: 0.00099945068359375,
    }
    for x, want in cases.items():
        assert mlp.bf16_round(x) == want, (x, mlp.bf16_round(x), want)


def test_gelu_values_and_slope():
    assert mlp.gelu(0.0) == 0.0
    # 0.5 (1 + erf(1/sqrt 2)) = Phi(1) = 0.8413447460685429
    assert abs(mlp.gelu(1.0) - 0.8413447460685429) < 1e-15
    assert abs(mlp.gelu(-1.0) + 1.0 - 0.8413447460685429) < 1e-15
    assert abs(mlp.gelu(8.0) - 8.0) < 1e-12 and abs(mlp.gelu(-8.0)) < 1e-12
    z = np.linspace(-4, 4, 41)
    h = 1e-6
    fd = (mlp.gelu(z + h) - mlp.gelu(z - h)) / (2 * h)
    np.testing.assert_allclose(mlp.gelu_grad(z), fd, rtol=0, atol=1e-9)


def test_gradients_match_finite_differences():
    d, w, m, B = 5, 7, 3, 4
    rng = np.random.default_rng(0)
    p = ws.mlp_init_params(d, w, m, seed=1).astype(np.float64)
    p += rng.normal(0, 0.1, size=p.shape)           # non-zero biases too
    X = rng.random((B, d))
    Y = rng.normal(size=(B, m))
    loss, g = mlp.loss_and_grads(p, X, Y, d, w, m, storage="exact")
    fd = np.empty_like(p)
    h = 1e-6
    for i in range(p.size):
        e = np.zeros_like(p)
        e[i] = h
        lp, _ = mlp.loss_and_grads(p + e, X, Y, d, w, m, storage="exact")
        lm, _ = mlp.loss_and_grads(p - e, X, Y, d, w, m, storage="exact")
        fd[i] = (lp - lm) / (2 * h)
    np.testing.assert_allclose(g, fd, rtol=1e-6, atol=1e-9)
    # the loss is the mean of squared differences
    out, _ = mlp.forward(p, X, d, w, m, storage="exact")
    assert abs(loss - np.mean((out - Y) ** 2)) < 1e-15


def test_adam_first_step_by_hand():
    # t = 1: mhat = g, vhat = g^2, step = lr g / (|g| + eps)
    p, g = np.array([1.0, -2.0, 0.5]), np.array([0.3, -0.04, 0.0])
    new, mom, vel = mlp.adam_step(p, g, np.zeros(3), np.zeros(3), 1, lr=0.01)
    np.testing.assert_allclose(mom, 0.1 * g, rtol=1e-15)
    np.testing.assert_allclose(vel, 0.001 * g * g, rtol=1e-15)
    want = p - 0.01 * np.array([0.3 / (0.3 + 1e-8), -0.04 / (0.04 + 1e-8), 0.0])
    np.testing.assert_allclose(new, want, rtol=0, atol=1e-15)
    # t = 2 with the same gradient: bias-corrected moments stay g and g^2
    new2, mom2, vel2 = mlp.adam_step(new, g, mom, vel, 2, lr=0.01)
    mhat = mom2 / (1 - 0.9 ** 2)
    np.testing.assert_allclose(mhat, g, rtol=1e-14, atol=1e-18)


def test_cosine_schedule_end_points():
    assert mlp.cosine_lr(0, 100, 1e-3) == 1e-3
    assert abs(mlp.cosine_lr(50, 100, 1e-3) - 5e-4) < 1e-18
    assert abs(mlp.cosine_lr(100, 100, 1e-3)) < 1e-18


def test_bf16_storage_is_close_to_exact():
    d, w, m = 6, 16, 4
    p = ws.mlp_init_params(d, w, m, seed=2).astype(np.float64)
    X = np.random.default_rng(3).random((10, d))
    a, _ = mlp.forward(p, X, d, w, m, storage="exact")
    b, _ = mlp.forward(p, X, d, w, m, storage="bf16")
    assert np.abs(a - b).max() <= 2e-2 * max(1.0, np.abs(a).max())
    assert not np.array_equal(a, b)
    assert math.isfinite(float(np.abs(a).sum()))
