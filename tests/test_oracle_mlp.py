"""Pins of the FP64 reference MLP: gradients against central finite
differences, the SiLU derivative against its closed form, and Adam's first
step against its closed form (a step of -lr * sign(g) for every weight)."""
import numpy as np

from oracle import mlp


def test_silu_derivative_closed_form():
    z = np.linspace(-6, 6, 101)
    h = 1e-6
    fd = (mlp.silu(z + h) - mlp.silu(z - h)) / (2 * h)
    np.testing.assert_allclose(mlp.silu_grad(z), fd, rtol=1e-8, atol=1e-10)
    assert mlp.silu(0.0) == 0.0 and abs(mlp.silu(20.0) - 20.0) < 1e-6


def test_backward_matches_finite_differences():
    rng = np.random.default_rng(0)
    sizes = [7, 11, 9, 5]
    params = mlp.init(sizes, seed=1)
    params = [(W, rng.standard_normal(b.shape) * 0.1) for W, b in params]
    x = rng.standard_normal((6, 7))
    t = rng.standard_normal((6, 5))
    grads = mlp.backward(params, x, t)
    h = 1e-6
    for k, (W, b) in enumerate(params):
        for arr_i, (arr, g) in enumerate(((W, grads[k][0]), (b, grads[k][1]))):
            flat = arr.reshape(-1)
            for idx in rng.choice(flat.size, size=min(6, flat.size), replace=False):
                old = flat[idx]
                flat[idx] = old + h
                lp = mlp.loss(params, x, t)
                flat[idx] = old - h
                lm = mlp.loss(params, x, t)
                flat[idx] = old
                fd = (lp - lm) / (2 * h)
                assert abs(fd - g.reshape(-1)[idx]) <= 1e-7 * max(1.0, abs(fd)), (k, arr_i, idx)


def test_adam_first_step_is_signed_lr():
    rng = np.random.default_rng(2)
    params = mlp.init([4, 3], seed=3)
    grads = [(rng.standard_normal((4, 3)), rng.standard_normal(3))]
    state = {}
    new = mlp.adam_step(params, grads, state, lr=1e-2)
    # bias-corrected first step: m_hat = g, v_hat = g^2 -> step = lr * g / (|g| + eps)
    np.testing.assert_allclose(new[0][0] - params[0][0], -1e-2 * np.sign(grads[0][0]), rtol=1e-6)
    np.testing.assert_allclose(new[0][1] - params[0][1], -1e-2 * np.sign(grads[0][1]), rtol=1e-6)


def test_training_reduces_loss_on_a_linear_map():
    rng = np.random.default_rng(4)
    A = rng.standard_normal((5, 3))
    x = rng.standard_normal((64, 5))
    t = x @ A
    params = mlp.init([5, 16, 3], seed=5)
    state = {}
    l0 = mlp.loss(params, x, t)
    for _ in range(300):
        params = mlp.adam_step(params, mlp.backward(params, x, t), state, lr=1e-2)
    assert mlp.loss(params, x, t) < 0.05 * l0
