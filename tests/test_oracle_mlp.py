"""Pins of the predictor-network oracle (CPU): backpropagation against central differences, closed
forms of the loss and of the first Adam step, and bfloat16 rounding against torch's conversion."""
import numpy as np
import pytest
import torch

from oracle import mlp


def _problem(seed=3, n=37, scale=0.3):
    rng = np.random.default_rng(seed)
    theta = rng.normal(0.0, scale, mlp.N_PARAMS)
    X = rng.normal(0.0, 1.0, (n, mlp.N_IN))
    Y = (rng.random((n, mlp.N_OUT)) < 0.4).astype(np.float64)
    return theta, X, Y


def test_parameter_count():
    assert mlp.N_PARAMS == 64 * 128 + 128 + 128 * 128 + 128 + 128 * 4 + 4 == 25348


def test_gradient_matches_central_differences():
    theta, X, Y = _problem()
    g = mlp.grad(theta, X, Y)
    rng = np.random.default_rng(7)
    # a sample of every block: W1, b1, W2, b2, W3, b3
    offs = np.cumsum([0] + [int(np.prod(s)) for s in mlp.SHAPES])
    idx = np.concatenate([rng.choice(np.arange(offs[k], offs[k + 1]), min(12, offs[k + 1] - offs[k]), replace=False)
                          for k in range(6)])
    h = 1e-6
    for i in idx:
        tp, tm = theta.copy(), theta.copy()
        tp[i] += h
        tm[i] -= h
        fd = (mlp.loss(tp, X, Y) - mlp.loss(tm, X, Y)) / (2 * h)
        assert abs(fd - g[i]) <= 1e-7 + 1e-5 * abs(fd), (i, fd, g[i])


def test_loss_closed_forms():
    theta, X, Y = _problem()
    # zero network: z = 0, p = 1/2, loss = log 2 whatever the labels
    assert mlp.loss(np.zeros(mlp.N_PARAMS), X, Y) == pytest.approx(np.log(2.0), rel=1e-15)
    # only the output bias: z = b3 for every sample
    parts = [np.zeros(s) for s in mlp.SHAPES]
    parts[5] = np.array([0.3, -1.2, 2.0, 0.0])
    th = mlp.pack(parts)
    b = parts[5]
    want = np.mean(np.log1p(np.exp(b))[None, :] - Y * b[None, :])
    assert mlp.loss(th, X, Y) == pytest.approx(want, rel=1e-14)
    # gradient of the output bias is mean(sigmoid(b) - y) / 4 per output
    g = mlp.grad(th, X, Y)
    gb3 = g[-4:]
    sig = 1 / (1 + np.exp(-b))
    assert np.allclose(gb3, (sig[None, :] - Y).mean(0) / 4, rtol=1e-13, atol=1e-16)


def test_first_adam_step_is_signed_learning_rate():
    theta = np.linspace(-1, 1, mlp.N_PARAMS)
    g = np.linspace(-2, 3, mlp.N_PARAMS) + 1e-3
    t1, m, v = mlp.adam_step(theta, g, np.zeros_like(g), np.zeros_like(g), 1, 1e-2)
    assert np.allclose(t1 - theta, -1e-2 * g / (np.abs(g) + 1e-8), rtol=1e-12, atol=1e-15)
    assert np.allclose(m, 0.1 * g) and np.allclose(v, 0.001 * g * g)


def test_bf16_rounding_matches_torch():
    rng = np.random.default_rng(11)
    x = np.concatenate([rng.normal(0, 1, 5000), rng.normal(0, 1e-3, 1000) * 10.0 ** rng.integers(-20, 20, 1000),
                        np.array([1.0, 1.0 + 2.0 ** -8, 1.0 + 3 * 2.0 ** -8, -(1.0 + 2.0 ** -8), 0.0])])
    x32 = x.astype(np.float32)
    ref = torch.from_numpy(x32).to(torch.bfloat16).to(torch.float64).numpy()
    assert np.array_equal(mlp.bf16(x32), ref)
    # ties go to even: 1 + 2^-8 -> 1, 1 + 3*2^-8 -> 1 + 2^-6
    assert mlp.bf16(np.array([1.0 + 2.0 ** -8]))[0] == 1.0
    assert mlp.bf16(np.array([1.0 + 3 * 2.0 ** -8]))[0] == 1.0 + 2.0 ** -6


def test_emulated_bf16_gradient_close_to_exact():
    """The bf16 rounding points change the gradient by the bf16 precision only."""
    theta, X, Y = _problem(n=64)
    g = mlp.grad(theta, X, Y)
    gb = mlp.grad(theta, X, Y, emulate_bf16=True)
    assert np.linalg.norm(gb - g) / np.linalg.norm(g) < 3e-2
