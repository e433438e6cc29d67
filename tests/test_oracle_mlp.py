"""Pins of the FP64 reference of the opening-angle network."""
import math

import numpy as np
import torch

from oracle import mlp


def _data(seed, b=32):
    rng = np.random.default_rng(seed)
    x = rng.normal(size=(b, mlp.N_IN)) * 2.0 + 1.0
    mu = rng.normal(size=mlp.N_IN) * 0.3
    sigma = rng.uniform(0.5, 2.0, mlp.N_IN)
    t = rng.uniform(0.3, 1.0, b)
    w = rng.uniform(1.0, 100.0, b)
    return x, mu, sigma, t, w


def test_forward_hand_computed():
    p = np.zeros(mlp.N_PARAMS)
    w = mlp.unpack(p)
    w["W1"][0, 0] = 1.0
    w["W2"][0, 0] = 1.0
    w["w3"][0] = 2.0
    w["b3"][0] = 0.5
    x = np.array([[0.7] + [5.0] * 11, [-1.3] + [-2.0] * 11])
    th, _ = mlp.forward(p, x, np.zeros(12), np.ones(12), shift=-0.25)
    y = 2.0 * np.tanh(np.tanh(x[:, 0])) + 0.5 - 0.25
    assert np.allclose(th, 0.3 + 0.7 / (1.0 + np.exp(-y)), rtol=0, atol=1e-15)
    # normalisation: (x - mu) / sigma
    th2, _ = mlp.forward(p, 2.0 * x + 3.0, np.full(12, 3.0), np.full(12, 2.0), shift=-0.25)
    assert np.allclose(th2, th, rtol=0, atol=1e-15)


def test_gradient_matches_central_differences():
    x, mu, sigma, t, wt = _data(1)
    p = mlp.init(7)
    p += np.random.default_rng(2).normal(size=p.shape) * 0.05  # non-zero biases
    loss, g = mlp.loss_and_grad(p, x, mu, sigma, t, wt)
    rng = np.random.default_rng(3)
    idx = np.concatenate([rng.choice(mlp.N_PARAMS, 300, replace=False), [mlp.N_PARAMS - 1]])
    h = 1e-6
    scale = np.max(np.abs(g))
    for k in idx:
        pp = p.copy()
        pp[k] += h
        lp, _ = mlp.loss_and_grad(pp, x, mu, sigma, t, wt)
        pp[k] -= 2 * h
        lm, _ = mlp.loss_and_grad(pp, x, mu, sigma, t, wt)
        fd = (lp - lm) / (2 * h)
        assert abs(fd - g[k]) <= 1e-7 * scale, (k, fd, g[k])
    assert loss > 0


def test_adam_first_step_is_signed_learning_rate():
    opt = mlp.Adam(5, lr=0.01)
    g = np.array([3.0, -2e-3, 0.5, -7.0, 1e-2])
    p1 = opt.step(np.zeros(5), g)
    # bias-corrected moments equal g and g^2 after one step
    assert np.allclose(p1, -0.01 * g / (np.abs(g) + 1e-8), rtol=0, atol=1e-15)


def test_bf16_rounding_is_round_to_nearest_even():
    v = np.array([1.0, 1.0 + 2.0 ** -8, 1.0 + 3 * 2.0 ** -8, -2.5, 3.14159265, 1e-30, 65504.0, 0.0])
    assert np.array_equal(mlp.bf16(v)[:3], [1.0, 1.0, 1.015625])
    ref = torch.tensor(v, dtype=torch.float32).to(torch.bfloat16).to(torch.float64).numpy()
    assert np.array_equal(mlp.bf16(v), ref)
    r = np.random.default_rng(4).normal(size=10000).astype(np.float32) * 100
    ref = torch.tensor(r).to(torch.bfloat16).to(torch.float64).numpy()
    assert np.array_equal(mlp.bf16(r), ref)


def test_training_fits_a_learnable_target():
    rng = np.random.default_rng(5)
    x = rng.normal(size=(512, mlp.N_IN))
    t = 0.3 + 0.7 / (1.0 + np.exp(-(1.5 * x[:, 0] - x[:, 1])))
    wt = np.ones(512)
    mu, sigma = x.mean(axis=0), x.std(axis=0)
    p = mlp.init(6)
    opt = mlp.Adam(mlp.N_PARAMS, lr=3e-3)
    l0, _ = mlp.loss_and_grad(p, x, mu, sigma, t, wt)
    for _ in range(300):
        _, g = mlp.loss_and_grad(p, x, mu, sigma, t, wt)
        p = opt.step(p, g)
    l1, _ = mlp.loss_and_grad(p, x, mu, sigma, t, wt)
    assert l1 < 0.05 * l0


def test_bf16_forward_close_to_fp64_forward():
    x, mu, sigma, _, _ = _data(8, 256)
    p = mlp.init(9)
    a, _ = mlp.forward(p, x, mu, sigma, 0.1)
    b = mlp.forward_bf16(p, x, mu, sigma, 0.1)
    # bf16 operands carry a relative error of 2^-9 per rounding
    assert np.max(np.abs(a - b)) < 0.7 * 0.25 * 64 * 3 * 2.0 ** -9 * 4
    assert np.max(np.abs(a - b)) > 0  # and it is not the same arithmetic
    assert math.isfinite(float(np.sum(b)))
