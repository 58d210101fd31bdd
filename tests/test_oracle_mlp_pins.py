"""Pins of the surrogate network's oracle (oracle/mlp.py) to values fixed
outside it: tabulated normal-CDF values, a hand-evaluated network, torch's
bfloat16 conversion, finite differences and the closed form of Adam's first
step. CPU only."""
import math

import numpy as np
import pytest
from scipy import stats

from oracle import mlp as O


def test_normal_cdf_and_gelu_at_tabulated_points():
    # Phi from standard tables (Abramowitz and Stegun 26.2)
    table = {0.0: 0.5, 1.0: 0.8413447460685429, -1.96: 0.024997895148220435,
             2.0: 0.9772498680518208, -0.5: 0.3085375387259869}
    for z, p in table.items():
        assert abs(float(O.phi_cdf(z)) - p) < 1e-15
    assert float(O.gelu(0.0)) == 0.0
    assert abs(float(O.gelu(1.0)) - 0.8413447460685429) < 1e-15
    assert abs(float(O.gelu(-1.0)) + 0.15865525393145707) < 1e-15
    # GELU(z) - GELU(-z) = z for every z (Phi(z) + Phi(-z) = 1)
    z = np.linspace(-6, 6, 101)
    assert np.max(np.abs(O.gelu(z) - O.gelu(-z) - z)) < 1e-14


def test_gelu_prime_matches_central_differences():
    z = np.linspace(-5, 5, 41)
    h = 1e-6
    fd = (O.gelu(z + h) - O.gelu(z - h)) / (2 * h)
    assert np.max(np.abs(O.gelu_prime(z) - fd)) < 1e-9
    assert float(O.gelu_prime(0.0)) == 0.5


def test_bf16_rounding_matches_torch_and_ties_go_to_even():
    torch = pytest.importorskip("torch")
    rng = np.random.default_rng(0)
    a = (rng.standard_normal(20000) * np.exp(rng.uniform(-20, 20, 20000))).astype(np.float32).astype(np.float64)
    ref = torch.from_numpy(a.astype(np.float32)).to(torch.bfloat16).to(torch.float64).numpy()
    assert np.array_equal(O.bf16(a), ref)
    # exact halfway cases: 1 + 2^-8 lies between 1 and 1 + 2^-7 -> the even one, 1
    assert O.bf16(1.0 + 2.0 ** -8) == 1.0
    # 1 + 3 2^-8 lies between 1 + 2^-7 (odd last bit) and 1 + 2^-6 (even) -> 1 + 2^-6
    assert O.bf16(1.0 + 3 * 2.0 ** -8) == 1.0 + 2.0 ** -6
    assert O.bf16(-1.0 - 2.0 ** -8) == -1.0
    # values already representable are unchanged
    v = np.array([1.0, -0.5, 3.0, 2.0 ** -20, 1.0 + 2.0 ** -7])
    assert np.array_equal(O.bf16(v), v)


def test_one_hidden_unit_network_by_hand():
    shapes = O.layer_dims(1, 1, 1, 1)
    flat = np.array([2.0, 0.0, 3.0, 0.25])  # W0, b0, W1, b1
    y, _ = O.forward(flat, shapes, np.array([[0.5]]), rounding=False)
    # z = 2 * 0.5 = 1, GELU(1) = Phi(1) = 0.8413447460685429, y = 3 GELU(1) + 0.25
    assert abs(y[0, 0] - 2.7740342382056287) < 1e-15
    # dy/dW1 = GELU(1), dy/db1 = 1, dy/dW0 = 3 GELU'(1) x, dy/db0 = 3 GELU'(1), dy/dx = 3 GELU'(1) 2
    g, dx = O.backward(flat, shapes, np.array([[0.5]]), np.array([[1.0]]), rounding=False)
    gp1 = 0.8413447460685429 + math.exp(-0.5) / math.sqrt(2 * math.pi)
    np.testing.assert_allclose(g, [3 * gp1 * 0.5, 3 * gp1, 0.8413447460685429, 1.0], rtol=1e-14)
    assert abs(dx[0, 0] - 6 * gp1) < 1e-13


def test_backward_matches_central_differences_of_forward():
    rng = np.random.default_rng(3)
    shapes = O.layer_dims(5, 7, 2, 4)
    P = O.num_params(shapes)
    flat = rng.standard_normal(P) * 0.5
    x = rng.standard_normal((6, 5))
    dy = rng.standard_normal((6, 4))

    def loss(fl, xx):
        return float(np.sum(O.forward(fl, shapes, xx, rounding=False)[0] * dy))

    g, dx = O.backward(flat, shapes, x, dy, rounding=False)
    h = 1e-6
    gfd = np.zeros(P)
    for i in range(P):
        e = np.zeros(P); e[i] = h
        gfd[i] = (loss(flat + e, x) - loss(flat - e, x)) / (2 * h)
    assert np.max(np.abs(g - gfd)) < 1e-7 * max(1, np.max(np.abs(g)))
    dxfd = np.zeros_like(x)
    for idx in np.ndindex(*x.shape):
        e = np.zeros_like(x); e[idx] = h
        dxfd[idx] = (loss(flat, x + e) - loss(flat, x - e)) / (2 * h)
    assert np.max(np.abs(dx - dxfd)) < 1e-7 * max(1, np.max(np.abs(dx)))


def test_rounded_network_stays_within_bf16_error_of_exact_one():
    rng = np.random.default_rng(4)
    shapes = O.layer_dims(20, 64, 2, 30)
    flat = rng.standard_normal(O.num_params(shapes)) * 0.15
    x = rng.uniform(-1, 1, (16, 20))
    y_r, _ = O.forward(flat, shapes, x, rounding=True)
    y_e, _ = O.forward(flat, shapes, x, rounding=False)
    rel = np.linalg.norm(y_r - y_e) / np.linalg.norm(y_e)
    # a handful of relative 2^-9 roundings per path: well above FP64 noise, well below 1e-1
    assert 1e-5 < rel < 3e-2


def test_mse_gradient_and_adam_first_step_closed_form():
    rng = np.random.default_rng(5)
    y, t = rng.standard_normal((3, 4)), rng.standard_normal((3, 4))
    L, dy = O.mse(y, t)
    assert abs(L - np.mean((y - t) ** 2)) < 1e-15
    h = 1e-7
    e = np.zeros_like(y); e[1, 2] = h
    assert abs((O.mse(y + e, t)[0] - O.mse(y - e, t)[0]) / (2 * h) - dy[1, 2]) < 1e-8
    # Adam at t = 1 from zero moments: m_hat = g, v_hat = g^2, step = lr g / (|g| + eps)
    w, g = rng.standard_normal(50), rng.standard_normal(50)
    w1, m, v = O.adam(w, g, np.zeros(50), np.zeros(50), 1, 1e-3)
    np.testing.assert_allclose(w1, w - 1e-3 * g / (np.abs(g) + 1e-8), rtol=0, atol=1e-15)
    np.testing.assert_allclose(m, 0.1 * g, rtol=1e-15)
    np.testing.assert_allclose(v, 0.001 * g * g, rtol=1e-12)


def test_surrogate_objective_is_poisson_log_likelihood_ratio():
    rng = np.random.default_rng(6)
    y = rng.standard_normal((2, 30)) * 0.3
    mean, std = rng.uniform(2, 5, 30), rng.uniform(0.1, 0.5, 30)
    mu = np.exp(y * std + mean)
    n = rng.poisson(mu).astype(float)
    n[0, :3] = 0.0
    x = rng.standard_normal((2, 4))
    xbar, w = rng.standard_normal(4), rng.uniform(0, 2, 4)
    got = O.surrogate_objective(y, n, mean, std, x, xbar, w)
    # deviance / 2 = ln P(n | n) - ln P(n | mu)
    ref = np.sum(stats.poisson.logpmf(n, n) - stats.poisson.logpmf(n, mu), axis=1)
    ref += 0.5 * np.sum(w * (x - xbar) ** 2, axis=1)
    np.testing.assert_allclose(got, ref, rtol=1e-12)
