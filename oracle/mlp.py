"""Dense GELU network of the warm-start surrogate, written out plainly in FP64.

TEST INFRASTRUCTURE ONLY: tests, the smoke check and the benchmark's CPU
baseline use this module; the product path never does.

The network is the textbook multilayer perceptron
    h_0 = x,  z_l = h_l W_l + b_l,  h_{l+1} = GELU(z_l)  (hidden layers),
    y = z_L  (last layer, no activation),
with GELU(z) = z Phi(z), Phi the standard normal CDF. Its gradient is the
chain rule taken backwards through those lines. The parameter vector is
W_0, b_0, W_1, b_1, ... with W_l stored row-major as (d_in, d_out).

`rounding=True` rounds, to bfloat16 (8 significant bits, round to nearest,
ties to even), exactly the quantities the matrix-core implementation feeds to
its products: the network input, every weight matrix, every hidden activation
and every back-propagated gradient entering a product. Biases, pre-activations
and sums stay unrounded (FP64 here). With `rounding=False` it is the exact
network.

Pins (tests/test_oracle_pins.py): Phi and GELU at tabulated points, the
bfloat16 rounding against torch's independent conversion, the gradient against
central differences of the forward pass, Adam's first step against its closed
form, and a one-hidden-unit network against its hand-evaluated value.
"""
from __future__ import annotations

import math

import numpy as np


def bf16(a):
    """Round to the nearest bfloat16 value (8 significant bits), ties to even;
    values are returned as float64. Finite, normal-range inputs only."""
    a = np.asarray(a, dtype=np.float64)
    m, e = np.frexp(a)                      # a = m 2^e, 0.5 <= |m| < 1
    return np.ldexp(np.rint(m * 256.0) / 256.0, e)


def phi_cdf(z):
    """Standard normal CDF, Phi(z) = (1 + erf(z / sqrt 2)) / 2."""
    z = np.asarray(z, dtype=np.float64)
    return 0.5 * (1.0 + np.vectorize(math.erf)(z / math.sqrt(2.0)))


def gelu(z):
    return np.asarray(z, dtype=np.float64) * phi_cdf(z)


def gelu_prime(z):
    z = np.asarray(z, dtype=np.float64)
    return phi_cdf(z) + z * np.exp(-0.5 * z * z) / math.sqrt(2.0 * math.pi)


def layer_dims(n_in, width, depth, n_out):
    dims = [n_in] + [width] * depth + [n_out]
    return [(dims[i], dims[i + 1]) for i in range(depth + 1)]


def num_params(shapes):
    return sum(a * b + b for a, b in shapes)


def unpack(flat, shapes):
    flat = np.asarray(flat, dtype=np.float64)
    out, o = [], 0
    for a, b in shapes:
        W = flat[o:o + a * b].reshape(a, b)
        o += a * b
        bias = flat[o:o + b]
        o += b
        out.append((W, bias))
    return out


def forward(flat, shapes, x, rounding=True):
    """Returns y and the per-layer (input, pre-activation) pairs."""
    r = bf16 if rounding else (lambda v: np.asarray(v, dtype=np.float64))
    layers = unpack(flat, shapes)
    h = r(x)
    cache = []
    for l, (W, b) in enumerate(layers):
        z = h @ r(W) + b
        cache.append((h, z))
        if l < len(layers) - 1:
            h = r(gelu(z))
        else:
            h = z
    return h, cache


def backward(flat, shapes, x, dy, rounding=True):
    """dL/d(parameters) (flat) and dL/dx for an upstream gradient dy = dL/dy."""
    r = bf16 if rounding else (lambda v: np.asarray(v, dtype=np.float64))
    layers = unpack(flat, shapes)
    _, cache = forward(flat, shapes, x, rounding)
    grads = [None] * len(layers)
    d = np.asarray(dy, dtype=np.float64)     # gradient w.r.t. z_l, unrounded
    dx = None
    for l in range(len(layers) - 1, -1, -1):
        W, _ = layers[l]
        h_in, _ = cache[l]
        dW = h_in.T @ r(d)
        db = d.sum(axis=0)
        grads[l] = (dW, db)
        dh = r(d) @ r(W).T                   # gradient w.r.t. this layer's input
        if l > 0:
            _, z_prev = cache[l - 1]
            d = dh * gelu_prime(z_prev)
        else:
            dx = dh
    flat_g = np.concatenate([np.concatenate([dW.ravel(), db]) for dW, db in grads])
    return flat_g, dx


def mse(y, t):
    """Mean squared error over all entries and its gradient dL/dy."""
    y = np.asarray(y, dtype=np.float64)
    t = np.asarray(t, dtype=np.float64)
    n = y.size
    return float(np.sum((y - t) ** 2) / n), 2.0 * (y - t) / n


def adam(w, g, m, v, t, lr, b1=0.9, b2=0.999, eps=1e-8):
    """One Adam step (Kingma and Ba 2015, Algorithm 1) at step count t >= 1."""
    m = b1 * m + (1.0 - b1) * g
    v = b2 * v + (1.0 - b2) * g * g
    mhat = m / (1.0 - b1 ** t)
    vhat = v / (1.0 - b2 ** t)
    return w - lr * mhat / (np.sqrt(vhat) + eps), m, v


def surrogate_objective(y, nobs, out_mean, out_std, x, x_prior, x_weight):
    """Per-row Poisson deviance of mu = exp(y out_std + out_mean) against
    observed counts, plus the Gaussian input prior 1/2 sum w (x - xbar)^2."""
    mu = np.exp(np.asarray(y, dtype=np.float64) * out_std + out_mean)
    n = np.asarray(nobs, dtype=np.float64)
    dev = np.where(n > 0, mu - n + n * np.log(np.where(n > 0, n, 1.0) / mu), mu)
    pri = 0.5 * np.sum(x_weight * (np.asarray(x, dtype=np.float64) - x_prior) ** 2, axis=1)
    return dev.sum(axis=1) + pri
