"""The surrogate network on the matrix cores (nf_mlp_*) against the FP64
oracle network with the same bfloat16 rounding points.

Hidden activations are rounded to bfloat16 from an FP32 pre-activation whose
summation order differs between the kernel and the oracle, so a value within
the FP32 accumulation error of a rounding boundary can round either way (one
bfloat16 unit, 2^-8 relative). Such a flip perturbs the rest of that row by
about 2^-8 / sqrt(width) relative. The parity bar is therefore per row: most
rows agree to FP32 accumulation accuracy, every row to the flip bound."""
import sys

import numpy as np
import pytest

from oracle import mlp as O
from paper_2502_15253_amd import nufold as nf

pytestmark = pytest.mark.gpu


def say(*a):
    print("[case]", *a, flush=True)
    sys.stdout.flush()


def init(shapes, rng, scale=1.0):
    parts = []
    for a, b in shapes:
        parts.append(rng.standard_normal(a * b) * scale * np.sqrt(2.0 / a))
        parts.append(rng.standard_normal(b) * 0.1)
    return np.concatenate(parts).astype(np.float32)


def row_errors(got, ref):
    scale = np.sqrt(np.mean(ref ** 2, axis=1)) + 1e-30
    return np.max(np.abs(got - ref), axis=1) / scale


@pytest.mark.parametrize("n_in,width,depth,n_out,B", [(20, 96, 2, 37, 70), (7, 64, 1, 5, 1),
                                                      (33, 130, 3, 65, 129)])
def test_forward_matches_oracle(n_in, width, depth, n_out, B):
    say("mlp forward", n_in, width, depth, n_out, B)
    rng = np.random.default_rng(n_in + width)
    net = nf.Mlp(n_in, width, depth, n_out, max_batch=B)
    shapes = O.layer_dims(n_in, width, depth, n_out)
    assert net.nparam == O.num_params(shapes)
    flat = init(shapes, rng)
    net.set_params(flat)
    np.testing.assert_array_equal(net.get_params(), flat)
    x = rng.uniform(-1, 1, (B, n_in)).astype(np.float32)
    y = net.forward(x)
    ref, _ = O.forward(flat.astype(np.float64), shapes, x.astype(np.float64))
    e = row_errors(y, ref)
    assert np.mean(e < 3e-5) >= 0.85, np.sort(e)[-10:]
    assert np.all(e < 1e-2), e.max()


def test_forward_full_surrogate_size():
    say("mlp forward 20-512x4-400")
    rng = np.random.default_rng(1)
    shapes = O.layer_dims(20, 512, 4, 400)
    net = nf.Mlp(20, 512, 4, 400, max_batch=256)
    flat = init(shapes, rng)
    net.set_params(flat)
    x = rng.uniform(-1, 1, (256, 20)).astype(np.float32)
    y = net.forward(x)
    ref, _ = O.forward(flat.astype(np.float64), shapes, x.astype(np.float64))
    e = row_errors(y, ref)
    assert np.all(e < 2e-2), e.max()
    assert np.linalg.norm(y - ref) / np.linalg.norm(ref) < 5e-3
    # without the emulated rounding the difference is the bfloat16 error itself
    ex, _ = O.forward(flat.astype(np.float64), shapes, x.astype(np.float64), rounding=False)
    assert np.linalg.norm(y - ex) / np.linalg.norm(ex) < 5e-2


def test_gradients_match_oracle():
    say("mlp grad")
    rng = np.random.default_rng(7)
    n_in, width, depth, n_out, B = 20, 96, 2, 37, 70
    shapes = O.layer_dims(n_in, width, depth, n_out)
    net = nf.Mlp(n_in, width, depth, n_out, max_batch=128)
    flat = init(shapes, rng)
    net.set_params(flat)
    x = rng.uniform(-1, 1, (B, n_in)).astype(np.float32)
    dy = rng.standard_normal((B, n_out)).astype(np.float32)
    g, dx = net.grad(x, dy)
    gr, dxr = O.backward(flat.astype(np.float64), shapes, x.astype(np.float64), dy.astype(np.float64))
    o = 0
    for a, b in shapes:
        for n in (a * b, b):
            seg, ref = g[o:o + n], gr[o:o + n]
            rel = np.abs(seg - ref) / np.max(np.abs(ref))
            assert np.linalg.norm(seg - ref) / np.linalg.norm(ref) < 3e-3, (o, n)
            assert np.mean(rel < 1e-4) >= 0.9, (o, n, np.sort(rel)[-5:])
            o += n
    e = row_errors(dx, dxr)
    assert np.mean(e < 1e-4) >= 0.85 and np.all(e < 2e-2), np.sort(e)[-5:]


def test_train_steps_match_oracle_adam():
    say("mlp train step")
    rng = np.random.default_rng(8)
    n_in, width, depth, n_out, B = 12, 64, 2, 24, 48
    shapes = O.layer_dims(n_in, width, depth, n_out)
    net = nf.Mlp(n_in, width, depth, n_out, max_batch=B)
    w = init(shapes, rng).astype(np.float64)
    net.set_params(w.astype(np.float32))
    m = np.zeros_like(w)
    v = np.zeros_like(w)
    lr = 1e-3
    for t in (1, 2):
        x = rng.uniform(-1, 1, (B, n_in)).astype(np.float32)
        tgt = rng.standard_normal((B, n_out)).astype(np.float32)
        loss = net.train_step(x, tgt, lr)
        y, _ = O.forward(w, shapes, x.astype(np.float64))
        L, dy = O.mse(y, tgt.astype(np.float64))
        g, _ = O.backward(w, shapes, x.astype(np.float64), dy)
        assert abs(loss - L) <= 1e-3 * L, (loss, L)
        w_new, m, v = O.adam(w, g, m, v, t, lr)
        got = net.get_params().astype(np.float64)
        big = np.abs(g) > 1e-2 * np.max(np.abs(g))
        # steps of well-determined gradients agree to a small fraction of lr;
        # every step is bounded by Adam's |step| <= lr sqrt((1 - b2^t)) / (1 - b1^t)
        assert np.max(np.abs((got - w_new)[big])) < 0.02 * lr
        assert np.max(np.abs(got - w_new)) < 3 * lr
        w = got  # continue from the device's weights


def test_fit_inputs_lowers_the_surrogate_objective_and_reports_it():
    say("mlp fit_inputs")
    rng = np.random.default_rng(9)
    n_in, width, depth, n_out, B = 6, 64, 2, 40, 16
    shapes = O.layer_dims(n_in, width, depth, n_out)
    net = nf.Mlp(n_in, width, depth, n_out, max_batch=B)
    flat = init(shapes, rng, scale=0.7)
    net.set_params(flat)
    mean = rng.uniform(3, 6, n_out).astype(np.float32)
    std = rng.uniform(0.05, 0.3, n_out).astype(np.float32)
    x_true = rng.uniform(-0.5, 0.5, (B, n_in)).astype(np.float32)
    y_true, _ = O.forward(flat.astype(np.float64), shapes, x_true.astype(np.float64))
    nobs = rng.poisson(np.exp(y_true * std + mean)).astype(np.float32)
    xbar = np.zeros(n_in, np.float32)
    xw = np.full(n_in, 0.5, np.float32)
    x0 = np.zeros((B, n_in), np.float32)
    y0, _ = O.forward(flat.astype(np.float64), shapes, x0.astype(np.float64))
    f0 = O.surrogate_objective(y0, nobs, mean, std, x0, xbar, xw)
    x1, nll = net.fit_inputs(x0, nobs, mean, std, xbar, xw, iters=300, lr=0.02)
    y1, _ = O.forward(flat.astype(np.float64), shapes, x1.astype(np.float64))
    f1 = O.surrogate_objective(y1, nobs, mean, std, x1, xbar, xw)
    assert np.all(f1 < f0)
    np.testing.assert_allclose(nll, f1, rtol=2e-3, atol=0.05)


def test_mlp_argument_errors():
    say("mlp errors")
    with pytest.raises(nf.NufoldError):
        nf.Mlp(0, 8, 1, 1, 4)
    net = nf.Mlp(4, 8, 1, 3, max_batch=4)
    with pytest.raises(nf.NufoldError) as ei:
        net.forward(np.zeros((5, 4), np.float32))
    assert ei.value.code == nf.NF_EINVAL
    with pytest.raises(nf.NufoldError):
        net.train_step(np.zeros((2, 4), np.float32), np.zeros((2, 3), np.float32), -1.0)


def test_train_step_graph_replays_match_launches():
    """The captured training step (replayed with each step's inputs, learning
    rate and bias corrections, other work and synchronisations in between)
    gives the same weights, bit for bit, as the same steps launched one kernel
    at a time; a change of batch size re-captures."""
    import torch
    say("mlp train step graph")
    rng = np.random.default_rng(9)
    n_in, width, depth, n_out = 20, 128, 3, 40
    shapes = O.layer_dims(n_in, width, depth, n_out)
    w = init(shapes, rng).astype(np.float32)
    nets = []
    for graphs in (False, True):
        net = nf.Mlp(n_in, width, depth, n_out, max_batch=512)
        net.set_params(w)
        net.use_graphs(graphs)
        nets.append(net)
    for step in range(8):
        B = 256 if step < 5 else 384
        x = torch.from_numpy(rng.uniform(-1, 1, (B, n_in)).astype(np.float32)).cuda()
        t = torch.from_numpy(rng.standard_normal((B, n_out)).astype(np.float32)).cuda()
        lr = 1e-3 * (1.0 + 0.1 * step)
        losses = [net.train_step(x, t, lr, want_loss=True) for net in nets]
        # unrelated eager work between the replays
        _ = [net.forward(rng.uniform(-1, 1, (7, n_in)).astype(np.float32)) for net in nets]
        torch.cuda.synchronize()
        p0, p1 = nets[0].get_params(), nets[1].get_params()
        assert losses[0] == losses[1], (step, losses)
        assert np.array_equal(p0, p1), (step, float(np.max(np.abs(p0 - p1))))
    for net in nets:
        net.close()
