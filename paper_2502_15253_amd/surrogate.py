"""Warm starts for fits from a learned surrogate of the expected spectrum.

The surrogate maps a subset of the model parameters (every free or
prior-constrained parameter except the per-bin flux and background shape
modes) to the standardised log expectations of all analysis bins. It is
trained on spectra from the exact engine (nf_expected_batch, one event fold
per oscillation point shared by many nuisance draws) with the library's
matrix-core network (nf_mlp_*), and used only to propose start points: a
batch of surrogate fits over a grid of starts in the free oscillation
parameters picks, per data set, the most likely basin; the exact fit then
starts there. Every reported NLL comes from the exact fold.

Host code here only draws parameter vectors, standardises arrays and moves
them; every evaluation of the spectrum or of the network runs in the
library's kernels.
"""
from __future__ import annotations

import math
import time

import numpy as np

from . import nufold as nf

# free oscillation parameters of the three-flavour fit: training box
DEFAULT_BOXES = {"osc.sin2_t13": (0.015, 0.030), "osc.dm2_31": (2.3, 2.8)}


class Space:
    """Input parameters of the surrogate, their training box and the map
    between parameter values and network inputs x in [-1, 1]."""

    def __init__(self, desc, boxes=None, nsigma=5.0, free_frac=0.5):
        boxes = dict(DEFAULT_BOXES if boxes is None else boxes)
        excluded = set()
        for ds in desc["datasets"]:
            fx = ds.get("flux")
            if fx:
                excluded.update(fx["params"])
            for b in ds.get("backgrounds", []):
                if b.get("shape"):
                    excluded.update(n for n in b["shape"] if n)
        osc_names = {v["param"] for v in desc["osc"].values() if isinstance(v, dict) and "param" in v}
        self.P = len(desc["params"])
        self.base = np.array([p["start"] for p in desc["params"]], dtype=np.float64)
        inputs, lo, hi, pm, ps, is_osc = [], [], [], [], [], []
        for i, p in enumerate(desc["params"]):
            name = p["name"]
            if name in excluded or p.get("fixed"):
                continue
            if name in boxes:
                a, b = boxes[name]
            elif p["prior"]:
                m, s = p["prior"]
                a, b = m - nsigma * s, m + nsigma * s
            else:
                s = abs(p["start"]) * free_frac or 1.0
                a, b = p["start"] - s, p["start"] + s
            inputs.append(i)
            lo.append(a)
            hi.append(b)
            pm.append(p["prior"][0] if p["prior"] else np.nan)
            ps.append(p["prior"][1] if p["prior"] else np.nan)
            is_osc.append(name in osc_names)
        self.inputs = np.array(inputs)
        self.names = [desc["params"][i]["name"] for i in inputs]
        self.lo, self.hi = np.array(lo), np.array(hi)
        self.center, self.half = 0.5 * (self.lo + self.hi), 0.5 * (self.hi - self.lo)
        self.is_osc = np.array(is_osc)
        pm, ps = np.array(pm), np.array(ps)
        has = np.isfinite(ps)
        # Gaussian priors in input units: 1/2 w (x - xbar)^2 with w = (half / sigma)^2
        self.x_prior = np.where(has, (pm - self.center) / self.half, 0.0)
        self.x_weight = np.where(has, (self.half / np.where(has, ps, 1.0)) ** 2, 0.0)
        self.free = ~has            # inputs without a prior: the ones the start grid covers
        self.n_in = len(inputs)

    def to_x(self, theta):
        return ((np.asarray(theta)[:, self.inputs] - self.center) / self.half).astype(np.float32)

    def to_theta(self, x, base=None):
        th = np.tile(self.base if base is None else base, (x.shape[0], 1))
        th[:, self.inputs] = self.center + self.half * np.asarray(x, dtype=np.float64)
        return th

    def sample(self, rng, n_osc, n_nuis):
        """n_osc oscillation points, each with n_nuis draws of the other inputs,
        all uniform over the training box; excluded parameters at their start."""
        x = rng.uniform(-1.0, 1.0, (n_osc * n_nuis, self.n_in))
        osc_x = rng.uniform(-1.0, 1.0, (n_osc, int(self.is_osc.sum())))
        x[:, self.is_osc] = np.repeat(osc_x, n_nuis, axis=0)
        return self.to_theta(x)


def generate(eng, space, n_osc, n_nuis, seed, rows_per_call=4096, log=None):
    """Training set: inputs x (float32, N x n_in) and log expectations of all
    analysis bins (float32, N x bins) from the exact engine."""
    rng = np.random.default_rng(seed)
    nb = sum(eng.nbins)
    N = n_osc * n_nuis
    X = np.empty((N, space.n_in), np.float32)
    Y = np.empty((N, nb), np.float32)
    per = max(1, rows_per_call // n_nuis)
    o = 0
    t0 = time.perf_counter()
    while o < N:
        k = min(per, (N - o) // n_nuis)
        th = space.sample(rng, k, n_nuis)
        mu, code = eng.expected_batch(th)
        if code != nf.NF_OK or not np.all(mu > 0):
            raise RuntimeError("training point out of the model's domain")
        X[o:o + len(th)] = space.to_x(th)
        Y[o:o + len(th)] = np.log(mu)
        o += len(th)
    if log:
        log(f"generated {N} spectra in {time.perf_counter() - t0:.2f} s")
    return X, Y


class Surrogate:
    """stream: a torch.cuda.Stream (default priority) shared by the network's
    kernels and the torch operations that feed it; None creates one."""

    def __init__(self, space, n_out, width=512, depth=4, max_batch=4096, seed=0, stream=None):
        import torch
        self.space = space
        self.stream = stream if stream is not None else torch.cuda.Stream()
        self.net = nf.Mlp(space.n_in, width, depth, n_out, max_batch, stream=self.stream.cuda_stream)
        rng = np.random.default_rng(seed)
        parts = []
        for a, b in self.net.layer_shapes():
            parts.append(rng.standard_normal(a * b) * math.sqrt(2.0 / a))  # He initialisation
            parts.append(np.zeros(b))
        self.net.set_params(np.concatenate(parts).astype(np.float32))
        self.out_mean = np.zeros(n_out, np.float32)
        self.out_std = np.ones(n_out, np.float32)

    def train(self, X, Ylog, epochs=10, batch=1024, lr=1e-3, lr_min=1e-5, seed=0, log=None):
        """Adam on the mean squared error of standardised log expectations,
        cosine learning-rate decay; the data set lives in device memory."""
        import torch
        self.out_mean = Ylog.mean(axis=0).astype(np.float32)
        self.out_std = (Ylog.std(axis=0) + 1e-6).astype(np.float32)
        T = ((Ylog - self.out_mean) / self.out_std).astype(np.float32)
        with torch.cuda.stream(self.stream):
            return self._train(torch, X, T, epochs, batch, lr, lr_min, seed, log)

    def _train(self, torch, X, T, epochs, batch, lr, lr_min, seed, log):
        Xd = torch.from_numpy(np.ascontiguousarray(X)).cuda()
        Td = torch.from_numpy(np.ascontiguousarray(T)).cuda()
        n = X.shape[0]
        spe = max(1, n // batch)
        total = epochs * spe
        gen = torch.Generator(device="cuda")
        gen.manual_seed(seed)
        losses = []
        step = 0
        t0 = time.perf_counter()
        for ep in range(epochs):
            perm = torch.randperm(n, device="cuda", generator=gen)
            for s in range(spe):
                idx = perm[s * batch:(s + 1) * batch]
                xb = Xd.index_select(0, idx).contiguous()
                tb = Td.index_select(0, idx).contiguous()
                a = lr_min + 0.5 * (lr - lr_min) * (1 + math.cos(math.pi * step / total))
                last = s == spe - 1
                out = self.net.train_step(xb, tb, a, want_loss=last)
                if last:
                    losses.append(out)
                step += 1
            if log:
                log(f"epoch {ep}: loss {losses[-1]:.3e} ({time.perf_counter() - t0:.1f} s)")
        self.stream.synchronize()
        return losses

    def predict_log_mu(self, theta):
        y = self.net.forward(self.space.to_x(theta))
        return y * self.out_std + self.out_mean

    def start_grid(self, grid=(4, 16)):
        """Start rows (x units) of the surrogate fits: a grid over the inputs
        without a prior, every other input at its prior mean."""
        sp = self.space
        free = np.where(sp.free)[0]
        axes = []
        for j, f in enumerate(free):
            n = grid[j] if j < len(grid) else 1
            axes.append((np.arange(n) + 0.5) / n * 2.0 - 1.0)
        mesh = np.array(np.meshgrid(*axes, indexing="ij")).reshape(len(free), -1).T
        x0 = np.tile(sp.x_prior, (mesh.shape[0], 1))
        x0[:, free] = mesh
        return x0.astype(np.float32)

    def attach(self, eng, grid=(4, 16), iters=200, lr=0.02):
        """Attach this network to an engine for warm starts inside the library's
        fits (nf_set_surrogate; fits then take warm_start=True): the same start
        grid, surrogate fits and choice as warm_start below."""
        sp = self.space
        return eng.set_surrogate(self.net, sp.inputs, sp.center, sp.half, self.out_mean, self.out_std,
                                 sp.x_prior.astype(np.float32), sp.x_weight.astype(np.float32),
                                 self.start_grid(grid), iters=iters, lr=lr)

    def warm_start(self, nobs, grid=(4, 16), iters=200, lr=0.02, base=None):
        """Start points for fits of each row of observed counts (E x bins).
        Surrogate fits from a grid over the inputs without a prior (others at
        their prior means), run together; the best per row wins."""
        sp = self.space
        E = nobs.shape[0]
        x0 = self.start_grid(grid)
        S = x0.shape[0]
        X0 = np.tile(x0, (E, 1)).astype(np.float32)
        N = np.repeat(np.asarray(nobs, np.float32), S, axis=0)
        out_x = np.empty_like(X0)
        out_f = np.empty(E * S, np.float32)
        mb = self.net.max_batch
        for o in range(0, E * S, mb):
            xs, fs = self.net.fit_inputs(X0[o:o + mb], N[o:o + mb], self.out_mean, self.out_std,
                                         sp.x_prior.astype(np.float32), sp.x_weight.astype(np.float32),
                                         iters, lr)
            out_x[o:o + mb], out_f[o:o + mb] = xs, fs
        out_f = np.where(np.isfinite(out_f), out_f, np.inf).reshape(E, S)
        best = np.argmin(out_f, axis=1)
        xb = out_x.reshape(E, S, -1)[np.arange(E), best]
        xb = np.clip(xb, -1.0, 1.0)
        return sp.to_theta(xb, base), out_f[np.arange(E), best]
