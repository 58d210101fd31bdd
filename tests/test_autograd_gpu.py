"""The adjoint gradient behind torch.autograd: against the oracle's gradient,
against central finite differences of the same operation, and inside a torch
optimiser."""
import sys

import numpy as np
import pytest

from oracle.model import Model
from oracle import likelihood as LK
from paper_2502_15253_amd import synth
import gradcheck

pytestmark = pytest.mark.gpu


def say(*a):
    print("[case]", *a, flush=True)
    sys.stdout.flush()


def test_backward_matches_oracle_gradient_and_finite_differences():
    import torch
    from paper_2502_15253_amd.autograd import NLL
    say("autograd c3")
    desc, events = synth.model_and_events(3, 200_000)
    m = Model(desc)
    th0 = synth.start_vector(desc)
    data = synth.poisson_data(LK.expected(m, events, th0)[0], 17)
    f = NLL.create(desc, events, data, "m64")
    th = th0.copy()
    th[m.index["osc.dm2_31"]] = 2.51
    th[m.index["escale.c1"]] = 0.004
    x = torch.tensor(th, dtype=torch.float64, device="cuda", requires_grad=True)
    y = f(x)
    (3.0 * y).backward()
    g = x.grad.cpu().numpy() / 3.0
    f_o, g_o, F = LK.nll_grad(m, events, data, th, fisher=True)
    assert abs(y.item() - f_o) <= 1e-9 * max(1.0, abs(f_o))
    assert np.max(np.abs(g - g_o)) <= 1e-9 * max(1.0, np.max(np.abs(g_o)))
    gradcheck.check(g, g_o, F, 1e-9, "autograd c3 m64", m.names)
    # central differences of the operation itself (h = 1e-6) on a few parameters
    for name in ("osc.dm2_31", "osc.sin2_t13", "norm", "escale.c1", "flux[40]"):
        i = m.index[name]
        e = torch.zeros_like(x)
        e[i] = 1e-6
        with torch.no_grad():
            fd = (f(x + e) - f(x - e)).item() / 2e-6
        assert abs(fd - g[i]) <= 1e-5 * max(1.0, abs(g[i])), (name, fd, g[i])


def test_torch_optimiser_reaches_the_device_fit_minimum():
    import torch
    from paper_2502_15253_amd.autograd import NLL
    say("autograd lbfgs c1")
    desc, events = synth.model_and_events(1, 30_000)
    m = Model(desc)
    th0 = synth.start_vector(desc)
    data = synth.poisson_data(LK.expected(m, events, th0)[0], 23)
    f = NLL.create(desc, events, data, "m64")
    r = f.engine.fit(th0, edm_tol=1e-10)
    assert r["status"] == 0
    # optimise z with theta = theta0 + scale * z on the free parameters (a
    # diagonal preconditioning: prior widths, else 5% of the start value)
    scale = np.array([p["prior"][1] if p["prior"] else 0.05 * max(abs(p["start"]), 0.02)
                      for p in desc["params"]]) * (~m.fixed)
    t0 = torch.tensor(th0, dtype=torch.float64, device="cuda")
    sc = torch.tensor(scale, dtype=torch.float64, device="cuda")
    z = torch.zeros(m.P, dtype=torch.float64, device="cuda", requires_grad=True)
    opt = torch.optim.LBFGS([z], lr=1, max_iter=500, tolerance_grad=1e-10, tolerance_change=1e-15,
                            history_size=50, line_search_fn="strong_wolfe")

    def closure():
        opt.zero_grad()
        y = f(t0 + sc * z)
        y.backward()
        return y

    for _ in range(5):
        opt.step(closure)
    with torch.no_grad():
        final = f(t0 + sc * z).item()
    assert abs(final - r["nll"]) < 1e-6, (final, r["nll"])
