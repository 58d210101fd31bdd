"""Device minimiser (nf_fit) against the oracle's fits and properties."""
import sys

import numpy as np
import pytest

from oracle.model import Model
from oracle import likelihood as LK
from oracle import fit as OFIT
from paper_2502_15253_amd import nufold as nf
from paper_2502_15253_amd import synth

pytestmark = pytest.mark.gpu


def say(*a):
    print("[case]", *a, flush=True)
    sys.stdout.flush()


def engine(desc, events, data, mode="m64"):
    eng = nf.Engine(desc, mode)
    for d, ev in enumerate(events):
        eng.set_events(d, ev["e_true"], ev["e_reco"], ev["source"], ev["weight"])
        eng.set_data(d, data[d])
    return eng


def displaced_start(desc, seed, frac=0.5):
    rng = np.random.default_rng(seed)
    th = synth.start_vector(desc).copy()
    for i, p in enumerate(desc["params"]):
        s = p["prior"][1] if p["prior"] else max(abs(p["start"]) * 0.03, 1e-3)
        th[i] += frac * s * rng.standard_normal()
    return th


def test_asimov_fit_recovers_truth_config1():
    say("fit asimov c1")
    desc, events = synth.model_and_events(1)
    m = Model(desc)
    truth = synth.start_vector(desc)
    data = LK.expected(m, events, truth)[0]
    eng = engine(desc, events, data)
    r = eng.fit(displaced_start(desc, 1), edm_tol=1e-9)
    assert r["code"] == nf.NF_OK and r["status"] == 0, r
    assert r["nll"] < 1e-6
    assert r["edm"] < 1e-9
    i13, iee = m.index["osc.sin2_2t13"], m.index["osc.dm2_ee"]
    assert abs(r["theta"][i13] - truth[i13]) < 2e-4
    assert abs(r["theta"][iee] - truth[iee]) < 2e-3


def test_poisson_fit_matches_oracle_minimum_config1():
    say("fit poisson c1 vs oracle")
    desc, events = synth.model_and_events(1, 30000)
    m = Model(desc)
    truth = synth.start_vector(desc)
    data = synth.poisson_data(LK.expected(m, events, truth)[0], synth.data_seed(1))
    eng = engine(desc, events, data)
    start = displaced_start(desc, 2)
    r = eng.fit(start, edm_tol=1e-9)
    ro = OFIT.fit(m, events, data, start, gtol=1e-8)
    assert r["status"] == 0
    # minimum NLL agrees; Delta chi^2 = 2 dNLL well below 1e-3
    assert abs(r["nll"] - ro["nll"]) < 1e-6, (r["nll"], ro["nll"])
    # the oracle agrees with the engine's NLL at the engine's optimum
    assert abs(LK.nll(m, events, data, r["theta"]) - r["nll"]) < 1e-9 * max(1, r["nll"])


def test_fixed_parameters_stay_fixed_and_profile_is_consistent():
    say("fit fixed / profile")
    desc, events = synth.model_and_events(1, 30000)
    m = Model(desc)
    truth = synth.start_vector(desc)
    data = synth.poisson_data(LK.expected(m, events, truth)[0], 7)
    eng = engine(desc, events, data)
    fixed = np.zeros(m.P, dtype=bool)
    i13, iee = m.index["osc.sin2_2t13"], m.index["osc.dm2_ee"]
    fixed[[i13, iee]] = True
    start = truth.copy()
    start[i13], start[iee] = 0.07, 2.4
    r = eng.fit(start, fixed=fixed, edm_tol=1e-9)
    assert r["status"] == 0
    assert r["theta"][i13] == 0.07 and r["theta"][iee] == 2.4
    rg = eng.fit(truth, edm_tol=1e-9)
    assert rg["status"] == 0
    # profile statistic of Eq. 7 at a displaced eta is positive
    assert r["nll"] - rg["nll"] > 0
    # the oracle's profile at the same point agrees
    fx = m.fixed.copy()
    fx[[i13, iee]] = True
    ro = OFIT.fit(m, events, data, start, fixed=fx, gtol=1e-8)
    assert abs(ro["nll"] - r["nll"]) < 1e-6


def test_covariance_matches_oracle_hessian():
    say("fit covariance")
    desc, events = synth.model_and_events(1, 30000)
    m = Model(desc)
    truth = synth.start_vector(desc)
    # Poisson data: at the Asimov truth the energy-scale map puts every analysis
    # edge on a fine-bin edge, where the spline's second derivative jumps, so
    # the Hessian there depends on the finite-difference step.
    data = synth.poisson_data(LK.expected(m, events, truth)[0], 11)
    eng = engine(desc, events, data)
    r = eng.fit(displaced_start(desc, 3), edm_tol=1e-10, want_cov=True)
    assert r["status"] == 0
    free = np.where(~m.fixed)[0]
    Ho = OFIT.hessian(m, events, data, r["theta"], free)
    cov_g = r["cov"][np.ix_(free, free)]
    Hg = np.linalg.inv(cov_g)
    # compare curvatures in units of the diagonal (the covariance itself amplifies
    # finite-difference errors by the Hessian's condition number)
    sd = np.sqrt(np.diag(Ho))
    err = np.max(np.abs(Hg - Ho) / np.outer(sd, sd))
    assert err < 1e-4, err
    assert np.all(np.diag(cov_g) > 0)


def test_config2_fit_converges_to_a_stationary_point():
    say("fit c2")
    desc, events = synth.model_and_events(2)
    m = Model(desc)
    truth = synth.start_vector(desc)
    data = synth.poisson_data(LK.expected(m, events, truth)[0], synth.data_seed(2))
    eng = engine(desc, events, data)
    r = eng.fit(displaced_start(desc, 4, 0.3), edm_tol=1e-8, max_iter=3000)
    assert r["status"] == 0, r
    f_o, g_o = LK.nll_grad(m, events, data, r["theta"])
    assert abs(f_o - r["nll"]) < 1e-9 * max(1, f_o)
    # gradient in units of each parameter's preconditioning scale is small
    scale = np.array([p["prior"][1] if p["prior"] else 0.01 for p in desc["params"]])
    assert np.max(np.abs(g_o * scale)) < 5e-3


@pytest.mark.parametrize("mode", ["m64", "m32"])
def test_config3_asimov_fit(mode):
    say("fit c3", mode)
    desc, events = synth.model_and_events(3, 2_000_000)
    m = Model(desc)
    truth = synth.start_vector(desc)
    data = LK.expected(m, events, truth)[0]
    eng = engine(desc, events, data, mode)
    start = truth.copy()
    start[m.index["osc.sin2_t13"]] = 0.0225
    start[m.index["osc.dm2_31"]] = 2.527
    r = eng.fit(start, edm_tol=1e-8)
    assert r["status"] == 0, r
    assert r["nll"] < (1e-6 if mode == "m64" else 1e-3)
    assert abs(r["theta"][m.index["osc.dm2_31"]] - 2.53) < 1e-3
    assert abs(r["theta"][m.index["osc.sin2_t13"]] - 0.0218) < 2e-4


def test_iteration_limit_and_domain_start():
    say("fit limits")
    desc, events = synth.model_and_events(1, 20000)
    m = Model(desc)
    truth = synth.start_vector(desc)
    data = synth.poisson_data(LK.expected(m, events, truth)[0], 9)
    eng = engine(desc, events, data)
    r = eng.fit(displaced_start(desc, 5), max_iter=1)
    assert r["code"] == nf.NF_WNOCONV and r["status"] == 2 and r["iters"] == 1
    bad = truth.copy()
    bad[m.index["escale.c1"]] = -2.0
    r = eng.fit(bad)
    assert r["code"] == nf.NF_WDOMAIN and r["status"] == 4
    # and a normal fit still works afterwards
    r = eng.fit(truth)
    assert r["status"] == 0
