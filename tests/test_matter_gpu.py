"""Exact three-flavour survival in matter of constant density (the matter step
of the medium-baseline analysis, which the paper takes from GLoBES): single
and batched device evaluations and fits against the oracle, and the size of
the matter effect against the same model in vacuum. Tolerances as in
test_parity_gpu."""
import sys

import numpy as np
import pytest

from oracle.model import Model
from oracle import likelihood as LK
from paper_2502_15253_amd import nufold as nf
from paper_2502_15253_amd import synth
import gradcheck
from test_parity_gpu import TOL, GRAD_TOL, GRAD_MAX_TOL, make_engine, oracle_data, compare, displaced

pytestmark = pytest.mark.gpu


def say(*a):
    print("[case]", *a, flush=True)
    sys.stdout.flush()


@pytest.mark.parametrize("mode", ["m64", "m32"])
def test_medium_baseline_in_matter(mode):
    say("medium baseline in matter", mode)
    desc, events = synth.model_and_events("c3_matter", 200_000)
    data = oracle_data(desc, events, 81)
    eng = make_engine(desc, events, data, mode)
    for j in range(2):
        compare(eng, desc, events, data, displaced(desc, 90 + j), TOL[mode], f"c3 matter {mode} {j}",
                gtol=GRAD_TOL[mode], gmax=GRAD_MAX_TOL[mode])
    # the same model in vacuum: the device reproduces the oracle's matter
    # effect bin by bin, and the effect is far above the tolerance
    vac = dict(desc)
    vac["osc"] = {k: v for k, v in desc["osc"].items() if k != "rho_ye"}
    vac["osc"]["formula"] = "3nu"
    eng_v = make_engine(vac, events, data, mode)
    th = displaced(desc, 95)
    mu_m, code_m = eng.expected(th)
    mu_v, code_v = eng_v.expected(th)
    assert code_m == nf.NF_OK and code_v == nf.NF_OK
    om, _ = LK.expected(Model(desc), events, th)
    ov, _ = LK.expected(Model(vac), events, th)
    for a, b, c, d in zip(mu_m, mu_v, om, ov):
        effect = np.max(np.abs(c / d - 1.0))
        say("largest relative matter effect on mu", effect)
        assert effect > 1e-4
        assert np.max(np.abs((a - b) - (c - d)) / np.abs(c)) <= 2 * TOL[mode]


@pytest.mark.parametrize("mode", ["m64", "m32"])
def test_batched_matter_matches_oracle_and_single_fits(mode):
    say("batched matter", mode)
    desc = synth.tiny_model(21, formula="3nu_matter", n_datasets=2, n_sources=2)
    events = synth.tiny_events(desc, 6000, 77)
    m = Model(desc)
    mus = LK.expected(m, events, synth.start_vector(desc))[0]
    rows = np.array([np.concatenate(synth.poisson_data(mus, 500 + j)) for j in range(4)])
    eng = make_engine(desc, events, None, mode)
    eng.set_data_batch(rows)
    rng = np.random.default_rng(7)
    B = 7
    thetas = np.array([displaced(desc, 200 + j) for j in range(B)])
    didx = rng.integers(0, 4, B).astype(np.int32)
    nll, grad, code = eng.eval_batch(thetas, didx)
    assert code == nf.NF_OK
    tol = TOL[mode]

    def split(row):
        out, o = [], 0
        for ds in desc["datasets"]:
            nb = len(ds["edges"]) - 1
            out.append(row[o:o + nb])
            o += nb
        return out
    for f in range(B):
        f_o, g_o, F = LK.nll_grad(m, events, split(rows[didx[f]]), thetas[f], fisher=True)
        assert abs(nll[f] - f_o) <= tol * max(1.0, abs(f_o)), (f, nll[f], f_o)
        assert np.max(np.abs(grad[f] - g_o)) <= GRAD_MAX_TOL[mode] * max(1.0, np.max(np.abs(g_o))), f
        gradcheck.check(grad[f], g_o, F, GRAD_TOL[mode], f"batch matter {mode} fit {f}", m.names)
    # batched fits against one-at-a-time fits of the same pseudo-experiments
    starts = np.tile(synth.start_vector(desc), (4, 1))
    rb = eng.fit_batch(starts, data_idx=np.arange(4, dtype=np.int32), edm_tol=1e-9, max_iter=3000)
    assert np.all(rb["status"] == 0)
    for j in range(4):
        for d, n in enumerate(split(rows[j])):
            eng.set_data(d, n)
        rs = eng.fit(synth.start_vector(desc), edm_tol=1e-9, max_iter=3000)
        say("fit", j, rb["nll"][j], rs["nll"])
        assert abs(rb["nll"][j] - rs["nll"]) < 1e-6 * max(1.0, abs(rs["nll"]))
