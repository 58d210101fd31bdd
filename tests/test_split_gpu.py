"""Conditional splitting of datasets (paper, "Conditional splitting of
datasets"; Eq. 9): 18 uneven histograms plus two one-bin reactor-off rate
terms in one model. Single evaluations against the oracle in both precision
modes, and batched pseudo-experiment fits against single fits."""
import sys

import numpy as np
import pytest

from oracle.model import Model
from oracle import likelihood as LK
from paper_2502_15253_amd import nufold as nf
from paper_2502_15253_amd import synth
from test_parity_gpu import compare, displaced, make_engine, TOL, GRAD_TOL, GRAD_MAX_TOL

pytestmark = pytest.mark.gpu


def say(*a):
    print("[case]", *a, flush=True)
    sys.stdout.flush()


@pytest.mark.parametrize("mode", ["m64", "m32"])
def test_split_model_matches_oracle(mode):
    say("split parity", mode)
    desc, events = synth.model_and_events("split")
    m = Model(desc)
    mus, _ = LK.expected(m, events, synth.start_vector(desc))
    data = synth.poisson_data(mus, synth.data_seed(6))
    eng = make_engine(desc, events, data, mode)
    assert eng.D == 20 and [eng.nbins[d] for d in range(18, 20)] == [1, 1]
    compare(eng, desc, events, data, synth.start_vector(desc), TOL[mode], "split start", gtol=GRAD_TOL[mode], gmax=GRAD_MAX_TOL[mode])
    compare(eng, desc, events, data, displaced(desc, 600), TOL[mode], "split displaced", gtol=GRAD_TOL[mode], gmax=GRAD_MAX_TOL[mode])


def test_split_batched_fits_match_single_fits():
    say("split batched fits")
    desc, events = synth.model_and_events("split", 0.3)
    m = Model(desc)
    mu0 = LK.expected(m, events, synth.start_vector(desc))[0]
    B = 12
    rows = np.array([np.concatenate(synth.poisson_data(mu0, synth.pseudo_seed(j))) for j in range(B)])
    eng = make_engine(desc, events, None, "m64")
    eng.set_data_batch(rows)
    start = np.tile(synth.start_vector(desc), (B, 1))
    rb = eng.fit_batch(start, edm_tol=1e-9, max_iter=3000)
    assert rb["code"] == nf.NF_OK, rb["status"]
    nb = np.cumsum([0] + [len(ds["edges"]) - 1 for ds in desc["datasets"]])
    for f in (0, 5, 11):
        for d in range(len(desc["datasets"])):
            eng.set_data(d, rows[f][nb[d]:nb[d + 1]])
        r1 = eng.fit(start[f], edm_tol=1e-9, max_iter=3000)
        assert r1["status"] == 0
        assert abs(rb["nll"][f] - r1["nll"]) < 5e-7, (f, rb["nll"][f], r1["nll"])
        # the reported minimum is the oracle's NLL at the reported point
        dat = [rows[f][nb[d]:nb[d + 1]] for d in range(len(desc["datasets"]))]
        f_o = LK.nll(m, events, dat, rb["theta"][f])
        assert abs(f_o - rb["nll"][f]) <= 1e-9 * max(1.0, f_o)
