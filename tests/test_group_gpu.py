"""Mixed ensembles (nf_fit_batch_group): pseudo-experiments of the
single-detector and the three-detector model fitted in one launch sequence,
against each model's own batched fits and single fits."""
import sys

import numpy as np
import pytest

from oracle.model import Model
from oracle import likelihood as LK
from paper_2502_15253_amd import nufold as nf
from paper_2502_15253_amd import synth

pytestmark = pytest.mark.gpu


def say(*a):
    print("[case]", *a, flush=True)
    sys.stdout.flush()


def member(config, n_events, B, seed0):
    desc, events = synth.model_and_events(config, n_events)
    m = Model(desc)
    mu0 = LK.expected(m, events, synth.start_vector(desc))[0]
    rows = np.array([np.concatenate(synth.poisson_data(mu0, seed0 + j)) for j in range(B)])
    eng = nf.Engine(desc, "m64")
    for d, ev in enumerate(events):
        eng.set_events(d, ev["e_true"], ev["e_reco"], ev["source"], ev["weight"])
    eng.set_data_batch(rows)
    start = np.tile(synth.start_vector(desc), (B, 1))
    return desc, eng, rows, start


def test_group_fits_match_separate_and_single_fits():
    say("group c1 + c2")
    d1, e1, r1, s1 = member(1, None, 40, 3000)
    d2, e2, r2, s2 = member(2, 100_000, 12, 3100)
    out, code = nf.fit_batch_group([(e1, s1, None, None), (e2, s2, None, None)], edm_tol=1e-9, max_iter=3000)
    assert code == nf.NF_OK, [o["status"] for o in out]
    for (desc, eng, rows, start), o in zip([(d1, e1, r1, s1), (d2, e2, r2, s2)], out):
        sep = eng.fit_batch(start, edm_tol=1e-9, max_iter=3000)
        assert sep["code"] == nf.NF_OK
        # the same minimiser on the same inputs: minima agree to rounding
        assert np.max(np.abs(sep["nll"] - o["nll"])) < 1e-7, np.max(np.abs(sep["nll"] - o["nll"]))
        nb = np.cumsum([0] + [len(ds["edges"]) - 1 for ds in desc["datasets"]])
        for f in (0, len(rows) - 1):
            for d in range(len(desc["datasets"])):
                eng.set_data(d, rows[f][nb[d]:nb[d + 1]])
            r = eng.fit(start[f], edm_tol=1e-9, max_iter=3000)
            assert r["status"] == 0
            assert abs(r["nll"] - o["nll"][f]) < 5e-7, (f, r["nll"], o["nll"][f])
        print(f"[group] {len(rows)} fits, mean iterations {o['iters'].mean():.1f}", flush=True)


def test_group_rejects_a_context_twice():
    say("group duplicate")
    d1, e1, r1, s1 = member(1, 20000, 4, 3000)
    with pytest.raises(nf.NufoldError):
        nf.fit_batch_group([(e1, s1, None, None), (e1, s1, None, None)])
