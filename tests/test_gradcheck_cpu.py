"""The per-component gradient scale of the parity tests (tests/gradcheck.py):
its Fisher diagonal equals the diagonal of the oracle's (pinned) Hessian at
Asimov data, and the per-component check catches an error that the
max-normalised check lets through (CPU)."""
import numpy as np

from oracle.model import Model
from oracle import likelihood as LK
from oracle import fit as FIT
from paper_2502_15253_amd import synth
import gradcheck


def test_fisher_diagonal_is_the_hessian_diagonal_at_asimov():
    desc = synth.tiny_model(51, formula="3nu", n_datasets=2, n_sources=2)
    m = Model(desc)
    ev = synth.tiny_events(desc, 3000, 52)
    th = synth.start_vector(desc)
    data = LK.expected(m, ev, th)[0]
    free = list(np.where(~m.fixed)[0])
    Hd = np.diag(FIT.hessian(m, ev, data, th, free))
    F = gradcheck.fisher_diagonal(m, ev, th)[free]
    assert np.max(np.abs(F - Hd) / Hd) < 1e-5


def test_per_component_check_catches_a_small_component_error():
    desc = synth.tiny_model(53, formula="eq1", n_datasets=1, n_sources=1)
    m = Model(desc)
    ev = synth.tiny_events(desc, 3000, 54)
    th = synth.start_vector(desc) * 1.01
    data = synth.poisson_data(LK.expected(m, ev, synth.start_vector(desc))[0], 55)
    _, g = LK.nll_grad(m, ev, data, th)
    F = gradcheck.fisher_diagonal(m, ev, th)
    j = int(np.argmin(np.maximum(np.abs(g), np.sqrt(F))))
    bad = g.copy()
    bad[j] += 1e-3 * max(abs(g[j]), np.sqrt(F[j])) + 0.0
    # within the max-normalised bar at 1e-3 ...
    assert np.max(np.abs(bad - g)) <= 1e-3 * max(1.0, np.max(np.abs(g)))
    # ... but at the per-component bar it is off by 1e-3 of its own scale
    r, jr, _, _ = gradcheck.component_errors(bad, g, F)
    assert jr == j and abs(r - 1e-3) < 1e-9


def test_oracle_fisher_output_matches_the_separate_route():
    desc = synth.tiny_model(56, formula="3nu", n_datasets=2, n_sources=2)
    m = Model(desc)
    ev = synth.tiny_events(desc, 2000, 57)
    th = synth.start_vector(desc) * 1.003
    data = synth.poisson_data(LK.expected(m, ev, synth.start_vector(desc))[0], 58)
    f, g = LK.nll_grad(m, ev, data, th)
    f2, g2, F = LK.nll_grad(m, ev, data, th, fisher=True)
    assert f == f2 and np.array_equal(g, g2)
    assert np.max(np.abs(F - gradcheck.fisher_diagonal(m, ev, th)) / F) < 1e-12
