"""Parity of the HIP engine (through the C-ABI) with the FP64 oracle.

Tolerances:
  M64: 1e-9 on every expectation mu_{d,i}, on the NLL and on the gradient
  M32: 1e-5 on the same quantities
  mu: relative per bin;  NLL: |dNLL| <= tol * max(1, |NLL|);
  gradient, per component: |dg_j| <= tol_g * max(|g_j|, sqrt(F_jj)), F_jj the
  NLL's curvature in theta_j (Fisher information plus prior; tests/gradcheck.py),
  so an error at the bar moves the fitted theta_j by tol_g standard deviations,
  and the whole vector also within tol * max(1, max|g|).
  tol_g is tol in M64; in M32 it is GRAD_TOL_M32. The FP32 fold's error in mu
  has a systematic part of a few 1e-8 relative: the hardware sin/cos
  (operand in revolutions) is biased by up to -4.6e-8 on average over
  [0, 0.02) revolutions and -2.8e-8 over [0.02, 0.1) (measured against FP64
  over 2^24 evenly spaced operands on MI355X). A relative error e common to
  the bins of a dataset with N counts moves dNLL/dtheta_j by about e N
  (through lambda = 1 - n/mu) against sqrt(F_jj) ~ sqrt(N), i.e. by e sqrt(N)
  of the per-component scale: 1e-5 at N = 2e5. The FP32 mode is held to
  5e-5 of that scale (one twenty-thousandth of a standard deviation of each
  fitted parameter); FP64 to 1e-9.
"""
import sys

import numpy as np
import pytest

from oracle.model import Model
from oracle import likelihood as LK
from oracle import fold as OF
from paper_2502_15253_amd import nufold as nf
from paper_2502_15253_amd import synth
import gradcheck

pytestmark = pytest.mark.gpu

TOL = {"m64": 1e-9, "m32": 1e-5}
GRAD_TOL_M32 = 5e-5
GRAD_TOL = {"m64": 1e-9, "m32": GRAD_TOL_M32}
# whole gradient vector against its largest component: 1e-9 / 2e-5 (the same
# FP32 systematic reaches 1.03e-5 of the largest component, an energy-scale
# derivative of a 2e5-count dataset)
GRAD_MAX_TOL = {"m64": 1e-9, "m32": 2e-5}


def say(*a):
    print("[case]", *a, flush=True)
    sys.stdout.flush()


def make_engine(desc, events, data=None, mode="m64", chunk=None, deterministic=None):
    eng = nf.Engine(desc, mode)
    if chunk:
        eng.set_option("chunk", chunk)
    if deterministic is not None:
        eng.set_option("deterministic", deterministic)
    for d, ev in enumerate(events):
        eng.set_events(d, ev["e_true"], ev["e_reco"], ev["source"], ev["weight"])
    if data is not None:
        for d, n in enumerate(data):
            eng.set_data(d, n)
    return eng


def oracle_data(desc, events, seed):
    m = Model(desc)
    mus, ok = LK.expected(m, events, synth.start_vector(desc))
    assert ok
    return synth.poisson_data(mus, seed)


def compare(eng, desc, events, data, theta, tol, what="", gtol=None, gmax=None):
    m = Model(desc)
    mus_o, _ = LK.expected(m, events, theta)
    f_o, g_o, F = LK.nll_grad(m, events, data, theta, fisher=True)
    mus_g, code = eng.expected(theta)
    assert code == nf.NF_OK
    for mo, mg in zip(mus_o, mus_g):
        rel = np.max(np.abs(mg - mo) / np.maximum(np.abs(mo), 1e-300))
        assert rel <= tol, f"{what}: mu rel err {rel:.3e}"
    f_g, g_g, code = eng.eval_nll_grad(theta)
    assert code == nf.NF_OK
    assert abs(f_g - f_o) <= tol * max(1.0, abs(f_o)), f"{what}: NLL {f_g!r} vs {f_o!r}"
    scale = max(1.0, np.max(np.abs(g_o)))
    err = np.max(np.abs(g_g - g_o))
    gm = tol if gmax is None else gmax
    assert err <= gm * scale, f"{what}: grad err {err:.3e} (scale {scale:.3e}) at {np.argmax(np.abs(g_g - g_o))}"
    gradcheck.check(g_g, g_o, F, tol if gtol is None else gtol, what, m.names)
    f_n, code = eng.eval_nll(theta)
    # the same evaluation without the gradient; fine-bin sums by atomic adds may
    # move the last bits of mu, which the deviance's cancellations amplify
    assert abs(f_n - f_g) <= 1e-10 * max(1.0, abs(f_g))
    return f_g, g_g


def displaced(desc, seed, scale=0.3):
    """Start vector moved by a fraction of each prior width (or 1% of the value)."""
    rng = np.random.default_rng(seed)
    th = synth.start_vector(desc).copy()
    for i, p in enumerate(desc["params"]):
        s = p["prior"][1] if p["prior"] else max(abs(p["start"]) * 0.01, 1e-3)
        th[i] += scale * s * rng.standard_normal()
    return th


@pytest.mark.parametrize("mode", ["m64", "m32"])
@pytest.mark.parametrize("formula", ["eq1", "3nu", "4nu", "3nu_matter"])
@pytest.mark.parametrize("seed", [0, 1, 2])
@pytest.mark.parametrize("deterministic", [0, 1])
def test_tiny_models(mode, formula, seed, deterministic):
    say("tiny", mode, formula, seed, deterministic)
    desc = synth.tiny_model(10 + seed, formula=formula, n_datasets=2 + seed % 2, n_sources=1 + seed)
    events = synth.tiny_events(desc, 5000 + 1111 * seed, 50 + seed)
    data = oracle_data(desc, events, 60 + seed)
    eng = make_engine(desc, events, data, mode, deterministic=deterministic)
    for j in range(3):
        compare(eng, desc, events, data, displaced(desc, 70 + j), TOL[mode], f"tiny {formula} {seed} {j}", gtol=GRAD_TOL[mode], gmax=GRAD_MAX_TOL[mode])


@pytest.mark.parametrize("mode", ["m64", "m32"])
def test_config1_full_size(mode):
    say("config1", mode)
    desc, events = synth.model_and_events(1)
    data = oracle_data(desc, events, synth.data_seed(1))
    eng = make_engine(desc, events, data, mode)
    assert eng.dropped(0) == OF.dropped_events(Model(desc), events)[0]
    compare(eng, desc, events, data, synth.start_vector(desc), TOL[mode], "c1 start", gtol=GRAD_TOL[mode], gmax=GRAD_MAX_TOL[mode])
    for j in range(3):
        compare(eng, desc, events, data, displaced(desc, 100 + j), TOL[mode], f"c1 displaced {j}", gtol=GRAD_TOL[mode], gmax=GRAD_MAX_TOL[mode])


@pytest.mark.parametrize("mode,deterministic", [("m64", 0), ("m32", 0), ("m64", 1)])
def test_config2_full_size(mode, deterministic):
    say("config2", mode, deterministic)
    desc, events = synth.model_and_events(2)
    data = oracle_data(desc, events, synth.data_seed(2))
    eng = make_engine(desc, events, data, mode, deterministic=deterministic)
    compare(eng, desc, events, data, synth.start_vector(desc), TOL[mode], "c2 start", gtol=GRAD_TOL[mode], gmax=GRAD_MAX_TOL[mode])
    compare(eng, desc, events, data, displaced(desc, 200), TOL[mode], "c2 displaced", gtol=GRAD_TOL[mode], gmax=GRAD_MAX_TOL[mode])


@pytest.mark.parametrize("mode", ["m64", "m32"])
def test_config3_full_size(mode):
    say("config3", mode)
    desc, events = synth.model_and_events(3)
    m = Model(desc)
    mus, _ = LK.expected(m, events, synth.start_vector(desc))
    data = [mu.copy() for mu in mus]  # Asimov, as in the medium-baseline study
    eng = make_engine(desc, events, data, mode)
    compare(eng, desc, events, data, displaced(desc, 300), TOL[mode], "c3 displaced", gtol=GRAD_TOL[mode], gmax=GRAD_MAX_TOL[mode])


@pytest.mark.parametrize("mode,dm2_41", [(m, v) for m in ("m64", "m32") for v in (0.0, 5.0, 50.0, 300.0)]
                         + [("m64", 1000.0)])
def test_sterile_full_size(mode, dm2_41):
    # 3+1 survival probability (sterile searches): near and far detector, two
    # reactors each; sterile mixing switched on at dm2_41 from 0 (no sterile
    # phase) to 1 eV^2 (up to 250 revolutions per event at the far detector).
    # M32 holds u = L/E in FP32, whose rounding alone moves a phase of p
    # revolutions by up to p 2^-25: at 1 eV^2 the dm2_41 derivative (a sum of
    # fast-alternating terms) is then off by about 1e-4 of its scale, so the
    # FP32 mode is checked up to 0.3 eV^2 and 1 eV^2 in FP64 only
    say("sterile", mode, dm2_41)
    desc, events = synth.model_and_events("sterile")
    data = oracle_data(desc, events, synth.data_seed(7))
    eng = make_engine(desc, events, data, mode)
    th = displaced(desc, 400)
    th[synth.param_index(desc, "osc.sin2_2t14")] = 0.04
    th[synth.param_index(desc, "osc.dm2_41")] = dm2_41
    compare(eng, desc, events, data, th, TOL[mode], f"sterile dm2_41={dm2_41}", gtol=GRAD_TOL[mode], gmax=GRAD_MAX_TOL[mode])


@pytest.mark.parametrize("mode", ["m64", "m32"])
def test_work_item_chunking_does_not_change_results(mode):
    # work items of 1, 2, 8 and up to 256 steps of 256 events: the fold's
    # pipelined loop at fewer steps than it loads ahead, at a multiple of its
    # unroll and at many iterations
    say("chunking", mode)
    desc = synth.tiny_model(21, formula="3nu", n_datasets=2, n_sources=3)
    events = synth.tiny_events(desc, 40000, 5)
    data = oracle_data(desc, events, 6)
    th = displaced(desc, 7)
    ref = None
    for chunk in (256, 512, 2048, 65536):
        eng = make_engine(desc, events, data, mode, chunk=chunk)
        f, g, _ = eng.eval_nll_grad(th)
        if mode == "m32":  # per-lane FP32 sums group the events differently per chunk size
            compare(eng, desc, events, data, th, TOL[mode], f"chunk {chunk}", gtol=GRAD_TOL[mode], gmax=GRAD_MAX_TOL[mode])
        elif ref is None:
            ref = (f, g)
            compare(eng, desc, events, data, th, 1e-9, "chunk")
        else:
            assert abs(f - ref[0]) <= 1e-12 * max(1, abs(f))
            assert np.max(np.abs(g - ref[1])) <= 1e-12 * max(1, np.max(np.abs(g)))


@pytest.mark.parametrize("mode", ["m64", "m32"])
def test_launch_options_do_not_change_results(mode):
    # every fold workgroup size (64, 128, 256 threads: blocks smaller than the
    # FP64 folds' sin/cos table fill the rest of it in a second pass) and
    # every bin-stage workgroup size the autotuner may choose, on every form.
    # Work items do not depend on these options, so the fold's sums are the
    # same; only the bin stages' block sums change order: every option agrees
    # with the default one to 1e-12, and the default one with the oracle (M64:
    # the 1e-9 bar throughout; M32: the per-component gradient bar; its
    # whole-vector bar is checked on the other workloads)
    say("launch options", mode)
    tol, gtol = TOL[mode], GRAD_TOL[mode]
    for formula in ("eq1", "3nu", "4nu", "3nu_matter"):
        desc = synth.tiny_model(31, formula=formula, n_datasets=2, n_sources=2)
        events = synth.tiny_events(desc, 20000, 8)
        data = oracle_data(desc, events, 9)
        th = displaced(desc, 10)
        m = Model(desc)
        mus_o, _ = LK.expected(m, events, th)
        f_o, g_o, F = LK.nll_grad(m, events, data, th, fisher=True)
        ref = None
        for fb in (256, 64, 128):
            for tt in (512, 256, 1024):
                what = f"{formula} fold_block {fb} tail_threads {tt}"
                eng = make_engine(desc, events, data, mode)
                eng.set_option("fold_block", fb)
                eng.set_option("tail_threads", tt)
                mus_g, code = eng.expected(th)
                assert code == nf.NF_OK, what
                f_g, g_g, code = eng.eval_nll_grad(th)
                assert code == nf.NF_OK, what
                eng.close()
                if ref is None:
                    ref = (mus_g, f_g, g_g)
                    for mo, mg in zip(mus_o, mus_g):
                        assert np.max(np.abs(mg - mo) / np.maximum(np.abs(mo), 1e-300)) <= tol, what
                    assert abs(f_g - f_o) <= tol * max(1.0, abs(f_o)), (what, f_g, f_o)
                    if mode == "m64":
                        assert np.max(np.abs(g_g - g_o)) <= tol * max(1.0, np.max(np.abs(g_o))), what
                    gradcheck.check(g_g, g_o, F, gtol, what, m.names)
                    continue
                for mr, mg in zip(ref[0], mus_g):
                    assert np.max(np.abs(mg - mr) / np.maximum(np.abs(mr), 1e-300)) <= 1e-12, what
                assert abs(f_g - ref[1]) <= 1e-12 * max(1.0, abs(ref[1])), what
                assert np.max(np.abs(g_g - ref[2])) <= 1e-12 * max(1.0, np.max(np.abs(ref[2]))), what


def test_repeated_evaluations_are_bitwise_identical():
    say("determinism")
    desc, events = synth.model_and_events(1)
    data = oracle_data(desc, events, 3)
    eng = make_engine(desc, events, data, deterministic=1)
    th = displaced(desc, 8)
    f0, g0, _ = eng.eval_nll_grad(th)
    for _ in range(5):
        f, g, _ = eng.eval_nll_grad(th)
        assert f == f0 and np.array_equal(g, g0)


def test_gradient_matches_central_differences_on_device():
    say("central differences")
    desc, events = synth.model_and_events(1)
    data = oracle_data(desc, events, 4)
    eng = make_engine(desc, events, data)
    th = displaced(desc, 9)
    f, g, _ = eng.eval_nll_grad(th)
    h = 1e-6
    for j in range(len(th)):
        e = np.zeros_like(th); e[j] = h
        fp, _ = eng.eval_nll(th + e)
        fm, _ = eng.eval_nll(th - e)
        fd = (fp - fm) / (2 * h)
        assert abs(fd - g[j]) <= 1e-5 * max(1.0, np.max(np.abs(g))), (j, fd, g[j])


def test_edge_cases_empty_single_bin_out_of_range_defaults():
    say("edge cases")
    desc = synth.tiny_model(31, formula="eq1", n_datasets=3, n_sources=2)
    ev = synth.tiny_events(desc, 3000, 9)
    # dataset 0: no events at all (background-only expectation)
    ev[0] = {k: v[:0] for k, v in ev[0].items()}
    # dataset 1: every event in one fine bin, a few exactly on edges and out of range
    f = desc["datasets"][1]["fine"]
    n1 = len(ev[1]["e_reco"])
    er = np.full(n1, f["y0"] + 3.5 * f["width"])
    er[:5] = f["y0"] + 3 * f["width"]              # on an edge: upper bin
    er[5:9] = f["y0"] + f["n"] * f["width"]        # top edge: dropped
    er[9:12] = f["y0"] - 1e-9                      # below: dropped
    ev[1]["e_reco"] = er
    # dataset 2: default source (all 0) and unit weights
    ev[2]["source"] = np.zeros_like(ev[2]["source"])
    ev[2]["weight"] = np.ones_like(ev[2]["weight"])
    data = oracle_data(desc, ev, 10)
    eng = nf.Engine(desc, "m64")
    eng.set_events(0, ev[0]["e_true"], ev[0]["e_reco"], ev[0]["source"], ev[0]["weight"])
    eng.set_events(1, ev[1]["e_true"], ev[1]["e_reco"], ev[1]["source"], ev[1]["weight"])
    eng.set_events(2, ev[2]["e_true"], ev[2]["e_reco"], None, None)
    for d in range(3):
        eng.set_data(d, data[d])
    assert eng.dropped(1) == 7
    compare(eng, desc, ev, data, displaced(desc, 11), 1e-9, "edge cases")


def test_error_paths():
    say("error paths")
    desc = synth.tiny_model(41, formula="eq1", n_datasets=1)
    ev = synth.tiny_events(desc, 2000, 3)
    eng = nf.Engine(desc, "m64")
    th = synth.start_vector(desc)
    with pytest.raises(nf.NufoldError) as e:
        eng.eval_nll(th)
    assert e.value.code == nf.NF_ESTATE
    eng.set_events(0, ev[0]["e_true"], ev[0]["e_reco"], ev[0]["source"], ev[0]["weight"])
    with pytest.raises(nf.NufoldError) as e:
        eng.eval_nll(th)
    assert e.value.code == nf.NF_ESTATE  # data missing
    data = oracle_data(desc, ev, 4)
    eng.set_data(0, data[0])
    bad = th.copy(); bad[0] = np.nan
    with pytest.raises(nf.NufoldError) as e:
        eng.eval_nll(bad)
    assert e.value.code == nf.NF_EINVAL
    with pytest.raises(nf.NufoldError) as e:
        eng.set_data(0, data[0][:-1])
    assert e.value.code == nf.NF_EINVAL
    # mu <= 0 -> domain warning, NLL = +inf, gradient 0
    neg = th.copy()
    neg[eng.param_index("ds0.norm")] = -1.0
    neg[eng.param_index("ds0.bkg.rate")] = -1.0
    f, g, code = eng.eval_nll_grad(neg)
    assert code == nf.NF_WDOMAIN and f == np.inf and np.all(g == 0)
    # energy map not monotone on the fine range -> domain warning
    bad_c = th.copy()
    bad_c[eng.param_index("ds0.c1")] = -1.5
    f, code = eng.eval_nll(bad_c)
    assert code == nf.NF_WDOMAIN and f == np.inf
    # and the engine keeps working afterwards
    f, g, code = eng.eval_nll_grad(th)
    assert code == nf.NF_OK and np.isfinite(f)


def test_device_pointer_entry_point_matches_host_path():
    say("device entry point")
    import torch
    desc, events = synth.model_and_events(1)
    data = oracle_data(desc, events, 5)
    eng = nf.Engine(desc, "m64", stream=torch.cuda.current_stream().cuda_stream)
    for d, ev in enumerate(events):
        eng.set_events(d, ev["e_true"], ev["e_reco"], ev["source"], ev["weight"])
        eng.set_data(d, torch.tensor(data[d], dtype=torch.float64, device="cuda"))
    th = displaced(desc, 12)
    theta_t = torch.tensor(th, dtype=torch.float64, device="cuda")
    out_t = torch.zeros(1 + len(th), dtype=torch.float64, device="cuda")
    st = torch.zeros(1, dtype=torch.int32, device="cuda")
    eng.eval_device(theta_t.data_ptr(), out_t.data_ptr(), st.data_ptr(), True)
    torch.cuda.synchronize()
    f, g, _ = eng.eval_nll_grad(th)
    o = out_t.cpu().numpy()
    # same kernels on the same inputs (fine-bin rows by atomic adds: last bits may move)
    assert abs(o[0] - f) <= 1e-13 * max(1.0, abs(f)) and int(st.item()) == 0
    assert np.max(np.abs(o[1:] - g)) <= 1e-12 * max(1.0, np.max(np.abs(g)))


@pytest.mark.parametrize("mode", ["m64", "m32"])
def test_deterministic_option_reproduces_bit_for_bit(mode):
    """With deterministic = 1 every fine bin is summed in source order by one
    wavefront: repeated evaluations (with other evaluations between them)
    agree bit for bit, and agree with the atomic accumulation to rounding."""
    say("deterministic option", mode)
    desc, events = synth.model_and_events(3, 400_000)
    m = Model(desc)
    data = [mu.copy() for mu in LK.expected(m, events, synth.start_vector(desc))[0]]
    eng = make_engine(desc, events, data, mode, deterministic=1)
    th = [displaced(desc, 500 + j) for j in range(3)]
    first = [eng.eval_nll_grad(t)[:2] for t in th]
    for rep in range(3):
        for t, (f0, g0) in zip(th, first):
            f, g, _ = eng.eval_nll_grad(t)
            assert f == f0 and np.array_equal(g, g0), rep
    assert eng.get_option("deterministic") == 1
    eng.set_option("deterministic", 0)
    assert eng.get_option("deterministic") == 0
    for t, (f0, g0) in zip(th, first):
        f, g, _ = eng.eval_nll_grad(t)
        assert abs(f - f0) <= 1e-12 * max(1.0, abs(f0))
        assert np.max(np.abs(g - g0)) <= 1e-11 * max(1.0, np.max(np.abs(g0)))


@pytest.mark.parametrize("mode", ["m64", "m32"])
def test_graph_of_device_evaluations_matches_single_evaluations(mode):
    """nf_eval_device_many: captured once, replayed on new parameter values,
    captured again for another count; every row equals the host path."""
    say("graph of device evaluations", mode)
    import torch
    desc, events = synth.model_and_events(1)
    data = oracle_data(desc, events, 6)
    stream = torch.cuda.Stream()
    eng = nf.Engine(desc, mode, stream=stream.cuda_stream)
    for d, ev in enumerate(events):
        eng.set_events(d, ev["e_true"], ev["e_reco"], ev["source"], ev["weight"])
        eng.set_data(d, data[d])
    P = eng.P
    out_t = torch.zeros((5, 1 + P), dtype=torch.float64, device="cuda")
    st = torch.full((5,), -7, dtype=torch.int32, device="cuda")
    for rnd, (n, seed0) in enumerate(((5, 20), (5, 40), (3, 60))):
        ths = np.stack([displaced(desc, seed0 + i) for i in range(5)])
        theta_t = torch.tensor(ths, dtype=torch.float64, device="cuda") if rnd == 0 else theta_t
        if rnd > 0:
            theta_t.copy_(torch.tensor(ths, dtype=torch.float64))  # same buffer: the graph reads it anew
        torch.cuda.synchronize()
        eng.eval_device_many(n, theta_t.data_ptr(), out_t.data_ptr(), st.data_ptr(), True)
        stream.synchronize()
        o = out_t.cpu().numpy()
        for i in range(n):
            f, g, code = eng.eval_nll_grad(ths[i])
            assert code == nf.NF_OK
            # same kernels on the same inputs; LDS atomic order may move the last bits
            assert abs(o[i, 0] - f) <= 1e-13 * max(1.0, abs(f)), (rnd, i)
            assert np.max(np.abs(o[i, 1:] - g)) <= 1e-12 * max(1.0, np.max(np.abs(g))), (rnd, i)
        assert np.all(st.cpu().numpy()[:n] == 0)
    with pytest.raises(nf.NufoldError) as e:
        eng.eval_device_many(0, theta_t.data_ptr(), out_t.data_ptr())
    assert e.value.code == nf.NF_EINVAL


@pytest.mark.parametrize("mode", ["m64", "m32"])
def test_stage_cache_reuses_the_fold_only_while_its_parameters_repeat(mode):
    """Option stage_cache: host evaluations that change only bin-stage
    parameters reuse the last fold; a change of an oscillation parameter or a
    source norm folds again; device evaluations in between clear the kept
    rows. Every result equals a full evaluation bit for bit (deterministic
    fine-bin sums on both engines) and the oracle at a reused fold."""
    say("stage cache", mode)
    import torch
    desc, events = synth.model_and_events(1)
    m = Model(desc)
    data = oracle_data(desc, events, 13)
    ref = make_engine(desc, events, data, mode, deterministic=1)
    eng = make_engine(desc, events, data, mode, deterministic=1)
    eng.set_option("stage_cache", 1)
    assert eng.get_option("stage_cache") == 1
    th = displaced(desc, 14)
    steps = [(None, 0.0), ("escale.c1", 0.003), ("bkg.flat.rate", 0.02), ("flux[2]", 0.01),
             ("osc.sin2_2t13", 0.004), ("escale.c0", -0.01), ("norm", 0.01), ("norm", 0.0),
             ("osc.dm2_ee", 0.03), ("flux[0]", -0.02)]
    names = set(m.names)
    seq = []
    for name, dv in steps:
        t = (seq[-1] if seq else th).copy()
        if name is not None:
            assert name in names, name
            t[m.index[name]] += dv
        seq.append(t)
    for i, t in enumerate(seq):
        f, g, code = eng.eval_nll_grad(t)
        f0, g0, _ = ref.eval_nll_grad(t)
        assert code == nf.NF_OK
        assert f == f0 and np.array_equal(g, g0), i
        mu, _ = eng.expected(t)
        mu0, _ = ref.expected(t)
        assert all(np.array_equal(a, b) for a, b in zip(mu, mu0)), i
        if i == 3:  # a device evaluation between two cached ones clears the rows
            tt = torch.tensor(seq[0], dtype=torch.float64, device="cuda")
            out = torch.zeros(1 + eng.P, dtype=torch.float64, device="cuda")
            eng.eval_device(tt.data_ptr(), out.data_ptr())
            torch.cuda.synchronize()
            fd, gd, _ = ref.eval_nll_grad(seq[0])
            assert out[0].item() == fd
    # the oracle at a point that reused the fold
    compare(eng, desc, events, data, seq[-1], TOL[mode], "stage cache", gtol=GRAD_TOL[mode], gmax=GRAD_MAX_TOL[mode])
    eng.set_option("stage_cache", 0)
    f, g, _ = eng.eval_nll_grad(seq[2])
    f0, g0, _ = ref.eval_nll_grad(seq[2])
    assert f == f0 and np.array_equal(g, g0)
