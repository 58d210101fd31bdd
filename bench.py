"""Benchmark: fold + NLL + adjoint-gradient evaluations per second on the
1e7-event medium-baseline (JUNO-like) workload, on one MI355X.

One step = one full model evaluation at a new parameter vector: the event fold
(HIP), the bin stages, the Poisson NLL with priors and the adjoint gradient
(HIP), for all 1e7 events, 10 reactor cores, 400 analysis bins, 120 parameters.
Inputs (events, data, 64 parameter vectors whose oscillation parameters all
differ) are resident in device memory before the timed region.

Prints one JSON line. Per-kernel durations come from HIP start/stop events
carried by the fold and bin-stage dispatches on the engine's stream; the
roofline entry prices the fold (the dominant kernel) against MI355X's 8 TB/s
HBM peak with the algorithmic bytes it must read (u = L/E and w per event:
12 B in FP64 mode, 8 B in FP32 mode), from evaluations cycled over engine
replicas whose event sets together exceed the 256 MB Infinity Cache (the
single-engine, cache-resident figure is reported beside it). Both precision
modes are measured. The CPU baseline is the FP64 oracle (NLL plus
complex-step gradient) timed on the host, on one core and on every core.
"""
import argparse
import hashlib
import json
import os
import sys
import tempfile
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
COLD_STEPS = 240  # evaluations of the replica-rotated loop (at least)
PROFILE_TRAFFIC = os.path.join(ROOT, "profiles", "fold_juno_like_1e7_traffic.json")


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def fold_source_hash():
    h = hashlib.sha256()
    for f in ("fold.hip", "fastmath.hpp", "sincos_coeffs.hpp", "osc.hpp", "kernels.hpp", "plan.hpp", "matter.hpp",
              "stages.hpp"):
        with open(os.path.join(ROOT, "paper_2502_15253_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def measured_traffic(mode, n_launch_bytes):
    """HBM bytes per fold launch from the committed rocprofv3 counter summary,
    or None when it was taken on a different fold source."""
    try:
        rec = json.load(open(PROFILE_TRAFFIC))
    except (OSError, ValueError):
        return None
    ent = rec.get(mode)
    if not ent or rec.get("fold_source_sha") != fold_source_hash():
        return None
    return ent.get("bytes_per_launch")


def cpu_baseline(desc, events, theta):
    from oracle.model import Model
    from oracle import likelihood as LK
    m = Model(desc)
    mus, _ = LK.expected(m, events, theta)
    data = [mu.copy() for mu in mus]
    from threadpoolctl import threadpool_limits
    n = 0
    with threadpool_limits(limits=1):  # numpy's library threads held to one
        t0 = time.perf_counter()
        while True:  # whole evaluations until about ten seconds of work
            LK.nll_grad(m, events, data, theta)
            n += 1
            if time.perf_counter() - t0 >= 10.0:
                break
        dt = time.perf_counter() - t0
    model = ""
    try:
        with open("/proc/cpuinfo") as f:
            model = next((ln.split(":", 1)[1].strip() for ln in f if ln.startswith("model name")), "")
    except OSError:
        pass
    return dict(value=n / dt, unit="evals/s", cores=1, kind="oracle",
                sample=f"{n} full evaluation(s) (NLL + complex-step gradient over {m.P} parameters) "
                       f"of the {sum(len(e['weight']) for e in events):.0e}-event workload, "
                       f"numpy FP64, single thread, {dt:.1f} s",
                host=dict(cpu=model, logical_cpus=os.cpu_count(),
                          usable_cpus=len(os.sched_getaffinity(0)) if hasattr(os, "sched_getaffinity") else None))


def _oracle_worker(args):
    """One worker of the all-cores CPU leg: builds the same workload from its
    seeds (spawned process, numpy only) and times whole oracle evaluations
    for about `seconds` seconds of work. Returns (evaluations, seconds)."""
    n_events, theta_seed, k, seconds = args
    from threadpoolctl import threadpool_limits
    from paper_2502_15253_amd import synth
    from oracle.model import Model
    from oracle import likelihood as LK
    desc, events = synth.model_and_events(3, n_events)
    m = Model(desc)
    thetas = synth.osc_theta_list(desc, 64, seed=theta_seed)
    data = [mu.copy() for mu in LK.expected(m, events, synth.start_vector(desc))[0]]
    n = 0
    with threadpool_limits(limits=1):
        t0 = time.perf_counter()
        while True:
            LK.nll_grad(m, events, data, thetas[(k + n) % 64])
            n += 1
            if time.perf_counter() - t0 >= seconds:
                break
        dt = time.perf_counter() - t0
    return n, dt


def cpu_baseline_all_cores(n_events, seconds=15.0):
    """The oracle as it stands on every usable host core: one spawned process
    per core, each timing whole evaluations of the same workload (numpy FP64,
    one library thread each); the rate is the sum of the per-process rates."""
    import multiprocessing as mp
    ncpu = len(os.sched_getaffinity(0)) if hasattr(os, "sched_getaffinity") else os.cpu_count()
    ncpu = max(1, min(ncpu, 16))
    ctx = mp.get_context("spawn")  # fresh interpreters: no device state inherited
    t0 = time.perf_counter()
    with ctx.Pool(ncpu) as pool:
        res = pool.map(_oracle_worker, [(n_events, 5, k, seconds) for k in range(ncpu)])
    wall = time.perf_counter() - t0
    rate = sum(n / dt for n, dt in res)
    return dict(value=rate, unit="evals/s", cores=ncpu, kind="oracle",
                sample=f"{sum(n for n, _ in res)} full evaluations over {ncpu} processes (one per core), "
                       f"about {seconds:.0f} s of work each, {wall:.0f} s wall including each process "
                       f"building the workload")


COPY_BYTES = 512 << 20


def mlp_profile(torch, batches=(1024, 4096), steps=100, warm=5):
    """Training steps of the surrogate network of the medium-baseline model
    (20 inputs, four hidden layers of 512, 400 outputs; random data) at each
    batch size, for a kernel trace: prints each step's products (pass, M, N,
    K, output tile, grid) and the step rate, so the trace's dispatches can be
    read per product shape."""
    import math
    from paper_2502_15253_amd import nufold as nf
    n_in, width, depth, n_out = 20, 512, 4, 400
    stream = torch.cuda.Stream()
    net = nf.Mlp(n_in, width, depth, n_out, max(batches), stream=stream.cuda_stream)
    rng = np.random.default_rng(0)
    parts = []
    for a, b in net.layer_shapes():
        parts.append(rng.standard_normal(a * b) * math.sqrt(2.0 / a))
        parts.append(np.zeros(b))
    net.set_params(np.concatenate(parts).astype(np.float32))
    dims = [n_in] + [width] * depth + [n_out]
    kin = (n_in + 7) // 8 * 8

    def grid(M, N, K, splits=1):
        kslice = max(32, ((K + splits - 1) // splits + 31) // 32 * 32)
        z = max(1, (K + kslice - 1) // kslice)
        t = 128 if ((N + 127) // 128) * ((M + 127) // 128) * z >= 512 else 64
        return t, ((N + t - 1) // t, (M + t - 1) // t, z)

    out = {"network": f"{n_in}-{'-'.join([str(width)] * depth)}-{n_out}", "params": net.nparam, "batches": []}
    for B in batches:
        prods = []
        for l in range(depth + 1):
            M, N, K = B, dims[l + 1], kin if l == 0 else dims[l]
            prods.append(("forward", l, M, N, K, *grid(M, N, K)))
        for l in range(depth, -1, -1):
            # the training step takes each layer's input gradient before its
            # weight gradient (the weights are updated right after the latter)
            if l > 0:
                M2, N2, K2 = B, dims[l], dims[l + 1]
                prods.append(("input grad", l, M2, N2, K2, *grid(M2, N2, K2)))
            M, N, K = dims[l], dims[l + 1], B
            tiles = ((M + 127) // 128) * ((N + 127) // 128)
            sp = min(32, max(1, min(512 // tiles, B // 256)))
            prods.append(("weight grad", l, M, N, K, *grid(M, N, K, sp)))
        x = torch.randn(B, n_in, device="cuda", dtype=torch.float32)
        t = torch.randn(B, n_out, device="cuda", dtype=torch.float32)
        torch.cuda.synchronize()
        for _ in range(warm):
            net.train_step(x, t, 1e-5, want_loss=False)
        stream.synchronize()
        t0 = time.perf_counter()
        for _ in range(steps):
            net.train_step(x, t, 1e-5, want_loss=False)
        stream.synchronize()
        dt = (time.perf_counter() - t0) / steps
        flop = sum(2.0 * M * N * K for (_, _, M, N, K, _, _) in prods)
        out["batches"].append({"batch": B, "steps": steps, "us_per_step": dt * 1e6,
                               "gemm_gflop_per_step": flop / 1e9, "tflops": flop / dt / 1e12,
                               "products": [dict(pass_=p_, layer=l, M=M, N=N, K=K, tile=tt, grid=list(g))
                                            for (p_, l, M, N, K, tt, g) in prods]})
        log(f"batch {B}: {dt * 1e6:.1f} us per step, {flop / dt / 1e12:.1f} TFLOP/s over its products")
    net.close()
    print(json.dumps(out))


def copy_probe(torch, reps=8):
    """Plain device-to-device copies of COPY_BYTES each: the reference that
    scales the memory counters of a profiled run to bytes."""
    src = torch.ones(COPY_BYTES // 4, dtype=torch.float32, device="cuda")
    dst = torch.empty_like(src)
    for _ in range(reps):
        dst.copy_(src)
    torch.cuda.synchronize()
    log(f"copy probe: {reps} copies of {COPY_BYTES} B")


def event_timed(torch, eng, run, steps, passes=3, warm=20):
    """Fold and bin-stage durations from the HIP start/stop events carried by
    every dispatch (option "timing"): a short warm-up of event-timed launches,
    then `passes` passes of `steps` evaluations; the pass with the median mean
    fold duration is reported, as (count, fold ms, bin-stage ms, seconds)."""
    eng.set_option("timing", 1)
    for k in range(warm):
        run(k)
    torch.cuda.synchronize()
    eng.timing(reset=True)
    res = []
    for _ in range(passes):
        e0 = time.perf_counter()
        for k in range(steps):
            run(k)
        torch.cuda.synchronize()
        e1 = time.perf_counter()
        cnt, fold_ms, tail_ms = eng.timing(reset=True)
        res.append((cnt, fold_ms, tail_ms, e1 - e0))
    eng.set_option("timing", 0)
    res.sort(key=lambda r: r[1] / max(1, r[0]))
    return res[len(res) // 2]


def pseudo_data(eng, desc, n, seed0=3000):
    """n Poisson pseudo-experiments around the expectations at the start point."""
    from paper_2502_15253_amd import synth
    mus, _ = eng.expected(synth.start_vector(desc))
    return np.array([np.concatenate(synth.poisson_data(mus, seed0 + j)) for j in range(n)])


def engine_for(nf, synth, config, stream, n_events=None):
    desc, events = synth.model_and_events(config, n_events)
    eng = nf.Engine(desc, "m64", stream=stream.cuda_stream)
    for d, ev in enumerate(events):
        eng.set_events(d, ev["e_true"], ev["e_reco"], ev["source"], ev["weight"])
    return desc, events, eng


def plain_fit(eng, desc, start, h=1e-6):
    """The paper's method on the GPU: one fit at a time, BFGS on the host with
    central finite-difference gradients, every function value one GPU
    evaluation (fold + bin stages + NLL) with stage caching (the fold is
    re-run only when an oscillation parameter or a source norm changed, as the
    paper's caches recompute a stage only when its parameters change; option
    stage_cache of the library). Like Minuit's internal parameters,
    the minimiser works in scaled variables z = (theta - start) / s, with s the
    prior width (else 5% of the start value), so that its initial metric is
    sensible; fixed parameters stay at their start. Returns (NLL, evaluations)."""
    from scipy.optimize import minimize
    free = np.array([not p["fixed"] for p in desc["params"]])
    scale = np.array([p["prior"][1] if p["prior"] else 0.05 * max(abs(p["start"]), 0.02)
                      for p in desc["params"]])
    idx = np.where(free)[0]
    n = [0]

    def theta(z):
        th = np.array(start, dtype=np.float64)
        th[idx] += scale[idx] * z
        return th

    def f(z):
        n[0] += 1
        return eng.eval_nll(theta(z))[0]

    def g(z):
        out = np.zeros_like(z)
        for j in range(len(z)):
            e = np.zeros_like(z)
            e[j] = h
            out[j] = (f(z + e) - f(z - e)) / (2 * h)
        return out

    eng.set_option("stage_cache", 1)
    try:
        r = minimize(f, np.zeros(len(idx)), jac=g, method="BFGS", options=dict(gtol=1e-6, maxiter=5000))
    finally:
        eng.set_option("stage_cache", 0)
    return r.fun, n[0]


def fits_section(nf, synth, torch, stream, n_plain, surrogate_samples, n_plain_c2=3, n_plain_c3=16):
    """Pseudo-experiment fits/s: batched adjoint fits (2048 + 2048 pseudo-experiments
    of the 1050 m single-detector and three-detector models, and a 200 x 200
    profile scan) against the plain per-fit GPU path; and the learned warm start
    on medium-baseline pseudo-experiments."""
    out = {}
    t_all = 0.0
    n_all = 0
    from paper_2502_15253_amd import autotune as AT
    tune_cache = os.path.join(tempfile.gettempdir(), "nufold_bench_autotune.json")
    for config, label in ((1, "single_detector"), (2, "three_detector")):
        desc, events, eng = engine_for(nf, synth, config, stream)
        data = pseudo_data(eng, desc, 2048)
        eng.set_data_batch(data)
        start = np.tile(synth.start_vector(desc), (2048, 1))
        # batched launch choices (fold tile, bin-stage threads) from the
        # library's autotuner, before the clock; the work-item size keeps its
        # default, which suits batches (the single-evaluation choice favours
        # small items)
        nb0 = np.cumsum([0] + [len(ds["edges"]) - 1 for ds in desc["datasets"]])
        for d in range(len(desc["datasets"])):
            eng.set_data(d, data[0][nb0[d]:nb0[d + 1]])
        tuned = AT.tune(eng, desc, [len(ev["weight"]) for ev in events], start[0], cache_path=tune_cache,
                        evals=0, batch=2048, force=True)
        log(f"autotuned {label}: {json.dumps(tuned)}")
        eng.fit_batch(start[:8], edm_tol=1e-7, max_iter=3000)  # graph capture and buffers
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        r = eng.fit_batch(start, edm_tol=1e-7, max_iter=3000)
        dt = time.perf_counter() - t0
        t_all += dt
        n_all += 2048
        ent = dict(fits=2048, seconds=dt, fits_per_s=2048 / dt, params=len(start[0]),
                   converged=int(np.sum(r["status"] == 0)), mean_iters=float(r["iters"].mean()),
                   launch_options=tuned["options"])
        log(f"batched {label}: {json.dumps(ent)}")
        if config == 1:
            # the plain per-fit GPU path on the first n_plain pseudo-experiments
            nb = np.cumsum([0] + [len(ds["edges"]) - 1 for ds in desc["datasets"]])
            t0 = time.perf_counter()
            dmax, nev = 0.0, 0
            for j in range(n_plain):
                for d in range(len(desc["datasets"])):
                    eng.set_data(d, data[j][nb[d]:nb[d + 1]])
                fmin, ne = plain_fit(eng, desc, start[j])
                nev += ne
                dmax = max(dmax, 2.0 * abs(fmin - r["nll"][j]))
            tp = time.perf_counter() - t0
            ent["plain"] = dict(fits=n_plain, seconds=tp, fits_per_s=n_plain / tp, evals_per_fit=nev / n_plain,
                                max_delta_chi2_vs_batched=dmax)
            ent["batched_over_plain"] = ent["fits_per_s"] / ent["plain"]["fits_per_s"]
            log(f"plain single_detector: {json.dumps(ent['plain'])}")
            # 200 x 200 profile scan of (sin2_2t13, dm2_ee) on one Poisson data set
            scan_data = np.concatenate(synth.poisson_data(eng.expected(synth.start_vector(desc))[0],
                                                          synth.data_seed(1)))
            eng.set_data_batch(scan_data[None, :])
            i13, iee = synth.param_index(desc, "osc.sin2_2t13"), synth.param_index(desc, "osc.dm2_ee")
            fixed = np.array([p["fixed"] for p in desc["params"]], dtype=bool)
            fixed[[i13, iee]] = True
            s13, dee = np.linspace(0.0, 0.2, 200), np.linspace(1.5, 3.5, 200)
            grid = np.array([(a, b) for a in s13 for b in dee])
            nll = np.empty(len(grid))
            t0 = time.perf_counter()
            conv = 0
            for o in range(0, len(grid), 4096):
                g = grid[o:o + 4096]
                st = np.tile(synth.start_vector(desc), (len(g), 1))
                st[:, i13], st[:, iee] = g[:, 0], g[:, 1]
                rs = eng.fit_batch(st, fixed=fixed, data_idx=np.zeros(len(g), np.int32), edm_tol=1e-7,
                                   max_iter=3000)
                nll[o:o + len(g)] = rs["nll"]
                conv += int(np.sum(rs["status"] == 0))
            ts = time.perf_counter() - t0
            t_all += ts
            n_all += len(grid)
            k = int(np.argmin(nll))
            out["scan_200x200"] = dict(fits=len(grid), seconds=ts, fits_per_s=len(grid) / ts, converged=conv,
                                       best=[float(grid[k, 0]), float(grid[k, 1])],
                                       delta_chi2_max=float(2 * (nll.max() - nll.min())))
            log(f"scan: {json.dumps(out['scan_200x200'])}")
        if config == 2 and n_plain_c2 > 0:
            # agreement of the batched 302-parameter fits with the plain path on
            # the first pseudo-experiments (a different minimiser: host BFGS on
            # finite differences)
            nb = np.cumsum([0] + [len(ds["edges"]) - 1 for ds in desc["datasets"]])
            t0 = time.perf_counter()
            dmax, nev = 0.0, 0
            for j in range(n_plain_c2):
                for d in range(len(desc["datasets"])):
                    eng.set_data(d, data[j][nb[d]:nb[d + 1]])
                fmin, ne = plain_fit(eng, desc, start[j])
                nev += ne
                dmax = max(dmax, 2.0 * (fmin - r["nll"][j]))
            tp = time.perf_counter() - t0
            ent["plain"] = dict(fits=n_plain_c2, seconds=tp, fits_per_s=n_plain_c2 / tp,
                                evals_per_fit=nev / n_plain_c2, max_delta_chi2_plain_minus_batched=dmax)
            ent["batched_over_plain"] = ent["fits_per_s"] / ent["plain"]["fits_per_s"]
            log(f"plain three_detector: {json.dumps(ent['plain'])}")
        out[label] = ent
        eng.close()
    out["ensemble_fits_per_s"] = n_all / t_all
    if surrogate_samples > 0:
        out["warm_start"] = warm_start_section(nf, synth, torch, stream, surrogate_samples, n_plain=n_plain_c3)
        out["mixed_ensemble"] = mixed_ensemble_section(nf, synth, torch, stream)
    out["sterile_raster"] = sterile_raster_section(nf, synth, torch, stream)
    return out


def mixed_ensemble_section(nf, synth, torch, stream, n_train=200_000, B=2048):
    """The mixed ensemble: 2048 pseudo-experiments of the single-detector model
    and 2048 of the three-detector model (uneven bin and parameter counts)
    fitted in one launch sequence (nf_fit_batch_group), from the start point
    (cold) and from warm starts of a surrogate network per model, each
    trained on spectra of its own model's exact fold and attached to its
    engine (nf_set_surrogate; the fits take nf_fit_opts.warm_start). The same
    fits as two separate batched launch sequences give the sequential time."""
    from paper_2502_15253_amd import surrogate as SG
    members, sur, res = [], [], {}
    t_train = 0.0
    for config in (1, 2):
        desc, _, eng = engine_for(nf, synth, config, stream)
        data = pseudo_data(eng, desc, B, seed0=3000 + 5000 * config)
        eng.set_data_batch(data)
        start = np.tile(synth.start_vector(desc), (B, 1))
        space = SG.Space(desc)
        t0 = time.perf_counter()
        X, Y = SG.generate(eng, space, n_train // 100, 100, seed=21 + config)
        net = SG.Surrogate(space, Y.shape[1], stream=stream, max_batch=4096)
        net.train(X, Y, epochs=8, batch=1024, lr=1e-3)
        torch.cuda.synchronize()
        t_train += time.perf_counter() - t0
        # the short-baseline likelihoods have one basin in the free inputs: a
        # coarse start grid suffices
        net.attach(eng, grid=(4, 2), iters=100)
        members.append((eng, start, None, None))
        sur.append(net)
    nf.fit_batch_group([(e, s[:8], f, d) for e, s, f, d in members], edm_tol=1e-7, max_iter=3000)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    cold, code = nf.fit_batch_group(members, edm_tol=1e-7, max_iter=3000)
    tc = time.perf_counter() - t0
    t0 = time.perf_counter()
    warm, _ = nf.fit_batch_group(members, edm_tol=1e-7, max_iter=3000, warm_start=True)
    tw = time.perf_counter() - t0
    t0 = time.perf_counter()
    seq = [e.fit_batch(s, edm_tol=1e-7, max_iter=3000) for e, s, _, _ in members]
    ts = time.perf_counter() - t0
    n = sum(len(s) for _, s, _, _ in members)
    dchi2 = max(float(np.max(2.0 * np.abs(c["nll"] - q["nll"]))) for c, q in zip(cold, seq))
    dwarm = max(float(np.max(2.0 * (w["nll"] - c["nll"]))) for c, w in zip(cold, warm))
    res = dict(fits=n, models=["single_detector (12 params, 40 bins)", "three_detector (302 params, 3 x 40 bins)"],
               cold=dict(seconds=tc, fits_per_s=n / tc, converged=int(sum(np.sum(c["status"] == 0) for c in cold)),
                         mean_iters=[float(c["iters"].mean()) for c in cold]),
               warm=dict(seconds=tw, fits_per_s=n / tw, converged=int(sum(np.sum(w["status"] == 0) for w in warm)),
                         mean_iters=[float(w["iters"].mean()) for w in warm],
                         max_delta_chi2_warm_minus_cold=dwarm, surrogate_training_s=t_train,
                         training_spectra_per_model=n_train),
               sequential=dict(seconds=ts, fits_per_s=n / ts, max_delta_chi2_vs_group=dchi2))
    for e, *_ in members:
        e.close()
    log(f"mixed ensemble: {json.dumps(res)}")
    return res


def sterile_raster_section(nf, synth, torch, stream, n_pe=100):
    """3+1 raster scan (sterile searches): 8 sin^2(2 theta14) x 10 dm2_41
    values over 5e-4 to 0.5 eV^2, each with its own ensemble of Poisson
    pseudo-experiments fitted twice (tested point fixed, sin^2(2 theta14) free)."""
    from paper_2502_15253_amd.sterile import RasterScan
    desc, events, eng = engine_for(nf, synth, "sterile", stream)
    mus, _ = eng.expected(synth.start_vector(desc))
    row = np.concatenate(synth.poisson_data(mus, synth.data_seed(7)))
    rs = RasterScan(eng, desc)
    s_values = np.linspace(0.0, 0.2, 8)
    m_values = np.geomspace(0.5, 500.0, 10)
    rs.run(row, s_values[:2], m_values[:2], n_pe=4, seed=1)  # buffers and graphs
    torch.cuda.synchronize()
    r = rs.run(row, s_values, m_values, n_pe=n_pe, cl=0.9, seed=2)
    eng.close()
    res = dict(points=len(s_values) * len(m_values), pseudo_experiments_per_point=n_pe, fits=r["fits"],
               seconds=r["seconds"], fit_seconds=r["fit_seconds"], fits_per_s=r["fits"] / r["fit_seconds"],
               fit_results=r["results"], converged=r["converged"], excluded_points=int(r["excluded"].sum()),
               dm2_41_range_ev2=[float(m_values[0]) * 1e-3, float(m_values[-1]) * 1e-3])
    log(f"sterile raster: {json.dumps(res)}")
    return res


def matter_section(nf, synth, torch, stream, events, thetas, steps=200):
    """The medium-baseline workload with the exact three-flavour probability in
    matter of constant density (rho Y_e = 1.3 g/cm^3) on the same 1e7 events, M64:
    evaluations per second (graph replays of consecutive evaluations, as the
    headline) and the fold and bin-stage durations (HIP events on each
    dispatch). The matter fold evaluates the eigen-system per event in FP64,
    so it is bound by FP64 arithmetic, not by HBM."""
    desc = synth.config3_matter_model()
    eng = nf.Engine(desc, "m64", stream=stream.cuda_stream)
    for d, ev in enumerate(events):
        eng.set_events(d, ev["e_true"], ev["e_reco"], ev["source"], ev["weight"])
    n_in = sum(len(ev["weight"]) for ev in events) - sum(eng.dropped(d) for d in range(eng.D))
    start = synth.start_vector(desc)
    for d, mu in enumerate(eng.expected(start)[0]):
        eng.set_data(d, mu)
    th_dev = torch.tensor(thetas, dtype=torch.float64, device="cuda")
    out_dev = torch.zeros((len(thetas), 1 + eng.P), dtype=torch.float64, device="cuda")
    torch.cuda.synchronize()
    n_graph = max(d for d in range(1, 65) if steps % d == 0)
    eng.eval_device_many(n_graph, th_dev.data_ptr(), out_dev.data_ptr())
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps // n_graph):
        eng.eval_device_many(n_graph, th_dev.data_ptr(), out_dev.data_ptr())
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    cnt, fold_ms, tail_ms, _ = event_timed(
        torch, eng, lambda k: eng.eval_device(th_dev[k % 64].data_ptr(), out_dev[k % 64].data_ptr()), steps)
    assert cnt == steps and bool(torch.isfinite(out_dev).all())
    eng.close()
    fold_us = fold_ms / cnt * 1e3
    res = dict(model="medium baseline, exact 3 flavours in matter, rho Y_e = 1.3 g/cm^3", mode="m64",
               events_in_range=n_in, evals_per_s=steps / (t1 - t0), ms_per_step=(t1 - t0) * 1e3 / steps,
               fold_us=fold_us, tail_us=tail_ms / cnt * 1e3, events_per_s_fold=n_in / (fold_us * 1e-6))
    log(f"matter: {json.dumps(res)}")
    return res


def warm_start_section(nf, synth, torch, stream, n_samples, E=256, n_plain=16):
    """Medium-baseline pseudo-experiments at random points of the training box:
    exact batched fits from the box centre (cold) and from the surrogate's
    proposal (warm). A third fit from the generating point gives the reference
    minimum; success = final NLL within 5e-4 of the best of the three."""
    from paper_2502_15253_amd import surrogate as SG
    desc, _, eng = engine_for(nf, synth, 3, stream)
    space = SG.Space(desc)
    t0 = time.perf_counter()
    X, Y = SG.generate(eng, space, n_samples // 100, 100, seed=11)
    t_gen = time.perf_counter() - t0
    sur = SG.Surrogate(space, Y.shape[1], stream=stream, max_batch=4096)
    t0 = time.perf_counter()
    losses = sur.train(X, Y, epochs=12, batch=1024, lr=1e-3)
    torch.cuda.synchronize()
    t_train = time.perf_counter() - t0
    steps = 12 * (len(X) // 1024)
    Xv, Yv = SG.generate(eng, space, 200, 5, seed=12)
    err = sur.predict_log_mu(space.to_theta(Xv)) - Yv
    rng = np.random.default_rng(5)
    base = synth.start_vector(desc)
    truths = np.tile(base, (E, 1))
    for i, p in enumerate(desc["params"]):
        if p["prior"]:
            truths[:, i] = p["prior"][0] + p["prior"][1] * rng.standard_normal(E)
    i13, i31 = synth.param_index(desc, "osc.sin2_t13"), synth.param_index(desc, "osc.dm2_31")
    truths[:, i13] = rng.uniform(0.017, 0.028, E)
    truths[:, i31] = rng.uniform(2.33, 2.77, E)
    mu, _ = eng.expected_batch(truths)
    data = rng.poisson(mu).astype(np.float64)
    eng.set_data_batch(data)
    cold = np.tile(base, (E, 1))
    for i, p in enumerate(desc["params"]):
        if p["prior"]:
            cold[:, i] = p["prior"][0]
    cold[:, i13], cold[:, i31] = 0.0225, 2.55
    eng.fit_batch(cold[:4], edm_tol=1e-6, max_iter=2000)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    rc = eng.fit_batch(cold, edm_tol=1e-6, max_iter=2000)
    tc = time.perf_counter() - t0
    # warm starts inside the library's batched fit (nf_set_surrogate +
    # nf_fit_opts.warm_start): surrogate fits over the start grid, the exact
    # NLL judging each proposal against the cold start, then the exact fits;
    # the whole call is timed
    sur.attach(eng)
    t0 = time.perf_counter()
    rw = eng.fit_batch(cold, edm_tol=1e-6, max_iter=2000, warm_start=True)
    tw = time.perf_counter() - t0
    t0 = time.perf_counter()
    warm, _ = sur.warm_start(data.astype(np.float32), base=cold[0])
    tsur = time.perf_counter() - t0
    rt = eng.fit_batch(truths, edm_tol=1e-6, max_iter=2000)
    # the start each warm fit used (the proposal where its exact NLL was lower)
    n_c, _, _ = eng.eval_batch(cold, want_grad=False)
    n_w, _, _ = eng.eval_batch(warm, want_grad=False)
    chosen = np.where((n_w < n_c)[:, None], warm, cold)
    best = np.minimum(np.minimum(rc["nll"], rw["nll"]), rt["nll"])
    # the plain per-fit GPU path on the first pseudo-experiments, from the same
    # surrogate starts (so both find the same minimum): host BFGS with central
    # finite-difference gradients, every value one GPU evaluation
    nb = np.cumsum([0] + [len(ds["edges"]) - 1 for ds in desc["datasets"]])
    t0 = time.perf_counter()
    dmax, nev = 0.0, 0
    for j in range(n_plain):
        for d in range(len(desc["datasets"])):
            eng.set_data(d, data[j][nb[d]:nb[d + 1]])
        fmin, ne = plain_fit(eng, desc, chosen[j])
        nev += ne
        dmax = max(dmax, 2.0 * abs(fmin - rw["nll"][j]))
    tp = time.perf_counter() - t0
    res = dict(pseudo_experiments=E, training_spectra=len(X), generate_s=t_gen, train_s=t_train,
               train_tflops=6.0 * sur.net.nparam * 1024 * steps / t_train / 1e12,
               heldout_rms_dlogmu=float(np.sqrt(np.mean(err ** 2))),
               cold=dict(seconds=tc, fits_per_s=E / tc, found_global_min=float(np.mean(rc["nll"] - best < 5e-4)),
                         correct_fits_per_s=float(np.sum(rc["nll"] - best < 5e-4)) / tc,
                         mean_iters=float(rc["iters"].mean())),
               warm=dict(seconds=tw, surrogate_s=tsur, fits_per_s=E / tw,
                         found_global_min=float(np.mean(rw["nll"] - best < 5e-4)),
                         correct_fits_per_s=float(np.sum(rw["nll"] - best < 5e-4)) / tw,
                         mean_iters=float(rw["iters"].mean())),
               plain=dict(fits=n_plain, seconds=tp, fits_per_s=n_plain / tp, evals_per_fit=nev / max(1, n_plain),
                          max_delta_chi2_vs_batched=dmax))
    res["warm_over_plain"] = res["warm"]["fits_per_s"] / res["plain"]["fits_per_s"]
    res["warm_over_cold_correct_fits"] = res["warm"]["correct_fits_per_s"] / max(res["cold"]["correct_fits_per_s"],
                                                                                 1e-300)
    eng.close()
    log(f"warm start: {json.dumps(res)}")
    return res


def copy_bandwidth(torch, nbytes=1 << 30, reps=10):
    """Achievable device-memory bandwidth: a plain device-to-device copy
    (bytes read + bytes written per second)."""
    src = torch.ones(nbytes // 4, dtype=torch.float32, device="cuda")
    dst = torch.empty_like(src)
    dst.copy_(src)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(reps):
        dst.copy_(src)
    torch.cuda.synchronize()
    dt = (time.perf_counter() - t0) / reps
    del src, dst
    return 2 * nbytes / dt / 1e9


def event_sweep(args, nf, synth, torch, counts):
    """Single-evaluation throughput and fold bandwidth of the medium-baseline
    model at several event counts (the asymptote of the streaming fold): graph
    replays for the rate, per-kernel dispatch events for the durations."""
    stream = torch.cuda.Stream()
    for n in counts:
        log(f"sweep: generating {n:.0e} events")
        desc, events = synth.model_and_events(3, n)
        thetas = synth.osc_theta_list(desc, 64, seed=5)
        for mode in ("m32", "m64"):
            eng = nf.Engine(desc, mode, stream=stream.cuda_stream)
            for d, ev in enumerate(events):
                eng.set_events(d, ev["e_true"], ev["e_reco"], ev["source"], ev["weight"])
            n_in = sum(len(ev["weight"]) for ev in events) - sum(eng.dropped(d) for d in range(eng.D))
            for d, mu in enumerate(eng.expected(synth.start_vector(desc))[0]):
                eng.set_data(d, mu)
            th_dev = torch.tensor(thetas, dtype=torch.float64, device="cuda")
            out_dev = torch.zeros((64, 1 + eng.P), dtype=torch.float64, device="cuda")
            torch.cuda.synchronize()
            n_graph = max(d for d in range(1, 65) if args.steps % d == 0)
            eng.eval_device_many(n_graph, th_dev.data_ptr(), out_dev.data_ptr())
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            for _ in range(args.steps // n_graph):
                eng.eval_device_many(n_graph, th_dev.data_ptr(), out_dev.data_ptr())
            torch.cuda.synchronize()
            t1 = time.perf_counter()
            cnt, fold_ms, tail_ms, _ = event_timed(
                torch, eng, lambda k: eng.eval_device(th_dev[k % 64].data_ptr(), out_dev[k % 64].data_ptr()),
                args.steps)
            eng.close()
            bpe = 12 if mode == "m64" else 8
            fold_us = fold_ms / cnt * 1e3
            gbs = n_in * bpe / (fold_us * 1e-6) / 1e9
            print(json.dumps(dict(events=n, events_in_range=n_in, mode=mode, evals_per_s=args.steps / (t1 - t0),
                                  us_per_eval=(t1 - t0) / args.steps * 1e6, fold_us=fold_us,
                                  tail_us=tail_ms / cnt * 1e3, fold_gbs=gbs, frac=gbs / HBM_PEAK_GBS)),
                  flush=True)
        del events


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=400)
    ap.add_argument("--warmup", type=int, default=20)
    ap.add_argument("--mode", default="m32", choices=["m32", "m64"])
    ap.add_argument("--events", type=float, default=1e7)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--one-mode", action="store_true", help="skip the other precision mode")
    ap.add_argument("--cold-only", action="store_true",
                    help="only the replica-rotated (cold) evaluation loop with the default launch choices "
                         "(for profiled runs) and exit")
    ap.add_argument("--no-cpu-all-cores", action="store_true", help="skip the all-cores oracle leg")
    ap.add_argument("--replicas", type=int, default=6,
                    help="event-set replicas cycled for the cold (HBM) figure; 0 skips it")
    ap.add_argument("--no-fits", action="store_true", help="skip the pseudo-experiment fits/s section")
    ap.add_argument("--plain-fits", type=int, default=64, help="fits of the plain per-fit GPU path")
    ap.add_argument("--surrogate-samples", type=int, default=1_000_000,
                    help="training spectra for the warm-start section (0 skips it)")
    ap.add_argument("--no-matter", action="store_true", help="skip the constant-density matter section")
    ap.add_argument("--matter-only", action="store_true",
                    help="only the constant-density matter section (for kernel traces and counters)")
    ap.add_argument("--mlp-profile", action="store_true",
                    help="surrogate-network training steps only (for a kernel trace per product shape)")
    ap.add_argument("--copy-probe", action="store_true",
                    help="only run a device copy of known size (counter calibration) and exit")
    ap.add_argument("--no-autotune", action="store_true",
                    help="keep the default launch choices (for profiling runs: the kernel statistics then "
                         "cover one configuration)")
    ap.add_argument("--event-sweep", default="",
                    help="comma-separated event counts (e.g. 1e6,1e7,1e8): only time the single "
                         "evaluation of the medium-baseline model at each count and exit")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for {args.gpus}); the event fold shards over "
              "events or fits as described in the design notes, but this build measures one GPU.",
              file=sys.stderr)
        sys.exit(2)

    import torch
    from paper_2502_15253_amd import nufold as nf
    from paper_2502_15253_amd import synth

    torch.cuda.set_device(0)
    if args.copy_probe:
        copy_probe(torch)
        return
    if args.mlp_profile:
        mlp_profile(torch)
        return
    if args.event_sweep:
        event_sweep(args, nf, synth, torch, [int(float(x)) for x in args.event_sweep.split(",")])
        return
    # one explicit stream (default priority) that every engine enqueues on
    stream = torch.cuda.Stream()
    n_events = int(args.events)
    log(f"generating {n_events:.0e} events")
    desc, events = synth.model_and_events(3, n_events)
    thetas = synth.osc_theta_list(desc, 64, seed=5)
    start = synth.start_vector(desc)
    if args.matter_only:
        print(json.dumps(dict(matter=matter_section(nf, synth, torch, stream, events, thetas, steps=args.steps))),
              flush=True)
        return

    def run(mode):
        eng = nf.Engine(desc, mode, stream=stream.cuda_stream)
        for d, ev in enumerate(events):
            eng.set_events(d, ev["e_true"], ev["e_reco"], ev["source"], ev["weight"])
        n_in = sum(len(ev["weight"]) for ev in events) - sum(eng.dropped(d) for d in range(eng.D))
        mus, _ = eng.expected(start)
        for d, mu in enumerate(mus):
            eng.set_data(d, mu)  # Asimov data at the start point
        # launch choices (work-item size, fold workgroup, bin-stage threads)
        # from the library's autotuner, before the clock
        from paper_2502_15253_amd import autotune as AT
        if args.no_autotune:
            tuned = dict(options={k: eng.get_option(k) for k in AT.OPTIONS}, cached=None)
        else:
            tuned = AT.tune(eng, desc, [len(ev["weight"]) for ev in events], thetas[0],
                            cache_path=os.path.join(tempfile.gettempdir(), "nufold_bench_autotune.json"),
                            evals=200, force=True)
        log(f"{mode} launch choices: {json.dumps(tuned)}")
        th_dev = torch.tensor(thetas, dtype=torch.float64, device="cuda")
        out_dev = torch.zeros((len(thetas), 1 + eng.P), dtype=torch.float64, device="cuda")
        ptr_t = [th_dev[i].data_ptr() for i in range(len(thetas))]
        ptr_o = [out_dev[i].data_ptr() for i in range(len(thetas))]
        torch.cuda.synchronize()  # the inputs were written on torch's default stream
        for k in range(args.warmup):
            eng.eval_device(ptr_t[k % 64], ptr_o[k % 64])
        # timed region: the evaluations as replays of one captured HIP graph of
        # n_graph consecutive evaluations (n_graph divides the step count, so
        # exactly `steps` evaluations run); the graph is captured and run once
        # before the clock starts
        n_graph = max(d for d in range(1, 65) if args.steps % d == 0)
        eng.eval_device_many(n_graph, th_dev.data_ptr(), out_dev.data_ptr())
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for r in range(args.steps // n_graph):
            eng.eval_device_many(n_graph, th_dev.data_ptr(), out_dev.data_ptr())
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        assert bool(torch.isfinite(out_dev[:n_graph]).all()), "non-finite NLL/gradient in the timed loop"
        # the same evaluations one launch pair at a time, without and with
        # per-kernel HIP events (the events give the fold and bin-stage
        # durations of the roofline figure)
        s0 = time.perf_counter()
        for k in range(args.steps):
            eng.eval_device(ptr_t[k % 64], ptr_o[k % 64])
        torch.cuda.synchronize()
        s1 = time.perf_counter()
        torch.cuda.synchronize()
        cnt, fold_ms, tail_ms, e_sec = event_timed(
            torch, eng, lambda k: eng.eval_device(ptr_t[k % 64], ptr_o[k % 64]), args.steps)
        assert cnt == args.steps
        # fixed cost inside every event-timed region (event packets, dispatch
        # and completion of the launch), measured on the same stream
        ev_over_us = eng.timing_overhead(200)
        assert bool(torch.isfinite(out_dev).all()), "non-finite NLL/gradient in the stream loops"
        # host C-ABI path, synchronous, including H2D of theta and D2H of NLL + gradient
        # (median of 5 rounds of 100: host-side stalls hit single rounds)
        th_np = thetas
        host_rates = []
        for _ in range(5):
            h0 = time.perf_counter()
            for k in range(100):
                eng.eval_nll_grad(th_np[k % 64])
            host_rates.append(100 / (time.perf_counter() - h0))
        host_rate = float(np.median(host_rates))
        bpe = 12 if mode == "m64" else 8
        fold_us = fold_ms / cnt * 1e3
        achieved = n_in * bpe / (fold_us * 1e-6) / 1e9
        traffic = measured_traffic(mode, n_in * bpe)
        res = dict(
            evals_per_s=args.steps / (t1 - t0), ms_per_step=(t1 - t0) * 1e3 / args.steps,
            graph_evals=n_graph, launch_options=tuned["options"],
            stream_loop_evals_per_s=args.steps / (s1 - s0),
            event_timed_evals_per_s=args.steps / e_sec,
            fold_us=fold_us, tail_us=tail_ms / cnt * 1e3, event_pair_gap_us=ev_over_us,
            host_path_evals_per_s=host_rate, events_in_range=n_in,
            roofline=dict(bound="hbm", achieved=achieved, peak=HBM_PEAK_GBS, unit="GB/s",
                          frac=achieved / HBM_PEAK_GBS, traffic=traffic,
                          algorithmic_bytes_per_launch=n_in * bpe,
                          duration="mean fold duration from HIP start/stop events carried by every "
                                   "fold dispatch (hipExtLaunchKernel) of event-timed passes over the "
                                   "same evaluations (same kernels and inputs) right after the timed "
                                   "graph replays, on the engine stream: 20 warm-up launches, then "
                                   "the median of three passes"))
        eng.close()
        log(f"{mode}: {json.dumps(res)}")
        return res

    def run_cold(mode, R, steps, options=None):
        """The same evaluations cycled over R engines that each hold their own
        copy of the event set, so that consecutive folds read different
        buffers whose total exceeds the 256 MB Infinity Cache."""
        engs = []
        for r in range(R):
            e = nf.Engine(desc, mode, stream=stream.cuda_stream)
            for k, v in (options or {}).items():
                e.set_option(k, v)
            for d, ev in enumerate(events):
                e.set_events(d, ev["e_true"], ev["e_reco"], ev["source"], ev["weight"])
            for d, mu in enumerate(e.expected(start)[0]):
                e.set_data(d, mu)
            engs.append(e)
        n_in = sum(len(ev["weight"]) for ev in events) - sum(engs[0].dropped(d) for d in range(engs[0].D))
        th_dev = torch.tensor(thetas, dtype=torch.float64, device="cuda")
        out_dev = torch.zeros((len(thetas), 1 + engs[0].P), dtype=torch.float64, device="cuda")
        torch.cuda.synchronize()
        for k in range(2 * R):
            engs[k % R].eval_device(th_dev[k % 64].data_ptr(), out_dev[k % 64].data_ptr())
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for k in range(steps):
            engs[k % R].eval_device(th_dev[k % 64].data_ptr(), out_dev[k % 64].data_ptr())
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        # the same loop again with per-kernel dispatch events for the durations
        for e in engs:
            e.set_option("timing", 1)
        for k in range(steps):
            engs[k % R].eval_device(th_dev[k % 64].data_ptr(), out_dev[k % 64].data_ptr())
        torch.cuda.synchronize()
        cnt = fold_ms = tail_ms = 0
        for e in engs:
            c_, f_, t_ = e.timing(reset=True)
            cnt, fold_ms, tail_ms = cnt + c_, fold_ms + f_, tail_ms + t_
            e.close()
        assert cnt == steps and bool(torch.isfinite(out_dev).all())
        bpe = 12 if mode == "m64" else 8
        fold_us = fold_ms / cnt * 1e3
        achieved = n_in * bpe / (fold_us * 1e-6) / 1e9
        res = dict(replicas=R, steps=steps, resident_bytes=R * n_in * bpe, evals_per_s=steps / (t1 - t0),
                   fold_us=fold_us, tail_us=tail_ms / cnt * 1e3,
                   achieved_gbs=achieved, frac=achieved / HBM_PEAK_GBS)
        log(f"{mode} cold: {json.dumps(res)}")
        return res

    if args.cold_only:
        # profiling run: only the replica-rotated loop, default launch choices
        res = run_cold(args.mode, max(args.replicas, 4), max(args.steps, COLD_STEPS))
        print(json.dumps(dict(mode=args.mode, cold=res)), flush=True)
        return

    def roofline(res, cold, copy_gbs):
        """The fold's roofline entry: HBM-bound, priced with the replica-rotated
        (cold) fold durations, whose event set does not fit the Infinity Cache;
        the single-engine (MALL-resident) figure is kept beside it."""
        warm = res["roofline"]
        rf = dict(warm)
        rf["frac_mall_warm"] = warm["frac"]
        rf["achieved_mall_warm"] = warm["achieved"]
        rf["fold_us_mall_warm"] = res["fold_us"]
        if cold is not None:
            rf["achieved"] = cold["achieved_gbs"]
            rf["frac"] = cold["frac"]
            rf["fold_us"] = cold["fold_us"]
            rf["duration"] = (f"mean fold duration from HIP start/stop events carried by every fold dispatch "
                              f"(hipExtLaunchKernel) of {cold['steps']} evaluations cycled over "
                              f"{cold['replicas']} engines holding their own copies of the event set "
                              f"({cold['resident_bytes'] / 1e6:.0f} MB, more than the 256 MB Infinity Cache), "
                              "on the engine stream")
        rf["frac_of_copy_bandwidth"] = rf["achieved"] / copy_gbs
        rf["copy_bandwidth_gbs"] = copy_gbs
        rf["frac_whole_evaluation"] = (rf["algorithmic_bytes_per_launch"] / (res["ms_per_step"] * 1e-3) / 1e9
                                       / HBM_PEAK_GBS)
        return rf

    copy_gbs = copy_bandwidth(torch)
    log(f"device copy bandwidth {copy_gbs:.0f} GB/s")
    cold_steps = max(args.steps, COLD_STEPS)
    main_res = run(args.mode)
    cold = (run_cold(args.mode, args.replicas, cold_steps, main_res["launch_options"]) if args.replicas > 0
            else None)
    main_res["roofline"] = roofline(main_res, cold, copy_gbs)
    other = None
    if not args.one_mode:
        om = "m64" if args.mode == "m32" else "m32"
        other = run(om)
        ocold = run_cold(om, args.replicas, cold_steps, other["launch_options"]) if args.replicas > 0 else None
        other["roofline"] = roofline(other, ocold, copy_gbs)
        other["cold"] = ocold
    fits = None
    if not args.no_fits:
        fits = fits_section(nf, synth, torch, stream, args.plain_fits, args.surrogate_samples)
    matter = None if args.no_matter else matter_section(nf, synth, torch, stream, events, thetas)
    cpu = None
    if not args.no_cpu_baseline:
        log("timing the CPU oracle (whole evaluations, about ten seconds)")
        cpu = cpu_baseline(desc, events, thetas[0])
        if not args.no_cpu_all_cores:
            log("timing the CPU oracle on every host core (one process per core)")
            cpu["all_cores"] = cpu_baseline_all_cores(n_events)

    line = {
        "metric": "fold+NLL+grad evals/s (1e7-event JUNO-like); pseudo-exp fits/s vs plain",
        "value": main_res["evals_per_s"],
        "unit": "evals/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": main_res["ms_per_step"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32+f64" if args.mode == "m32" else "f64",
        "data": "synthetic (seeded MC events and Asimov data)",
        "config": {
            "workload": "medium-baseline three-flavour fold: 1e7 MC events, 10 cores at "
                        "52-53 km, 400 bins on 0.8-12 MeV, 120 parameters, NLL + adjoint gradient",
            "events": n_events, "bins": 400, "params": len(start),
            "mode": args.mode,
        },
        "timed_region": f"replays of one HIP graph of {main_res['graph_evals']} consecutive "
                        "evaluations (nf_eval_device_many), parameters and outputs resident in HBM",
        "launch_options": main_res["launch_options"],
        "fold_us": main_res["fold_us"],
        "tail_us": main_res["tail_us"],
        "stream_loop_evals_per_s": main_res["stream_loop_evals_per_s"],
        "event_timed_evals_per_s": main_res["event_timed_evals_per_s"],
        "host_path_evals_per_s": main_res["host_path_evals_per_s"],
        "roofline": main_res["roofline"],
        "cold": cold,
        "fits": fits,
        "cpu_baseline": cpu,
    }
    if other is not None:
        line["other_mode"] = {"mode": "m64" if args.mode == "m32" else "m32", **other}
    if matter is not None:
        line["matter"] = matter
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
