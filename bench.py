"""Benchmark: fold + NLL + adjoint-gradient evaluations per second on the
1e7-event medium-baseline (JUNO-like) workload, on one MI355X.

One step = one full model evaluation at a new parameter vector: the event fold
(HIP), the bin stages, the Poisson NLL with priors and the adjoint gradient
(HIP), for all 1e7 events, 10 reactor cores, 400 analysis bins, 120 parameters.
Inputs (events, data, 64 parameter vectors whose oscillation parameters all
differ) are resident in device memory before the timed region.

Prints one JSON line. Per-kernel durations come from HIP events recorded on
the engine's stream around every fold and bin-stage launch of the timed
region; the roofline entry prices the fold (the dominant kernel) against
MI355X's 8 TB/s HBM peak with the algorithmic bytes it must read
(u = L/E and w per event: 12 B in FP64 mode, 8 B in FP32 mode).
The CPU baseline is the FP64 oracle (NLL plus complex-step gradient) timed on
the host for one evaluation of the same workload.
"""
import argparse
import hashlib
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
PROFILE_TRAFFIC = os.path.join(ROOT, "profiles", "fold_c3_traffic.json")


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def fold_source_hash():
    h = hashlib.sha256()
    for f in ("fold.hip", "fastmath.hpp", "sincos_coeffs.hpp", "kernels.hpp", "plan.hpp"):
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
    t0 = time.perf_counter()
    LK.nll_grad(m, events, data, theta)
    dt = time.perf_counter() - t0
    return dict(value=1.0 / dt, unit="evals/s", cores=1, kind="oracle",
                sample=f"1 full evaluation (NLL + complex-step gradient over {m.P} parameters) "
                       f"of the {sum(len(e['weight']) for e in events):.0e}-event workload, "
                       f"numpy FP64, single thread, {dt:.1f} s")


COPY_BYTES = 512 << 20


def copy_probe(torch, reps=8):
    """Plain device-to-device copies of COPY_BYTES each: the reference that
    scales the memory counters of a profiled run to bytes."""
    src = torch.ones(COPY_BYTES // 4, dtype=torch.float32, device="cuda")
    dst = torch.empty_like(src)
    for _ in range(reps):
        dst.copy_(src)
    torch.cuda.synchronize()
    log(f"copy probe: {reps} copies of {COPY_BYTES} B")


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=400)
    ap.add_argument("--warmup", type=int, default=20)
    ap.add_argument("--mode", default="m32", choices=["m32", "m64"])
    ap.add_argument("--events", type=float, default=1e7)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--both-modes", action="store_true", help="also measure the other precision mode")
    ap.add_argument("--replicas", type=int, default=6,
                    help="event-set replicas cycled for the cold (HBM) figure; 0 skips it")
    ap.add_argument("--copy-probe", action="store_true",
                    help="only run a device copy of known size (counter calibration) and exit")
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
    stream = torch.cuda.current_stream()
    n_events = int(args.events)
    log(f"generating {n_events:.0e} events")
    desc, events = synth.model_and_events(3, n_events)
    thetas = synth.osc_theta_list(desc, 64, seed=5)
    start = synth.start_vector(desc)

    def run(mode):
        eng = nf.Engine(desc, mode, stream=stream.cuda_stream)
        for d, ev in enumerate(events):
            eng.set_events(d, ev["e_true"], ev["e_reco"], ev["source"], ev["weight"])
        n_in = sum(len(ev["weight"]) for ev in events) - sum(eng.dropped(d) for d in range(eng.D))
        mus, _ = eng.expected(start)
        for d, mu in enumerate(mus):
            eng.set_data(d, mu)  # Asimov data at the start point
        th_dev = torch.tensor(thetas, dtype=torch.float64, device="cuda")
        out_dev = torch.zeros((len(thetas), 1 + eng.P), dtype=torch.float64, device="cuda")
        ptr_t = [th_dev[i].data_ptr() for i in range(len(thetas))]
        ptr_o = [out_dev[i].data_ptr() for i in range(len(thetas))]
        for k in range(args.warmup):
            eng.eval_device(ptr_t[k % 64], ptr_o[k % 64])
        torch.cuda.synchronize()
        eng.set_option("timing", 1)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for k in range(args.steps):
            eng.eval_device(ptr_t[k % 64], ptr_o[k % 64])
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        cnt, fold_ms, tail_ms = eng.timing(reset=True)
        eng.set_option("timing", 0)
        assert cnt == args.steps
        assert bool(torch.isfinite(out_dev).all()), "non-finite NLL/gradient in the timed loop"
        # host C-ABI path, synchronous, including H2D of theta and D2H of NLL + gradient
        th_np = thetas
        h0 = time.perf_counter()
        nh = 50
        for k in range(nh):
            eng.eval_nll_grad(th_np[k % 64])
        h1 = time.perf_counter()
        bpe = 12 if mode == "m64" else 8
        fold_avg_s = fold_ms / cnt / 1e3
        achieved = n_in * bpe / fold_avg_s / 1e9
        traffic = measured_traffic(mode, n_in * bpe)
        res = dict(
            evals_per_s=args.steps / (t1 - t0), ms_per_step=(t1 - t0) * 1e3 / args.steps,
            fold_us=fold_ms / cnt * 1e3, tail_us=tail_ms / cnt * 1e3,
            host_path_evals_per_s=nh / (h1 - h0), events_in_range=n_in,
            roofline=dict(bound="hbm", achieved=achieved, peak=HBM_PEAK_GBS, unit="GB/s",
                          frac=achieved / HBM_PEAK_GBS, traffic=traffic,
                          algorithmic_bytes_per_launch=n_in * bpe))
        eng.close()
        log(f"{mode}: {json.dumps(res)}")
        return res

    def run_cold(mode, R, steps):
        """The same evaluations cycled over R engines that each hold their own
        copy of the event set, so that consecutive folds read different
        buffers whose total exceeds the 256 MB Infinity Cache."""
        engs = []
        for r in range(R):
            e = nf.Engine(desc, mode, stream=stream.cuda_stream)
            for d, ev in enumerate(events):
                e.set_events(d, ev["e_true"], ev["e_reco"], ev["source"], ev["weight"])
            for d, mu in enumerate(e.expected(start)[0]):
                e.set_data(d, mu)
            engs.append(e)
        n_in = sum(len(ev["weight"]) for ev in events) - sum(engs[0].dropped(d) for d in range(engs[0].D))
        th_dev = torch.tensor(thetas, dtype=torch.float64, device="cuda")
        out_dev = torch.zeros((len(thetas), 1 + engs[0].P), dtype=torch.float64, device="cuda")
        for k in range(2 * R):
            engs[k % R].eval_device(th_dev[k % 64].data_ptr(), out_dev[k % 64].data_ptr())
        torch.cuda.synchronize()
        for e in engs:
            e.set_option("timing", 1)
        t0 = time.perf_counter()
        for k in range(steps):
            engs[k % R].eval_device(th_dev[k % 64].data_ptr(), out_dev[k % 64].data_ptr())
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        cnt = fold_ms = tail_ms = 0
        for e in engs:
            c_, f_, t_ = e.timing(reset=True)
            cnt, fold_ms, tail_ms = cnt + c_, fold_ms + f_, tail_ms + t_
            e.close()
        assert cnt == steps and bool(torch.isfinite(out_dev).all())
        bpe = 12 if mode == "m64" else 8
        achieved = n_in * bpe / (fold_ms / cnt / 1e3) / 1e9
        res = dict(replicas=R, resident_bytes=R * n_in * bpe, evals_per_s=steps / (t1 - t0),
                   fold_us=fold_ms / cnt * 1e3, tail_us=tail_ms / cnt * 1e3,
                   achieved_gbs=achieved, frac=achieved / HBM_PEAK_GBS)
        log(f"{mode} cold: {json.dumps(res)}")
        return res

    main_res = run(args.mode)
    cold = None
    if args.replicas > 0:
        cold = run_cold(args.mode, args.replicas, max(args.steps, 4 * args.replicas))
    other = None
    if args.both_modes:
        other = run("m64" if args.mode == "m32" else "m32")
    cpu = None
    if not args.no_cpu_baseline:
        log("timing the CPU oracle (one evaluation)")
        cpu = cpu_baseline(desc, events, thetas[0])

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
        "fold_us": main_res["fold_us"],
        "tail_us": main_res["tail_us"],
        "host_path_evals_per_s": main_res["host_path_evals_per_s"],
        "roofline": main_res["roofline"],
        "cold": cold,
        "cpu_baseline": cpu,
    }
    if other is not None:
        line["other_mode"] = {"mode": "m64" if args.mode == "m32" else "m32", **other}
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
