#!/usr/bin/env python3
"""Throughput of the DEM step (sphere-steps per second) on one MI355X.

Workload: gravitational collapse of 25,000 rigid aggregates of 2-8 spheres
(about 125k spheres, radius U[0.8, 1.2], density 1) at rest in a ball sized
for an initial packing fraction of 0.15; G = 1, Plummer softening 0.5 of the
mean pair radius, contact constants k_n = 1e5, k_t = 2/7 k_n, restitution 0.5,
mu_s = 0.5, mu_r = mu_t = 0.1; dt = 5e-4.  Synthetic, seeded inputs.

One step is the whole hot path: kick/drift/rotate, member reconstruction,
cell binning, contact search, contact forces with spring history, softened
all-pairs gravity, aggregate reduction and kick.  The timed region replays K
steps with an event around every kernel (per-kernel durations on the
library's stream); the roofline object describes the dominant kernel
(gravity).  The CPU baseline times the FP64 oracle on the host.

  python bench.py [--steps K] [--warmup W] [--precision fp64|fp32] [--n-agg N]
"""
import argparse
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "sphere-steps/sec at 125k spheres (plain vs FP32-force batched); p50/p99 run latency"
PEAK_TFLOPS = {"fp64": 78.6, "fp32": 157.3}     # MI355X vector peaks
GRAVITY_FLOP_PER_PAIR = 20                      # 3 sub, 3 fma, rsqrt, 2 mul, 1 mul, 3 fma
PEAK_HBM_GBS = 8000.0                           # MI355X HBM3E
# algorithmic bytes of the contact path per sphere-step: about 390 B for the
# aggregate update, reconstruction, binning, search and force-side reads, plus
# 64 B per contact of the sphere (keys and FP64 spring history, read and written)
CONTACT_BYTES_FIXED = 390
CONTACT_BYTES_PER_CONTACT = 64


# HBM traffic of the gravity stage per launch (bytes), from rocprofv3 --pmc
# FETCH_SIZE and WRITE_SIZE runs scaled by a plain-copy calibration (see the
# profile summaries); valid only for the gravity source it was measured on.
MEASURED_TRAFFIC = {
    # (precision, spheres, tile, form of the exact sum):
    #     (bytes per launch, source_hash("kernels_gravity.hip"))
    ("fp64", 124958, 512, 1): (2299.0e6, "065b5f21aae1cf9c"),
    ("fp32", 124958, 1024, 1): (539.8e6, "065b5f21aae1cf9c"),
    ("fp64", 124958, 512, 2): (196.9e6, "065b5f21aae1cf9c"),
    ("fp64", 499845, 512, 1): (26922.6e6, "065b5f21aae1cf9c"),
}


# Executed FP64 FLOP of the tree walk per launch (64 x SQ_INSTS_VALU_FLOPS_FP64
# from rocprofv3 --pmc), for the tree run's roofline; valid only for the
# gravity source it was measured on.
MEASURED_TREE_FLOP = {
    # (spheres, opening angle, leaf, order): (FLOP per launch, source_hash("kernels_tree.hip"))
    (124958, 0.5, 32, 4): (3.609e10, "471bb11951ce97d0"),
    (999660, 0.5, 32, 4): (3.797e11, "471bb11951ce97d0"),
}


def source_hash(name):
    """sha256[:16] of a gravity kernel source together with the header the
    gravity sources share."""
    import hashlib
    h = hashlib.sha256()
    for f in (name, "gravity_common.h"):
        with open(os.path.join(ROOT, "paper_2311_11322_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def log(*a):
    print("[bench]", *a, file=sys.stderr, flush=True)


def _cpu_model():
    """The host CPU's model name with its family, model and stepping numbers
    (a virtual machine may report only a generic name)."""
    try:
        with open("/proc/cpuinfo") as f:
            first = f.read().split("\n\n", 1)[0]
    except OSError:
        return ""
    fields = {}
    for ln in first.splitlines():
        if ":" in ln:
            k, v = ln.split(":", 1)
            fields.setdefault(k.strip(), v.strip())
    name = fields.get("model name", "")
    ids = [f"{k} {fields[k]}" for k in ("cpu family", "model", "stepping") if k in fields]
    return f"{name} ({', '.join(ids)})" if ids else name


def cpu_baseline(inp, n_sample, seconds_cap):
    """The FP64 oracle on the host, as it stands: its gravity and sampled
    evaluation loops are shared among threads with OpenMP (each target's sum
    keeps its order, so the thread count changes no result).

    * headline (collapse): the t0 force evaluation (brute-force contacts and
      direct-sum gravity at full N) of a sample of spheres, on all allowed
      cores and on one core, scaled by N to a whole step;
    * cfg0 (the contact-only periodic box) run in full, 200 steps (no
      gravity: the step is single-threaded);
    * 8 of the spin-up piles, one step each, all cores."""
    import numpy as np
    import oracle as O
    cores = len(os.sched_getaffinity(0))
    w = inp["collapse"]
    o = O.Oracle(w.params).add_workload(w, evaluate=False)
    rng = np.random.default_rng(0)
    idx = np.sort(rng.choice(w.n_sph, n_sample, replace=False))

    def sampled(threads, cap_s):
        used = O.set_threads(threads)
        done, t_used, chunk = 0, 0.0, max(64, 16 * used)
        while done < n_sample and t_used < cap_s:
            sl = idx[done:done + chunk]
            t0 = time.perf_counter()
            o.eval_subset(sl)
            t_used += time.perf_counter() - t0
            done += len(sl)
        return used, done, t_used

    used_n, done_n, t_n = sampled(cores, seconds_cap / 2)
    _, done_1, t_1 = sampled(1, seconds_cap / 2)
    log(f"cpu baseline: {done_n} spheres on {used_n} threads in {t_n:.1f} s, "
        f"{done_1} on 1 in {t_1:.1f} s")
    out = {"value": round(done_n / t_n, 1), "unit": "sphere-steps/s", "cores": used_n,
           "kind": "oracle",
           "sample": f"t0 force evaluation of {done_n} of {w.n_sph} spheres of the collapse at "
                     f"full N (brute-force contacts + direct-sum gravity, {used_n} OpenMP "
                     f"threads, {t_n:.1f} s), scaled by N to a whole step",
           "one_core": {"value": round(done_1 / t_1, 1), "cores": 1,
                        "sample": f"{done_1} spheres, {t_1:.1f} s"},
           "host_cores_allowed": cores, "cpu_model": _cpu_model()}
    # cfg0 in full
    w0 = inp.get("cfg0")
    if w0 is not None:
        O.set_threads(1)
        t0 = time.perf_counter()
        o0 = O.Oracle(w0.params).add_workload(w0)
        o0.step(w0.n_steps)
        t = time.perf_counter() - t0
        out["cfg0"] = {"value": round(w0.n_sph * w0.n_steps / t, 1), "unit": "sphere-steps/s",
                       "cores": 1, "steps": w0.n_steps, "seconds": round(t, 2),
                       "contacts_at_end": o0.counts()[2],
                       "sample": f"the whole run: {w0.n_steps} steps of {w0.n_sph} spheres "
                                 "(set-up and t0 evaluation included)"}
    # 8 of the spin-up piles, one step each
    piles = inp.get("piles")
    if piles:
        used = O.set_threads(cores)
        pick = np.sort(np.random.default_rng(8).choice(len(piles), min(8, len(piles)),
                                                       replace=False))
        t_sum, ss = 0.0, 0
        for k in pick:
            p = piles[int(k)]
            op = O.Oracle(p.params).add_workload(p)
            t0 = time.perf_counter()
            op.step(1)
            t_sum += time.perf_counter() - t0
            ss += p.n_sph
        out["cfg3_subset"] = {"value": round(ss / t_sum, 1), "unit": "sphere-steps/s",
                              "cores": used, "piles": [int(k) for k in pick],
                              "spheres": ss, "seconds": round(t_sum, 2),
                              "sample": "one step of each of 8 spin-up piles (FP64 oracle, "
                                        "brute-force contacts single-threaded, gravity on "
                                        f"{used} threads)"}
    O.set_threads(cores)
    return out


def prepare_inputs(args, workers, sections):
    """Every CPU-side input, generated before anything touches the GPU, on
    one process pool (its workers are forked from a process that has not
    initialised a device)."""
    from concurrent.futures import ProcessPoolExecutor
    from paper_2311_11322_amd import serve
    from paper_2311_11322_amd import workloads as W
    t = time.time()
    inp, fut = {}, {}
    with ProcessPoolExecutor(max_workers=max(1, workers)) as ex:
        if "big" in sections and args.big_agg > 0:
            fut["big"] = ex.submit(W.collapse_cloud, 2, n_agg=args.big_agg)
        if "headline" in sections:
            fut["collapse"] = ex.submit(W.collapse_cloud, 1, n_agg=args.n_agg)
            fut["cfg0"] = ex.submit(W.periodic_box, 0)
        if "ablation" in sections:
            fut["ablation"] = ex.submit(W.collapse_cloud, seed=5, n_agg=4444, cmin=1, cmax=8)
        if "contact_path" in sections:
            fut["lattices"] = [ex.submit(W.dense_lattice, n_side=n) for n in args.lattice_sides]
            if not args.no_lattice_morton:
                fut["lattices"].append(ex.submit(W.dense_lattice, n_side=max(args.lattice_sides),
                                                 order="morton"))
        if "walled" in sections:
            fut["fills"] = {sh: ex.submit(W.box_fill, seed=8, shape=sh)
                            for sh in ("sphere", "dumbbell", "cube", "mixed")}
            fut["boxes"] = [ex.submit(W.box_fill, seed=100 + k, shape="mixed")
                            for k in range(args.box_batch)]
            fut["brazil"] = ex.submit(W.brazil_nut)
        if "batched" in sections:
            inp["piles"] = W.pile_batch(seed=3, n_piles=args.piles, executor=ex)
        if "served" in sections and args.requests > 0:
            inp["requests"] = serve.request_stream(seed=4, n_requests=args.requests,
                                                   rate_per_s=20.0, executor=ex)
        for k, f in fut.items():
            if isinstance(f, dict):
                inp[k] = {a: b.result() for a, b in f.items()}
            elif isinstance(f, list):
                inp[k] = [b.result() for b in f]
            else:
                inp[k] = f.result()
    log(f"inputs generated in {time.time() - t:.1f} s on {workers} workers")
    return inp


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--precision", choices=["fp64", "fp32"], default="fp64")
    ap.add_argument("--gravity", choices=["direct", "tree"], default="direct",
                    help="gravity of the headline run: exact direct sum, or the tree "
                         "(opening angle 0.5, leaves of 32, FP64)")
    ap.add_argument("--n-agg", type=int, default=25000)
    ap.add_argument("--gravity-tile", type=int, default=0, help="0: library default")
    ap.add_argument("--gravity-form", type=int, default=0, choices=[0, 1, 2],
                    help="exact sum: 0 library choice, 1 pairs, 2 per target")
    ap.add_argument("--cell-scale", type=float, default=1.0)
    ap.add_argument("--full-run-steps", type=int, default=2000,
                    help="steps of the whole-run leg of the headline workload (0: skip)")
    ap.add_argument("--cpu-sample", type=int, default=4096)
    ap.add_argument("--cpu-seconds", type=float, default=20.0)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-extra", action="store_true",
                    help="only the headline workload (skip FP32-force, batched and served)")
    ap.add_argument("--piles", type=int, default=256)
    ap.add_argument("--settle-steps", type=int, default=5600,
                    help="steps that collapse and settle each spin-up pile first "
                         "(5600 x 5e-4 = 2 free-fall times of the packing-0.15 cloud)")
    ap.add_argument("--campaign-steps", type=int, default=4000,
                    help="step limit of the spin-up campaign to failure")
    ap.add_argument("--big-agg", type=int, default=100000,
                    help="aggregates of the FP32-force 500k-sphere gravity run (0: skip)")
    ap.add_argument("--requests", type=int, default=200)
    ap.add_argument("--lattice-sides", type=int, nargs="+", default=[50, 100],
                    help="lattice edge lengths of the contact-path runs (n^3 spheres)")
    ap.add_argument("--no-lattice-morton", action="store_true",
                    help="skip the largest lattice with its aggregates in Morton order")
    ap.add_argument("--fill-steps", type=int, default=10000,
                    help="steps of the box-filling runs (the paper profiles 10^4)")
    ap.add_argument("--box-batch", type=int, default=64, help="box fills batched in one engine")
    ap.add_argument("--only", choices=["contact_path", "walled", "batched"], default=None,
                    help="run only this section and print its result (for profiler runs)")
    ap.add_argument("--calibrate-copy", type=int, default=0, metavar="BYTES",
                    help="only run a plain device copy of BYTES (counter calibration)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for {args.gpus}): the library has no "
              "multi-GPU decomposition", file=sys.stderr)
        sys.exit(2)

    import torch
    if args.calibrate_copy:
        # a plain copy kernel of known size, for scaling the HBM byte counters
        x = torch.empty(args.calibrate_copy // 4, dtype=torch.float32, device="cuda")
        y = torch.empty_like(x)
        x.fill_(1.0)
        torch.cuda.synchronize()
        for _ in range(3):
            y.copy_(x)
        torch.cuda.synchronize()
        print(json.dumps({"calibration_copy_bytes": args.calibrate_copy, "copies": 3}))
        return
    workers = min(16, len(os.sched_getaffinity(0)))
    if args.only:
        sections = {args.only}
    else:
        sections = {"headline"}
        if not args.no_extra:
            sections |= {"big", "ablation", "contact_path", "walled", "batched", "served"}
        if not args.no_cpu_baseline:
            sections |= {"batched"}
    inp = prepare_inputs(args, workers, sections)
    from paper_2311_11322_amd import dem
    torch.cuda.init()
    dem.lib()
    if args.only:
        part = {}
        if args.only == "contact_path":
            contact_path_run(args, inp, part)
        elif args.only == "batched":
            batched_run(args, inp, part, plain=False)
        else:
            walled_runs(args, inp, part)
        print(json.dumps(part), flush=True)
        return

    w = inp["collapse"]
    log(f"workload: {w.n_agg} aggregates, {w.n_sph} spheres")
    prec = dem.PREC_FP32_FORCE if args.precision == "fp32" else dem.PREC_FP64
    if args.gravity == "tree":
        w.params.update(gravity_tree=1, theta=0.5, tree_leaf=32, tree_order=4)
    alloc = dem.TorchAllocator(0)
    sim = dem.Sim(w.params, precision=prec, allocator=alloc, stream=dem.torch_stream())
    sim.set_tuning(args.gravity_tile, args.cell_scale, gravity_form=args.gravity_form)
    sim.add_workload(w)
    log("added; warmup", args.warmup)
    sim.step(args.warmup)
    torch.cuda.synchronize()

    # timed region: K steps launched in the order and on the streams of the
    # step graph (gravity on the second stream beside the contact kernels),
    # with a HIP event before and after the gravity stage on that stream
    sim.set_profiling(True, graph_order=True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    sim.step(args.steps)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    prof = sim.profile()
    sim.set_profiling(False)
    wall = t1 - t0
    ms_per_step = 1e3 * wall / args.steps
    value = w.n_sph * args.steps / wall
    log(f"timed: {args.steps} steps in {wall:.3f} s -> {value:.4g} sphere-steps/s")

    # the same steps as graph replays (no events)
    torch.cuda.synchronize()
    g0 = time.perf_counter()
    sim.step(args.steps)
    torch.cuda.synchronize()
    graph_value = w.n_sph * args.steps / (time.perf_counter() - g0)

    # per-kernel breakdown (outside the timed region): the same number of
    # steps launched kernel by kernel with an event between consecutive ones
    sim.set_profiling(True)
    sim.step(args.steps)
    torch.cuda.synchronize()
    staged = sim.profile()
    sim.set_profiling(False)
    staged_ms = sum(v for k, v in staged.items() if not k.startswith("_")) / staged["_steps"]

    # per-step latency over repeated single steps (outside the timed region)
    lat = []
    for _ in range(max(50, args.steps)):
        s0 = time.perf_counter()
        sim.step(1)
        torch.cuda.synchronize()
        lat.append(1e3 * (time.perf_counter() - s0))
    lat.sort()
    step_latency = {"p50_ms": round(lat[len(lat) // 2], 4),
                    "p99_ms": round(lat[min(len(lat) - 1, int(0.99 * len(lat)))], 4),
                    "steps": len(lat)}

    n = w.n_sph
    grav_ms = prof["gravity"] / prof["_steps"]
    flop = GRAVITY_FLOP_PER_PAIR * n * (n - 1)
    if args.gravity == "tree":
        mt = MEASURED_TREE_FLOP.get((n, 0.5, 32, 4))
        flop = mt[0] if mt and mt[1] == source_hash("kernels_tree.hip") else float("nan")
    achieved = flop / (grav_ms * 1e-3) / 1e12
    dt_key = "fp32" if prec == dem.PREC_FP32_FORCE else "fp64"
    tile = args.gravity_tile or dem.gravity_tiles(prec)[0]
    meas = MEASURED_TRAFFIC.get((dt_key, n, tile, args.gravity_form or 1))
    traffic = (meas[0] if meas and meas[1] == source_hash("kernels_gravity.hip")
               and args.gravity == "direct"
               else None)
    roofline = {"kernel": "gravity" if args.gravity == "direct" else "gravity (tree)",
                "bound": "alu", "achieved": round(achieved, 3) if achieved == achieved else None,
                "peak": PEAK_TFLOPS[dt_key], "unit": "TFLOP/s",
                "frac": round(achieved / PEAK_TFLOPS[dt_key], 4) if achieved == achieved else None,
                "traffic": traffic,
                "avg_ms": round(grav_ms, 4),
                "algorithmic": (f"{GRAVITY_FLOP_PER_PAIR} FLOP x N(N-1) ordered pairs per launch"
                                if args.gravity == "direct" else
                                "FP64 FLOP the tree kernels execute per launch (64 x "
                                "SQ_INSTS_VALU_FLOPS_FP64, rocprofv3 --pmc)")}
    per_kernel = {k: round(v / staged["_steps"], 4) for k, v in staged.items()
                  if not k.startswith("_")}
    state = sim.read_state(["agg_pos"])
    out = {
        "metric": METRIC, "value": round(value, 1), "unit": "sphere-steps/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": round(ms_per_step, 4),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f64" if prec == dem.PREC_FP64 else "f32-force/f64-state",
        "data": "synthetic",
        "config": {"workload": f"gravitational collapse, {w.n_agg} aggregates of 2-8 spheres "
                               f"({w.n_sph} spheres), ball at packing 0.15, G=1, softening 0.5, "
                               f"dt=5e-4, {'plain FP64' if prec == 0 else 'FP32-force'}"
                               + (", tree gravity (opening angle 0.5, leaves of 32)"
                                  if args.gravity == "tree" else "")
                               + (", per-target form of the exact sum"
                                  if args.gravity == "direct" and args.gravity_form == 2
                                  else ""),
                   "n_spheres": w.n_sph, "n_aggregates": w.n_agg, "contacts": state["n_pairs"]},
        "graph_replay_value": round(graph_value, 1),
        "timing": ("value: K steps launched as the step graph orders them, gravity on a "
                   "second stream beside the contact kernels, with HIP events around the "
                   "gravity stage on that stream (roofline.avg_ms); graph_replay_value: the "
                   "same steps as graph replays; kernel_ms_per_step: K more steps with an "
                   "event between consecutive kernels, run one after another "
                   f"({staged_ms:.4f} ms of kernels per step)"),
        "step_latency": step_latency,
        "kernel_ms_per_step": per_kernel,
        "roofline": roofline,
    }
    sim.close()
    if not args.no_extra and args.full_run_steps > 0:
        full_run(w, prec, args.full_run_steps, out)
    cfg0_run(inp["cfg0"], out)
    if not args.no_extra:
        extra_runs(args, inp, out, prec)
    if not args.no_cpu_baseline:
        log("cpu baseline (oracle) ...")
        out["cpu_baseline"] = cpu_baseline(inp, args.cpu_sample, args.cpu_seconds)
    print(json.dumps(out), flush=True)


def full_run(w, prec, steps, out):
    """The whole run the collapse configuration names (2,000 steps from
    rest), one graph replay per step, timed in ten chunks: sphere-steps/s
    over the run, and the step time and contact count as the cloud falls in."""
    from paper_2311_11322_amd import dem
    sf = dem.Sim(w.params, precision=prec)
    sf.add_workload(w)
    chunk = max(1, steps // 10)
    done, wall, trace = 0, 0.0, []
    while done < steps:
        k = min(chunk, steps - done)
        t = timed_steps(sf, k)
        wall += t
        done += k
        trace.append({"step": done, "ms_per_step": round(1e3 * t / k, 4),
                      "contacts": sf.counts()[2]})
    sf.close()
    out["full_run"] = {"workload": f"the collapse above, all {steps} steps from rest, "
                                   "graph replay",
                       "value": round(w.n_sph * steps / wall, 1), "unit": "sphere-steps/s",
                       "seconds": round(wall, 2), "trace": trace}
    log(f"full run: {out['full_run']['value']:.4g} sphere-steps/s over {steps} steps")


def cfg0_run(w0, out):
    """The contact-only periodic box (500 aggregates of 1-8 spheres, packing
    0.2, velocities N(0, 0.05), dt 1e-4), plain FP64, its whole 200-step run
    replayed as graphs after a t0 evaluation."""
    from paper_2311_11322_amd import dem
    s0 = dem.Sim(w0.params)
    s0.add_workload(w0)
    c0 = s0.counts()[2]
    wall = timed_steps(s0, w0.n_steps)
    out["cfg0"] = {"workload": f"periodic box, {w0.n_agg} aggregates of 1-8 spheres "
                               f"({w0.n_sph} spheres), packing 0.2, v ~ N(0, 0.05), dt=1e-4, "
                               f"{w0.n_steps} steps, plain FP64",
                   "value": round(w0.n_sph * w0.n_steps / wall, 1), "unit": "sphere-steps/s",
                   "ms_per_step": round(1e3 * wall / w0.n_steps, 4),
                   "contacts_at_t0": c0, "contacts_at_end": s0.counts()[2]}
    s0.close()
    log(f"cfg0: {out['cfg0']}")


def timed_steps(sim, steps):
    import torch
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    sim.step(steps)
    torch.cuda.synchronize()
    return time.perf_counter() - t0


def contact_path_run(args, inp, out):
    """The contact path alone on contact-dense periodic lattices (no
    gravity): every non-gravity kernel of the step, against the HBM roofline,
    at 125k spheres (launch-latency bound) and at 1M spheres."""
    from paper_2311_11322_amd import dem
    from paper_2311_11322_amd import workloads as W
    res = []
    for wl in inp["lattices"]:
        sl = dem.Sim(wl.params)
        sl.add_workload(wl)
        sl.step(2)
        wall = timed_steps(sl, args.steps)          # graph replay, no per-kernel events
        sl.set_profiling(True)
        timed_steps(sl, args.steps)
        pl = sl.profile()
        n_pairs = sl.counts()[2]
        sl.close()
        kms = {k: v / pl["_steps"] for k, v in pl.items() if not k.startswith("_") and k != "gravity"}
        contact_ms = sum(kms.values())
        zbar = 2.0 * n_pairs / wl.n_sph
        bytes_per_sphere = CONTACT_BYTES_FIXED + CONTACT_BYTES_PER_CONTACT * zbar
        gbs = bytes_per_sphere * wl.n_sph / (contact_ms * 1e-3) / 1e9
        res.append({
            "workload": f"periodic lattice of {wl.n_sph} unit spheres (dumbbells + lone), "
                        f"{n_pairs} contacts (z = {zbar:.2f}), FP64, no gravity"
                        + (", aggregates in Morton order of their cells"
                           if wl.notes.endswith("morton order") else ""),
            "value": round(wl.n_sph * args.steps / wall, 1), "unit": "sphere-steps/s",
            "ms_per_step": round(1e3 * wall / args.steps, 4),
            "kernel_ms_per_step": {k: round(v, 4) for k, v in kms.items()},
            "roofline": {"bound": "hbm", "achieved": round(gbs, 1), "peak": PEAK_HBM_GBS,
                         "unit": "GB/s", "frac": round(gbs / PEAK_HBM_GBS, 4),
                         "algorithmic": f"{CONTACT_BYTES_FIXED} B + {CONTACT_BYTES_PER_CONTACT} B "
                                        "x z per sphere-step over the summed contact-path "
                                        "kernel times"}})
        log(f"contact path: {res[-1]}")
    out["contact_path"] = res[0] if len(res) == 1 else res


def walled_runs(args, inp, out):
    """The box-filling profiling workload (6,400 unit spheres in a 40 x 40 x
    240 open-topped box under a uniform field; the first 10^4 steps of the
    fill, as profiled in the paper) for each aggregate shape, the member
    search ablation on it, many box fills batched in one engine, and the
    Brazil-nut set-up with shaken walls."""
    from paper_2311_11322_amd import dem, serve
    n_fill = args.fill_steps
    shapes = ("sphere", "dumbbell", "cube", "mixed")
    fills = inp["fills"]
    per_shape = {}
    prof = None
    for shape in shapes:
        wb = fills[shape]
        sb = dem.Sim(wb.params)
        sb.add_workload(wb)
        wall = timed_steps(sb, n_fill)
        per_shape[shape] = {"aggregates": wb.n_agg, "ms_per_step": round(1e3 * wall / n_fill, 4),
                            "contacts_at_end": sb.counts()[2]}
        if shape == "mixed":
            # per-kernel times over further steps, with an event around each kernel
            sb.set_profiling(True)
            timed_steps(sb, max(100, n_fill // 20))
            prof = sb.profile()
        sb.close()
    wm = fills["mixed"]
    abl = {}
    for scan in (0, 1):
        sa = dem.Sim(wm.params)
        sa.set_tuning(0, 1.0, scan)
        sa.add_workload(wm)
        abl[scan] = 1e3 * timed_steps(sa, n_fill // 5) / (n_fill // 5)
        sa.close()
    out["box_fill"] = {
        "workload": f"box filling, {wm.n_sph} unit spheres, 40x40x240 open box, g = 2 along -z, "
                    f"first {n_fill} steps from rest, FP64",
        "value": round(wm.n_sph * n_fill / (per_shape["mixed"]["ms_per_step"] * 1e-3 * n_fill), 1),
        "unit": "sphere-steps/s", "per_shape": per_shape,
        "kernel_ms_per_step_mixed": {k: round(v / prof["_steps"], 5) for k, v in prof.items()
                                     if not k.startswith("_")},
        "member_search_ablation": {"improved_ms_per_step": round(abl[0], 4),
                                   "original_ms_per_step": round(abl[1], 4),
                                   "speedup": round(abl[1] / abl[0], 3)}}
    log(f"box fill: {out['box_fill']}")
    # many box fills in one engine (seeds differ, mixed shapes)
    nb = args.box_batch
    if nb > 0:
        boxes = inp["boxes"]
        steps_b = max(50, n_fill // 20)
        rb = serve.run_batch(boxes, steps_b, dem.PREC_FP64, warmup=2)
        for s in rb["sims"]:
            s.close()
        out["box_fill"]["batched"] = {
            "boxes": nb, "spheres": rb["spheres"], "steps": steps_b,
            "value": round(rb["sphere_steps_per_s"], 1), "unit": "sphere-steps/s",
            "ms_per_step": round(rb["ms_per_step"], 4)}
        log(f"box fill batched: {out['box_fill']['batched']}")
    # Brazil-nut set-up, walls shaken at Froude number 3
    wn = inp["brazil"]
    sn = dem.Sim(wn.params)
    sn.add_workload(wn)
    sn.step(2)
    n_bne = max(200, n_fill // 10)
    wall = timed_steps(sn, n_bne)
    sn.set_profiling(True)
    timed_steps(sn, max(100, n_bne // 4))
    pn = sn.profile()
    out["brazil_nut"] = {
        "workload": f"intruder R=6 among {wn.n_sph - 1} grain spheres ({wn.n_agg - 1} aggregates), "
                    "40x40 box, all walls shaken, Froude 3, FP64",
        "value": round(wn.n_sph * n_bne / wall, 1), "unit": "sphere-steps/s",
        "ms_per_step": round(1e3 * wall / n_bne, 4),
        "kernel_ms_per_step": {k: round(v / pn["_steps"], 5) for k, v in pn.items()
                               if not k.startswith("_")}}
    sn.close()
    log(f"brazil nut: {out['brazil_nut']}")


def tree_run(w, steps, theta=0.5, leaf=32, order=4):
    """Tree gravity (FP64) on a workload: ms per step and gravity ms."""
    from paper_2311_11322_amd import dem
    prm = dict(w.params, gravity_tree=1, theta=theta, tree_leaf=leaf, tree_order=order)
    st = dem.Sim(prm)
    st.add_workload(w)
    st.step(1)
    wall = timed_steps(st, steps)
    st.set_profiling(True)
    timed_steps(st, steps)
    pt = st.profile()
    st.close()
    return {"value": round(w.n_sph * steps / wall, 1), "unit": "sphere-steps/s",
            "ms_per_step": round(1e3 * wall / steps, 4),
            "gravity_ms": round(pt["gravity"] / pt["_steps"], 4),
            "theta": theta, "leaf": leaf, "order": order}


def big_run(args, out, wbig):
    """FP32-force gravity at 500k spheres (100,000 aggregates): a few steps."""
    from paper_2311_11322_amd import dem
    sb = dem.Sim(wbig.params, precision=dem.PREC_FP32_FORCE)
    sb.add_workload(wbig)
    sb.step(1)
    nbig = 3
    wall = timed_steps(sb, nbig)
    sb.set_profiling(True)
    timed_steps(sb, nbig)
    pb = sb.profile()
    sb.close()
    gb_ms = pb["gravity"] / pb["_steps"]
    nb = wbig.n_sph
    achb = GRAVITY_FLOP_PER_PAIR * nb * (nb - 1) / (gb_ms * 1e-3) / 1e12
    out["fp32_force_500k"] = {
        "workload": f"collapse, {wbig.n_agg} aggregates of 2-8 spheres ({nb} spheres), FP32-force",
        "value": round(nb * nbig / wall, 1), "unit": "sphere-steps/s",
        "ms_per_step": round(1e3 * wall / nbig, 3), "gravity_ms": round(gb_ms, 3),
        "gravity_frac_of_fp32_peak": round(achb / PEAK_TFLOPS["fp32"], 4)}
    log(f"fp32-force 500k: {out['fp32_force_500k']}")
    out["tree_500k"] = dict(tree_run(wbig, 5, leaf=32),
                            workload=f"collapse, {nb} spheres, tree gravity (multipoles to "
                                     "hexadecapole order), FP64")
    log(f"tree 500k: {out['tree_500k']}")


def _one_at_a_time(piles, steps, precision, cache):
    """Sphere-steps/s of the piles run one system at a time (each after a
    warm-up step), summed over the piles' timed steps; each pile with the
    tuning the autotuner picks for its size (one measurement per shape
    bucket, cached)."""
    from paper_2311_11322_amd import dem, serve
    t_sum = 0.0
    for p in piles:
        tune = serve.autotune([p], precision, steps=2, cell_scales=(1.0, 1.5), cache=cache)
        sp = dem.Sim(p.params, precision=precision)
        sp.set_tuning(tune["gravity_tile"], tune["cell_scale"])
        sp.set_forcing(p.params["spin_dw"])
        sp.add_workload(p)
        sp.step(1)
        t_sum += timed_steps(sp, steps)
        sp.close()
    return sum(p.n_sph for p in piles) * steps / t_sum


def batched_run(args, inp, out, plain=True):
    """The spin-up piles (Sec. 4.1 shape): each cloud first collapsed and
    settled on the GPU (all piles in one engine, FP32-force, no forcing),
    then spun up from its settled state.  Timed in one engine in the
    FP32-force form with the tuning the autotuner picks (or, for a profiler
    run of this section alone, the --gravity-tile / --cell-scale given);
    per-kernel times of the batched step give the contact path's HBM
    fraction.  With ``plain``, also the same piles batched in FP64 and one
    at a time in both forms (the gain of batching apart from that of the
    precision), and the whole spin-up campaign to each pile's failure (its
    bulk radius grown by 5 %, the device's stop rule).  Returns the tuning."""
    from paper_2311_11322_amd import dem, serve
    clouds = inp["piles"]
    n_tot = sum(p.n_sph for p in clouds)
    t = time.perf_counter()
    piles = serve.settle(clouds, args.settle_steps, dem.PREC_FP32_FORCE)
    t_settle = time.perf_counter() - t
    log(f"{len(piles)} piles, {n_tot} spheres, settled over {args.settle_steps} steps "
        f"in {t_settle:.1f} s")
    if not plain and args.gravity_tile:
        tune = {"gravity_tile": args.gravity_tile, "cell_scale": args.cell_scale}
    else:
        tune = serve.autotune(piles, dem.PREC_FP32_FORCE, steps=3)
    log(f"tuning: tile {tune['gravity_tile']}, cell scale {tune['cell_scale']}")
    bsteps = max(5, args.steps // 2)
    batch = serve.run_batch(piles, bsteps, dem.PREC_FP32_FORCE,
                            tuning=(tune["gravity_tile"], tune["cell_scale"]), warmup=2,
                            profile=True)
    for s in batch["sims"]:
        s.close()
    prof = batch["profile"]
    kms = {k: v / prof["_steps"] for k, v in prof.items() if not k.startswith("_")}
    contact_ms = sum(v for k, v in kms.items() if k != "gravity")
    zbar = 2.0 * batch["contacts"] / n_tot
    gbs = (CONTACT_BYTES_FIXED + CONTACT_BYTES_PER_CONTACT * zbar) * n_tot / (contact_ms * 1e-3) / 1e9
    out["batched"] = {
        "workload": f"{len(piles)} independent spin-up piles, 500-20000 spheres each "
                    f"(log-uniform), {n_tot} spheres, each a cloud at packing 0.15 collapsed and "
                    f"settled on the GPU for {args.settle_steps} steps, spin ramp 1e-6 rad/step^2, "
                    "FP32-force, one engine",
        "value": round(batch["sphere_steps_per_s"], 1), "unit": "sphere-steps/s",
        "ms_per_step": round(batch["ms_per_step"], 4),
        "gravity_pairs_per_step": batch["sum_n2"],
        "contacts": batch["contacts"],
        "settle_seconds": round(t_settle, 1),
        "kernel_ms_per_step": {k: round(v, 4) for k, v in kms.items()},
        "contact_path_roofline": {
            "bound": "hbm", "achieved": round(gbs, 1), "peak": PEAK_HBM_GBS, "unit": "GB/s",
            "frac": round(gbs / PEAK_HBM_GBS, 4),
            "algorithmic": f"{CONTACT_BYTES_FIXED} B + {CONTACT_BYTES_PER_CONTACT} B x z per "
                           f"sphere-step (z = {zbar:.2f}) over the summed non-gravity kernel times"},
        "tuning": {"gravity_tile": tune["gravity_tile"], "cell_scale": tune["cell_scale"],
                   "candidates": len(tune.get("candidates", []))}}
    if plain:
        b64 = serve.run_batch(piles, bsteps, dem.PREC_FP64, warmup=2)
        for s in b64["sims"]:
            s.close()
        cache = {}
        one64 = _one_at_a_time(piles, bsteps, dem.PREC_FP64, cache)
        one32 = _one_at_a_time(piles, bsteps, dem.PREC_FP32_FORCE, cache)
        v32 = batch["sphere_steps_per_s"]
        v64 = b64["sphere_steps_per_s"]
        out["batched"].update(
            batched_fp64=round(v64, 1),
            plain_fp64_one_pile_at_a_time=round(one64, 1),
            fp32_force_one_pile_at_a_time=round(one32, 1),
            speedup_vs_plain=round(v32 / one64, 2),
            gain_of_batching={"fp64": round(v64 / one64, 2), "fp32_force": round(v32 / one32, 2)},
            gain_of_precision={"batched": round(v32 / v64, 2),
                               "one_at_a_time": round(one32 / one64, 2)})
        camp = serve.spin_campaign(piles, dem.PREC_FP32_FORCE,
                                   (tune["gravity_tile"], tune["cell_scale"]), stop_growth=1.05,
                                   max_steps=args.campaign_steps)
        import numpy as np
        crit = []
        for p, wf in zip(piles, camp["spin_at_failure"]):
            if wf is None:
                continue
            m = p.mass
            com = (m[:, None] * p.pos).sum(0) / m.sum()
            R = math.sqrt(5.0 / 3.0 * float((m * ((p.pos - com) ** 2).sum(1)).sum() / m.sum()))
            rho = float(m.sum()) / (4.0 / 3.0 * math.pi * R ** 3)
            crit.append(wf / math.sqrt(4.0 * math.pi * p.params["G"] * rho / 3.0))
        stf = [d for d in camp["steps_to_failure"] if d is not None]
        out["batched"]["spin_campaign"] = {
            "piles": camp["piles"], "stopped": camp["stopped"], "steps": camp["steps"],
            "seconds": round(camp["seconds"], 2),
            "sphere_steps_per_s": round(camp["sphere_steps_per_s"], 1),
            "steps_to_failure_p50": float(np.percentile(stf, 50)) if stf else None,
            "steps_to_failure_max": max(stf) if stf else None,
            "spin_at_failure_over_nominal_critical_p50":
                round(float(np.percentile(crit, 50)), 3) if crit else None}
    log(f"batched: {out['batched']}")
    return tune


def extra_runs(args, inp, out, prec):
    """The FP32-force form on the same collapse, the batched spin-up piles
    (plain FP64 one pile at a time vs FP32-force batched in one engine) and
    a served request stream."""
    from paper_2311_11322_amd import dem, serve
    w = inp["collapse"]
    # -- FP32-force form at 125k spheres
    if prec == dem.PREC_FP64:
        s32 = dem.Sim(w.params, precision=dem.PREC_FP32_FORCE)
        s32.add_workload(w)
        s32.step(2)
        s32.set_profiling(True)
        wall = timed_steps(s32, args.steps)
        p32 = s32.profile()
        s32.close()
        g_ms = p32["gravity"] / p32["_steps"]
        ach = GRAVITY_FLOP_PER_PAIR * w.n_sph * (w.n_sph - 1) / (g_ms * 1e-3) / 1e12
        out["fp32_force"] = {"value": round(w.n_sph * args.steps / wall, 1),
                             "ms_per_step": round(1e3 * wall / args.steps, 4),
                             "gravity_ms": round(g_ms, 4),
                             "gravity_frac_of_fp32_peak": round(ach / PEAK_TFLOPS["fp32"], 4)}
        log(f"fp32-force: {out['fp32_force']}")
    if prec == dem.PREC_FP64:
        out["tree"] = dict(tree_run(w, args.steps, leaf=32),
                           workload=f"collapse, {w.n_sph} spheres, tree gravity (multipoles to "
                                    "hexadecapole order), FP64")
        log(f"tree: {out['tree']}")
    contact_path_run(args, inp, out)
    # -- the paper's efficiency experiment: original (full-scan) vs improved
    #    (contiguous) member search, on its collapse shape (2e4 spheres)
    wa = inp["ablation"]
    abl = {}
    for scan in (0, 1):
        sa = dem.Sim(wa.params)
        sa.set_tuning(0, 1.0, scan)
        sa.add_workload(wa)
        sa.step(2)
        sa.set_profiling(True)
        wall = timed_steps(sa, 10)
        pa = sa.profile()
        sa.close()
        abl[scan] = (1e3 * wall / 10, pa["reduce"] / pa["_steps"])
    out["member_search_ablation"] = {
        "workload": f"collapse, {wa.n_agg} aggregates of 1-8 spheres ({wa.n_sph} spheres), FP64",
        "improved_ms_per_step": round(abl[0][0], 4), "original_ms_per_step": round(abl[1][0], 4),
        "improved_reduce_ms": round(abl[0][1], 4), "original_reduce_ms": round(abl[1][1], 4),
        "speedup": round(abl[1][0] / abl[0][0], 3)}
    log(f"member search ablation: {out['member_search_ablation']}")
    walled_runs(args, inp, out)
    tune = batched_run(args, inp, out)
    # -- served stream
    if args.requests > 0:
        reqs = inp["requests"]
        srv = serve.Server(64 << 30, precision=dem.PREC_FP32_FORCE, chunk_steps=50,
                           tuning=(tune["gravity_tile"], tune["cell_scale"]))
        st = srv.run(reqs)
        out["served"] = {
            "workload": f"{len(reqs)} requests, Poisson arrivals at 20/s, collapse, spin-up or flyby, "
                        "1k-50k spheres, 100-5000 steps, FP32-force, 64 GiB admission budget",
            "p50_latency_s": round(st["p50_latency_s"], 3),
            "p99_latency_s": round(st["p99_latency_s"], 3),
            "sphere_steps_per_s": round(st["sphere_steps_per_s"], 1),
            "offered_rate_per_s": 20.0,
            "service_rate_per_s": round(st["service_rate_per_s"], 2),
            "makespan_s": round(st["makespan_s"], 2), "completed": st["completed"],
            "failed": st["failed"]}
        log(f"served: {out['served']}")
        # the same stream under shortest-remaining-work-first chunks (up to
        # 1e10 gravity pairs per step attached at a time)
        reqs_s = [serve.Request(r.rid, r.kind, r.workload, r.steps, r.arrival) for r in reqs]
        srv_s = serve.Server(64 << 30, precision=dem.PREC_FP32_FORCE, chunk_steps=50,
                             tuning=(tune["gravity_tile"], tune["cell_scale"]), policy="srpt",
                             pairs_per_step_cap=1e10)
        st_s = srv_s.run(reqs_s)
        out["served_srpt"] = {
            "workload": "the same requests and arrivals; each chunk steps the runs with the least "
                        "remaining work (spheres^2 x steps) up to 1e10 gravity pairs per step",
            "p50_latency_s": round(st_s["p50_latency_s"], 3),
            "p99_latency_s": round(st_s["p99_latency_s"], 3),
            "sphere_steps_per_s": round(st_s["sphere_steps_per_s"], 1),
            "service_rate_per_s": round(st_s["service_rate_per_s"], 2),
            "makespan_s": round(st_s["makespan_s"], 2), "completed": st_s["completed"],
            "failed": st_s["failed"]}
        log(f"served (srpt): {out['served_srpt']}")
        # the first half of the same requests offered at 80 % of the measured
        # service rate (same workloads, arrival times stretched)
        rate2 = round(0.8 * st["service_rate_per_s"], 2)
        if rate2 > 0:
            half = reqs[: max(1, len(reqs) // 2)]
            reqs2 = [serve.Request(r.rid, r.kind, r.workload, r.steps, r.arrival * 20.0 / rate2)
                     for r in half]
            srv2 = serve.Server(64 << 30, precision=dem.PREC_FP32_FORCE, chunk_steps=50,
                                tuning=(tune["gravity_tile"], tune["cell_scale"]))
            st2 = srv2.run(reqs2)
            out["served_sustainable"] = {
                "workload": f"the first {len(reqs2)} of those requests, Poisson arrivals at "
                            f"{rate2}/s (80 % of the measured service rate)",
                "p50_latency_s": round(st2["p50_latency_s"], 3),
                "p99_latency_s": round(st2["p99_latency_s"], 3),
                "sphere_steps_per_s": round(st2["sphere_steps_per_s"], 1),
                "offered_rate_per_s": rate2,
                "service_rate_per_s": round(st2["service_rate_per_s"], 2),
                "makespan_s": round(st2["makespan_s"], 2), "completed": st2["completed"],
                "failed": st2["failed"]}
            log(f"served at a sustainable rate: {out['served_sustainable']}")
    # -- FP32-force gravity at 500k spheres
    if "big" in inp:
        big_run(args, out, inp["big"])


if __name__ == "__main__":
    main()
