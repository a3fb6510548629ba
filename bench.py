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
    # (precision, spheres, default tile): (bytes per launch, source_hash("kernels_gravity.hip"))
    ("fp64", 124958, 512): (2299.3e6, "4819b4985e946fcb"),
    ("fp32", 124958, 1024): (539.8e6, "4819b4985e946fcb"),
}


# Executed FP64 FLOP of the tree walk per launch (64 x SQ_INSTS_VALU_FLOPS_FP64
# from rocprofv3 --pmc), for the tree run's roofline; valid only for the
# gravity source it was measured on.
MEASURED_TREE_FLOP = {
    # (spheres, opening angle, leaf, order): (FLOP per launch, source_hash("kernels_tree.hip"))
    (124958, 0.5, 32, 4): (3.665e10, "823728918897e80c"),
    (999660, 0.5, 32, 4): (3.844e11, "823728918897e80c"),
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


def cpu_baseline(w, n_sample, seconds_cap):
    """FP64 oracle on the host: force evaluation (brute-force contacts and
    direct-sum gravity at full N) of a sample of spheres, scaled to
    sphere-steps/s (one step evaluates every sphere at the same cost)."""
    import numpy as np
    import oracle as O
    o = O.Oracle(w.params).add_workload(w, evaluate=False)
    rng = np.random.default_rng(0)
    idx = np.sort(rng.choice(w.n_sph, n_sample, replace=False))
    done, t_used = 0, 0.0
    chunk = 64
    while done < n_sample and t_used < seconds_cap:
        sl = idx[done:done + chunk]
        t0 = time.perf_counter()
        o.eval_subset(sl)
        t_used += time.perf_counter() - t0
        done += len(sl)
    per_sphere = t_used / done
    model = ""
    try:
        with open("/proc/cpuinfo") as f:
            model = next((ln.split(":", 1)[1].strip() for ln in f if ln.startswith("model name")), "")
    except OSError:
        pass
    return {"value": 1.0 / per_sphere, "unit": "sphere-steps/s", "cores": 1, "kind": "oracle",
            "sample": f"t0 force evaluation of {done} of {w.n_sph} spheres at full N "
                      f"(brute-force contacts + direct-sum gravity, single thread, "
                      f"{t_used:.1f} s), scaled by N to a whole step",
            "host_cores_allowed": len(os.sched_getaffinity(0)), "cpu_model": model}


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
    ap.add_argument("--cell-scale", type=float, default=1.0)
    ap.add_argument("--cpu-sample", type=int, default=4096)
    ap.add_argument("--cpu-seconds", type=float, default=20.0)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-extra", action="store_true",
                    help="only the headline workload (skip FP32-force, batched and served)")
    ap.add_argument("--piles", type=int, default=256)
    ap.add_argument("--big-agg", type=int, default=100000,
                    help="aggregates of the FP32-force 500k-sphere gravity run (0: skip)")
    ap.add_argument("--requests", type=int, default=200)
    ap.add_argument("--lattice-sides", type=int, nargs="+", default=[50, 100],
                    help="lattice edge lengths of the contact-path runs (n^3 spheres)")
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
    from paper_2311_11322_amd import dem
    from paper_2311_11322_amd import workloads as W
    if args.only:
        dem.lib()
        part = {}
        workers = min(16, len(os.sched_getaffinity(0)))
        if args.only == "contact_path":
            contact_path_run(args, part)
        elif args.only == "batched":
            batched_run(args, part, workers, plain=False)
        else:
            walled_runs(args, part, workers)
        print(json.dumps(part), flush=True)
        return

    t = time.time()
    w = W.collapse_cloud(1, n_agg=args.n_agg)
    log(f"workload: {w.n_agg} aggregates, {w.n_sph} spheres ({time.time() - t:.1f} s to place)")
    prec = dem.PREC_FP32_FORCE if args.precision == "fp32" else dem.PREC_FP64
    if args.gravity == "tree":
        w.params.update(gravity_tree=1, theta=0.5, tree_leaf=32, tree_order=4)
    torch.cuda.init()
    alloc = dem.TorchAllocator(0)
    sim = dem.Sim(w.params, precision=prec, allocator=alloc, stream=dem.torch_stream())
    sim.set_tuning(args.gravity_tile, args.cell_scale)
    sim.add_workload(w)
    log("added; warmup", args.warmup)
    sim.step(args.warmup)
    torch.cuda.synchronize()

    # timed region: K steps, an event around every kernel on the library's stream
    sim.set_profiling(True)
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

    # same work replayed as one HIP graph per step (no per-kernel events)
    torch.cuda.synchronize()
    g0 = time.perf_counter()
    sim.step(args.steps)
    torch.cuda.synchronize()
    graph_value = w.n_sph * args.steps / (time.perf_counter() - g0)

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
    meas = MEASURED_TRAFFIC.get((dt_key, n, tile))
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
    per_kernel = {k: round(v / prof["_steps"], 4) for k, v in prof.items() if not k.startswith("_")}
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
                                  if args.gravity == "tree" else ""),
                   "n_spheres": w.n_sph, "n_aggregates": w.n_agg, "contacts": state["n_pairs"]},
        "graph_replay_value": round(graph_value, 1),
        "step_latency": step_latency,
        "kernel_ms_per_step": per_kernel,
        "roofline": roofline,
    }
    sim.close()
    if not args.no_extra:
        extra_runs(args, w, out, prec)
    if not args.no_cpu_baseline:
        log("cpu baseline (oracle) ...")
        out["cpu_baseline"] = cpu_baseline(w, args.cpu_sample, args.cpu_seconds)
    print(json.dumps(out), flush=True)


def timed_steps(sim, steps):
    import torch
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    sim.step(steps)
    torch.cuda.synchronize()
    return time.perf_counter() - t0


def _box(seed_shape):
    from paper_2311_11322_amd import workloads as W
    seed, shape = seed_shape
    return W.box_fill(seed=seed, shape=shape)


def contact_path_run(args, out):
    """The contact path alone on contact-dense periodic lattices (no
    gravity): every non-gravity kernel of the step, against the HBM roofline,
    at 125k spheres (launch-latency bound) and at 1M spheres."""
    from paper_2311_11322_amd import dem
    from paper_2311_11322_amd import workloads as W
    res = []
    for n_side in args.lattice_sides:
        wl = W.dense_lattice(n_side=n_side)
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
                        f"{n_pairs} contacts (z = {zbar:.2f}), FP64, no gravity",
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


def walled_runs(args, out, workers):
    """The box-filling profiling workload (6,400 unit spheres in a 40 x 40 x
    240 open-topped box under a uniform field; the first 10^4 steps of the
    fill, as profiled in the paper) for each aggregate shape, the member
    search ablation on it, many box fills batched in one engine, and the
    Brazil-nut set-up with shaken walls."""
    from concurrent.futures import ProcessPoolExecutor
    from paper_2311_11322_amd import dem, serve
    from paper_2311_11322_amd import workloads as W
    n_fill = args.fill_steps
    shapes = ("sphere", "dumbbell", "cube", "mixed")
    with ProcessPoolExecutor(max_workers=max(1, min(workers, 8))) as ex:
        fills = dict(zip(shapes, ex.map(_box, [(8, s) for s in shapes])))
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
        with ProcessPoolExecutor(max_workers=max(1, workers)) as ex:
            boxes = list(ex.map(_box, [(100 + k, "mixed") for k in range(nb)]))
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
    wn = W.brazil_nut()
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


def _big_collapse(n_agg):
    from paper_2311_11322_amd import workloads as W
    return W.collapse_cloud(2, n_agg=n_agg)


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


def batched_run(args, out, workers, plain=True):
    """The spin-up piles in one engine, FP32-force, with the tuning the
    autotuner picks (or, for a profiler run of this section alone, the
    --gravity-tile / --cell-scale given); with ``plain``, also the same piles
    in plain FP64 one at a time.  Returns the tuning."""
    from paper_2311_11322_amd import dem, serve
    from paper_2311_11322_amd import workloads as W
    t = time.time()
    piles = W.pile_batch(seed=3, n_piles=args.piles, workers=workers)
    n_tot = sum(p.n_sph for p in piles)
    log(f"{len(piles)} piles, {n_tot} spheres ({time.time() - t:.1f} s to place)")
    if not plain and args.gravity_tile:
        tune = {"gravity_tile": args.gravity_tile, "cell_scale": args.cell_scale}
    else:
        tune = serve.autotune(piles, dem.PREC_FP32_FORCE, steps=3)
    log(f"tuning: tile {tune['gravity_tile']}, cell scale {tune['cell_scale']}")
    bsteps = max(5, args.steps // 2)
    batch = serve.run_batch(piles, bsteps, dem.PREC_FP32_FORCE,
                            tuning=(tune["gravity_tile"], tune["cell_scale"]), warmup=2)
    for s in batch["sims"]:
        s.close()
    out["batched"] = {
        "workload": f"{len(piles)} independent spin-up piles, 500-20000 spheres each "
                    f"(log-uniform), {n_tot} spheres, FP32-force, one engine",
        "value": round(batch["sphere_steps_per_s"], 1), "unit": "sphere-steps/s",
        "ms_per_step": round(batch["ms_per_step"], 4),
        "gravity_pairs_per_step": batch["sum_n2"],
        "tuning": {"gravity_tile": tune["gravity_tile"], "cell_scale": tune["cell_scale"]}}
    if plain:
        # the same piles, FP64, one at a time
        plain_time = 0.0
        for p in piles:
            sp = dem.Sim(p.params)
            sp.add_workload(p)
            sp.set_forcing(p.params["spin_dw"])
            sp.step(1)
            plain_time += timed_steps(sp, bsteps)
            sp.close()
        plain_value = n_tot * bsteps / plain_time
        out["batched"].update(
            plain_fp64_one_pile_at_a_time=round(plain_value, 1),
            speedup_vs_plain=round(batch["sphere_steps_per_s"] / plain_value, 2))
    log(f"batched: {out['batched']}")
    return tune


def extra_runs(args, w, out, prec):
    """The FP32-force form on the same collapse, the batched spin-up piles
    (plain FP64 one pile at a time vs FP32-force batched in one engine) and
    a served request stream."""
    import numpy as np
    import torch
    from paper_2311_11322_amd import dem, serve
    from paper_2311_11322_amd import workloads as W
    workers = min(16, len(os.sched_getaffinity(0)))
    from concurrent.futures import ProcessPoolExecutor
    big_pool = ProcessPoolExecutor(max_workers=1) if args.big_agg > 0 else None
    big_fut = big_pool.submit(_big_collapse, args.big_agg) if big_pool else None
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
    contact_path_run(args, out)
    # -- the paper's efficiency experiment: original (full-scan) vs improved
    #    (contiguous) member search, on its collapse shape (2e4 spheres)
    wa = W.collapse_cloud(seed=5, n_agg=4444, cmin=1, cmax=8)
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
    walled_runs(args, out, workers)
    tune = batched_run(args, out, workers)
    # -- served stream
    if args.requests > 0:
        t = time.time()
        reqs = serve.request_stream(seed=4, n_requests=args.requests, rate_per_s=20.0,
                                    workers=workers)
        log(f"{len(reqs)} requests generated ({time.time() - t:.1f} s)")
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
    # -- FP32-force gravity at 500k spheres, placed in the background meanwhile
    if big_fut is not None:
        t = time.time()
        wbig = big_fut.result()
        big_pool.shutdown()
        log(f"big collapse: {wbig.n_sph} spheres (waited {time.time() - t:.1f} s)")
        big_run(args, out, wbig)


if __name__ == "__main__":
    main()
