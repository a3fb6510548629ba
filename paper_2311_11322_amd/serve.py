"""Batched and served DEM runs on one GPU.

* :func:`run_batch` steps many independent piles together through one
  engine (every kernel of a step covers all piles; one HIP graph per step).
* :class:`Server` is a continuous-batching request loop: requests arrive over
  time, are admitted while the engine's HBM budget allows (footprint from the
  library), join the running batch at the next chunk boundary, and leave it
  when their step count is reached; latency is completion minus arrival.
  Policy "fifo" steps every admitted run in every chunk; policy "srpt" steps,
  chunk by chunk, the runs with the least remaining work (spheres^2 x steps
  left) up to a cap on gravity pairs per step, the others staying resident
  on the device, detached, until they are among the shortest again.

All stepping runs in the HIP library; this module only schedules.
"""
from __future__ import annotations

import collections
import dataclasses
import math
import time
from typing import Dict, List, Optional, Sequence

import numpy as np

from . import dem


@dataclasses.dataclass
class Request:
    rid: int
    kind: str                       # "collapse", "spinup" or "flyby"
    workload: object                # workloads.Workload
    steps: int
    arrival: float                  # seconds after the stream starts
    admitted: Optional[float] = None
    done: Optional[float] = None
    status: int = 0
    result: Optional[Dict] = None

    @property
    def latency(self) -> Optional[float]:
        return None if self.done is None else self.done - self.arrival


def make_sim(w, precision: int, tuning=None, allocator=None, stream=None) -> dem.Sim:
    """A system for a workload: tuning, forcing (spin-up, perturber), then the
    aggregates (so the perturber's t0 acceleration is evaluated)."""
    sim = dem.Sim(w.params, precision=precision, allocator=allocator, stream=stream)
    if tuning:
        sim.set_tuning(*tuning)
    pert = w.params.get("perturber")
    stop = float(w.params.get("stop_growth", 0.0))
    if w.params.get("spin_dw", 0.0) or pert or stop:
        if pert:
            sim.set_forcing(w.params.get("spin_dw", 0.0), pert[0], pert[1], pert[2],
                            stop_growth=stop)
        else:
            sim.set_forcing(w.params.get("spin_dw", 0.0), stop_growth=stop)
    sim.add_workload(w)
    return sim


def settle(workloads: Sequence, steps: int, precision: int = dem.PREC_FP32_FORCE,
           tuning=None) -> List:
    """Self-gravitating clouds collapsed and settled together in one engine
    (no forcing), then each made into a new workload from its settled state:
    sphere centres, centre-of-mass velocities and space-frame spins, the
    forcing of the original kept.  Deterministic: the engine's result for a
    pile does not depend on the rest of the batch."""
    import copy
    quiet = []
    for w in workloads:
        q = copy.copy(w)
        q.params = {k: v for k, v in w.params.items()
                    if k not in ("spin_dw", "stop_growth", "perturber")}
        quiet.append(q)
    eng = dem.Engine(1 << 40)
    sims = [make_sim(q, precision, tuning) for q in quiet]
    for sm in sims:
        eng.attach(sm)
    code = eng.step(steps)
    if code != dem.DEM_OK:
        raise dem.DemError(code, "settling failed")
    out = []
    for w, sm in zip(workloads, sims):
        eng.detach(sm)
        st = sm.read_state(["sph_pos", "agg_vel", "agg_spin"])
        sm.close()
        n = copy.copy(w)
        n.pos, n.agg_vel, n.agg_spin = st["sph_pos"], st["agg_vel"], st["agg_spin"]
        n.params = dict(w.params)
        n.notes = (w.notes + f"; settled {steps} steps").lstrip("; ")
        out.append(n)
    eng.close()
    return out


def spin_campaign(workloads: Sequence, precision: int = dem.PREC_FP32_FORCE, tuning=None,
                  stop_growth: float = 1.05, max_steps: int = 20000, chunk: int = 100) -> Dict:
    """Spin-up of every pile in one engine until each one's stop rule fires
    (its bulk radius grown by ``stop_growth``; Sec. 4.1): the steps to
    failure and spin at failure of each pile, and the throughput of the
    campaign in sphere-steps of running piles per second."""
    import copy
    ws = []
    for w in workloads:
        c = copy.copy(w)
        c.params = dict(w.params, stop_growth=stop_growth)
        ws.append(c)
    eng = dem.Engine(1 << 40)
    sims = [make_sim(w, precision, tuning) for w in ws]
    for sm in sims:
        eng.attach(sm)
    done = [None] * len(sims)
    steps, t_run = 0, 0.0
    while steps < max_steps and any(d is None for d in done):
        t0 = time.perf_counter()
        code = eng.step(chunk)
        t_run += time.perf_counter() - t0
        if code != dem.DEM_OK:
            raise dem.DemError(code, "spin-up failed")
        steps += chunk
        for k, sm in enumerate(sims):
            if done[k] is None and sm.status() == dem.DEM_STOPPED:
                # steps committed before the stopping step, plus that step
                done[k] = sm.read_state(["agg_mass"])["step"] + 1
    # sphere-steps evaluated: each pile up to and including its stopping step
    sphere_steps = sum(w.n_sph * (steps if d is None else d) for w, d in zip(ws, done))
    for sm in sims:
        eng.detach(sm)
        sm.close()
    eng.close()
    fail = [d for d in done if d is not None]
    return {"piles": len(ws), "stopped": len(fail), "steps": steps, "seconds": t_run,
            "steps_to_failure": done,
            "spin_at_failure": [None if d is None else d * w.params["spin_dw"]
                                for d, w in zip(done, ws)],
            "sphere_steps_per_s": sphere_steps / t_run if t_run > 0 else 0.0}


def add_flyby(w, mass_ratio: float = 1000.0, periapsis_radii: float = 3.0,
              start_factor: float = 3.0, ecc: float = 2.0) -> None:
    """Give a pile a tidal perturber: a point mass of ``mass_ratio`` pile
    masses on an inbound hyperbola (eccentricity ``ecc``) with periapsis
    ``periapsis_radii`` bulk radii from the pile's centre of mass, starting at
    ``start_factor`` periapses."""
    from . import workloads as W
    M = float(w.mass.sum())
    com = (w.mass[:, None] * w.pos).sum(0) / M
    r2 = float((w.mass * ((w.pos - com) ** 2).sum(1)).sum() / M)
    R = math.sqrt(5.0 / 3.0 * r2)
    pos, vel = W.flyby_orbit(M, mass_ratio * M, periapsis_radii * R, ecc=ecc,
                             start_factor=start_factor, G=w.params["G"])
    w.params["perturber"] = (mass_ratio * M, pos + com, vel)


def bulk_radius(sim: dem.Sim) -> float:
    """Uniform-sphere equivalent radius sqrt(5/3 <|r - r_com|^2>_m) of the
    aggregate centres (the disruption diagnostic of the spin-up test)."""
    st = sim.read_state(["agg_pos", "agg_mass"])
    m = st["agg_mass"]
    r = st["agg_pos"]
    com = (m[:, None] * r).sum(0) / m.sum()
    return math.sqrt(5.0 / 3.0 * float((m * ((r - com) ** 2).sum(1)).sum() / m.sum()))


def run_batch(workloads: Sequence, steps: int, precision: int = dem.PREC_FP32_FORCE,
              tuning=None, budget_bytes: int = 1 << 40, warmup: int = 1,
              profile: bool = False) -> Dict:
    """Step every workload ``steps`` times in one engine; returns timing.
    dem_engine_step returns after the device work is complete."""
    eng = dem.Engine(budget_bytes)
    sims = [make_sim(w, precision, tuning) for w in workloads]
    for s in sims:
        eng.attach(s)
    if warmup:
        code = eng.step(warmup)
        if code != dem.DEM_OK:
            raise dem.DemError(code, "warm-up step failed")
    t0 = time.perf_counter()
    code = eng.step(steps)
    wall = time.perf_counter() - t0
    n_sph = sum(w.n_sph for w in workloads)
    out = {"wall_s": wall, "ms_per_step": 1e3 * wall / steps, "spheres": n_sph,
           "sphere_steps_per_s": n_sph * steps / wall, "status": code,
           "sum_n2": float(sum(float(w.n_sph) ** 2 for w in workloads))}
    if profile:
        # per-kernel times over further steps (an event between kernels)
        eng.set_profiling(True)
        eng.step(steps)
        out["profile"] = eng.profile()
        eng.set_profiling(False)
        out["contacts"] = sum(s.counts()[2] for s in sims)
    for s in sims:
        eng.detach(s)
    out["sims"] = sims
    eng.close()
    return out


_TUNE_CACHE: Dict = {}


def shape_bucket(workloads: Sequence, precision: int):
    """What the tuning of a batch depends on: precision, gravity kind, the
    number of piles and the total and largest sphere counts, each rounded to
    a power of two."""
    n = [w.n_sph for w in workloads]
    grav = "tree" if any(w.params.get("gravity_tree") for w in workloads) else (
        "direct" if any(w.params.get("G", 0.0) != 0.0 for w in workloads) else "none")
    b = lambda x: int(round(math.log2(max(1, x))))
    return (int(precision), grav, b(len(n)), b(sum(n)), b(max(n)))


def autotune(workloads: Sequence, precision: int, steps: int = 3,
             cell_scales=(1.0, 1.25, 1.5, 2.0), tiles=None, cache: Optional[Dict] = None) -> Dict:
    """Pick the gravity tile and cell scale that minimise the measured step
    time of this batch (a few steps per candidate).  The choice is cached
    per shape bucket (``shape_bucket``): a later batch of the same shape
    reuses it without measuring."""
    cache = _TUNE_CACHE if cache is None else cache
    key = shape_bucket(workloads, precision)
    if key in cache:
        return dict(cache[key], cached=True)
    tiles = list(tiles) if tiles else dem.gravity_tiles(precision)
    has_grav = any(w.params.get("G", 0.0) != 0.0 for w in workloads)
    if not has_grav:
        tiles = tiles[:1]
    timings = []
    for tile in tiles:
        for cs in cell_scales:
            r = run_batch(workloads, steps, precision, tuning=(tile, cs), warmup=1)
            for s in r["sims"]:
                s.close()
            timings.append({"gravity_tile": tile, "cell_scale": cs, "ms_per_step": r["ms_per_step"]})
    best = min(timings, key=lambda t: t["ms_per_step"])
    out = {"gravity_tile": best["gravity_tile"], "cell_scale": best["cell_scale"],
           "candidates": timings, "bucket": list(key)}
    cache[key] = out
    return dict(out, cached=False)


class Server:
    """Continuous batching of DEM runs on one engine."""

    def __init__(self, hbm_budget_bytes: int, precision: int = dem.PREC_FP32_FORCE,
                 chunk_steps: int = 50, tuning=None, capture_state: bool = False,
                 policy: str = "fifo", pairs_per_step_cap: float = 5e9):
        if policy not in ("fifo", "srpt"):
            raise ValueError("policy must be 'fifo' or 'srpt'")
        self.policy = policy
        self.cap = float(pairs_per_step_cap)
        self.engine = dem.Engine(hbm_budget_bytes)
        self.budget = int(hbm_budget_bytes)
        self.used = 0
        self.precision = precision
        self.chunk = int(chunk_steps)
        self.tuning = tuning
        self.capture = capture_state
        self.active: Dict[int, List] = {}    # rid -> [request, sim, remaining, bytes]
        self.attached: set = set()           # rids attached to the engine
        self.log: List[str] = []

    def footprint(self, w) -> int:
        return dem.footprint_bytes(w.params, w.n_agg, w.n_sph, self.precision)

    def _admit(self, req: Request, now: float) -> bool:
        need = self.footprint(req.workload)
        if self.used + need > self.budget:
            return False
        sim = make_sim(req.workload, self.precision, self.tuning)
        self.active[req.rid] = [req, sim, req.steps, need]
        self.used += need
        req.admitted = now
        return True

    def _finish(self, rid: int, now: float, status: int = 0):
        req, sim, _rem, need = self.active.pop(rid)
        if rid in self.attached:
            self.engine.detach(sim)
            self.attached.discard(rid)
        req.status = status
        req.result = {"bulk_radius": bulk_radius(sim), "steps": sim.read_state(["agg_mass"])["step"]}
        if self.capture:
            req.result["state"] = sim.read_state(["agg_pos", "agg_vel", "agg_quat"], pairs=True)
        req.done = now
        sim.close()
        self.used -= need

    def _select(self) -> set:
        """The runs stepped in the next chunk."""
        if self.policy == "fifo":
            return set(self.active)
        order = sorted(self.active, key=lambda rid: (
            self.active[rid][0].workload.n_sph ** 2 * self.active[rid][2], rid))
        run, pairs = set(), 0.0
        for rid in order:
            p = float(self.active[rid][0].workload.n_sph) ** 2
            if run and pairs + p > self.cap:
                continue
            run.add(rid)
            pairs += p
        return run

    def run(self, requests: Sequence[Request], clock=time.perf_counter) -> Dict:
        """Serve requests with their arrival offsets in real time."""
        pending = collections.deque(sorted(requests, key=lambda r: r.arrival))
        waiting: collections.deque = collections.deque()
        t0 = clock()
        busy = 0.0
        sphere_steps = 0
        while pending or waiting or self.active:
            now = clock() - t0
            while pending and pending[0].arrival <= now:
                waiting.append(pending.popleft())
            # admit in arrival order while memory allows (no overtaking)
            while waiting:
                if self.footprint(waiting[0].workload) > self.budget:
                    r = waiting.popleft()
                    r.status = dem.DEM_ERR_OOM
                    r.done = clock() - t0
                    continue
                if not self._admit(waiting[0], clock() - t0):
                    break
                waiting.popleft()
            if not self.active:
                if pending:
                    time.sleep(max(0.0, pending[0].arrival - (clock() - t0)))
                continue
            run = self._select()
            for rid in list(self.attached - run):
                self.engine.detach(self.active[rid][1])
                self.attached.discard(rid)
            for rid in sorted(run - self.attached):
                self.engine.attach(self.active[rid][1])
                self.attached.add(rid)
            n = min(self.chunk, min(self.active[rid][2] for rid in run))
            s0 = clock()
            code = self.engine.step(n)
            busy += clock() - s0
            now = clock() - t0
            for rid in sorted(run):
                req, sim, rem, _ = self.active[rid]
                st = sim.status()
                sphere_steps += req.workload.n_sph * n
                if st != dem.DEM_OK:
                    # a stop rule that fired ends the run normally
                    self._finish(rid, now, 0 if st == dem.DEM_STOPPED else st)
                    continue
                self.active[rid][2] = rem - n
                if self.active[rid][2] <= 0:
                    self._finish(rid, now)
        makespan = clock() - t0
        lat = np.array([r.latency for r in requests if r.latency is not None and r.status == 0])
        return {
            "requests": len(requests),
            "completed": int(sum(1 for r in requests if r.done is not None and r.status == 0)),
            "failed": int(sum(1 for r in requests if r.status != 0)),
            "p50_latency_s": float(np.percentile(lat, 50)) if lat.size else None,
            "p99_latency_s": float(np.percentile(lat, 99)) if lat.size else None,
            "makespan_s": makespan,
            "gpu_busy_s": busy,
            "sphere_steps_per_s": sphere_steps / makespan if makespan > 0 else 0.0,
            # requests this mix completes per second of engine time: the
            # highest arrival rate the server sustains for it
            "service_rate_per_s": (sum(1 for r in requests if r.done is not None and r.status == 0)
                                   / busy if busy > 0 else 0.0),
        }


def request_stream(seed: int, n_requests: int, rate_per_s: float, nmin: int = 1000,
                   nmax: int = 50000, smin: int = 100, smax: int = 5000,
                   kinds=("collapse", "spinup", "flyby"), workers: int = 0,
                   executor=None) -> List[Request]:
    """Poisson arrivals at ``rate_per_s``; sphere counts and step counts
    log-uniform; kind uniform.  Inputs are generated up front (in ``workers``
    processes, or on an existing process pool ``executor``)."""
    from . import workloads as W
    rng = np.random.default_rng(seed)
    gaps = rng.exponential(1.0 / rate_per_s, n_requests)
    arrivals = np.cumsum(gaps) - gaps[0]
    n_sph = np.floor(np.exp(rng.uniform(math.log(nmin), math.log(nmax), n_requests))).astype(int)
    steps = np.floor(np.exp(rng.uniform(math.log(smin), math.log(smax), n_requests))).astype(int)
    kind = [kinds[int(k)] for k in rng.integers(len(kinds), size=n_requests)]
    seeds = rng.integers(2 ** 31, size=n_requests)
    jobs = [(k, int(seeds[k]), max(1, int(round(n_sph[k] / 4.5))), 1, 8, 0.15, 5e-4, int(steps[k]),
             1.0, 0.5, 1e-6 if kind[k] == "spinup" else 0.0) for k in range(n_requests)]
    if executor is not None:
        wl = list(executor.map(W._one_pile, jobs, chunksize=1))
    elif workers and workers > 1:
        from concurrent.futures import ProcessPoolExecutor
        with ProcessPoolExecutor(max_workers=workers) as ex:
            wl = list(ex.map(W._one_pile, jobs, chunksize=1))
    else:
        wl = [W._one_pile(j) for j in jobs]
    for k in range(n_requests):
        if kind[k] == "flyby":
            add_flyby(wl[k])
    return [Request(k, kind[k], wl[k], int(steps[k]), float(arrivals[k])) for k in range(n_requests)]
