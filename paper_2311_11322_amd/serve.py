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
    if w.params.get("spin_dw", 0.0) or pert:
        if pert:
            sim.set_forcing(w.params.get("spin_dw", 0.0), pert[0], pert[1], pert[2])
        else:
            sim.set_forcing(w.params["spin_dw"])
    sim.add_workload(w)
    return sim


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
    for s in sims:
        eng.detach(s)
    out["sims"] = sims
    eng.close()
    return out


def autotune(workloads: Sequence, precision: int, steps: int = 3,
             cell_scales=(1.0, 1.5), tiles=None) -> Dict:
    """Pick the gravity tile and cell scale that minimise the measured step
    time of this batch (a few steps per candidate)."""
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
    return {"gravity_tile": best["gravity_tile"], "cell_scale": best["cell_scale"],
            "candidates": timings}


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
                    self._finish(rid, now, st)
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
