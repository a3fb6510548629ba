"""Writes the oracle's bulk observables of a reduced collapse and spin-up.

Runs only the FP64 oracle (``oracle/``) on the seeded generator's input and
stores what the GPU observables test compares with:

* collapse: a self-gravitating cloud of 1,100 aggregates of 1-8 spheres
  (4,907 spheres, seed 21, packing 0.15 at rest, G = 1, softening 0.5,
  dt = 5e-4) run for 8 free-fall times; the final bulk radius and packing
  fraction (the collapse runs of Sec. 3.3 and Table 1, reduced in size so
  that the oracle finishes);
* the settled pile it ends with (sphere centres, centre-of-mass velocities,
  space-frame spins), saved as the input of the spin-up;
* spin-up (Sec. 4.1: a constant spin increment each step about +z through
  the centre of mass; 1e-6 rad/step^2, i.e. 1e-6/dt per step in rad per time
  unit) of a new system made from the settled pile, until the bulk radius
  first reaches 1.05 times its starting value (the failure criterion of
  Sec. 4.1); the spin then applied, checked every step.

Bulk radius sqrt(5/3 <|r - r_com|^2>_m) (the oracle's diagnostic) and
packing sum s^3 / R^3 (a uniform-sphere equivalent volume).

Usage:  python tests/golden/make_observables.py [--threads N]
Takes about 35 minutes with 6 threads (the oracle's gravity loop is shared
among threads; its results do not depend on the count).
"""
import argparse
import json
import math
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

import oracle as O  # noqa: E402
from paper_2311_11322_amd import workloads as W  # noqa: E402

SEED, N_AGG, CMIN, CMAX, PHI0 = 21, 1100, 1, 8, 0.15
FF_TIMES = 8.0
SPIN_PER_STEP2 = 1e-6          # rad / step^2
FAIL_GROWTH = 1.05
MAX_SPIN_STEPS = 6000


def observables_workload():
    return W.collapse_cloud(seed=SEED, n_agg=N_AGG, cmin=CMIN, cmax=CMAX, phi0=PHI0)


def collapse_steps(w):
    t_ff = math.sqrt(3 * math.pi / (32 * w.params["G"] * PHI0))
    return int(FF_TIMES * t_ff / w.params["dt"])


def bulk(o, radius):
    R = float(o.diagnostics()["R_bulk"])
    return R, float((radius ** 3).sum()) / R ** 3


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--threads", type=int, default=6)
    a = ap.parse_args()
    O.set_threads(a.threads)
    w = observables_workload()
    steps = collapse_steps(w)
    t0 = time.time()
    o = O.Oracle(w.params).add_workload(w)
    done = 0
    while done < steps:
        k = min(1000, steps - done)
        o.step(k)
        done += k
        print(f"collapse {done}/{steps} steps, {time.time() - t0:.0f} s", flush=True)
    R_c, phi_c = bulk(o, w.radius)
    s = o.spheres()
    ag = o.aggregates()
    spin = np.einsum("nij,nj->ni", quat_R(ag["q"]), ag["wb"])
    np.savez_compressed(os.path.join(HERE, "observables_pile.npz"), sph_pos=s["r"],
                        agg_vel=ag["vA"], agg_spin=spin)
    # spin-up of a new system made from the settled pile
    dw = SPIN_PER_STEP2 / w.params["dt"]
    p2 = dict(w.params, spin_dw=dw)
    o2 = O.Oracle(p2).add(w.counts, s["r"], w.radius, w.mass, ag["vA"], spin)
    R0, _ = bulk(o2, w.radius)
    n = 0
    fail = None
    while n < MAX_SPIN_STEPS:
        o2.step(1)
        n += 1
        R, _ = bulk(o2, w.radius)
        if n % 100 == 0:
            print(f"spin-up {n} steps, R/R0 {R / R0:.4f}, {time.time() - t0:.0f} s", flush=True)
        if R >= FAIL_GROWTH * R0:
            fail = n
            break
    if fail is None:
        raise SystemExit("the pile did not fail within the step limit")
    out = {
        "source": "FP64 oracle (oracle/oracle.c), written by tests/golden/make_observables.py",
        "workload": {"seed": SEED, "n_agg": N_AGG, "n_sph": int(w.n_sph), "cmin": CMIN,
                     "cmax": CMAX, "phi0": PHI0, "dt": w.params["dt"], "G": w.params["G"],
                     "soft_frac": w.params["soft_frac"]},
        "collapse": {"steps": steps, "free_fall_times": FF_TIMES, "R_bulk": R_c,
                     "packing": phi_c},
        "spin_up": {"spin_dw": dw, "R0": R0, "fail_growth": FAIL_GROWTH,
                    "steps_to_failure": fail, "spin_at_failure": fail * dw},
        "seconds": round(time.time() - t0, 1),
        "threads": O.set_threads(0),
    }
    with open(os.path.join(HERE, "observables.json"), "w") as f:
        json.dump(out, f, indent=1)
    print(json.dumps(out, indent=1))


def quat_R(q):
    """Rotation matrices of unit quaternions (w, x, y, z), body to space."""
    w, x, y, z = q[:, 0], q[:, 1], q[:, 2], q[:, 3]
    return np.stack([1 - 2 * (y * y + z * z), 2 * (x * y - w * z), 2 * (x * z + w * y),
                     2 * (x * y + w * z), 1 - 2 * (x * x + z * z), 2 * (y * z - w * x),
                     2 * (x * z - w * y), 2 * (y * z + w * x), 1 - 2 * (x * x + y * y)],
                    -1).reshape(-1, 3, 3)


if __name__ == "__main__":
    main()
