"""Bulk observables of the FP32-force form against the plain FP64 form.

Runs long enough to settle a self-gravitating pile and to spin it up to
mass shedding are far beyond what the CPU oracle can finish, so the reference
here is the plain FP64 GPU path (itself held to the oracle step by step in
test_gpu_parity.py).  Both forms start from the same state with the same
seeds; the final packing fraction of a collapse and the spin at which a
spun-up pile's bulk radius has grown by 5 % must agree within 1 %.
"""
import math
import sys

import numpy as np
import pytest

from paper_2311_11322_amd import workloads as W

pytestmark = pytest.mark.gpu


def say(*a):
    print("[case]", *a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def D():
    from paper_2311_11322_amd import dem
    dem.lib()
    return dem


def bulk(sim, radius):
    st = sim.read_state(["sph_pos"])
    r = st["sph_pos"]
    m = radius ** 3
    com = (m[:, None] * r).sum(0) / m.sum()
    R = math.sqrt(5.0 / 3.0 * float((m * ((r - com) ** 2).sum(1)).sum() / m.sum()))
    phi = float((radius ** 3).sum()) / R ** 3
    return R, phi


def collapse(D, w, precision, steps):
    sim = D.Sim(w.params, precision=precision)
    sim.add_workload(w)
    sim.step(steps)
    return sim


def restart(D, sim, w, precision, spin_dw):
    """A new system from another's current positions and velocities."""
    st = sim.read_state(["sph_pos", "agg_vel", "agg_spin"])
    s2 = D.Sim(w.params, precision=precision)
    s2.set_forcing(spin_dw)
    s2.add_aggregates(w.counts, st["sph_pos"], w.radius, w.mass, st["agg_vel"], st["agg_spin"])
    return s2


def spin_to_failure(sim, radius, dw, every=20, max_steps=6000):
    R0, _ = bulk(sim, radius)
    n = 0
    while n < max_steps:
        sim.step(every)
        n += every
        R, _ = bulk(sim, radius)
        if R >= 1.05 * R0:
            return n * dw
    return None


def test_collapse_packing_and_spin_at_failure_fp32_vs_fp64(D):
    w = W.collapse_cloud(seed=21, n_agg=1100, cmin=1, cmax=8, phi0=0.15)
    t_ff = math.sqrt(3 * math.pi / (32 * 1.0 * 0.15))
    steps = int(8 * t_ff / w.params["dt"])
    say("collapse", w.n_sph, "spheres,", steps, "steps")
    s64 = collapse(D, w, D.PREC_FP64, steps)
    s32 = collapse(D, w, D.PREC_FP32_FORCE, steps)
    R64, phi64 = bulk(s64, w.radius)
    R32, phi32 = bulk(s32, w.radius)
    print(f"packing fp64 {phi64:.5f} fp32 {phi32:.5f}  R {R64:.4f} {R32:.4f}")
    assert abs(phi32 - phi64) <= 0.01 * phi64
    # spin-up of the settled FP64 pile in both forms
    dw = 1e-6 / w.params["dt"]
    say("spin-up")
    w64 = spin_to_failure(restart(D, s64, w, D.PREC_FP64, dw), w.radius, dw)
    w32 = spin_to_failure(restart(D, s64, w, D.PREC_FP32_FORCE, dw), w.radius, dw)
    rho = float(W.sphere_mass(w.radius).sum()) / (4 / 3 * math.pi * R64 ** 3)
    w_crit = math.sqrt(4 * math.pi * 1.0 * rho / 3)
    print(f"spin at failure fp64 {w64} fp32 {w32}  nominal critical {w_crit:.4f}")
    assert w64 is not None and w32 is not None
    assert abs(w32 - w64) <= 0.01 * w64
