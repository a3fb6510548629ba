"""The fused per-pile step against the staged step (needs an MI355X).

A system of at most 256 spheres (or any system tuned so) runs its whole
step in one workgroup (k_fused); the staged step launches one kernel per
stage.  Both evaluate every element with the same device functions, so a
run without spin-up must agree bit for bit between the two; with spin-up the
pile's centre of mass is summed in another order, so the runs agree to
rounding.  The fused step is also checked against the oracle directly.
"""
import sys

import numpy as np
import pytest

import oracle as O
from paper_2311_11322_amd import workloads as W
from tests.gpu_util import compare_states

pytestmark = pytest.mark.gpu

FIELDS = ("agg_pos", "agg_vel", "agg_acc", "agg_torque", "agg_quat", "agg_spin_body",
          "sph_pos", "sph_vel", "sph_force", "sph_torque", "pair_keys", "pair_hist")


def say(*a):
    print("[case]", *a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def D():
    from paper_2311_11322_amd import dem
    dem.lib()
    return dem


def _run(D, w, fused, steps, precision=0, spin=0.0):
    from paper_2311_11322_amd import serve
    sim = D.Sim(w.params, precision=precision)
    sim.set_tuning(fused=fused)
    if spin:
        sim.set_forcing(spin)
    sim.add_workload(w)
    sim.step(steps)
    return sim.read_state(list(FIELDS[:-2]), pairs=True)


def _cases():
    box = W.periodic_box(31, n_agg=300, contact_seeded=True, spin_sigma=0.5, vel_sigma=0.2)
    cloud = W.collapse_cloud(41, n_agg=250, contact_seeded=True, spin_sigma=0.3, vel_sigma=0.1)
    fill = W.box_fill(seed=2, n_sph=240, shape="mixed", base=14, height=40, z_range=(0, 30),
                      floor_seeded=0.3, contact_seeded=True)
    nut = W.brazil_nut(seed=9, n_sph=600, base=16.0, fill_height=50.0)
    return {"periodic box": box, "gravity cloud": cloud, "box fill": fill, "brazil nut": nut}


@pytest.mark.parametrize("name", ["periodic box", "gravity cloud", "box fill", "brazil nut"])
def test_fused_step_equals_staged_step(D, name):
    w = _cases()[name]
    for prec in (D.PREC_FP64, D.PREC_FP32_FORCE):
        say("fused vs staged", name, "precision", prec, w.n_sph, "spheres")
        a = _run(D, w, 1, 12, prec)
        b = _run(D, w, 2, 12, prec)
        assert a["step"] == b["step"] == 12
        for k in FIELDS:
            assert np.array_equal(a[k], b[k]), (name, prec, k)


def test_fused_step_with_spin_up_agrees_to_rounding(D):
    w = W.collapse_cloud(43, n_agg=250, contact_seeded=True, spin_sigma=0.3, vel_sigma=0.1)
    say("fused vs staged with spin-up")
    a = _run(D, w, 1, 5, spin=0.01)
    b = _run(D, w, 2, 5, spin=0.01)
    assert np.array_equal(a["pair_keys"], b["pair_keys"])
    for k in ("agg_pos", "agg_vel", "agg_spin_body", "sph_force"):
        scale = float(np.abs(b[k]).max())
        assert np.abs(a[k] - b[k]).max() <= 1e-13 * scale, k


def test_fused_piles_in_an_engine_with_staged_ones(D):
    """Small (fused) and large (staged) piles in one engine: every pile
    bit-identical to its own run alone; the fused and staged parts of a step
    share one graph, with gravity batched over both."""
    from paper_2311_11322_amd import serve
    small = [W.collapse_cloud(50 + k, n_agg=n, contact_seeded=True, spin_sigma=0.2,
                              vel_sigma=0.1) for k, n in enumerate((20, 40, 55))]
    big = W.collapse_cloud(60, n_agg=2500, contact_seeded=False)      # staged
    assert big.n_sph > 256 and all(p.n_sph <= 256 for p in small)
    piles = small + [big]
    say("engine: 3 fused + 1 staged piles")
    alone = []
    for p in piles:
        sim = serve.make_sim(p, D.PREC_FP64)
        sim.step(6)
        alone.append(sim.read_state(list(FIELDS[:-2]), pairs=True))
        sim.close()
    eng = D.Engine(1 << 36)
    sims = [serve.make_sim(p, D.PREC_FP64) for p in piles]
    for s in sims:
        eng.attach(s)
    assert eng.step(6) == D.DEM_OK
    for s, ref in zip(sims, alone):
        eng.detach(s)
        got = s.read_state(list(FIELDS[:-2]), pairs=True)
        for k in FIELDS:
            assert np.array_equal(got[k], ref[k]), k


def test_fused_step_parity_with_oracle(D):
    """The fused step of a contact-seeded cloud with gravity, spins and a
    perturber against the oracle (one step at 1e-12, three more at 1e-10)."""
    from paper_2311_11322_amd import serve
    w = W.collapse_cloud(47, n_agg=200, contact_seeded=True, spin_sigma=0.2, vel_sigma=0.05)
    serve.add_flyby(w, start_factor=1.2)
    Mp, rp, vp = w.params["perturber"]
    say("fused step parity, flyby cloud")
    sim = D.Sim(w.params)
    sim.set_tuning(fused=1)
    sim.set_forcing(0.0, Mp, rp, vp)
    sim.add_workload(w)
    o = O.Oracle(w.params).set_perturber(Mp, rp, vp).add_workload(w)
    compare_states(sim, o)
    sim.step(1)
    o.step(1)
    compare_states(sim, o)
    sim.step(3)
    o.step(3)
    compare_states(sim, o, tol=1e-10)
