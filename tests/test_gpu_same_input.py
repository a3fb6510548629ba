"""Contact forces on identical FP64 input: the library against the oracle.

The state comparisons of test_gpu_parity.py start the two sides from the
same aggregates; their sphere positions then agree only to rounding, and the
overlap's conditioning sets the force bound there.  Here both sides are fed
exactly the same sphere positions, velocities, spins, masses and previous
contacts with their spring history (from the seeded generator and the
oracle's brute-force search, never from the library), so the only
differences left are the rounding of the force arithmetic itself: contact
lists and keys bit for bit, per-sphere forces, torques and the updated
history within 1e-12 of each array's largest oracle value in the FP64 form,
1e-5 in the FP32-force form (torques and history included).
"""
import sys

import numpy as np
import pytest

import oracle as O
from paper_2311_11322_amd import workloads as W
from tests.gpu_util import rel_err

pytestmark = pytest.mark.gpu


def say(*a):
    print("[case]", *a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def D():
    from paper_2311_11322_amd import dem
    dem.lib()
    return dem


def same_input(kind, seed):
    """Sphere states and a previous contact list with history: 70 % of the
    current contacts carried (history drawn from a seeded generator, some
    large enough to sit beyond the friction caps) plus stale keys that are
    no longer contacts."""
    rng = np.random.default_rng(seed)
    if kind == "periodic":
        w = W.periodic_box(seed, n_agg=300, contact_seeded=True)
        L = w.params["box"][0]
        box = (L, L, L)
    elif kind == "cloud":
        w = W.collapse_cloud(seed, n_agg=300, contact_seeded=True)
        w.params["G"] = 0.0
        box = None
    else:
        w = W.box_fill(seed, n_sph=500, shape="mixed", base=16.0, height=40.0,
                       z_range=(0.0, 16.0), floor_seeded=0.5, contact_seeded=True)
        box = None
    n = w.n_sph
    agg = w.agg_of_sphere()
    off = w.offsets()
    agg_mass = np.add.reduceat(w.mass, off[:-1])
    vel = rng.normal(0.0, 0.3, (n, 3))
    spin = rng.normal(0.0, 0.8, (w.n_agg, 3))
    cur = O.find_contacts(w.pos, w.radius, agg, box)
    keep = cur[rng.random(cur.size) < 0.7]
    if kind == "walls":
        # wall contacts of floor spheres: sphere i, partner n + 0 (the floor)
        floor = np.nonzero(w.pos[:, 2] < w.radius)[0][::2].astype(np.uint64)
        keep = np.concatenate([keep, (floor << np.uint64(32)) | np.uint64(n)])
    i = rng.integers(0, n - 1, 60)
    j = np.minimum(i + rng.integers(1, 40, 60), n - 1)
    stale = (i.astype(np.uint64) << np.uint64(32)) | j.astype(np.uint64)
    stale = stale[(agg[i] != agg[j]) & (i < j)]
    old = np.unique(np.concatenate([keep, stale]))
    hist = rng.normal(0.0, 2e-4, (old.size, 7))
    hist[::5] *= 50.0                       # beyond the caps: the slider branch
    return w, dict(pos=w.pos, vel=vel, radius=w.radius, agg=agg, agg_mass=agg_mass,
                   agg_spin=spin, old_keys=old, old_hist=hist)


@pytest.mark.parametrize("kind,seed", [("periodic", 71), ("cloud", 72), ("walls", 73)])
def test_contact_forces_same_input(D, kind, seed):
    w, x = same_input(kind, seed)
    say("same input", kind, w.n_sph, "spheres,", x["old_keys"].size, "old contacts")
    ref = O.contact_forces(w.params, **x)
    assert ref["keys"].size > 100 if kind != "walls" else ref["keys"].size > 40
    g64 = D.contact_forces(w.params, **x, precision=D.PREC_FP64)
    assert np.array_equal(g64["keys"], ref["keys"])
    e = {k: rel_err(g64[k], ref[k]) for k in ("F", "tau", "hist")}
    print("FP64 same-input errors", e, flush=True)
    assert all(v <= 1e-12 for v in e.values()), e
    say("same input fp32-force", kind)
    g32 = D.contact_forces(w.params, **x, precision=D.PREC_FP32_FORCE)
    assert np.array_equal(g32["keys"], ref["keys"])
    e32 = {k: rel_err(g32[k], ref[k]) for k in ("F", "tau", "hist")}
    print("FP32-force same-input errors", e32, flush=True)
    assert all(v <= 1e-5 for v in e32.values()), e32
