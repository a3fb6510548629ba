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


@pytest.mark.parametrize("prec", [0, 1])
def test_both_spheres_of_a_contact_see_the_same_force(D, prec):
    """Each contact is evaluated by both of its spheres; with isolated pairs
    (one contact per sphere) the two contact forces must be exact negatives
    of each other, bit for bit, in both precision forms."""
    say("isolated pairs, antisymmetry, precision", prec)
    rng = np.random.default_rng(77 + prec)
    n_pair = 400
    ra = rng.uniform(0.5, 1.5, n_pair)
    rb = rng.uniform(0.5, 1.5, n_pair)
    u = rng.normal(size=(n_pair, 3))
    u /= np.linalg.norm(u, axis=1, keepdims=True)
    d = (ra + rb) * rng.uniform(0.97, 0.999, n_pair)
    base = np.stack(np.meshgrid(np.arange(8), np.arange(8), np.arange(8), indexing="ij"),
                    -1).reshape(-1, 3)[:n_pair] * 10.0
    pos = np.empty((2 * n_pair, 3))
    pos[0::2] = base
    pos[1::2] = base + d[:, None] * u
    radius = np.empty(2 * n_pair)
    radius[0::2], radius[1::2] = ra, rb
    agg = np.arange(2 * n_pair, dtype=np.int32)
    mass = rng.uniform(0.5, 2.0, 2 * n_pair)
    vel = rng.normal(0.0, 0.3, (2 * n_pair, 3))
    spin = rng.normal(0.0, 0.5, (2 * n_pair, 3))
    # previous contacts: every other pair, with a spring history
    old = np.arange(0, n_pair, 2)
    keys = (old * 2).astype(np.uint64) << np.uint64(32) | (old * 2 + 1).astype(np.uint64)
    hist = rng.normal(0.0, 0.02, (old.size, 7))
    prm = dict(W.CONTACT_PARAMS, dt=1e-4, G=0.0, soft_frac=0.5, periodic=0)
    g = D.contact_forces(prm, pos, vel, radius, agg, mass, spin, keys, hist, precision=prec)
    assert g["keys"].size == n_pair
    Fa, Fb = g["F"][0::2], g["F"][1::2]
    assert np.all(np.abs(Fa).max(axis=1) > 0)
    assert np.array_equal(Fa, -Fb)
