"""Pins of the oracle's periodic cube: the wrap of aggregate centres in the
drift and the minimum-image rule of the contact geometry.

Periodic boundaries are a property of the workload (the contact-only box),
not of the method: inside a cube of side L much larger than the interaction
range, a system must move exactly as the same system in open space, with
each aggregate centre reduced into [0, L).  These tests run the same bodies
in open space and straddling faces, edges and a corner of the cube, and
require the periodic run to reproduce the open-space one.  No GPU needed.
"""
import math

import numpy as np
import pytest

import oracle as O
from paper_2311_11322_amd import workloads as W

M1 = 4.0 / 3.0 * math.pi


def params(periodic, L, **kw):
    p = dict(W.CONTACT_PARAMS, dt=2e-4, G=0.0, soft_frac=0.5, periodic=int(periodic),
             box=(L, L, L) if periodic else (0.0, 0.0, 0.0))
    p.update(kw)
    return p


def run(counts, pos, rad, vel, spin, periodic, L, steps, every, **kw):
    """Aggregate centres, velocities and space-frame spins every `every`
    steps, and the contact count seen at each sample."""
    o = O.Oracle(params(periodic, L, **kw))
    o.add(counts, pos, rad, W.sphere_mass(rad), vel, spin)
    out = []
    for _ in range(steps // every):
        o.step(every)
        a = o.aggregates()
        out.append((a["rA"].copy(), a["vA"].copy(), a["wA"].copy(), o.counts()[2]))
    return out


def min_image(d, L):
    return d - L * np.round(d / L)


@pytest.mark.parametrize("sign", [1.0, -1.0])
def test_free_flight_crosses_every_face(sign):
    """Two spinning aggregates flying side by side (same velocity, so they
    never meet) through three faces; the opposite velocity takes them through
    the other three.  Centres stay in [0, L) and equal the open-space centres
    modulo L; velocities and spins are untouched by the wrap."""
    L = 10.0
    rng = np.random.default_rng(5)
    rel_a, rad_a = W.random_cluster(rng, 3)
    rel_b, rad_b = W.random_cluster(rng, 4)
    pos = np.concatenate([rel_a + [2.0, 2.0, 2.0], rel_b + [7.0, 7.0, 7.0]])
    rad = np.concatenate([rad_a, rad_b])
    v = sign * np.array([-30.0, 25.0, -21.0])          # 3-4 box lengths in the run
    vel = np.array([v, v])
    spin = np.array([[0.5, -1.0, 2.0], [-1.5, 0.3, 0.7]])
    per = run([3, 4], pos, rad, vel, spin, True, L, 5000, 250)
    opn = run([3, 4], pos, rad, vel, spin, False, L, 5000, 250)
    crossed = np.zeros((2, 3), dtype=bool)
    prev = None
    for (rp, vp, wp, cp), (ro, vo, wo, co) in zip(per, opn):
        assert cp == 0 and co == 0
        assert np.all(rp >= 0.0) and np.all(rp < L)
        assert np.abs(min_image(rp - ro, L)).max() < 1e-12 * np.abs(ro).max()
        assert np.array_equal(vp, vo) and np.abs(wp - wo).max() < 1e-14
        if prev is not None:
            # a jump by about L against the motion is a wrap through the
            # face the velocity points at
            crossed |= (rp - prev) * np.sign(v) < -L / 2
        prev = rp
    assert crossed.all()


@pytest.mark.parametrize("corner", [False, True])
def test_rebound_straddling_faces_matches_open_space(corner):
    """An oblique frictional collision of a spinning dumbbell and a sphere
    whose contact straddles one face (or the corner where three faces meet),
    drifting across it so that the centres are wrapped during the run:
    velocities and spins equal those of the same collision in open space at
    every sample, and the contact forms and breaks at the same samples."""
    L = 12.0
    d = np.array([1.0, 0.0, 0.0]) if not corner else np.array([1.0, 1.0, 1.0]) / math.sqrt(3)
    # dumbbell (two unit spheres along its axis) approaching the sphere
    e = np.array([0.3, 1.0, -0.2])
    e /= np.linalg.norm(e)
    c_a = -1.7 * d + np.array([0.0, 0.15, -0.1])
    pos = np.array([c_a - e, c_a + e, 1.2 * d])
    rad = np.array([1.0, 1.0, 0.9])
    # approaching at 4 with a common drift of 5 across the face(s): the
    # centres cross the face during the run, the contact straddles it
    vel = np.array([7.0 * d, 3.0 * d])
    spin = np.array([[0.2, -0.4, 0.3], [0.0, 0.5, -0.6]])
    kw = dict(dt=1e-4)
    per = run([2, 1], pos, rad, vel, spin, True, L, 4000, 100, **kw)
    opn = run([2, 1], pos + L / 2, rad, vel, spin, False, L, 4000, 100, **kw)
    touched = False
    for (rp, vp, wp, cp), (ro, vo, wo, co) in zip(per, opn):
        assert np.all(rp >= 0.0) and np.all(rp < L)
        assert np.abs(min_image(rp - (ro - L / 2), L)).max() < 1e-9
        assert np.abs(vp - vo).max() <= 1e-9 * np.abs(vo).max()
        assert np.abs(wp - wo).max() <= 1e-9 * max(np.abs(wo).max(), 1.0)
        assert cp == co
        touched |= cp > 0
    assert touched and per[-1][3] == 0         # a collision happened and ended
    # the collision changed the motion (not a miss)
    assert np.abs(per[-1][1] - vel).max() > 0.1


def test_periodic_search_pairs_across_faces_equal_open_space():
    """Contact lists of a cluster placed across a corner equal those of the
    same cluster in open space (brute force on both sides)."""
    L = 15.0
    w = W.periodic_box(7, n_agg=60, contact_seeded=True)
    pos = w.pos - w.pos.mean(0)
    scale = 4.0 / np.abs(pos).max()
    pos = pos * scale                           # squeeze into |x| < 4
    rad = w.radius * scale
    agg = w.agg_of_sphere()
    ref = O.find_contacts(pos, rad, agg)        # open space
    wrapped = pos - L * np.floor(pos / L)       # every sphere reduced into [0, L)
    got = O.find_contacts(wrapped, rad, agg, (L, L, L))
    assert ref.size > 10
    assert np.array_equal(got, ref)
