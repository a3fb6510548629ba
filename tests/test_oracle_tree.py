"""Pins of the oracle's tree gravity (multipoles to the quadrupole or the
hexadecapole, plus the softening term of the quadrupole's order).

The paper's gravity is a tree code; the tree here is an approximation with
no closed form, so it is pinned to things other than itself: it must reduce
to the exact direct sum when every node is opened; its truncation error must
fall with distance d as the power the expansion leaves (monopole only: d^-2;
to the quadrupole: d^-3, the octupole being the first neglected term; to the
hexadecapole: d^-5); with softened pairs, the kept eps^2 term must remove the
softening mismatch down to a small fraction of each of its three parts; and
the error must shrink with the opening angle and with the order.
"""
import math

import numpy as np
import pytest

import oracle as O
from paper_2311_11322_amd import workloads as W

pytestmark = pytest.mark.filterwarnings("ignore::RuntimeWarning")


def test_tree_reduces_to_direct_sum_when_every_node_opens():
    w = W.collapse_cloud(3, n_agg=400)
    Fd = O.gravity(w.pos, w.mass, w.radius, 1.0, 0.5)
    for order in (2, 4):
        Ft = O.tree_gravity(w.pos, w.mass, w.radius, 1.0, 0.5, theta=1e-6, order=order)
        assert np.abs(Ft - Fd).max() <= 1e-13 * np.abs(Fd).max()


def _cluster_and_target(d, seed=4, radii=None):
    rng = np.random.default_rng(seed)
    # an irregular cluster of 128 spheres (nonzero octupole and hexadecapole)
    # near the origin, and one target sphere at distance d
    c = rng.normal(0.0, 1.0, (128, 3)) * np.array([2.5, 1.5, 1.0])
    c[:, 0] += 0.3 * c[:, 1] ** 2
    u = np.array([1.0, 0.8, 0.6])
    u /= np.linalg.norm(u)
    pos = np.vstack([c, d * u])
    radius = np.full(129, 0.5) if radii is None else radii(rng)
    mass = W.sphere_mass(radius)
    return pos, mass, radius


def _target_error(d, order=2, soft_frac=0.0, radii=None):
    """Relative error of the tree's force on the target against the direct
    sum; order -1 is the bare monopole written out here."""
    pos, mass, radius = _cluster_and_target(d, radii=radii)
    Fd = O.gravity(pos, mass, radius, 1.0, soft_frac, idx=np.array([128]))[0]
    if order < 0:
        M = mass[:128].sum()
        com = (mass[:128, None] * pos[:128]).sum(0) / M
        R = pos[128] - com
        Ft = -mass[128] * M * R / np.linalg.norm(R) ** 3
    else:
        Ft = O.tree_gravity(pos, mass, radius, 1.0, soft_frac, theta=0.5, order=order)[128]
    return np.linalg.norm(Ft - Fd) / np.linalg.norm(Fd)


def test_truncation_error_falls_as_the_expansion_order_says():
    m1, m2 = _target_error(40.0, -1), _target_error(80.0, -1)
    o1, o2 = _target_error(40.0, 0), _target_error(80.0, 0)
    q1, q2 = _target_error(40.0, 2), _target_error(80.0, 2)
    h1, h2 = _target_error(40.0, 4), _target_error(80.0, 4)
    assert 3.0 < m1 / m2 < 5.0           # monopole only: (a/d)^2
    assert abs(o1 / m1 - 1.0) < 1e-6     # the tree's order 0 is that monopole
    assert 6.0 < q1 / q2 < 10.0          # to the quadrupole: (a/d)^3, octupole first neglected
    assert 25.0 < h1 / h2 < 45.0         # to the hexadecapole: (a/d)^5
    assert q1 < 0.2 * m1 and h1 < 0.2 * q1


def test_softening_term_removes_the_softening_mismatch():
    """Spheres of mixed radii and a large target: with eps_ij = f (s_i + s_j)/2
    the eps^2 term has three parts, s_i^2 M, 2 s_i sum m s and sum m s^2.  Each
    part's relative pull 3/2 G E_part / (M R^2) is written out here; the tree's
    error against the softened direct sum must sit far below the smallest, so
    a dropped part, a wrong sign or a wrong factor fails."""
    d, f = 80.0, 1.0
    radii = lambda rng: np.concatenate([rng.uniform(0.3, 0.7, 128), [1.5]])
    pos, mass, radius = _cluster_and_target(d, radii=radii)
    m, s, si = mass[:128], radius[:128], radius[128]
    M = m.sum()
    com = (m[:, None] * pos[:128]).sum(0) / M
    R = np.linalg.norm(pos[128] - com)
    parts = (f / 2) ** 2 * np.array([si * si * M, 2 * si * (m * s).sum(), (m * s * s).sum()])
    rel = 1.5 * parts / (M * R * R)
    e = _target_error(d, 4, f, radii)
    assert e < 0.2 * rel.min()
    # without softening the same tree is the unsoftened expansion
    assert _target_error(d, 4, 0.0, radii) < 0.2 * rel.min()


def test_tree_error_shrinks_with_opening_angle_and_order():
    w = W.collapse_cloud(3, n_agg=400)
    Fd = O.gravity(w.pos, w.mass, w.radius, 1.0, 0.5)
    rms = {}
    for order in (2, 4):
        for th in (0.3, 0.5, 0.7):
            Ft = O.tree_gravity(w.pos, w.mass, w.radius, 1.0, 0.5, theta=th, order=order)
            e = np.linalg.norm(Ft - Fd, axis=1) / np.linalg.norm(Fd, axis=1)
            rms[order, th] = math.sqrt(float((e ** 2).mean()))
    for order in (2, 4):
        assert rms[order, 0.3] < rms[order, 0.5] < rms[order, 0.7]
        for th in (0.3, 0.5, 0.7):
            assert rms[4, th] < 0.25 * rms[2, th]
    assert rms[2, 0.5] < 1e-3 and rms[4, 0.5] < 1e-4
