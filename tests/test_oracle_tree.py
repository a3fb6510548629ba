"""Pins of the oracle's tree gravity (monopole + quadrupole multipoles).

The paper's gravity is a tree code; the tree here is an approximation with
no closed form, so it is pinned to things other than itself: it must reduce
to the exact direct sum when every node is opened, its truncation error must
fall as the cube of the distance (the first neglected term is the octupole;
a monopole-only expansion falls as the square), and its error must shrink
with the opening angle.
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
    Ft = O.tree_gravity(w.pos, w.mass, w.radius, 1.0, 0.5, theta=1e-6)
    assert np.abs(Ft - Fd).max() <= 1e-13 * np.abs(Fd).max()


def _cluster_and_target(d, seed=4):
    rng = np.random.default_rng(seed)
    # an irregular cluster of 128 unit spheres (nonzero octupole) near the origin
    c = rng.normal(0.0, 1.0, (128, 3)) * np.array([2.5, 1.5, 1.0])
    c[:, 0] += 0.3 * c[:, 1] ** 2
    u = np.array([1.0, 0.8, 0.6])
    u /= np.linalg.norm(u)
    pos = np.vstack([c, d * u])
    radius = np.full(129, 0.5)
    mass = W.sphere_mass(radius)
    return pos, mass, radius


def _target_error(d, monopole=False):
    pos, mass, radius = _cluster_and_target(d)
    Fd = O.gravity(pos, mass, radius, 1.0, 0.0, idx=np.array([128]))[0]
    if monopole:
        M = mass[:128].sum()
        com = (mass[:128, None] * pos[:128]).sum(0) / M
        R = pos[128] - com
        Ft = -mass[128] * M * R / np.linalg.norm(R) ** 3
    else:
        Ft = O.tree_gravity(pos, mass, radius, 1.0, 0.0, theta=0.5)[128]
    return np.linalg.norm(Ft - Fd) / np.linalg.norm(Fd)


def test_quadrupole_truncation_error_falls_as_cube_of_distance():
    e1, e2 = _target_error(40.0), _target_error(80.0)
    m1, m2 = _target_error(40.0, True), _target_error(80.0, True)
    assert 6.0 < e1 / e2 < 10.0          # (a/d)^3: the octupole is the first neglected term
    assert 3.0 < m1 / m2 < 5.0           # a monopole-only expansion: (a/d)^2
    assert e1 < 0.2 * m1


def test_tree_error_shrinks_with_opening_angle():
    w = W.collapse_cloud(3, n_agg=400)
    Fd = O.gravity(w.pos, w.mass, w.radius, 1.0, 0.5)
    rms = []
    for th in (0.3, 0.5, 0.7):
        Ft = O.tree_gravity(w.pos, w.mass, w.radius, 1.0, 0.5, theta=th)
        e = np.linalg.norm(Ft - Fd, axis=1) / np.linalg.norm(Fd, axis=1)
        rms.append(math.sqrt(float((e ** 2).mean())))
    assert rms[0] < rms[1] < rms[2]
    assert rms[1] < 1e-3
