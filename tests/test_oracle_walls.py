"""Pins of the oracle's planar walls, uniform field and wall shaking.

The box-filling and Brazil-nut workloads of the paper (Sec. 3.3 performance scaling,
Sec. 4.3) put the spheres under a uniform gravitational field inside a
container whose walls may oscillate sinusoidally.  The paper gives no wall
model of its own; the oracle treats each wall as a contact partner of
infinite mass and no spin, with the same spring-dashpot and friction model as
sphere pairs.  Every check below is a textbook result of rigid-body
mechanics, with a negative control where a plausible mistake would survive a
weaker test.
"""
import math

import numpy as np
import pytest

import oracle as O
from paper_2311_11322_amd import workloads as W

pytestmark = pytest.mark.filterwarnings("ignore::RuntimeWarning")

M1 = 4.0 / 3.0 * math.pi   # unit sphere at density 1
FLOOR = (0.0, 0.0, 1.0, 0.0)


def params(**kw):
    p = dict(W.CONTACT_PARAMS, dt=1e-4, G=0.0, soft_frac=0.5, periodic=0, box=(0, 0, 0),
             mu_r=0.0, mu_t=0.0)
    p.update(kw)
    return p


def one_sphere(prm, pos, vel=(0, 0, 0), spin=(0, 0, 0)):
    o = O.Oracle(prm)
    o.add([1], [pos], [1.0], [M1], [vel], [spin])
    return o


def test_wall_contact_is_strict_and_walls_follow_spheres():
    """A sphere touches a wall iff its centre is closer than its radius; the
    wall partner's index is n_spheres + wall, after every sphere partner."""
    walls = [FLOOR, (1.0, 0.0, 0.0, -5.0)]
    prm = params(walls=walls)
    o = O.Oracle(prm)
    o.add([1, 1], [[0, 0, 1.0], [1.5, 0, 1.0 - 1e-12]], [1, 1], [M1, M1])
    p = o.pairs()
    assert list(zip(p["i"], p["j"])) == [(0, 1), (1, 2)]
    o = O.Oracle(prm)
    o.add([1], [[-4.5, 0, 0.5]], [1], [M1])
    p = o.pairs()
    assert list(zip(p["i"], p["j"])) == [(0, 1), (0, 2)]
    assert np.allclose(p["diag"][:, 4], [0.5, 0.5])       # overlaps s - d


@pytest.mark.parametrize("h", [2e-4, 1e-4])
def test_wall_rebound_restitution_uses_body_mass(h):
    """Normal impact on a fixed wall rebounds at eps_n times the incoming
    speed when the dashpot takes the body's own mass (the wall is infinitely
    heavy); the reduced mass of two equal bodies would give another value."""
    prm = params(dt=h, mu_s=0.0, walls=[FLOOR])
    o = one_sphere(prm, (0, 0, 1.01), vel=(0, 0, -1))
    o.step(int(0.08 / h))
    assert o.counts()[2] == 0
    e = o.aggregates()["vA"][0, 2]
    le = math.log(prm["eps_n"])
    zeta = -le / math.sqrt(math.pi ** 2 + le * le)
    tc = math.pi / (math.sqrt(prm["k_n"] / M1) * math.sqrt(1 - zeta * zeta))
    assert abs(e - prm["eps_n"]) <= h / tc
    # restitution if the dashpot used half the mass
    C = 2 * zeta * math.sqrt(prm["k_n"] * M1 / 2)
    z2 = C / (2 * math.sqrt(prm["k_n"] * M1))
    e_wrong = math.exp(-z2 * math.pi / math.sqrt(1 - z2 * z2))
    assert abs(e_wrong - prm["eps_n"]) > 0.1


def test_resting_sphere_static_overlap_and_load():
    """At rest on a floor under g the spring carries the weight: overlap
    M g / k_n and normal force M g."""
    g = 2.0
    prm = params(g=(0, 0, -g), walls=[FLOOR])
    o = one_sphere(prm, (0, 0, 1.0))
    o.step(30000)
    p = o.pairs()
    assert p["j"].tolist() == [1]
    assert abs(p["diag"][0, 4] - M1 * g / prm["k_n"]) < 1e-6 * M1 * g / prm["k_n"]
    assert abs(p["diag"][0, 0] - M1 * g) < 1e-6 * M1 * g
    assert abs(o.aggregates()["vA"][0, 2]) < 1e-9


def _slide(torque_at_centre):
    g, v0, mu = 1.0, 1.0, 0.5
    prm = params(g=(0, 0, -g), walls=[FLOOR], mu_s=mu, torque_at_centre=torque_at_centre)
    o = one_sphere(prm, (0, 0, 1.0 - M1 * g / prm["k_n"]), vel=(v0, 0, 0))
    n = int((2 * v0 / (7 * mu * g) + 0.4) / prm["dt"])
    o.step(n)
    a = o.aggregates()
    return a["vA"][0, 0], a["wA"][0, 1], v0 - mu * g * n * prm["dt"]


def test_sliding_sphere_ends_rolling_at_five_sevenths():
    """A sphere launched sliding without spin on a frictional floor ends
    rolling without slipping at 5/7 of its initial speed, whatever mu_s; the
    friction acts at the contact point (Eq. 9).  Applied at the centre, no
    spin develops and the sphere keeps sliding at deceleration mu_s g."""
    v, w, _ = _slide(0)
    assert abs(v - 5.0 / 7.0) < 5e-3
    assert abs(w - v) < 5e-3            # v_x = w_y s: contact point at rest
    v_c, w_c, v_kin = _slide(1)
    assert abs(v_c - v_kin) < 5e-3 and abs(w_c) < 1e-12


def _incline(torque_at_centre, T=1.0):
    th, g = math.radians(20.0), 1.0
    s, c = math.sin(th), math.cos(th)
    n = (-s, 0.0, c)
    prm = params(g=(0, 0, -g), walls=[(n[0], n[1], n[2], 0.0)], mu_s=0.5,
                 torque_at_centre=torque_at_centre)
    d = 1.0 - M1 * g * c / prm["k_n"]
    o = one_sphere(prm, (n[0] * d, 0.0, n[2] * d))
    o.step(int(T / prm["dt"]))
    down = -np.array([c, 0.0, s])
    v = float(o.aggregates()["vA"][0] @ down)
    return v, o.pairs()["diag"][0, 0], s, c, g, T


def test_sphere_rolls_down_incline_at_five_sevenths_g_sin():
    """On an inclined plane steeper friction than needed for rolling, a
    sphere rolls with acceleration (5/7) g sin(theta) and presses on the
    plane with M g cos(theta); forced through the centre it would stick."""
    v, fN, s, c, g, T = _incline(0)
    assert abs(v - 5.0 / 7.0 * g * s * T) < 0.01 * v
    assert abs(fN - M1 * g * c) < 1e-3 * M1 * g
    v_c, _, _, _, _, _ = _incline(1, T=0.3)
    assert abs(v_c) < 1e-3


def _shaken(a_over_g, phase, n_per=1.0):
    g, om = 1.0, math.pi
    A = a_over_g * g / om ** 2
    prm = params(g=(0, 0, -g), walls=[FLOOR], shake_amp=[(0, 0, A)], shake_omega=om,
                 shake_phase=phase, mu_s=0.0)
    acc0 = g + A * om * om * -math.sin(phase)          # floor acceleration is -A w^2 sin
    z0 = A * math.sin(phase) + 1.0 - M1 * acc0 / prm["k_n"]
    o = one_sphere(prm, (0, 0, z0))
    h = prm["dt"]
    out = []
    for k in range(int(n_per * 2.0 / h)):
        o.step(1)
        t = (k + 1) * h
        out.append((t, o.aggregates()["rA"][0, 2], o.counts()[2],
                    A * math.sin(om * t + phase)))
    return np.array(out), A, om, prm


def test_shaken_floor_carries_sphere_below_one_g():
    """Peak floor acceleration below g: the sphere rides the floor, never
    losing contact, its centre one radius (less the load overlap) above the
    displaced plane."""
    out, A, om, prm = _shaken(0.5, -math.pi / 2)
    assert out[:, 2].min() == 1
    gap = out[:, 1] - out[:, 3] - 1.0
    assert np.abs(gap).max() < 3 * M1 * 1.5 / prm["k_n"]


def test_shaken_floor_throws_sphere_at_predicted_phase():
    """Peak floor acceleration 2 g from the lowest point: the sphere leaves
    the floor when the floor's downward acceleration first exceeds g, at
    phase w t - pi/2 = pi/6; the wall's displacement, velocity and
    acceleration signs all enter."""
    out, A, om, prm = _shaken(2.0, -math.pi / 2)
    t_lift = out[np.argmax(out[:, 2] == 0), 0]
    assert abs(t_lift - (math.pi / 6 + math.pi / 2) / om) < 0.02
    # a floor displaced the other way would not be touched after its first move
    assert out[: int(0.5 / prm["dt"]), 2].min() == 1


def test_side_wall_shaken_along_itself_drags_sphere_by_two_sevenths():
    """A sphere pressed against a wall that slides along its own plane,
    without slipping, moves its centre by 2/7 of the wall's displacement
    (the rest of the contact point's motion is rolling): wall velocity and the
    lever arm of the friction both enter."""
    g, om = 1.0, math.pi
    A = 1.0 / om ** 2
    wall = (1.0, 0.0, 0.0, 0.0)
    prm = params(g=(-g, 0, 0), walls=[wall], shake_amp=[(0, 0, A)], shake_omega=om,
                 shake_phase=-math.pi / 2, mu_s=0.5)
    x0 = 1.0 - M1 * g / prm["k_n"]
    o = one_sphere(prm, (x0, 0, 0))
    h = prm["dt"]
    worst = 0.0
    for k in range(int(2.0 / h) // 50):
        o.step(50)
        t = (k + 1) * 50 * h
        wall_dz = A * math.sin(om * t - math.pi / 2) + A
        worst = max(worst, abs(o.aggregates()["rA"][0, 2] - 2.0 / 7.0 * wall_dz))
    assert o.counts()[2] == 1
    assert worst < 0.02 * A


def test_closed_box_conserves_energy_without_damping():
    """Elastic, frictionless spheres bouncing in a closed box under g:
    kinetic + spring + field energy is conserved to O(h^2), and no sphere
    leaves the box."""
    L = 12.0
    walls = [(1, 0, 0, 0), (-1, 0, 0, -L), (0, 1, 0, 0), (0, -1, 0, -L), (0, 0, 1, 0),
             (0, 0, -1, -L)]
    drift = []
    for h in (2e-4, 1e-4):
        prm = params(dt=h, eps_n=1.0, eps_t=1.0, mu_s=0.0, g=(0.3, -0.2, -1.0), walls=walls)
        rng = np.random.default_rng(5)
        pos = np.array([[x, y, z] for x in (2.5, 6.0, 9.5) for y in (2.5, 6.0, 9.5)
                        for z in (2.5, 6.0)], dtype=float)
        pos += rng.uniform(-0.3, 0.3, pos.shape)
        vel = rng.normal(0, 3.0, pos.shape)
        o = O.Oracle(prm)
        n = pos.shape[0]
        o.add([1] * n, pos, [1.0] * n, [M1] * n, vel)
        e0 = o.diagnostics()["E"]
        worst = 0.0
        for _ in range(10):
            o.step(int(0.1 / h))
            worst = max(worst, abs(o.diagnostics()["E"] - e0) / e0)
            r = o.spheres()["r"]
            assert r.min() > 0.0 and r.max() < L
        drift.append(worst)
    assert drift[1] < 1e-3
    assert drift[1] < 0.4 * drift[0]
