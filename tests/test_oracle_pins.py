"""Pins of the FP64 oracle against what the paper and the mathematics fix.

Each test checks the oracle against something other than itself: a closed
form, an invariant, a special case that reduces to a textbook result, an
independent library routine, or brute force on a tiny input.  None of these
tests needs a GPU.
"""
import math

import numpy as np
import pytest

import oracle as O
from paper_2311_11322_amd import workloads as W

pytestmark = pytest.mark.filterwarnings("ignore::RuntimeWarning")

M1 = 4.0 / 3.0 * math.pi   # mass of a unit sphere at density 1


def frictionless(**kw):
    p = dict(W.CONTACT_PARAMS, dt=1e-4, G=0.0, soft_frac=0.5, periodic=0, box=(0, 0, 0),
             mu_s=0.0, mu_r=0.0, mu_t=0.0)
    p.update(kw)
    return p


def collision_time(k, mu, eps):
    le = math.log(eps)
    zeta = -le / math.sqrt(math.pi ** 2 + le * le)
    return math.pi / (math.sqrt(k / mu) * math.sqrt(1.0 - zeta * zeta))


# ---------------------------------------------------------------------------
# V1 / V2: head-on rebound, closed form of the linear damped oscillator
# ---------------------------------------------------------------------------

@pytest.mark.parametrize("h", [4e-4, 2e-4, 1e-4, 5e-5])
def test_two_sphere_rebound_restitution(h):
    """Outgoing/incoming speed equals eps_n (unclamped spring-dashpot); the
    scheme is first order (predicted velocities), so the error is O(h/t_c)."""
    prm = frictionless(dt=h)
    o = O.Oracle(prm)
    o.add([1, 1], [[-1.01, 0, 0], [1.01, 0, 0]], [1, 1], [M1, M1], [[1, 0, 0], [-1, 0, 0]])
    o.step(int(0.05 / h))
    v = o.aggregates()["vA"]
    assert o.counts()[2] == 0                      # separated again
    e = v[1, 0] / 1.0
    tc = collision_time(prm["k_n"], M1 / 2, prm["eps_n"])
    assert abs(e - prm["eps_n"]) <= h / tc
    if tc / h >= 100:
        assert abs(e - prm["eps_n"]) < 1e-2
    assert abs(v[0, 0] + v[1, 0]) < 1e-13          # momentum


def test_dumbbell_rebound_uses_aggregate_mass():
    """Two aligned dumbbells colliding end-on rebound with eps_n when the
    dashpot uses the reduced mass of the *aggregates* (SetMassDEM); the
    sphere-mass reading would give a visibly different restitution.  No spin
    is induced by a central collision."""
    h = 5e-5
    prm = frictionless(dt=h)
    pos = [[-3.01, 0, 0], [-1.01, 0, 0], [1.01, 0, 0], [3.01, 0, 0]]
    o = O.Oracle(prm)
    o.add([2, 2], pos, [1] * 4, [M1] * 4, [[1, 0, 0], [-1, 0, 0]])
    o.step(int(0.06 / h))
    a = o.aggregates()
    e = a["vA"][1, 0]
    assert abs(e - 0.5) < 3e-3
    # restitution that the sphere-mass reading would produce
    mu_wrong = M1 / 2
    C = -2 * math.log(0.5) * math.sqrt(prm["k_n"] * mu_wrong / (math.pi ** 2 + math.log(0.5) ** 2))
    zeta_true = C / (2 * math.sqrt(prm["k_n"] * M1))        # true reduced mass is M1
    e_wrong = math.exp(-zeta_true * math.pi / math.sqrt(1 - zeta_true ** 2))
    assert abs(e_wrong - 0.5) > 0.05
    assert np.abs(a["wA"]).max() < 1e-12


# ---------------------------------------------------------------------------
# V3 / V4 / V5: invariants
# ---------------------------------------------------------------------------

def _seeded_cluster(seed=3, n_agg=40, G=0.0, spin=0.2, vel=0.05):
    w = W.periodic_box(seed, n_agg=n_agg, contact_seeded=True, spin_sigma=spin, vel_sigma=vel)
    # same placement, open space, optional gravity
    w.params.update(periodic=0, box=(0, 0, 0), G=G, soft_frac=0.5)
    return w


def test_linear_momentum_conserved():
    w = _seeded_cluster(G=1.0)
    o = O.Oracle(w.params).add_workload(w)
    P0 = o.diagnostics()["P"]
    scale = float((o.aggregates()["M"][:, None] * np.abs(o.aggregates()["vA"])).sum())
    o.step(60)
    assert o.counts()[2] > 0
    P1 = o.diagnostics()["P"]
    assert np.abs(P1 - P0).max() <= 1e-13 * max(scale, 1.0) * 60


def _oblique_collision(h, torque_at_centre=0):
    """Spinning rod and diamond colliding off-centre with sliding, rolling and
    twisting friction; no contacts at the start or at the end."""
    prm = dict(W.CONTACT_PARAMS, dt=h, G=0.0, soft_frac=0.5, periodic=0, box=(0, 0, 0),
               torque_at_centre=torque_at_centre)
    rot = W._random_rotation(np.random.default_rng(7))
    w = W.fixture_system(["rod", "diamond"], [[-4.6, 0.7, 0.2], [4.6, -0.9, 0.0]],
                         vel=[[2.0, 0.1, 0.0], [-2.0, 0.0, 0.1]],
                         spin=[[0.0, 0.0, 3.0], [1.0, -2.0, 0.5]], rot=[rot, None], params=prm)
    o = O.Oracle(prm).add_workload(w)
    L0 = o.diagnostics()["L"]
    n_contacts_seen = 0
    for _ in range(int(1.6 / h) // 50):
        o.step(50)
        n_contacts_seen += o.counts()[2]
    assert o.counts()[2] == 0
    return L0, o.diagnostics()["L"], n_contacts_seen


def test_angular_momentum_conserved_and_needs_contact_point():
    """Forces applied at the shared contact point give zero net torque about
    the origin at every evaluation.  Over an isolated collision (no contact
    at either end) the leapfrog's orbital torque (half at n, half at n+1)
    and the lagged spin torque (all of step n) then sum to the same total,
    so L is conserved to rounding.  Applying the forces at sphere centres
    instead (negative control) breaks it at the percent level."""
    for h in (2e-4, 1e-4, 5e-5):
        L0, L1, seen = _oblique_collision(h)
        assert seen > 0
        assert np.linalg.norm(L1 - L0) / np.linalg.norm(L0) < 1e-11
    L0, L1, _ = _oblique_collision(1e-4, torque_at_centre=1)
    bad = np.linalg.norm(L1 - L0) / np.linalg.norm(L0)
    assert bad > 1e-2


def _energy_run(h, shapes):
    prm = dict(W.CONTACT_PARAMS, dt=h, G=1.0, soft_frac=0.5, periodic=0, box=(0, 0, 0),
               eps_n=1.0, eps_t=1.0, mu_s=0.0, mu_r=0.0, mu_t=0.0)
    rng = np.random.default_rng(11)
    centres = [[-3.2, 0.3, 0.0], [3.2, -0.2, 0.4], [0.1, 3.4, -0.3], [0.2, -3.3, 0.1]]
    vel = rng.normal(0, 0.3, (4, 3))
    w = W.fixture_system(shapes, centres, vel=vel, params=prm)
    o = O.Oracle(prm).add_workload(w)
    E0 = o.diagnostics()["E"]
    o.step(int(3.0 / h))
    return abs(o.diagnostics()["E"] - E0) / abs(E0), o


def test_energy_conserved_without_damping_second_order_for_spheres():
    """eps = 1 and zero friction leave only springs and gravity: leapfrog
    energy error is O(h^2) for lone spheres."""
    shapes = ["sphere"] * 4
    e1, o = _energy_run(2e-4, shapes)
    e2, _ = _energy_run(1e-4, shapes)
    assert e1 < 1e-4
    assert e2 < e1 / 2.5


def test_energy_conserved_for_aggregates_first_order():
    shapes = ["dumbbell", "rod", "tetrahedron", "cube"]
    e1, _ = _energy_run(2e-4, shapes)
    e2, _ = _energy_run(1e-4, shapes)
    assert e1 < 1e-2
    assert e2 < e1 / 1.6


# ---------------------------------------------------------------------------
# V6 / V10: per-contact invariants
# ---------------------------------------------------------------------------

def test_coulomb_caps_and_lever_arms():
    w = W.periodic_box(5, n_agg=80, contact_seeded=True, spin_sigma=0.5, vel_sigma=0.3)
    prm = dict(w.params)
    o = O.Oracle(prm).add_workload(w)
    checked = 0
    for _ in range(5):
        o.step(4)
        p = o.pairs()
        if p["i"].size == 0:
            continue
        d = p["diag"]
        fN, FT, Fr, Fq, delta, li, lj, sliding = d.T
        tol = 1e-12 * (1 + fN)
        assert np.all(FT[sliding == 1] <= prm["mu_s"] * fN[sliding == 1] + tol[sliding == 1])
        assert np.all(Fr <= prm["mu_r"] * fN + tol)
        assert np.all(Fq <= prm["mu_t"] * fN + tol)
        xi_t = np.linalg.norm(p["hist"][:, 0:3], axis=1)
        assert np.all(prm["k_t"] * xi_t <= prm["mu_s"] * fN + tol)
        # lever arms: l_i + l_j = |d| = S - delta, contact point shared
        S = w.radius[p["i"]] + w.radius[p["j"]]
        assert np.allclose(li + lj, S - delta, rtol=0, atol=1e-13)
        si, sj = w.radius[p["i"]], w.radius[p["j"]]
        dist = S - delta
        assert np.allclose(li, (si ** 2 - sj ** 2 + dist ** 2) / (2 * dist), atol=1e-13)
        checked += p["i"].size
    assert checked > 50


def test_equal_radii_lever_arm_is_half_distance():
    prm = frictionless()
    o = O.Oracle(prm)
    o.add([1, 1], [[0, 0, 0], [1.998, 0, 0]], [1, 1], [M1, M1])
    d = o.pairs()["diag"][0]
    assert d[5] == pytest.approx(0.999, abs=1e-15) and d[6] == pytest.approx(0.999, abs=1e-15)


# ---------------------------------------------------------------------------
# spring history: closed forms with quasi-static heavy bodies
# ---------------------------------------------------------------------------

def _heavy_pair(vB=(0, 0, 0), wA=(0, 0, 0), h=1e-4):
    prm = dict(W.CONTACT_PARAMS, dt=h, G=0.0, soft_frac=0.5, periodic=0, box=(0, 0, 0),
               eps_n=1.0, eps_t=1.0)
    Mh = 1e15
    o = O.Oracle(prm)
    o.add([1, 1], [[0, 0, 0], [1.999, 0, 0]], [1, 1], [Mh, Mh], [[0, 0, 0], list(vB)],
          [list(wA), [0, 0, 0]])
    return o, prm


def test_tangential_spring_accumulates_history_then_caps():
    """B slides tangentially at u past A (both ~immovable): the spring grows
    by k_t h u per evaluation (history carried), until it reaches mu_s f_N."""
    u, h = 1.0, 1e-4
    o, prm = _heavy_pair(vB=(0, u, 0), h=h)
    for n in range(1, 30):
        o.step(1)
        d = o.pairs()["diag"][0]
        cap = prm["mu_s"] * prm["k_n"] * d[4]       # f_N = k_n delta (no dashpot)
        expect = min(prm["k_t"] * (n + 1) * h * u, cap)
        assert d[1] == pytest.approx(expect, rel=2e-3)
    assert o.pairs()["diag"][0][7] == 1.0          # sliding at the end


def test_rolling_and_twisting_springs_oppose_relative_spin():
    h, w = 1e-4, 0.3
    Rij = 0.5
    # rolling: A spins about z, contact normal along x
    o, prm = _heavy_pair(wA=(0, 0, w), h=h)
    for n in range(1, 6):
        o.step(1)
        p = o.pairs()
        F, ti = p["force"][0, :3], p["force"][0, 3:6]
        li = p["diag"][0, 5]
        tau_couple = ti - np.cross([li, 0, 0], F)
        expect = prm["k_r"] * (n + 1) * h * Rij * w
        assert expect < prm["mu_r"] * prm["k_n"] * p["diag"][0, 4]     # below the cap
        assert p["diag"][0, 2] == pytest.approx(expect, rel=1e-9)
        assert tau_couple[2] == pytest.approx(-Rij * expect, rel=1e-9)   # opposes w_A
    # twisting: A spins about the contact normal
    o, prm = _heavy_pair(wA=(w, 0, 0), h=h)
    for n in range(1, 6):
        o.step(1)
        p = o.pairs()
        expect = prm["k_q"] * (n + 1) * h * Rij * w
        assert expect < prm["mu_t"] * prm["k_n"] * p["diag"][0, 4]
        assert p["diag"][0, 3] == pytest.approx(expect, rel=1e-9)
        assert p["force"][0, 3] == pytest.approx(-Rij * expect, rel=1e-9)


# ---------------------------------------------------------------------------
# V7: torque-free rotation (closed form) and the RK5 order
# ---------------------------------------------------------------------------

def _precession_error(h, T=2.0):
    I = np.array([2.0, 2.0, 0.8])          # axisymmetric about body z
    w1, w3 = 0.7, 2.5
    q = np.array([1.0, 0, 0, 0])
    wb = np.array([w1, 0.0, w3])
    N = np.zeros(3)
    L0 = O.quat_matrix(q) @ (I * wb)
    n = int(round(T / h))
    for _ in range(n):
        q, wb, _ = O.rotate(q, wb, I, N, h)
    Om = w3 * (I[2] - I[0]) / I[0]
    exact = np.array([w1 * math.cos(Om * T), w1 * math.sin(Om * T), w3])
    L1 = O.quat_matrix(q) @ (I * wb)
    return np.abs(wb - exact).max(), np.abs(L1 - L0).max()


def test_torque_free_axisymmetric_precession_and_fifth_order():
    e1, l1 = _precession_error(0.04)
    e2, l2 = _precession_error(0.02)
    assert e1 < 1e-6 and l1 < 1e-6
    assert e1 / e2 > 20.0                   # ~2^5 for a fifth-order step


def test_torque_free_asymmetric_conserves_L_and_energy():
    I = np.array([1.0, 2.0, 3.5])
    q = np.array([0.9, 0.1, -0.3, 0.2]); q /= np.linalg.norm(q)
    wb = np.array([0.3, 1.7, -0.4])
    L0 = O.quat_matrix(q) @ (I * wb)
    E0 = 0.5 * np.dot(wb, I * wb)
    for _ in range(2000):
        q, wb, _ = O.rotate(q, wb, I, np.zeros(3), 1e-3)
    L1 = O.quat_matrix(q) @ (I * wb)
    assert np.abs(L1 - L0).max() < 1e-10
    assert abs(0.5 * np.dot(wb, I * wb) - E0) < 1e-10


def _euler_closed_form(I, w0, t):
    """Torque-free body-frame spin of an asymmetric body, I1 < I2 < I3, with
    L^2 > 2 E I2 (the spin circulates about the axis of largest moment):
    w1 = A1 cn(u), w2 = A2 sn(u), w3 = A3 dn(u), u = lam t + u0, the
    textbook solution of Euler's equations by Jacobi elliptic functions.
    Amplitudes and rate from the two invariants 2E = sum I w^2 and
    L^2 = sum I^2 w^2; u0 from the initial phase by the incomplete integral
    of the first kind."""
    from scipy.special import ellipj, ellipkinc
    I1, I2, I3 = I
    E2 = float(np.dot(I, w0 * w0))
    L2 = float(np.dot(I * I, w0 * w0))
    assert I1 < I2 < I3 and L2 > E2 * I2
    A1 = math.sqrt((E2 * I3 - L2) / (I1 * (I3 - I1)))
    A3 = math.copysign(math.sqrt((L2 - E2 * I1) / (I3 * (I3 - I1))), w0[2])
    lam = math.sqrt((I3 - I2) * (L2 - E2 * I1) / (I1 * I2 * I3))
    A2 = (I3 - I1) * A3 * A1 / (I2 * lam)
    m = (I2 - I1) * (E2 * I3 - L2) / ((I3 - I2) * (L2 - E2 * I1))
    phi0 = math.atan2(w0[1] / A2, w0[0] / A1)
    u0 = ellipkinc(phi0, m)
    sn, cn, dn, _ = ellipj(lam * np.asarray(t) + u0, m)
    return np.stack([A1 * cn, A2 * sn, A3 * dn], -1)


def test_torque_free_asymmetric_matches_jacobi_elliptic_solution():
    """V7 for a body with three different moments: the RK5 spin follows the
    Jacobi-elliptic closed form over several tumbling periods, and the
    orientation carries the body-frame angular momentum I w_b(t) of that
    closed form onto the fixed space-frame L (so the quaternion kinematics
    are pinned too, not only Euler's equations)."""
    I = np.array([1.0, 2.0, 3.5])
    w0 = np.array([0.3, 1.7, -0.4])
    q = np.array([0.9, 0.1, -0.3, 0.2])
    q /= np.linalg.norm(q)
    L0 = O.quat_matrix(q) @ (I * w0)
    h, n_out, every = 1e-3, 20, 500            # 10 time units, ~3 tumbling periods
    ts, got, Rs = [], [], []
    wb = w0.copy()
    for k in range(1, n_out + 1):
        for _ in range(every):
            q, wb, _ = O.rotate(q, wb, I, np.zeros(3), h)
        ts.append(k * every * h)
        got.append(wb.copy())
        Rs.append(O.quat_matrix(q))
    exact = _euler_closed_form(I, w0, np.array(ts))
    assert np.abs(np.array(got) - exact).max() < 1e-9
    # the spin really tumbles: w2 changes sign along the run
    assert exact[:, 1].min() < -1.0 and exact[:, 1].max() > 1.0
    for R, we in zip(Rs, exact):
        # R(q(t)) I w_b(t) with the closed-form w_b is the fixed L
        assert np.abs(R @ (I * we) - L0).max() < 1e-9


def test_constant_torque_spin_up_about_principal_axis():
    """Constant space-frame torque along a principal axis of a body at rest:
    w(t) = N t / I exactly (linear), so RK5 is exact up to rounding."""
    I = np.array([1.5, 2.5, 4.0])
    q = np.array([1.0, 0, 0, 0])
    wb = np.zeros(3)
    for _ in range(100):
        q, wb, _ = O.rotate(q, wb, I, np.array([0, 0, 2.0]), 1e-2)
    assert wb[2] == pytest.approx(2.0 * 1.0 / 4.0, rel=1e-12)
    assert abs(wb[0]) < 1e-14 and abs(wb[1]) < 1e-14


# ---------------------------------------------------------------------------
# V8 / V11: set-up closed forms
# ---------------------------------------------------------------------------

INERTIA = {  # principal moments in units of m s^2 (equal touching spheres)
    "sphere": (0.4, 0.4, 0.4),
    "dumbbell": (0.8, 2.8, 2.8),
    "rod": (1.6, 21.6, 21.6),
    "cube": (19.2, 19.2, 19.2),
    "tetrahedron": (5.6, 5.6, 5.6),
    "diamond": (3.6, 7.6, 9.6),
}


@pytest.mark.parametrize("name", list(INERTIA))
def test_inertia_of_paper_shapes(name):
    s, m = 0.7, 2.3
    rot = W._random_rotation(np.random.default_rng(len(name)))
    pos = W.shape_fixture(name, s) @ rot.T + np.array([5.0, -2.0, 1.0])
    n = pos.shape[0]
    M, r, I, q, b = O.setup_body(pos, np.full(n, s), np.full(n, m))
    assert M == pytest.approx(n * m, rel=1e-15)
    assert np.allclose(r, [5.0, -2.0, 1.0], atol=1e-13)
    assert np.allclose(np.sort(I), np.array(INERTIA[name]) * m * s * s, rtol=1e-12)
    R = O.quat_matrix(q)
    assert np.allclose(R @ R.T, np.eye(3), atol=1e-14)
    assert np.linalg.det(R) == pytest.approx(1.0, abs=1e-14)
    assert np.allclose(b @ R.T + r, pos, atol=1e-13)     # SetBodyPos inverts SetSpacePos


def test_lone_sphere_special_case():
    """Single spheres: I = 2/5 m s^2, no gravity torque, and the member
    velocity of Eq. 3 reduces to the predicted centre-of-mass velocity."""
    prm = dict(W.CONTACT_PARAMS, dt=1e-3, G=1.0, soft_frac=0.5, periodic=0, box=(0, 0, 0))
    rng = np.random.default_rng(2)
    pos = rng.uniform(-10, 10, (6, 3))
    rad = rng.uniform(0.8, 1.2, 6)
    o = O.Oracle(prm).add([1] * 6, pos, rad, W.sphere_mass(rad), rng.normal(0, 0.1, (6, 3)))
    a = o.aggregates()
    assert np.allclose(a["I"], 0.4 * W.sphere_mass(rad)[:, None] * rad[:, None] ** 2, rtol=1e-14)
    for _ in range(3):
        a_prev = o.aggregates()["aA"]
        o.step(1)
        a = o.aggregates()
        F = o.spheres()["F"]
        # gravity acts at sphere centres: no torque beyond rounding of b_i ~ 0
        assert np.abs(a["NA"]).max() <= 1e-14 * np.abs(F).max()
        v_half = a["vA"] - 0.5 * prm["dt"] * a["aA"]
        expect = v_half + 0.5 * prm["dt"] * a_prev          # Eq. 3 with w = 0
        assert np.allclose(o.spheres()["v"], expect, rtol=0, atol=1e-15)


def test_predicted_velocity_matches_rigid_motion():
    """For a force-free spinning aggregate the member velocity of Eq. 3 is
    the time derivative of r_A + R b_i (central difference, O(h^2))."""
    prm = frictionless(dt=1e-3)
    rot = W._random_rotation(np.random.default_rng(4))
    w = W.fixture_system(["diamond"], [[0, 0, 0]], vel=[[0.3, -0.2, 0.1]],
                         spin=[[0.4, 1.1, -0.7]], rot=[rot], params=prm)
    o = O.Oracle(prm).add_workload(w)
    rs, vs = [], []
    for _ in range(3):
        o.step(1)
        s = o.spheres()
        rs.append(s["r"]); vs.append(s["v"])
    fd = (rs[2] - rs[0]) / (2 * prm["dt"])
    assert np.abs(fd - vs[1]).max() < 1e-5


# ---------------------------------------------------------------------------
# V9: pair search against an independent k-d tree query
# ---------------------------------------------------------------------------

@pytest.mark.parametrize("periodic", [False, True])
def test_pair_search_matches_kdtree(periodic):
    from scipy.spatial import cKDTree
    w = W.periodic_box(9, n_agg=150, contact_seeded=True)
    L = w.params["box"][0]
    agg = w.agg_of_sphere()
    box = (L, L, L) if periodic else None
    keys = O.find_contacts(w.pos, w.radius, agg, box)
    pos = np.mod(w.pos, L) if periodic else w.pos
    tree = cKDTree(pos, boxsize=L if periodic else None)
    cand = np.array(sorted(tree.query_pairs(2.4 + 1e-9)), dtype=np.int64)
    d = pos[cand[:, 1]] - pos[cand[:, 0]]
    if periodic:
        d -= L * np.round(d / L)
    dist = np.sqrt((d * d).sum(1))
    S = w.radius[cand[:, 0]] + w.radius[cand[:, 1]]
    other = agg[cand[:, 0]] != agg[cand[:, 1]]
    assert np.abs(dist - S)[other].min() > 1e-9       # no threshold coin-flips
    sel = (dist < S) & other
    ref = (cand[sel, 0].astype(np.uint64) << np.uint64(32)) | cand[sel, 1].astype(np.uint64)
    assert keys.size > 100
    assert np.array_equal(keys, np.sort(ref))


def test_pair_search_skips_same_aggregate_and_is_strict():
    pos = np.array([[0, 0, 0], [2.0, 0, 0], [4.0, 0, 0], [5.5, 0, 0]])
    rad = np.array([1.0, 1.0, 1.0, 1.0])
    agg = np.array([0, 1, 1, 2], dtype=np.int32)
    keys = O.find_contacts(pos, rad, agg)
    # (0,1): touching exactly -> strict test excludes; (1,2) same aggregate;
    # (2,3): overlapping
    assert keys.tolist() == [(2 << 32) | 3]


# ---------------------------------------------------------------------------
# V12 / V13: gravity closed forms
# ---------------------------------------------------------------------------

def test_softened_pair_gravity_closed_form():
    for dist in (0.3, 1.0, 7.0):
        pos = np.array([[0, 0, 0], [dist, 0, 0]], dtype=float)
        m = np.array([2.0, 3.0])
        s = np.array([0.9, 1.1])
        F = O.gravity(pos, m, s, 1.7, 0.5, [0, 1])
        eps = 0.5 * (0.9 + 1.1) / 2
        f = 1.7 * 6.0 * dist / (dist ** 2 + eps ** 2) ** 1.5
        assert F[0, 0] == pytest.approx(f, rel=1e-14)
        assert F[1, 0] == pytest.approx(-f, rel=1e-14)


def test_circular_two_body_orbit_period():
    G, m, d = 1.0, 5.0, 20.0
    v = math.sqrt(G * m / (2 * d))                     # each body, equal masses
    T = 2 * math.pi * math.sqrt(d ** 3 / (G * 2 * m))
    errs = []
    for h in (T / 400, T / 800):
        prm = dict(W.CONTACT_PARAMS, dt=h, G=G, soft_frac=1e-3, periodic=0, box=(0, 0, 0))
        o = O.Oracle(prm).add([1, 1], [[-d / 2, 0, 0], [d / 2, 0, 0]], [0.5, 0.5], [m, m],
                              [[0, -v, 0], [0, v, 0]])
        o.step(int(round(T / h)))
        errs.append(np.linalg.norm(o.aggregates()["rA"][1] - [d / 2, 0, 0]) / d)
    assert errs[0] < 2e-3
    assert errs[0] / errs[1] > 3.0                     # second order


def _fibonacci_shell(n, R):
    k = np.arange(n) + 0.5
    phi = np.arccos(1 - 2 * k / n)
    th = math.pi * (1 + 5 ** 0.5) * k
    return R * np.stack([np.cos(th) * np.sin(phi), np.sin(th) * np.sin(phi), np.cos(phi)], 1)


def test_shell_theorem_and_third_law():
    n, R = 4000, 10.0
    shell = _fibonacci_shell(n, R)
    probes = np.array([[0.0, 0, 0], [3.0, 1.0, -2.0], [25.0, 0, 0], [0, -40.0, 3.0]])
    pos = np.concatenate([shell, probes])
    m = np.concatenate([np.full(n, 1.0 / n), np.full(4, 1e-9)])
    s = np.full(n + 4, 1e-6)
    F = O.gravity(pos, m, s, 1.0, 0.0, np.arange(n, n + 4))
    f = F / 1e-9
    assert np.linalg.norm(f[0]) < 1e-3 and np.linalg.norm(f[1]) < 1e-3
    for k in (2, 3):
        r = np.linalg.norm(probes[k])
        assert np.linalg.norm(f[k]) == pytest.approx(1.0 / r ** 2, rel=2e-3)
        assert np.dot(f[k], probes[k]) < 0
    Fall = O.gravity(pos[:300], m[:300], s[:300], 1.0, 0.3)
    assert np.abs(Fall.sum(0)).max() < 1e-15 * np.abs(Fall).sum()


# ---------------------------------------------------------------------------
# V14: invariances of the force evaluation
# ---------------------------------------------------------------------------

def test_galilean_rotation_and_relabel_invariance():
    w = _seeded_cluster(seed=8, n_agg=30, G=1.0)
    base = O.Oracle(w.params).add_workload(w)
    F0 = base.spheres()["F"]
    T0 = base.spheres()["tau"]
    assert base.counts()[2] > 0
    # Galilean boost
    o = O.Oracle(w.params).add(w.counts, w.pos, w.radius, w.mass, w.agg_vel + [3.0, -1.0, 2.0],
                               w.agg_spin)
    assert np.allclose(o.spheres()["F"], F0, rtol=0, atol=1e-9 * np.abs(F0).max())
    # global rotation
    Rg = W._random_rotation(np.random.default_rng(1))
    o = O.Oracle(w.params).add(w.counts, w.pos @ Rg.T, w.radius, w.mass, w.agg_vel @ Rg.T,
                               w.agg_spin @ Rg.T)
    assert np.allclose(o.spheres()["F"], F0 @ Rg.T, rtol=0, atol=1e-9 * np.abs(F0).max())
    assert np.allclose(o.spheres()["tau"], T0 @ Rg.T, rtol=0, atol=1e-9 * np.abs(T0).max())
    # relabel aggregates (reverse order)
    off = w.offsets()
    order = np.arange(w.n_agg)[::-1]
    sph = np.concatenate([np.arange(off[a], off[a + 1]) for a in order])
    o = O.Oracle(w.params).add(w.counts[order], w.pos[sph], w.radius[sph], w.mass[sph],
                               w.agg_vel[order], w.agg_spin[order])
    assert np.allclose(o.spheres()["F"], F0[sph], rtol=0, atol=1e-9 * np.abs(F0).max())


def test_subset_evaluation_matches_full_evaluation():
    """The one-sphere-at-a-time evaluation used for sampled checks at full
    size reproduces the full evaluation at t0 (same pair order)."""
    w = _seeded_cluster(seed=12, n_agg=50, G=1.0)
    o = O.Oracle(w.params).add_workload(w)
    s = o.spheres()
    idx = np.arange(0, w.n_sph, 3)
    F, T = o.eval_subset(idx)
    assert np.array_equal(F, s["F"][idx])
    assert np.array_equal(T, s["tau"][idx])


# ---------------------------------------------------------------------------
# spin-up forcing and the bulk radius diagnostic
# ---------------------------------------------------------------------------

def test_spin_up_forcing_adds_spin_and_angular_momentum():
    """Each step adds dw about +z through the pile's centre of mass to every
    body: space spins grow by n dw exactly, and L_z grows by
    dw sum(M r_perp^2 + I_zz) per step (bodies barely move here)."""
    dw = 1e-3
    prm = dict(W.CONTACT_PARAMS, dt=1e-3, G=0.0, soft_frac=0.5, periodic=0, box=(0, 0, 0),
               spin_dw=dw)
    ang = np.linspace(0, 2 * np.pi, 9)[:-1]
    pos = np.stack([5 * np.cos(ang), 5 * np.sin(ang), np.linspace(-1, 1, 8)], 1) + [1.0, 2.0, 0.0]
    rad = np.full(8, 0.9)
    m = W.sphere_mass(rad)
    o = O.Oracle(prm).add([1] * 8, pos, rad, m)
    L0 = o.diagnostics()["L"][2]
    n = 20
    o.step(n)
    a = o.aggregates()
    w_space = np.array([O.quat_matrix(q) @ wb for q, wb in zip(a["q"], a["wb"])])
    assert np.allclose(w_space[:, 2], n * dw, rtol=1e-12)
    assert np.abs(w_space[:, :2]).max() < 1e-15
    com = (m[:, None] * pos).sum(0) / m.sum()
    rp2 = ((pos - com)[:, :2] ** 2).sum(1)
    expect = n * dw * (m * rp2 + 0.4 * m * rad ** 2).sum()
    # the orbital part about the origin also picks up r_A x (dw z x (r_A - com))
    assert o.diagnostics()["L"][2] - L0 == pytest.approx(
        expect + n * dw * (m * ((pos[:, :2] - com[:2]) * com[:2]).sum(1)).sum(), rel=1e-4)


def test_bulk_radius_of_uniform_ball():
    """A uniform ball of radius R has sqrt(5/3 <r^2>) = R."""
    g = np.arange(-20, 21) * 0.5
    p = np.stack(np.meshgrid(g, g, g, indexing="ij"), -1).reshape(-1, 3)
    p = p[np.linalg.norm(p, axis=1) <= 10.0]
    rad = np.full(len(p), 0.01)
    prm = dict(W.CONTACT_PARAMS, dt=1e-3, G=0.0, soft_frac=0.5, periodic=0, box=(0, 0, 0))
    o = O.Oracle(prm).add([1] * len(p), p, rad, W.sphere_mass(rad))
    assert o.diagnostics()["R_bulk"] == pytest.approx(10.0, rel=2e-2)


# ---------------------------------------------------------------------------
# point-mass perturber (tidal flyby)
# ---------------------------------------------------------------------------

def _kepler_pair(h_frac):
    G, m, Mp, d = 1.0, 4.0, 12.0, 30.0
    v = math.sqrt(G * (m + Mp) / d)
    T = 2 * math.pi * math.sqrt(d ** 3 / (G * (m + Mp)))
    h = T * h_frac
    prm = dict(W.CONTACT_PARAMS, dt=h, G=G, soft_frac=0.5, periodic=0, box=(0, 0, 0))
    o = O.Oracle(prm)
    o.set_perturber(Mp, [d * m / (m + Mp), 0, 0], [0, v * m / (m + Mp), 0])
    o.add([1], [[-d * Mp / (m + Mp), 0, 0]], [0.5], [m], [[0, -v * Mp / (m + Mp), 0]])
    P0 = m * o.aggregates()["vA"][0] + Mp * o.perturber()[1]
    o.step(int(round(1.0 / h_frac)))
    rp, vp, _ = o.perturber()
    P1 = m * o.aggregates()["vA"][0] + Mp * vp
    return np.linalg.norm(rp - [d * m / (m + Mp), 0, 0]) / d, np.abs(P1 - P0).max()


def test_perturber_two_body_orbit_and_momentum():
    """A lone sphere and the perturber on a circular orbit about their common
    centre of mass return after one period (second order); total momentum
    (spheres + perturber) is conserved to rounding."""
    e1, dp1 = _kepler_pair(1 / 400)
    e2, dp2 = _kepler_pair(1 / 800)
    assert e1 < 5e-3 and e1 / e2 > 3.0
    assert dp1 < 1e-12 and dp2 < 1e-12


def test_flyby_orbit_reaches_its_periapsis():
    """The inbound hyperbolic initial condition (e = 2) passes a point-like
    pile at the requested periapsis."""
    G, m, Mp, q = 1.0, 1.0, 1000.0, 10.0
    pos, vel = W.flyby_orbit(m, Mp, q, ecc=2.0, start_factor=10.0, G=G)
    h = 2e-3
    prm = dict(W.CONTACT_PARAMS, dt=h, G=G, soft_frac=0.5, periodic=0, box=(0, 0, 0))
    # the pile is at rest at the origin, the perturber carries the relative
    # velocity; move to the centre-of-mass frame so the relative orbit holds
    vc = Mp * vel / (m + Mp)
    rc = Mp * pos / (m + Mp)
    o = O.Oracle(prm)
    o.set_perturber(Mp, pos - rc, vel - vc)
    o.add([1], [-rc], [0.5], [m], [-vc])
    dmin = np.inf
    for _ in range(600):
        o.step(10)
        rp = o.perturber()[0]
        dmin = min(dmin, np.linalg.norm(rp - o.aggregates()["rA"][0]))
    assert dmin == pytest.approx(q, rel=2e-3)
