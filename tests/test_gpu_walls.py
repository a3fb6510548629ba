"""Parity of the walled workloads with the FP64 oracle (needs an MI355X).

Box filling under a uniform field (open-topped box, wall contacts seeded on
the floor) and the Brazil-nut set-up (a large intruder among aggregates, all
walls shaken sinusoidally).  Each test prints its case before the GPU runs.
"""
import sys

import numpy as np
import pytest

import oracle as O
from paper_2311_11322_amd import workloads as W
from tests.gpu_util import compare_states, oracle_keys, rel_err

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def D():
    from paper_2311_11322_amd import dem
    dem.lib()
    return dem


def say(*a):
    print("[case]", *a, flush=True)
    sys.stdout.flush()


def _pair(D, w, precision=0):
    sim = D.Sim(w.params, precision=precision)
    sim.add_workload(w)
    o = O.Oracle(w.params).add_workload(w)
    return sim, o


def _small_box(seed=2, shape="mixed"):
    """A partly filled box with floor and aggregate contacts seeded, and
    random velocities and spins so that every friction term is active."""
    w = W.box_fill(seed=seed, n_sph=240, shape=shape, base=14, height=40, z_range=(0, 30),
                   floor_seeded=0.3, contact_seeded=True)
    rng = np.random.default_rng(seed + 100)
    w.agg_vel[:] = rng.normal(0.0, 0.1, w.agg_vel.shape)
    w.agg_spin[:] = rng.normal(0.0, 0.3, w.agg_spin.shape)
    return w


@pytest.mark.parametrize("shape", ["mixed", "sphere", "cube"])
def test_box_fill_parity(D, shape):
    """t0, one step and then 40 more: contacts with the floor and side walls
    in the contact list, forces and the uniform field in the state."""
    say("box fill", shape)
    w = _small_box(shape=shape)
    sim, o = _pair(D, w)
    compare_states(sim, o)
    keys = oracle_keys(o)
    assert (keys & np.uint64(0xFFFFFFFF) >= np.uint64(w.n_sph)).any()     # wall contacts
    sim.step(1)
    o.step(1)
    compare_states(sim, o)
    for _ in range(4):
        sim.step(10)
        o.step(10)
        compare_states(sim, o, tol=1e-10)


@pytest.mark.parametrize("gravity", ["direct", "tree"])
def test_walled_box_with_self_gravity_parity(D, gravity):
    """Walls, the uniform field and self-gravity in one pile (exact sum, or
    the tree): the same bar as without gravity."""
    say("walled box + self-gravity", gravity)
    w = _small_box(shape="mixed", seed=9)
    w.params.update(G=0.05)
    if gravity == "tree":
        w.params.update(gravity_tree=1, theta=0.5, tree_leaf=16, tree_order=4)
    sim, o = _pair(D, w)
    compare_states(sim, o)
    sim.step(1)
    o.step(1)
    compare_states(sim, o)
    sim.step(10)
    o.step(10)
    compare_states(sim, o, tol=1e-10)


def test_box_fill_wall_contacts_form_and_break(D):
    """Aggregates dropped from just above the floor hit it and bounce: the
    wall contacts of the last step agree with the oracle throughout."""
    say("box fill drop")
    w = W.box_fill(seed=4, n_sph=200, base=24, height=40, z_range=(0.0, 2.5))
    w.agg_vel[:, 2] = -5.0
    sim, o = _pair(D, w)
    n_wall = []
    for _ in range(8):
        sim.step(50)
        o.step(50)
        compare_states(sim, o, tol=1e-9)
        n_wall.append(int((oracle_keys(o) & np.uint64(0xFFFFFFFF) >= np.uint64(w.n_sph)).sum()))
    print("wall contacts", n_wall)
    assert max(n_wall) > 10 and min(n_wall) < max(n_wall)


def test_brazil_nut_shaken_walls_parity(D):
    """Large intruder among aggregates, every wall oscillating: the floor
    comes up into the bed in the first steps."""
    say("brazil nut small")
    w = W.brazil_nut(seed=3, n_sph=300, intruder_radius=4.0, base=16, fill_height=30.0,
                     floor_seeded=0.5)
    sim, o = _pair(D, w)
    compare_states(sim, o)
    for n in (1, 9, 40, 150):
        sim.step(n)
        o.step(n)
        compare_states(sim, o, tol=1e-9)
    walls = oracle_keys(o) & np.uint64(0xFFFFFFFF) >= np.uint64(w.n_sph)
    assert walls.sum() >= 5


def test_box_fill_fp32_force_form(D):
    """FP32 pair forces: sphere forces within 1e-5 of the oracle (max norm),
    contact list exact."""
    say("box fill fp32-force")
    w = _small_box(seed=5)
    sim, o = _pair(D, w, precision=D.PREC_FP32_FORCE)
    sim.step(1)
    o.step(1)
    g = sim.read_state(["sph_force", "agg_pos"], pairs=True)
    assert np.array_equal(g["pair_keys"], oracle_keys(o))
    assert rel_err(g["sph_force"], o.spheres()["F"]) <= 1e-5


def test_walled_piles_in_engine_match_alone(D):
    """A box fill, a Brazil-nut set-up and a self-gravitating pile stepped
    together in one engine give the states each gives alone, bit for bit."""
    say("engine walls + pile")
    ws = [_small_box(seed=6), W.brazil_nut(seed=7, n_sph=200, intruder_radius=3.0, base=14,
                                            fill_height=24.0),
          W.collapse_cloud(8, n_agg=60, contact_seeded=True)]
    alone = []
    for w in ws:
        s = D.Sim(w.params)
        s.add_workload(w)
        s.step(7)
        alone.append(s.read_state(pairs=True))
        s.close()
    eng = D.Engine(1 << 33)
    sims = []
    for w in ws:
        s = D.Sim(w.params)
        s.add_workload(w)
        eng.attach(s)
        sims.append(s)
    assert eng.step(7) == D.DEM_OK
    for s in list(eng.sims):
        eng.detach(s)
    for k, s in enumerate(sims):
        got = s.read_state(pairs=True)
        for f in ("agg_pos", "agg_vel", "agg_quat", "pair_keys", "pair_hist", "sph_force"):
            assert np.array_equal(got[f], alone[k][f]), (k, f)


def test_box_fill_full_size_parity(D):
    """The box-filling workload at its full size (6,400 spheres, 40 x 40 x 240
    box), floor and aggregate contacts seeded: t0, one step and 20 more
    against the brute-force oracle, in the configuration the bench runs."""
    w = W.box_fill(seed=11, floor_seeded=0.3, contact_seeded=True, z_range=(0, 120))
    say("box fill full size", w.n_sph)
    sim, o = _pair(D, w)
    compare_states(sim, o)
    sim.step(1)
    o.step(1)
    compare_states(sim, o)
    sim.step(20)
    o.step(20)
    compare_states(sim, o, tol=1e-10)
    assert (oracle_keys(o) & np.uint64(0xFFFFFFFF) >= np.uint64(w.n_sph)).sum() > 50


def test_brazil_nut_full_size_parity(D):
    """The Brazil-nut set-up at its full size (intruder + 4,000 grain spheres),
    walls shaken, grains seeded on the floor: t0, one step and 30 more."""
    w = W.brazil_nut(seed=12, floor_seeded=0.3)
    say("brazil nut full size", w.n_sph)
    sim, o = _pair(D, w)
    compare_states(sim, o)
    sim.step(1)
    o.step(1)
    compare_states(sim, o)
    sim.step(30)
    o.step(30)
    compare_states(sim, o, tol=1e-10)


def test_walled_checkpoint_restore_bit_identical(D):
    """A box fill with floor and wall contacts checkpointed after 3 steps
    and restored into a fresh system (wall partners n_sph + w in the keys)
    continues bit for bit like the uninterrupted run."""
    say("walled checkpoint/restore")
    w = _small_box(seed=4)
    a = D.Sim(w.params)
    a.add_workload(w)
    a.step(3)
    ck = a.checkpoint()
    assert (ck["pair_keys"] & np.uint64(0xFFFFFFFF) >= np.uint64(w.n_sph)).any()
    a.step(5)
    ref = a.read_state(pairs=True)
    b = D.Sim(w.params)
    b.add_workload(w)
    b.restore(ck)
    b.step(5)
    got = b.read_state(pairs=True)
    for k in ("agg_pos", "agg_vel", "agg_acc", "agg_torque", "agg_quat", "pair_keys", "pair_hist",
              "sph_force"):
        assert np.array_equal(got[k], ref[k]), k


def _walled_lattice():
    """Lone unit spheres stacked 6 x 6 x 8 in a box whose side walls and
    floor they touch, falling onto each other: the contacts grow from about
    1.1 to 2.8 per sphere within a few steps."""
    B = 11.998
    g = np.arange(6) * 2.0 + 0.999
    z = np.arange(8) * 2.01 + 0.999
    pos = np.stack(np.meshgrid(g, g, z, indexing="ij"), -1).reshape(-1, 3)
    n = len(pos)
    prm = dict(W.CONTACT_PARAMS, dt=5e-4, G=0.0, soft_frac=0.5, periodic=0, box=(0, 0, 0),
               g=(0.0, 0.0, -2.0), walls=W.open_box_walls(B, B))
    vel = np.zeros((n, 3))
    vel[:, 2] = -1.0
    one = np.ones(n)
    return W.Workload("walled lattice", np.ones(n, np.int32), pos, one, W.sphere_mass(one), vel,
                      np.zeros((n, 3)), prm, 1)


def test_walled_capacity_overflow_then_reserve(D):
    """A walled system with room for two contacts per sphere overflows
    (CAPACITY, state rolled back to the failing step's start); growing the
    capacity keeps every contact's spring history, wall contacts included,
    and the run then continues bit for bit like a roomy one."""
    say("walled capacity overflow + reserve")
    w = _walled_lattice()
    small = D.Sim(w.params, max_contacts=2)
    small.add_workload(w)
    code = None
    for _ in range(40):
        try:
            small.step(1)
        except D.DemError as e:
            code = e.code
            break
    assert code == D.DEM_ERR_CAPACITY
    st = small.read_state(["agg_pos"], pairs=True)
    k = st["step"]
    assert k >= 1 and (st["pair_keys"] & np.uint64(0xFFFFFFFF) >= np.uint64(w.n_sph)).any()
    ref = D.Sim(w.params, max_contacts=16)
    ref.add_workload(w)
    ref.step(k)
    rs = ref.read_state(["agg_pos"], pairs=True)
    for f in ("agg_pos", "pair_keys", "pair_hist"):
        assert np.array_equal(st[f], rs[f]), f
    small.reserve_contacts(16)
    got = small.read_state(["agg_pos"], pairs=True)
    for f in ("agg_pos", "pair_keys", "pair_hist"):
        assert np.array_equal(got[f], rs[f]), f
    small.step(10)
    ref.step(10)
    a, b = small.read_state(pairs=True), ref.read_state(pairs=True)
    assert a["n_pairs"] > 2 * w.n_sph
    for f in ("agg_pos", "agg_vel", "pair_keys", "pair_hist", "sph_force"):
        assert np.array_equal(a[f], b[f]), f


def test_search_lane_counts_agree(D):
    """The contact search gives each sphere eight lanes in launches of few
    spheres and four in launches of many: a Brazil-nut set-up (big intruder
    searched apart, shaken walls) alone, and together with eight more in one
    engine (36k spheres), gives the same state, contacts and history bit for
    bit (grains seeded on the floor, so contacts and wall contacts exist
    from the start)."""
    say("Brazil nut alone (8 lanes) vs in a 36k-sphere engine (4 lanes)")
    w = W.brazil_nut(seed=7, floor_seeded=0.3)
    s = D.Sim(w.params)
    s.add_workload(w)
    s.step(30)
    alone = s.read_state(pairs=True)
    s.close()
    assert alone["pair_keys"].size > 0
    others = [W.brazil_nut(seed=20 + k, floor_seeded=0.3) for k in range(8)]
    assert w.n_sph + sum(o.n_sph for o in others) >= 32768
    eng = D.Engine(1 << 34)
    sims = []
    for x in [w] + others:
        t = D.Sim(x.params)
        t.add_workload(x)
        eng.attach(t)
        sims.append(t)
    assert eng.step(30) == D.DEM_OK
    for t in list(eng.sims):
        eng.detach(t)
    got = sims[0].read_state(pairs=True)
    for t in sims:
        t.close()
    for f in ("agg_pos", "agg_vel", "agg_quat", "agg_spin_body", "pair_keys", "pair_hist",
              "sph_force", "sph_torque"):
        assert np.array_equal(got[f], alone[f]), f
