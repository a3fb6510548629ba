"""Parity of the HIP library with the FP64 oracle (needs an MI355X).

Each test prints the case it runs before touching the GPU.
"""
import sys

import numpy as np
import pytest

import oracle as O
from paper_2311_11322_amd import workloads as W
from tests.gpu_util import compare_states, rel_err

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def D():
    from paper_2311_11322_amd import dem
    dem.lib()
    return dem


def say(*a):
    print("[case]", *a, flush=True)
    sys.stdout.flush()


# ---------------------------------------------------------------------------
# contact search: bit-exact against brute force
# ---------------------------------------------------------------------------

@pytest.mark.parametrize("n_agg,periodic", [(1, False), (2, True), (150, True), (150, False),
                                            (700, True), (700, False), (2500, True)])
def test_find_contacts_bit_exact(D, n_agg, periodic):
    say("find_contacts", n_agg, periodic)
    w = W.periodic_box(21 + n_agg, n_agg=n_agg, contact_seeded=True)
    L = w.params["box"][0]
    agg = w.agg_of_sphere()
    box = (L, L, L) if periodic else None
    ref = O.find_contacts(w.pos, w.radius, agg, box)
    got = D.find_contacts(w.pos, w.radius, agg, box)
    assert np.array_equal(got, ref)
    if n_agg >= 150:
        assert ref.size > n_agg // 2


def test_degenerate_systems(D):
    """An empty contact search finds nothing; one lone sphere drifts and
    spins freely (its gravity excludes itself); one spinning 8-sphere
    aggregate alone feels no net force or torque from its own members'
    gravity and rotates torque-free -- each against the oracle."""
    say("degenerate systems")
    z = np.zeros((0, 3))
    assert D.find_contacts(z, np.zeros(0), np.zeros(0, np.int32)).size == 0
    prm = dict(W.CONTACT_PARAMS, dt=5e-4, G=1.0, soft_frac=0.5, periodic=0, box=(0, 0, 0))
    rng = np.random.default_rng(8)
    rel, rad = W.random_cluster(rng, 8)
    for counts, pos, r in (([1], np.array([[0.3, -0.2, 0.1]]), np.array([1.1])),
                           ([8], rel + 5.0, rad)):
        w = W.Workload("degenerate", np.array(counts, np.int32), pos, r, W.sphere_mass(r),
                       np.array([[0.2, -0.1, 0.05]]), np.array([[0.1, 0.4, -0.3]]), prm, 5)
        sim, o = _pair(D, w)
        compare_states(sim, o)
        sim.step(5)
        o.step(5)
        compare_states(sim, o, tol=1e-10)
        a = sim.read_state(["agg_acc", "agg_torque"])
        scale = float(np.abs(o.spheres()["F"]).max()) if counts[0] > 1 else 1.0
        assert np.abs(a["agg_acc"]).max() <= 1e-12 * max(scale, 1.0)


def test_find_contacts_wrapped_positions(D):
    """Whole aggregates shifted by +-L: binning wraps the centres and both
    sides apply the same minimum-image rule."""
    say("find_contacts wrapped")
    w = W.periodic_box(5, n_agg=200, contact_seeded=True)
    L = w.params["box"][0]
    rng = np.random.default_rng(0)
    shift = np.repeat(rng.integers(-1, 2, w.n_agg), w.counts)[:, None] * L
    pos = w.pos + shift * np.array([1.0, 0.0, 1.0])
    agg = w.agg_of_sphere()
    ref = O.find_contacts(pos, w.radius, agg, (L, L, L))
    got = D.find_contacts(pos, w.radius, agg, (L, L, L))
    assert np.array_equal(got, ref)


# ---------------------------------------------------------------------------
# one step and a few steps against the oracle
# ---------------------------------------------------------------------------

def _pair(D, w, precision=0):
    sim = D.Sim(w.params, precision=precision)
    sim.add_workload(w)
    o = O.Oracle(w.params).add_workload(w)
    return sim, o


def test_step_parity_periodic_contacts(D):
    """Contact-only periodic box, contact-seeded, spinning aggregates: the
    t0 evaluation, one step and five steps agree with the oracle."""
    say("periodic contacts n_agg=300")
    w = W.periodic_box(31, n_agg=300, contact_seeded=True, spin_sigma=0.5, vel_sigma=0.2)
    L = w.params["box"][0]
    sim, o = _pair(D, w)
    e0 = compare_states(sim, o, box=L)
    assert sim.counts()[2] > 250
    sim.step(1)
    o.step(1)
    e1 = compare_states(sim, o, box=L)
    sim.step(4)
    o.step(4)
    e5 = compare_states(sim, o, box=L, tol=1e-10)
    print("t0", e0, "\nstep1", e1, "\nstep5", e5)


def test_step_parity_gravity_and_contacts(D):
    say("gravity + contacts n_agg=250")
    w = W.collapse_cloud(41, n_agg=250, contact_seeded=True, spin_sigma=0.3, vel_sigma=0.1)
    sim, o = _pair(D, w)
    compare_states(sim, o)
    sim.step(1)
    o.step(1)
    e1 = compare_states(sim, o)
    sim.step(3)
    o.step(3)
    e4 = compare_states(sim, o, tol=1e-10)
    print("step1", e1, "\nstep4", e4)


def test_far_outliers_parity(D):
    """An open pile with pairs of touching spheres far outside it: the grid
    then covers only the pile's core and the outliers fall into its
    outermost cells; contacts (those of the outlier pairs included) and the
    state still agree with the oracle."""
    say("collapse cloud with far outlier pairs")
    w = W.collapse_cloud(45, n_agg=250, contact_seeded=True, spin_sigma=0.3, vel_sigma=0.1)
    com = (w.mass[:, None] * w.pos).sum(0) / w.mass.sum()
    r0 = float(w.radius[0])
    pos, rad = [], []
    for d, u in (((1000.0, 0.0, 0.0), (0.0, 0.6, 0.8)), ((0.0, -800.0, 0.0), (1.0, 0.0, 0.0)),
                 ((0.0, 0.0, 1500.0), (0.6, 0.0, 0.8)), ((-700.0, 600.0, -500.0), (0.0, 0.0, 1.0))):
        a = com + np.array(d)
        pos += [a, a + 0.99 * 2.0 * r0 * np.array(u)]
        rad += [r0, r0]
    pos, rad = np.array(pos), np.array(rad)
    w = W.Workload("outliers", np.concatenate([w.counts, np.ones(8, np.int32)]),
                   np.concatenate([w.pos, pos]), np.concatenate([w.radius, rad]),
                   np.concatenate([w.mass, W.sphere_mass(rad)]),
                   np.concatenate([w.agg_vel, np.zeros((8, 3))]),
                   np.concatenate([w.agg_spin, np.zeros((8, 3))]), w.params, w.n_steps)
    sim, o = _pair(D, w)
    compare_states(sim, o)
    keys = sim.read_state([], pairs=True)["pair_keys"]
    n = w.n_sph
    for k in range(4):
        pair = (np.uint64(n - 8 + 2 * k) << np.uint64(32)) | np.uint64(n - 7 + 2 * k)
        assert pair in keys
    sim.step(3)
    o.step(3)
    compare_states(sim, o, tol=1e-10)


def test_fp32_force_form_parity(D):
    """FP32 pair forces and gravity on relative coordinates: per-sphere
    force within 1e-5 of the FP64 oracle (max norm), contact list exact."""
    say("fp32-force n_agg=250")
    w = W.collapse_cloud(43, n_agg=250, contact_seeded=True, spin_sigma=0.3, vel_sigma=0.1)
    sim, o = _pair(D, w, precision=D.PREC_FP32_FORCE)
    g = sim.read_state(["sph_force"], pairs=True)
    assert rel_err(g["sph_force"], o.spheres()["F"]) <= 1e-5
    sim.step(1)
    o.step(1)
    g = sim.read_state(["sph_force", "agg_pos"], pairs=True)
    assert np.array_equal(g["pair_keys"], (o.pairs()["i"].astype(np.uint64) << np.uint64(32))
                          | o.pairs()["j"].astype(np.uint64))
    assert rel_err(g["sph_force"], o.spheres()["F"]) <= 1e-5
    assert rel_err(g["agg_pos"], o.aggregates()["rA"]) <= 1e-12


def test_flyby_perturber_parity(D):
    """A point-mass perturber passing a contact-seeded cloud: state and the
    perturber's own position and velocity agree with the oracle."""
    say("flyby perturber n_agg=200")
    from paper_2311_11322_amd import serve
    w = W.collapse_cloud(47, n_agg=200, contact_seeded=True, spin_sigma=0.2, vel_sigma=0.05)
    serve.add_flyby(w, start_factor=1.2)
    Mp, rp, vp = w.params["perturber"]
    sim = serve.make_sim(w, D.PREC_FP64)
    o = O.Oracle(w.params).set_perturber(Mp, rp, vp).add_workload(w)
    compare_states(sim, o)
    for n in (1, 3):
        sim.step(n)
        o.step(n)
        compare_states(sim, o, tol=1e-12 if n == 1 else 1e-10)
        f = sim.get_forcing()
        orp, ovp, _ = o.perturber()
        assert rel_err(f["pert_pos"], orp) <= 1e-13
        assert rel_err(f["pert_vel"], ovp) <= 1e-12


def test_lone_spheres_and_large_aggregate(D):
    """Degenerate cases: 1-sphere aggregates (I = 2/5 m s^2) beside one
    155-sphere aggregate spanning several blocks."""
    say("lone spheres + 155-sphere aggregate")
    rng = np.random.default_rng(3)
    big_rel, big_r = W.random_cluster(rng, 155)
    parts_p = [big_rel]
    parts_r = [big_r]
    counts = [155]
    for k in range(300):
        p = rng.uniform(-30, 30, 3)
        parts_p.append(p[None] + 40.0)
        parts_r.append(rng.uniform(0.8, 1.2, 1))
        counts.append(1)
    pos = np.concatenate(parts_p)
    rad = np.concatenate(parts_r)
    prm = dict(W.CONTACT_PARAMS, dt=5e-4, G=1.0, soft_frac=0.5, periodic=0, box=(0, 0, 0))
    w = W.Workload("mixed", np.array(counts, np.int32), pos, rad, W.sphere_mass(rad),
                   rng.normal(0, 0.1, (len(counts), 3)), rng.normal(0, 0.2, (len(counts), 3)),
                   prm, 3)
    sim, o = _pair(D, w)
    compare_states(sim, o)
    sim.step(2)
    o.step(2)
    compare_states(sim, o)


# ---------------------------------------------------------------------------
# full size: the collapse at 125k spheres, sampled
# ---------------------------------------------------------------------------

@pytest.fixture(scope="module")
def collapse125k():
    return W.collapse_cloud(1, n_agg=25000)


def test_full_size_initial_forces_sampled(D, collapse125k):
    """At 125k spheres in the benchmark's launch configuration: the t0 force
    on 192 sampled spheres equals the oracle's one-sphere-at-a-time
    evaluation (contacts by brute force, direct-sum gravity)."""
    say("full size sampled", collapse125k.n_sph)
    sim = D.Sim(collapse125k.params)
    sim.add_workload(collapse125k)
    g = sim.read_state(["sph_force", "sph_torque"])
    o = O.Oracle(collapse125k.params).add_workload(collapse125k, evaluate=False)
    rng = np.random.default_rng(9)
    idx = np.sort(rng.choice(collapse125k.n_sph, 192, replace=False))
    F, T = o.eval_subset(idx)
    assert rel_err(g["sph_force"][idx], F) <= 1e-12
    assert np.abs(g["sph_torque"][idx] - T).max() <= 1e-12 * max(np.abs(F).max(), 1.0)
    # linear momentum of one step at full size (property at any size)
    a0 = sim.read_state(["agg_vel", "agg_mass"])
    P0 = (a0["agg_mass"][:, None] * a0["agg_vel"]).sum(0)
    sim.step(2)
    a1 = sim.read_state(["agg_vel", "agg_mass", "agg_acc"])
    P1 = (a1["agg_mass"][:, None] * a1["agg_vel"]).sum(0)
    Fscale = (a1["agg_mass"][:, None] * np.abs(a1["agg_acc"])).sum()
    assert np.abs(P1 - P0).max() <= 1e-12 * Fscale * 2 * collapse125k.params["dt"]


# ---------------------------------------------------------------------------
# determinism, checkpoint, failure handling, batching
# ---------------------------------------------------------------------------

def test_bitwise_deterministic(D):
    say("determinism")
    w = W.collapse_cloud(51, n_agg=300, contact_seeded=True, spin_sigma=0.3)
    outs = []
    for _ in range(2):
        sim = D.Sim(w.params)
        sim.add_workload(w)
        sim.step(3)
        outs.append(sim.read_state(pairs=True))
        sim.close()
    for k in outs[0]:
        assert np.array_equal(outs[0][k], outs[1][k]), k


def test_profiling_modes_do_not_change_results(D):
    """Launches one after another with events between kernels (mode 1) and
    launches ordered as in the step graph with events around the gravity
    stage (mode 2) step the system exactly as the graph does; mode 2 keeps
    only the gravity span."""
    say("profiling modes")
    w = W.collapse_cloud(52, n_agg=300, contact_seeded=True, spin_sigma=0.3, vel_sigma=0.1)
    outs = []
    profs = []
    for mode in (0, 1, 2):
        sim = D.Sim(w.params)
        sim.add_workload(w)
        if mode:
            sim.set_profiling(True, graph_order=mode == 2)
        sim.step(4)
        profs.append(sim.profile())
        sim.set_profiling(False)
        sim.step(2)
        outs.append(sim.read_state(pairs=True))
        sim.close()
    for m in (1, 2):
        for k in outs[0]:
            assert np.array_equal(outs[0][k], outs[m][k]), (m, k)
    assert profs[1]["_steps"] == 4 and profs[2]["_steps"] == 4
    assert profs[1]["gravity"] > 0 and profs[1]["forces"] > 0
    assert profs[2]["gravity"] > 0
    assert all(v == 0 for k, v in profs[2].items() if k not in ("gravity", "_steps"))
    sim = D.Sim(w.params)
    with pytest.raises(D.DemError):
        D._check(D.lib().dem_set_profiling(sim.h, 3), sim.h)
    sim.close()


def test_checkpoint_restore_bit_identical(D):
    say("checkpoint/restore")
    w = W.periodic_box(61, n_agg=300, contact_seeded=True, spin_sigma=0.4, vel_sigma=0.2)
    a = D.Sim(w.params)
    a.add_workload(w)
    a.step(3)
    ck = a.checkpoint()
    a.step(4)
    ref = a.read_state(pairs=True)
    b = D.Sim(w.params)
    b.add_workload(w)
    b.restore(ck)
    b.step(4)
    got = b.read_state(pairs=True)
    for k in ("agg_pos", "agg_vel", "agg_acc", "agg_torque", "agg_quat", "pair_keys", "pair_hist",
              "sph_force"):
        assert np.array_equal(got[k], ref[k]), k
    assert got["step"] == ref["step"] == 7


def _lattice(n=8, gap=0.01, squeeze=0.5):
    """Lone unit spheres on a cubic lattice, contracting toward the centre,
    so that contacts (about 3 per sphere) appear after some steps."""
    g = np.arange(n) * (2.0 + gap)
    pos = np.stack(np.meshgrid(g, g, g, indexing="ij"), -1).reshape(-1, 3)
    pos -= pos.mean(0)
    m = W.sphere_mass(np.ones(len(pos)))
    prm = dict(W.CONTACT_PARAMS, dt=1e-4, G=0.0, soft_frac=0.5, periodic=0, box=(0, 0, 0))
    return W.Workload("lattice", np.ones(len(pos), np.int32), pos, np.ones(len(pos)), m,
                      -squeeze * pos / np.abs(pos).max(), np.zeros_like(pos), prm, 1)


def test_capacity_error_rolls_back(D):
    """With room for one contact per sphere the contracting lattice
    overflows: the call fails with CAPACITY and the state is that at the
    start of the failing step (checked bitwise against a roomy run); after
    growing the capacity the run continues bit-identically."""
    say("capacity rollback")
    w = _lattice()
    small = D.Sim(w.params, max_contacts=1)
    small.add_workload(w)
    code = None
    for _ in range(100):
        try:
            small.step(20)
        except D.DemError as e:
            code = e.code
            break
    assert code == D.DEM_ERR_CAPACITY
    st = small.read_state(["agg_pos", "agg_vel"], pairs=True)
    k = st["step"]
    ref = D.Sim(w.params, max_contacts=16)
    ref.add_workload(w)
    ref.step(k)
    rs = ref.read_state(["agg_pos", "agg_vel"], pairs=True)
    for f in ("agg_pos", "agg_vel", "pair_keys", "pair_hist"):
        assert np.array_equal(st[f], rs[f]), f
    with pytest.raises(D.DemError):
        small.step(1)                      # a failed system refuses to step
    small.reserve_contacts(16)
    small.step(30)
    ref.step(30)
    a, b = small.read_state(pairs=True), ref.read_state(pairs=True)
    assert a["n_pairs"] > w.n_sph          # more contacts than the old capacity
    for f in ("agg_pos", "agg_vel", "pair_keys", "pair_hist"):
        assert np.array_equal(a[f], b[f]), f


def test_invalid_input_rejected(D):
    say("invalid input")
    w = W.periodic_box(3, n_agg=20)
    bad = w.pos.copy()
    bad[5, 1] = np.nan
    sim = D.Sim(w.params)
    for bad_tuning in ((0, 1.0, 2, 0), (0, 1.0, 0, 3), (0, 0.5, 0, 0)):
        with pytest.raises(D.DemError) as ei:
            sim.set_tuning(*bad_tuning)
        assert ei.value.code == D.DEM_ERR_INVALID_ARG
    with pytest.raises(D.DemError) as ei:
        sim.add_aggregates(w.counts, bad, w.radius, w.mass)
    assert ei.value.code == D.DEM_ERR_INVALID_ARG
    with pytest.raises(D.DemError) as ei:
        sim.step(1)
    assert ei.value.code == D.DEM_ERR_STATE


def test_spin_up_parity(D):
    """Spin-up forcing (the body-frame spin increment after the second kick,
    Sec. 4.1) on the exact sum against the oracle: three steps within the
    parity bar."""
    say("direct + spin-up")
    w = W.collapse_cloud(78, n_agg=300, contact_seeded=True, spin_sigma=0.1)
    w.params["spin_dw"] = 1e-3
    sim = D.Sim(w.params)
    sim.add_workload(w)
    sim.set_forcing(w.params["spin_dw"])
    o = O.Oracle(w.params).add_workload(w)
    compare_states(sim, o)
    sim.step(3)
    o.step(3)
    compare_states(sim, o, tol=1e-10)


@pytest.mark.parametrize("case", ["lone+big", "collapse"])
def test_member_read_paths_bit_identical(D, case):
    """The member reduction read directly and staged through LDS (forced by
    the tuning; a launch picks staging only from 131,072 aggregates) gives
    bit-identical states, and the staged run matches the oracle -- with lone
    spheres and a 155-sphere aggregate spanning several 64-sphere slices, and
    with aggregates of 2-8 spheres."""
    say("member read paths", case)
    if case == "lone+big":
        rng = np.random.default_rng(5)
        big_rel, big_r = W.random_cluster(rng, 155)
        parts_p, parts_r, counts = [big_rel], [big_r], [155]
        for k in range(200):
            parts_p.append(rng.uniform(-30, 30, 3)[None] + 40.0)
            parts_r.append(rng.uniform(0.8, 1.2, 1))
            counts.append(1)
        rad = np.concatenate(parts_r)
        prm = dict(W.CONTACT_PARAMS, dt=5e-4, G=1.0, soft_frac=0.5, periodic=0, box=(0, 0, 0))
        w = W.Workload("mixed", np.array(counts, np.int32), np.concatenate(parts_p), rad,
                       W.sphere_mass(rad), rng.normal(0, 0.1, (len(counts), 3)),
                       rng.normal(0, 0.2, (len(counts), 3)), prm, 3)
    else:
        w = W.collapse_cloud(62, n_agg=500, contact_seeded=True, spin_sigma=0.2)
    out = []
    for read in (1, 2):
        sim = D.Sim(w.params)
        sim.set_tuning(0, 1.0, 0, read)
        sim.add_workload(w)
        sim.step(3)
        out.append(sim.read_state(pairs=True))
        if read == 2:
            o = O.Oracle(w.params).add_workload(w)
            o.step(3)
            compare_states(sim, o, tol=1e-10)
        sim.close()
    for k in out[0]:
        assert np.array_equal(out[0][k], out[1][k]), k


def test_engine_alone_vs_mix_bit_identical(D):
    say("engine alone vs mix")
    piles = W.pile_batch(seed=3, n_piles=6, nmin=300, nmax=3000, n_steps=5)
    alone = []
    for w in piles:
        s = D.Sim(w.params)
        s.add_workload(w)
        s.set_forcing(w.params["spin_dw"])
        s.step(5)
        alone.append(s.read_state(pairs=True))
        s.close()
    eng = D.Engine(1 << 34)
    sims = []
    for w in piles:
        s = D.Sim(w.params)
        s.add_workload(w)
        s.set_forcing(w.params["spin_dw"])
        eng.attach(s)
        sims.append(s)
    assert eng.step(2) == D.DEM_OK
    eng.detach(sims[2])       # a request leaves mid-run ...
    sims[2].step(3)           # ... and finishes on its own
    assert eng.step(3) == D.DEM_OK
    for s in list(eng.sims):
        eng.detach(s)
    for k, s in enumerate(sims):
        got = s.read_state(pairs=True)
        for f in ("agg_pos", "agg_vel", "agg_quat", "pair_keys", "pair_hist", "sph_force"):
            assert np.array_equal(got[f], alone[k][f]), (k, f)


def test_member_scan_ablation_gives_identical_results(D):
    """The paper's original member search (full scan per aggregate) and its
    improvement (contiguous segments) give bit-identical states."""
    say("member scan ablation")
    w = W.collapse_cloud(61, n_agg=400, contact_seeded=True, spin_sigma=0.2)
    out = []
    for scan in (0, 1):
        sim = D.Sim(w.params)
        sim.set_tuning(0, 1.0, scan)
        sim.add_workload(w)
        sim.step(3)
        out.append(sim.read_state(pairs=True))
        sim.close()
    for k in out[0]:
        assert np.array_equal(out[0][k], out[1][k]), k


def test_dense_lattice_parity(D):
    """Contact-dense periodic lattice (five contacts per sphere): one and
    three steps against the oracle."""
    say("dense lattice 10^3")
    w = W.dense_lattice(n_side=10)
    L = w.params["box"][0]
    sim, o = _pair(D, w)
    compare_states(sim, o, box=L)
    assert sim.counts()[2] == 2500
    sim.step(1)
    o.step(1)
    compare_states(sim, o, box=L)
    sim.step(2)
    o.step(2)
    compare_states(sim, o, box=L, tol=1e-10)


def test_boulders_periodic_parity(D):
    """Boulders (radius 4) among aggregates of unit-size spheres in a periodic
    cube: the boulders are searched apart from the cell grid (sized for the
    small spheres), across the periodic wrap, with boulder-boulder and
    boulder-aggregate contacts seeded."""
    say("boulders periodic")
    w = W.boulders(seed=13)
    L = w.params["box"][0]
    sim, o = _pair(D, w)
    compare_states(sim, o, box=L)
    p = o.pairs()
    assert ((p["i"] < 6) & (p["j"] < 6)).sum() >= 2 and (p["j"] >= 6).sum() >= 20
    sim.step(1)
    o.step(1)
    compare_states(sim, o, box=L)
    for _ in range(3):
        sim.step(20)
        o.step(20)
        compare_states(sim, o, box=L, tol=1e-10)
