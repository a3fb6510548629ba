"""Tree gravity on the GPU against the oracle's tree and the exact sum
(needs an MI355X).  Each test prints its case before the GPU runs."""
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


def _tree(w, theta=0.5, leaf=16, order=4):
    w.params.update(gravity_tree=1, theta=theta, tree_leaf=leaf, tree_order=order)
    return w


@pytest.mark.parametrize("theta,leaf,order,soft", [(0.5, 16, 4, 0.5), (0.3, 4, 4, 0.5),
                                                   (0.8, 64, 4, 0.5), (0.5, 16, 2, 0.5),
                                                   (0.8, 64, 2, 0.5), (0.5, 16, 4, 0.0)])
def test_tree_gravity_parity(D, theta, leaf, order, soft):
    """Same tree, same groups, same opening decisions as the oracle's tree:
    t0, one step and three more within the parity bar (softened, and
    unsoftened where each sphere's own term must be skipped)."""
    say("tree parity", theta, leaf, order, soft)
    w = _tree(W.collapse_cloud(71, n_agg=500, contact_seeded=True, spin_sigma=0.2), theta, leaf,
              order)
    w.params["soft_frac"] = soft
    sim = D.Sim(w.params)
    sim.add_workload(w)
    o = O.Oracle(w.params).add_workload(w)
    compare_states(sim, o)
    sim.step(1)
    o.step(1)
    compare_states(sim, o)
    sim.step(3)
    o.step(3)
    compare_states(sim, o, tol=1e-10)


@pytest.mark.parametrize("n_agg,leaf,order", [(1, 16, 4), (3, 4, 4), (3, 16, 2), (12, 4, 4),
                                               (40, 4, 4), (40, 64, 2)])
def test_tree_small_piles_parity(D, n_agg, leaf, order):
    """Piles of 2 to 192 spheres: a root of at most tree_leaf spheres acting
    as one set of pairs, finest cells above the split level, groups shorter
    than a wave.  Random spins and velocities keep every compared quantity
    above rounding noise (a lone aggregate's own pulls cancel)."""
    say("tree small pile", n_agg, leaf, order)
    w = _tree(W.collapse_cloud(80 + n_agg, n_agg=n_agg, spin_sigma=0.3, vel_sigma=0.1), 0.5, leaf,
              order)
    sim = D.Sim(w.params)
    sim.add_workload(w)
    o = O.Oracle(w.params).add_workload(w)
    compare_states(sim, o)
    sim.step(2)
    o.step(2)
    compare_states(sim, o, tol=1e-10)


def test_tree_in_fp32_force_form(D):
    """FP32 contact forces beside the tree (FP64 in both forms): per-sphere
    force within 1e-5 of the oracle's tree, contact list exact, positions
    after a step within 1e-12."""
    say("tree fp32-force")
    w = _tree(W.collapse_cloud(76, n_agg=300, contact_seeded=True, spin_sigma=0.3, vel_sigma=0.1))
    sim = D.Sim(w.params, precision=D.PREC_FP32_FORCE)
    sim.add_workload(w)
    o = O.Oracle(w.params).add_workload(w)
    g = sim.read_state(["sph_force"], pairs=True)
    assert rel_err(g["sph_force"], o.spheres()["F"]) <= 1e-5
    sim.step(1)
    o.step(1)
    g = sim.read_state(["sph_force", "agg_pos"], pairs=True)
    keys = (o.pairs()["i"].astype(np.uint64) << np.uint64(32)) | o.pairs()["j"].astype(np.uint64)
    assert np.array_equal(g["pair_keys"], keys)
    assert rel_err(g["sph_force"], o.spheres()["F"]) <= 1e-5
    assert rel_err(g["agg_pos"], o.aggregates()["rA"]) <= 1e-12


def test_tree_with_perturber_parity(D):
    say("tree + flyby")
    from paper_2311_11322_amd import serve
    w = _tree(W.collapse_cloud(72, n_agg=300, contact_seeded=True))
    serve.add_flyby(w, start_factor=1.2)
    Mp, rp, vp = w.params["perturber"]
    sim = serve.make_sim(w, D.PREC_FP64)
    o = O.Oracle(w.params).set_perturber(Mp, rp, vp).add_workload(w)
    compare_states(sim, o)
    sim.step(2)
    o.step(2)
    compare_states(sim, o, tol=1e-10)
    f = sim.get_forcing()
    orp, ovp, _ = o.perturber()
    assert rel_err(f["pert_pos"], orp) <= 1e-13
    assert rel_err(f["pert_vel"], ovp) <= 1e-12


@pytest.mark.parametrize("order,theta,rms_max,max_max", [(4, 0.5, 1e-4, 1e-3), (2, 0.5, 1e-3, 1e-2),
                                                         (4, 0.7, 1e-3, 1e-2)])
def test_tree_at_full_size_against_exact_sum(D, order, theta, rms_max, max_max):
    """The 125k-sphere collapse with tree gravity: the force on sampled
    spheres against the oracle's exact one-at-a-time evaluation (contacts +
    direct sum) -- the difference is the tree's truncation error only."""
    w = _tree(W.collapse_cloud(1, n_agg=25000), theta=theta, order=order)
    say("tree full size", w.n_sph, order, theta)
    sim = D.Sim(w.params)
    sim.add_workload(w)
    F = sim.read_state(["sph_force"])["sph_force"]
    sim.close()
    o = O.Oracle(w.params).add_workload(w, evaluate=False)
    idx = np.random.default_rng(0).choice(w.n_sph, 192, replace=False)
    Fo, _ = o.eval_subset(idx)
    err = np.linalg.norm(F[idx] - Fo, axis=1) / np.linalg.norm(Fo, axis=1)
    print("tree relative error: max", err.max(), "rms", np.sqrt((err ** 2).mean()))
    assert np.sqrt((err ** 2).mean()) < rms_max and err.max() < max_max


def test_tree_and_direct_piles_in_one_engine(D):
    """Tree-gravity piles of both orders and a direct-sum pile stepped
    together give the states each gives alone, bit for bit."""
    say("engine tree + direct")
    ws = [_tree(W.collapse_cloud(73, n_agg=400, contact_seeded=True)),
          W.collapse_cloud(74, n_agg=300, contact_seeded=True),
          _tree(W.collapse_cloud(75, n_agg=350, contact_seeded=True), order=2)]
    alone = []
    for w in ws:
        s = D.Sim(w.params)
        s.add_workload(w)
        s.step(4)
        alone.append(s.read_state(pairs=True))
        s.close()
    eng = D.Engine(1 << 33)
    sims = []
    for w in ws:
        s = D.Sim(w.params)
        s.add_workload(w)
        eng.attach(s)
        sims.append(s)
    assert eng.step(4) == D.DEM_OK
    for s in list(eng.sims):
        eng.detach(s)
    for k, s in enumerate(sims):
        got = s.read_state(pairs=True)
        for f in ("agg_pos", "agg_vel", "agg_quat", "pair_keys", "sph_force"):
            assert np.array_equal(got[f], alone[k][f]), (k, f)


def test_tree_piles_of_different_depths_in_one_engine(D):
    """Tree piles of 2 to 5 pyramid levels (and both orders, different
    opening angles and leaves) batched with a direct-sum pile: a level is the
    finest of one pile while others build it from their children, and every
    pile's state equals its state alone, bit for bit."""
    say("engine, tree piles of different depths")
    specs = [(3, 0.5, 16, 4), (60, 0.6, 8, 2), (2500, 0.5, 32, 4), (400, 0.8, 64, 4)]
    ws = [_tree(W.collapse_cloud(90 + k, n_agg=n, contact_seeded=True, spin_sigma=0.2), th, lf,
                od) for k, (n, th, lf, od) in enumerate(specs)]
    ws.append(W.collapse_cloud(95, n_agg=200, contact_seeded=True))
    alone = []
    for w in ws:
        s = D.Sim(w.params)
        s.add_workload(w)
        s.step(3)
        alone.append(s.read_state(pairs=True))
        s.close()
    eng = D.Engine(1 << 33)
    sims = []
    for w in ws:
        s = D.Sim(w.params)
        s.add_workload(w)
        eng.attach(s)
        sims.append(s)
    assert eng.step(3) == D.DEM_OK
    for s in list(eng.sims):
        eng.detach(s)
    for k, s in enumerate(sims):
        got = s.read_state(pairs=True)
        for f in ("agg_pos", "agg_vel", "agg_quat", "pair_keys", "sph_force"):
            assert np.array_equal(got[f], alone[k][f]), (k, f)


def test_tree_checkpoint_restore_bit_identical(D):
    """A tree pile checkpointed after 3 steps and restored into a fresh
    system continues exactly as the original."""
    say("tree checkpoint/restore")
    w = _tree(W.collapse_cloud(77, n_agg=300, contact_seeded=True, spin_sigma=0.3))
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


def test_tree_with_spin_up_parity(D):
    """Spin-up forcing (the YORP-like ramp) on a tree pile against the
    oracle: three steps within the parity bar."""
    say("tree + spin-up")
    w = _tree(W.collapse_cloud(78, n_agg=300, contact_seeded=True, spin_sigma=0.1))
    w.params["spin_dw"] = 1e-3
    sim = D.Sim(w.params)
    sim.add_workload(w)
    sim.set_forcing(w.params["spin_dw"])
    o = O.Oracle(w.params).add_workload(w)
    compare_states(sim, o)
    sim.step(3)
    o.step(3)
    compare_states(sim, o, tol=1e-10)

