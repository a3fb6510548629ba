"""The two forms of the exact softened gravity sum (Eq. 4) against the
oracle and against each other (needs an MI355X).

The pair form evaluates each unordered pair once, a wave per pair of
super-tiles (runs of ceil(tiles / 256) tiles), and keeps one partial sum per
sphere and super-tile; the per-target form evaluates each ordered pair from
its target's side and keeps one partial per sphere and source split (16).
Both are the same sum in another order, so each is compared with the oracle
at the FP64 parity bar, and a pile's result must not depend on the form of
the other piles in its engine.
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


def _pair(D, w, form, tile=0, precision=0):
    sim = D.Sim(w.params, precision=precision)
    sim.set_tuning(gravity_tile=tile, gravity_form=form)
    sim.add_workload(w)
    o = O.Oracle(w.params).add_workload(w)
    return sim, o


@pytest.mark.parametrize("tile", [0, 128])
def test_per_target_form_parity(D, tile):
    """FP64, per-target form: t0, one step and three more against the
    oracle (tile 128 on 2.7k spheres: 22 tiles in 11 splits of two)."""
    w = W.collapse_cloud(44, n_agg=600, contact_seeded=True, spin_sigma=0.3, vel_sigma=0.1)
    say("per-target gravity, tile", tile, w.n_sph, "spheres")
    sim, o = _pair(D, w, 2, tile)
    compare_states(sim, o)
    sim.step(1)
    o.step(1)
    compare_states(sim, o)
    sim.step(3)
    o.step(3)
    compare_states(sim, o, tol=1e-10)


def test_per_target_form_unsoftened_and_fp32(D):
    """Unsoftened (a sphere's own term is skipped by r^-3 = 0) in FP64, and
    the FP32-force form on relative coordinates within 1e-5."""
    w = W.collapse_cloud(45, n_agg=300, contact_seeded=True, spin_sigma=0.3, vel_sigma=0.1,
                         soft_frac=0.0)
    say("per-target gravity, unsoftened", w.n_sph)
    sim, o = _pair(D, w, 2, 128)
    compare_states(sim, o)
    sim.step(2)
    o.step(2)
    compare_states(sim, o, tol=1e-10)
    w2 = W.collapse_cloud(46, n_agg=300, contact_seeded=True, spin_sigma=0.3, vel_sigma=0.1)
    say("per-target gravity, FP32-force", w2.n_sph)
    sim2, o2 = _pair(D, w2, 2, 256, precision=D.PREC_FP32_FORCE)
    g = sim2.read_state(["sph_force"])
    assert rel_err(g["sph_force"], o2.spheres()["F"]) <= 1e-5
    sim2.step(1)
    o2.step(1)
    g = sim2.read_state(["sph_force"])
    assert rel_err(g["sph_force"], o2.spheres()["F"]) <= 1e-5


def test_forms_agree_and_mix_in_an_engine(D):
    """The two forms agree to rounding, and piles of both forms stepped in
    one engine give what each gives alone, bit for bit."""
    ws = [W.collapse_cloud(47 + k, n_agg=400, contact_seeded=True, spin_sigma=0.2) for k in range(2)]
    say("tile pairs vs per target, engine mix")
    alone = []
    for w, form in zip(ws, (1, 2)):
        s = D.Sim(w.params)
        s.set_tuning(gravity_tile=128, gravity_form=form)
        s.add_workload(w)
        s.step(4)
        alone.append(s.read_state(pairs=True))
        s.close()
    other = D.Sim(ws[1].params)
    other.set_tuning(gravity_tile=128, gravity_form=1)
    other.add_workload(ws[1])
    other.step(4)
    sym = other.read_state(["sph_force", "agg_pos"])
    other.close()
    scale = float(np.abs(sym["sph_force"]).max())
    assert np.abs(alone[1]["sph_force"] - sym["sph_force"]).max() <= 1e-10 * scale
    eng = D.Engine(1 << 33)
    sims = []
    for w, form in zip(ws, (1, 2)):
        s = D.Sim(w.params)
        s.set_tuning(gravity_tile=128, gravity_form=form)
        s.add_workload(w)
        eng.attach(s)
        sims.append(s)
    assert eng.step(4) == D.DEM_OK
    for s in list(eng.sims):
        eng.detach(s)
    for k, s in enumerate(sims):
        got = s.read_state(pairs=True)
        s.close()
        for f in ("agg_pos", "agg_vel", "agg_quat", "pair_keys", "sph_force"):
            assert np.array_equal(got[f], alone[k][f]), (k, f)


@pytest.mark.parametrize("n_agg,tile,prec,soft", [(7000, 128, 0, 0.5), (14000, 128, 0, 0.5),
                                                   (14000, 256, 1, 0.5), (7000, 128, 0, 0.0),
                                                   (14000, 256, 1, 0.0)])
def test_super_tiles_sampled(D, n_agg, tile, prec, soft):
    """More tiles than super-tiles (35k and 70k spheres in tiles of 128: two
    and three tiles per super-tile, the last one short; 70k in tiles of 256:
    two), softened and not: sampled spheres against the oracle's exact sum,
    both forms."""
    w = W.collapse_cloud(50 + n_agg // 7000, n_agg=n_agg, soft_frac=soft)
    idx = np.sort(np.random.default_rng(5).choice(w.n_sph, 160, replace=False))
    o = O.Oracle(w.params).add_workload(w, evaluate=False)
    F, _ = o.eval_subset(idx)
    nt = -(-w.n_sph // tile)
    span = -(-nt // 256)
    assert span >= 2
    for form in (1, 2):
        say("super-tiles", w.n_sph, "spheres, tile", tile, "span", span, "form", form, "prec", prec,
            "soft", soft)
        sim = D.Sim(w.params, precision=prec)
        sim.set_tuning(gravity_tile=tile, gravity_form=form)
        sim.add_workload(w)
        g = sim.read_state(["sph_force"])["sph_force"]
        sim.close()
        assert rel_err(g[idx], F) <= (1e-12 if prec == 0 else 1e-5), form


def test_super_tiles_default_tiles_unsoftened(D):
    """The default tiles (512 in FP64, eight targets per lane) past 256
    tiles, unsoftened: 140k spheres, super-tiles of two, sampled spheres
    against the oracle's exact sum."""
    w = W.collapse_cloud(53, n_agg=28000, soft_frac=0.0)
    assert -(-w.n_sph // 512) > 256
    idx = np.sort(np.random.default_rng(6).choice(w.n_sph, 128, replace=False))
    o = O.Oracle(w.params).add_workload(w, evaluate=False)
    F, _ = o.eval_subset(idx)
    for prec, tile in ((0, 0), (1, 512)):
        say("super-tiles at the default tile", w.n_sph, "spheres, unsoftened, prec", prec)
        sim = D.Sim(w.params, precision=prec)
        sim.set_tuning(gravity_tile=tile)
        sim.add_workload(w)
        g = sim.read_state(["sph_force"])["sph_force"]
        sim.close()
        assert rel_err(g[idx], F) <= (1e-12 if prec == 0 else 1e-5), prec


def test_super_tile_and_tile_pair_piles_in_one_engine(D):
    """A pile on super-tiles and a pile of single tile pairs in one engine
    (two launches of the pair kernel for one tile size) give their runs
    alone bit for bit."""
    ws = [W.collapse_cloud(54, n_agg=7000), W.collapse_cloud(55, n_agg=400, contact_seeded=True)]
    say("super-tile and tile-pair piles in one engine", [w.n_sph for w in ws])
    alone = []
    for w in ws:
        s = D.Sim(w.params)
        s.set_tuning(gravity_tile=128)
        s.add_workload(w)
        s.step(2)
        alone.append(s.read_state(["agg_pos", "agg_vel", "sph_force"], pairs=True))
        s.close()
    eng = D.Engine(1 << 33)
    sims = []
    for w in ws:
        s = D.Sim(w.params)
        s.set_tuning(gravity_tile=128)
        s.add_workload(w)
        eng.attach(s)
        sims.append(s)
    assert eng.step(2) == D.DEM_OK
    for s in list(eng.sims):
        eng.detach(s)
    for k, s in enumerate(sims):
        got = s.read_state(["agg_pos", "agg_vel", "sph_force"], pairs=True)
        s.close()
        for f in ("agg_pos", "agg_vel", "pair_keys", "sph_force"):
            assert np.array_equal(got[f], alone[k][f]), (k, f)
