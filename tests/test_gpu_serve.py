"""Batching and serving on the GPU: each run gives the same result alone and
inside a running batch; admission respects the memory budget."""
import sys

import numpy as np
import pytest

from paper_2311_11322_amd import workloads as W

pytestmark = pytest.mark.gpu


def say(*a):
    print("[case]", *a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def D():
    from paper_2311_11322_amd import dem
    dem.lib()
    return dem


@pytest.mark.parametrize("policy", ["fifo", "srpt"])
def test_served_stream_matches_alone(D, policy):
    """Requests of different sizes arrive while others run; every served
    result equals the same request run alone, bit for bit.  Under "srpt" a
    small pair cap keeps one or two runs attached per chunk, so runs are
    detached and re-attached many times on the way."""
    from paper_2311_11322_amd import serve
    say("served stream vs alone", policy)
    reqs = serve.request_stream(seed=11, n_requests=6, rate_per_s=50.0, nmin=300, nmax=2500,
                                smin=10, smax=60)
    srv = serve.Server(1 << 34, precision=D.PREC_FP32_FORCE, chunk_steps=8, capture_state=True,
                       policy=policy, pairs_per_step_cap=2.5e6)
    stats = srv.run(reqs)
    assert stats["completed"] == len(reqs)
    for r in reqs:
        sim = serve.make_sim(r.workload, D.PREC_FP32_FORCE)
        sim.step(r.steps)
        ref = sim.read_state(["agg_pos", "agg_vel", "agg_quat"], pairs=True)
        got = r.result["state"]
        assert got["step"] == ref["step"] == r.steps
        for f in ("agg_pos", "agg_vel", "agg_quat", "pair_keys", "pair_hist"):
            assert np.array_equal(got[f], ref[f]), (r.rid, f)
        sim.close()


def test_admission_waits_for_memory(D):
    """With room for one request at a time the stream still completes, and
    the second request is admitted only after the first finished."""
    from paper_2311_11322_amd import serve
    say("admission under a small budget")
    reqs = serve.request_stream(seed=12, n_requests=3, rate_per_s=1000.0, nmin=400, nmax=600,
                                smin=20, smax=30)
    need = max(D.footprint_bytes(r.workload.params, r.workload.n_agg, r.workload.n_sph,
                                 D.PREC_FP32_FORCE) for r in reqs)
    srv = serve.Server(int(need * 1.5), precision=D.PREC_FP32_FORCE, chunk_steps=10)
    stats = srv.run(reqs)
    assert stats["completed"] == 3
    order = sorted(reqs, key=lambda r: r.admitted)
    for a, b in zip(order, order[1:]):
        assert b.admitted >= a.done


def test_autotune_picks_a_measured_candidate(D):
    from paper_2311_11322_amd import serve
    say("autotune")
    piles = W.pile_batch(seed=5, n_piles=4, nmin=500, nmax=3000)
    cache = {}
    res = serve.autotune(piles, D.PREC_FP32_FORCE, steps=2, cache=cache)
    assert not res["cached"]
    assert (res["gravity_tile"], res["cell_scale"]) in [
        (c["gravity_tile"], c["cell_scale"]) for c in res["candidates"]]
    assert len(res["candidates"]) == len(D.gravity_tiles(D.PREC_FP32_FORCE)) * 4
    # a batch of the same shape bucket reuses the choice without measuring
    again = serve.autotune(W.pile_batch(seed=6, n_piles=4, nmin=500, nmax=3000)[:4],
                           D.PREC_FP32_FORCE, steps=2, cache=cache)
    if serve.shape_bucket(piles, D.PREC_FP32_FORCE) == serve.shape_bucket(
            W.pile_batch(seed=6, n_piles=4, nmin=500, nmax=3000), D.PREC_FP32_FORCE):
        assert again["cached"] and again["gravity_tile"] == res["gravity_tile"]
