"""Host logic of the served loop's scheduling (no GPU): which admitted runs
a chunk steps under each policy."""
import types

import pytest

from paper_2311_11322_amd import serve


def _server(policy, cap, runs):
    srv = serve.Server.__new__(serve.Server)      # no engine: selection only
    srv.policy, srv.cap = policy, cap
    srv.active = {rid: [types.SimpleNamespace(rid=rid, workload=types.SimpleNamespace(n_sph=n)),
                        None, steps, 0] for rid, (n, steps) in runs.items()}
    return srv


RUNS = {0: (2000, 50), 1: (500, 10), 2: (1500, 5), 3: (1000, 100)}


def test_fifo_steps_every_admitted_run():
    assert _server("fifo", 1.0, RUNS)._select() == {0, 1, 2, 3}


def test_srpt_takes_least_remaining_work_up_to_the_pair_cap():
    # remaining work n^2 x steps: run 1 2.5e6, run 2 1.1e7, run 3 1e8, run 0 2e8;
    # pairs per step 2.5e5 + 2.25e6 fill a cap of 2.5e6, run 3 would exceed it
    assert _server("srpt", 2.5e6, RUNS)._select() == {1, 2}
    # a cap above everything steps every run
    assert _server("srpt", 1e12, RUNS)._select() == {0, 1, 2, 3}


def test_srpt_always_steps_at_least_one_run():
    assert _server("srpt", 1.0, RUNS)._select() == {1}


def test_unknown_policy_is_refused():
    with pytest.raises(ValueError):
        serve.Server(1 << 30, policy="lifo")


def test_shape_bucket_groups_batches_by_size_and_kind():
    mk = lambda n, G=1.0, tree=0: types.SimpleNamespace(
        n_sph=n, params={"G": G, "gravity_tree": tree})
    a = serve.shape_bucket([mk(1000), mk(3000)], 1)
    assert a == serve.shape_bucket([mk(1100), mk(2900)], 1)       # same powers of two
    assert a != serve.shape_bucket([mk(1000), mk(3000)], 0)       # precision
    assert a != serve.shape_bucket([mk(1000, G=0.0), mk(3000, G=0.0)], 1)
    assert a != serve.shape_bucket([mk(1000, tree=1), mk(3000, tree=1)], 1)
    assert a != serve.shape_bucket([mk(1000), mk(3000), mk(2000), mk(2000)], 1)
