"""Seeded input generators: determinism, placement constraints, shapes."""
import numpy as np
import pytest

from paper_2311_11322_amd import workloads as W


def _min_gap_other(w, periodic):
    from scipy.spatial import cKDTree
    agg = w.agg_of_sphere()
    L = w.params["box"][0] if periodic else None
    pos = np.mod(w.pos, L) if periodic else w.pos
    t = cKDTree(pos, boxsize=L)
    c = np.array(sorted(t.query_pairs(2.5)), dtype=np.int64)
    d = pos[c[:, 1]] - pos[c[:, 0]]
    if periodic:
        d -= L * np.round(d / L)
    gap = np.sqrt((d * d).sum(1)) - w.radius[c[:, 0]] - w.radius[c[:, 1]]
    other = agg[c[:, 0]] != agg[c[:, 1]]
    return gap[other]


def test_periodic_box_deterministic_and_non_overlapping():
    a = W.periodic_box(0, n_agg=120)
    b = W.periodic_box(0, n_agg=120)
    assert np.array_equal(a.pos, b.pos) and np.array_equal(a.agg_vel, b.agg_vel)
    assert a.counts.min() >= 1 and a.counts.max() <= 8
    assert a.radius.min() >= 0.8 and a.radius.max() <= 1.2
    assert _min_gap_other(a, True).min() >= W.MIN_GAP
    c = W.periodic_box(1, n_agg=120)
    assert not np.array_equal(a.pos, c.pos)


def test_contact_seeded_has_overlaps_in_range():
    w = W.periodic_box(2, n_agg=100, contact_seeded=True)
    g = _min_gap_other(w, True)
    ov = -g[g < 0]
    assert ov.size >= 99 - 5
    assert ov.max() <= 1e-3 + 1e-12
    assert np.abs(g).min() > 1e-9


def test_collapse_cloud_inside_ball_at_rest():
    w = W.collapse_cloud(1, n_agg=400)
    R = float(w.notes.split("R=")[1].split(",")[0])
    assert np.linalg.norm(w.pos, axis=1).max() <= R + 8.0    # centres inside, members may poke out
    assert w.counts.min() >= 2 and w.counts.max() <= 8
    assert np.all(w.agg_vel == 0) and w.params["G"] == 1.0
    assert _min_gap_other(w, False).min() >= W.MIN_GAP
    phi = (W.sphere_mass(w.radius).sum()) / (4 / 3 * np.pi * R ** 3)
    assert phi == pytest.approx(0.15, rel=1e-3)


def test_clusters_are_touching_and_rigid():
    rng = np.random.default_rng(5)
    for n in range(1, 9):
        p, r = W.random_cluster(rng, n)
        if n == 1:
            continue
        d = np.linalg.norm(p[:, None] - p[None], axis=2)
        S = r[:, None] + r[None]
        np.fill_diagonal(d, np.inf)
        assert np.all(d >= S * (1 - 1e-12))
        # every sphere touches at least one other
        assert np.all(np.min(np.abs(d - S), axis=1) < 1e-12)


@pytest.mark.parametrize("name", W.SHAPES)
def test_shape_fixtures_touching(name):
    p = W.shape_fixture(name, 1.0)
    assert np.allclose(p.mean(0), 0)
    if p.shape[0] > 1:
        d = np.linalg.norm(p[:, None] - p[None], axis=2)
        np.fill_diagonal(d, np.inf)
        assert d.min() == pytest.approx(2.0, abs=1e-12)


def test_request_stream_is_seeded():
    from paper_2311_11322_amd import serve
    a = serve.request_stream(seed=1, n_requests=5, rate_per_s=20.0, nmin=300, nmax=900,
                             smin=10, smax=50)
    b = serve.request_stream(seed=1, n_requests=5, rate_per_s=20.0, nmin=300, nmax=900,
                             smin=10, smax=50)
    assert [r.arrival for r in a] == [r.arrival for r in b]
    assert all(np.array_equal(x.workload.pos, y.workload.pos) for x, y in zip(a, b))
    assert a[0].arrival == 0.0 and all(x.arrival <= y.arrival for x, y in zip(a, a[1:]))
    assert all(10 <= r.steps <= 50 for r in a)
