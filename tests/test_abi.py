"""The C-ABI library loads, exports every symbol include/dem.h declares, and
validates parameters on the host (no GPU needed)."""
import ctypes as C
import os
import re
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "dem.h")
LIB = os.path.join(ROOT, "paper_2311_11322_amd", "libdem.so")


def declared():
    txt = open(HEADER).read()
    txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
    return sorted(set(re.findall(r"\b(dem_[a-z_]+)\s*\(", txt)))


def test_header_declares_the_boundary():
    names = declared()
    for n in ("dem_create", "dem_add_aggregates", "dem_step", "dem_read_state", "dem_get_counts",
              "dem_set_forcing", "dem_restore_state", "dem_find_contacts", "dem_destroy",
              "dem_last_error", "dem_engine_create", "dem_engine_attach", "dem_engine_step",
              "dem_engine_detach", "dem_engine_destroy", "dem_footprint_bytes"):
        assert n in names


@pytest.mark.skipif(not os.path.exists(LIB), reason="libdem.so not built")
def test_library_exports_every_declared_symbol():
    out = subprocess.run(["nm", "-D", "--defined-only", LIB], capture_output=True, text=True,
                         check=True).stdout
    exported = set(re.findall(r"\bT (dem_\w+)", out))
    missing = [n for n in declared() if n not in exported]
    assert not missing, missing
    C.CDLL(LIB)   # loads without a GPU


@pytest.mark.skipif(not os.path.exists(LIB), reason="libdem.so not built")
def test_parameter_validation_on_host():
    from paper_2311_11322_amd import dem
    from paper_2311_11322_amd import workloads as W
    good = dict(W.CONTACT_PARAMS, dt=1e-4, G=0.0, soft_frac=0.5, periodic=0, box=(0, 0, 0))
    for bad in (dict(dt=0.0), dict(eps_n=0.0), dict(eps_t=1.5), dict(k_n=-1.0), dict(mu_s=-0.1),
                dict(periodic=1, box=(10.0, 10.0, 9.0)), dict(dt=float("nan")),
                dict(walls=[(0.0, 0.0, 2.0, 0.0)]),                        # not a unit normal
                dict(walls=[(0.0, 0.0, 1.0, 0.0)], periodic=1, box=(9.0, 9.0, 9.0)),
                dict(walls=[(0.0, 0.0, 1.0, float("inf"))]),
                dict(walls=[(0.0, 0.0, 1.0, 0.0)], shake_amp=[(0.0, 0.0, float("nan"))]),
                dict(g=(0.0, 0.0, float("nan"))),
                dict(G=1.0, gravity_tree=1, tree_order=3),
                dict(G=1.0, gravity_tree=1, tree_order=0),
                dict(G=1.0, gravity_tree=1, theta=1.5),
                dict(G=1.0, gravity_tree=1, tree_leaf=0),
                dict(G=1.0, gravity_tree=1, periodic=1, box=(9.0, 9.0, 9.0))):
        p = dict(good, **bad)
        with pytest.raises(dem.DemError) as ei:
            dem.Sim(p)
        assert ei.value.code == dem.DEM_ERR_INVALID_ARG
    with pytest.raises(ValueError):
        dem.Sim(dict(good, walls=[(0.0, 0.0, 1.0, 0.0)] * 7))
    dem.Sim(dict(good, walls=W.open_box_walls(10, 10), g=(0, 0, -1))).close()
    # footprint is pure host arithmetic and grows with size
    f1 = dem.footprint_bytes(good, 1000, 4500)
    f2 = dem.footprint_bytes(good, 2000, 9000)
    assert 0 < f1 < f2
    assert f1 > 4500 * 500
    # with gravity the exact sum's partials are at most 256 x 3 per sphere
    # beyond 256 tiles: the footprint grows linearly in the sphere count
    grav = dict(good, G=1.0)
    f3 = dem.footprint_bytes(grav, 200000, 1000000)
    f4 = dem.footprint_bytes(grav, 400000, 2000000)
    assert 1.9 < f4 / f3 < 2.1
    assert f4 < 2000000 * (256 * 3 * 8 + 4000)


@pytest.mark.skipif(not os.path.exists(LIB) or os.path.exists("/dev/kfd"),
                    reason="needs the built library on a machine without a GPU")
def test_no_device_fails_loudly():
    """Without a device the first call that needs one reports DEVICE with a
    message (not an allocation failure)."""
    import numpy as np
    from paper_2311_11322_amd import dem
    from paper_2311_11322_amd import workloads as W
    w = W.periodic_box(3, n_agg=5)
    sim = dem.Sim(w.params)
    with pytest.raises(dem.DemError) as ei:
        sim.add_workload(w)
    assert ei.value.code == dem.DEM_ERR_DEVICE
    assert "device" in str(ei.value)
    with pytest.raises(dem.DemError) as ei:
        dem.find_contacts(w.pos, w.radius, np.zeros(w.n_sph, np.int32))
    assert ei.value.code == dem.DEM_ERR_DEVICE
