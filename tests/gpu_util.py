"""Shared helpers of the GPU parity tests (comparison norms, runners)."""
import numpy as np

import oracle as O


def rel_err(gpu, ora, box=None):
    """max |gpu - ora| / max |ora| (minimum image if a periodic side is
    given).  The parity norm: per state array, relative to its largest
    oracle entry."""
    g = np.asarray(gpu, dtype=np.float64)
    o = np.asarray(ora, dtype=np.float64)
    d = g - o
    if box is not None:
        d = d - box * np.round(d / box)
    scale = np.abs(o).max()
    if scale == 0.0:
        return float(np.abs(d).max())
    return float(np.abs(d).max() / scale)


def hist_tolerance(r, delta):
    """Relative tolerance of the spring history, derived from the arithmetic.

    Positions agree only to rounding (a few ulp of |r|), so the overlap
    delta = S - |d| carries an absolute error of about 4 ulp(max |r|).  The
    history saturates at mu f_N / k with f_N = k_n delta, so its error relative
    to its largest value is about 4 ulp(max|r|) / max(delta); 4x margin."""
    ulp = np.spacing(np.abs(r).max())
    return float(16.0 * ulp / max(float(np.max(delta)), 1e-300))


def oracle_keys(o: O.Oracle) -> np.ndarray:
    p = o.pairs()
    return (p["i"].astype(np.uint64) << np.uint64(32)) | p["j"].astype(np.uint64)


def compare_states(sim, o: O.Oracle, box=None, tol=1e-12, with_pairs=True):
    """Compare the GPU system with the oracle in the space frame; returns a
    dict of relative errors and asserts the pair list is identical."""
    g = sim.read_state(pairs=with_pairs)
    a = o.aggregates()
    s = o.spheres()
    errs = {
        "agg_pos": rel_err(g["agg_pos"], a["rA"], box),
        "agg_vel": rel_err(g["agg_vel"], a["vA"]),
        "agg_acc": rel_err(g["agg_acc"], a["aA"]),
        "agg_torque": rel_err(g["agg_torque"], a["NA"]),
        "agg_spin": rel_err(g["agg_spin"], a["wA"]),
        "agg_mass": rel_err(g["agg_mass"], a["M"]),
        "sph_pos": rel_err(g["sph_pos"], s["r"], box),
        "sph_vel": rel_err(g["sph_vel"], s["v"]),
        "sph_force": rel_err(g["sph_force"], s["F"]),
        "sph_torque": rel_err(g["sph_torque"], s["tau"]),
    }
    tols = {k: tol for k in errs}
    if with_pairs:
        keys = oracle_keys(o)
        assert np.array_equal(g["pair_keys"], keys), "contact lists differ"
        if keys.size:
            op = o.pairs()
            errs["pair_hist"] = rel_err(g["pair_hist"], op["hist"])
            tols["pair_hist"] = max(tol, hist_tolerance(s["r"], op["diag"][:, 4]))
    bad = {k: (v, tols[k]) for k, v in errs.items() if not v <= tols[k]}
    assert not bad, f"parity above {tol}: {bad}"
    return errs
