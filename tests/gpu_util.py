"""Shared helpers of the GPU parity tests (comparison norms, runners)."""
import numpy as np

import oracle as O


def rel_err(gpu, ora, box=None, scale=None):
    """max |gpu - ora| / max |ora| (minimum image if a periodic side is
    given).  The parity norm: per state array, relative to its largest
    oracle entry, or to ``scale`` when that is larger."""
    g = np.asarray(gpu, dtype=np.float64)
    o = np.asarray(ora, dtype=np.float64)
    d = g - o
    if box is not None:
        d = d - box * np.round(d / box)
    s = float(np.abs(o).max()) if o.size else 0.0
    if scale is not None:
        s = max(s, float(scale))
    if s == 0.0:
        return float(np.abs(d).max()) if d.size else 0.0
    return float(np.abs(d).max() / s)


def sum_scales(o: O.Oracle):
    """Magnitudes of the terms the force and torque sums are made of.

    A sum computed in another order differs from the oracle's by rounding
    relative to the sum of the terms' magnitudes, not to the result: forces
    that nearly cancel (a sphere squeezed evenly by its neighbours) or torques
    of purely normal forces (zero up to rounding) are compared against these
    scales.  Per sphere: sum of |F| over its contacts plus the magnitude of
    its total force (which covers the gravity terms: an aggregate alone in
    space has a torque of its members' mutual pulls that is zero up to
    rounding), and sum of |tau| + l |F| (lever times force); per aggregate:
    the members' force scale over M, and sum of |b| F-scale + torque scale."""
    a = o.aggregates()
    s = o.spheres()
    p = o.pairs()
    ns = s["r"].shape[0]
    SF = np.linalg.norm(s["F"], axis=1) if ns else np.zeros(0)
    ST = np.zeros(ns)
    if p["i"].size:
        F = np.linalg.norm(p["force"][:, 0:3], axis=1)
        ti = np.linalg.norm(p["force"][:, 3:6], axis=1)
        tj = np.linalg.norm(p["force"][:, 6:9], axis=1)
        li, lj = p["diag"][:, 5], p["diag"][:, 6]
        np.add.at(SF, p["i"], F)
        np.add.at(ST, p["i"], ti + np.abs(li) * F)
        sph = p["j"] < ns
        np.add.at(SF, p["j"][sph], F[sph])
        np.add.at(ST, p["j"][sph], tj[sph] + np.abs(lj[sph]) * F[sph])
    return SF, ST, a, s


def agg_scales(o: O.Oracle):
    SF, ST, a, s = sum_scales(o)
    off = np.concatenate([[0], np.cumsum(o.agg_counts)]).astype(np.int64)
    b = np.linalg.norm(s["b"], axis=1)
    AF = np.add.reduceat(SF, off[:-1]) if SF.size else SF
    AT = np.add.reduceat(b * SF + ST, off[:-1]) if SF.size else SF
    return SF, ST, AF / a["M"], AT


def hist_tolerance(r, delta):
    """Relative tolerance of the spring history, derived from the arithmetic.

    Positions agree only to rounding (a few ulp of |r|), so the overlap
    delta = S - |d| carries an absolute error of about 4 ulp(max |r|).  The
    history saturates at mu f_N / k with f_N = k_n delta, so its error relative
    to its largest value is about 4 ulp(max|r|) / max(delta); 4x margin."""
    ulp = np.spacing(np.abs(r).max())
    return float(16.0 * ulp / max(float(np.max(delta)), 1e-300))


def space_spin(q: np.ndarray, wb: np.ndarray) -> np.ndarray:
    """R(q) w_b for unit quaternions q = (w, x, y, z): the space-frame spin
    of a state (the state's own, after every increment of the step)."""
    w, x, y, z = q[:, 0], q[:, 1], q[:, 2], q[:, 3]
    R = np.stack([1 - 2 * (y * y + z * z), 2 * (x * y - w * z), 2 * (x * z + w * y),
                  2 * (x * y + w * z), 1 - 2 * (x * x + z * z), 2 * (y * z - w * x),
                  2 * (x * z - w * y), 2 * (y * z + w * x), 1 - 2 * (x * x + y * y)], -1)
    return np.einsum("nij,nj->ni", R.reshape(-1, 3, 3), wb)


def oracle_keys(o: O.Oracle) -> np.ndarray:
    p = o.pairs()
    return (p["i"].astype(np.uint64) << np.uint64(32)) | p["j"].astype(np.uint64)


def compare_states(sim, o: O.Oracle, box=None, tol=1e-12, with_pairs=True):
    """Compare the GPU system with the oracle in the space frame; returns a
    dict of relative errors and asserts the pair list is identical."""
    g = sim.read_state(pairs=with_pairs)
    SF, ST, AF, AT = agg_scales(o)
    a = o.aggregates()
    s = o.spheres()
    mx = lambda x: float(x.max()) if x.size else 0.0
    errs = {
        "agg_pos": rel_err(g["agg_pos"], a["rA"], box),
        "agg_vel": rel_err(g["agg_vel"], a["vA"]),
        "agg_acc": rel_err(g["agg_acc"], a["aA"], scale=mx(AF)),
        "agg_torque": rel_err(g["agg_torque"], a["NA"], scale=mx(AT)),
        # the oracle keeps w_A from the evaluation (the contact velocities'
        # spin); a spin-up increment after the second kick changes w_b only,
        # so the state's spin is compared as R(q) w_b
        "agg_spin": rel_err(g["agg_spin"], space_spin(a["q"], a["wb"])),
        "agg_mass": rel_err(g["agg_mass"], a["M"]),
        "sph_pos": rel_err(g["sph_pos"], s["r"], box),
        "sph_vel": rel_err(g["sph_vel"], s["v"]),
        "sph_force": rel_err(g["sph_force"], s["F"], scale=mx(SF)),
        "sph_torque": rel_err(g["sph_torque"], s["tau"], scale=mx(ST)),
    }
    tols = {k: tol for k in errs}
    op = o.pairs()
    if op["i"].size:
        # the contact forces inherit the overlap's conditioning: each contact
        # force carries an error of k_n times a few ulp of |r| (the spring
        # history's bound), a sphere sums up to z of them, and the largest
        # force is at least k_n max(delta); so forces, torques, accelerations
        # and aggregate torques carry `cond` relative to their scales
        ns = s["r"].shape[0]
        z = np.bincount(np.concatenate([op["i"], op["j"][op["j"] < ns]]), minlength=ns)
        cond = hist_tolerance(s["r"], op["diag"][:, 4]) * max(1.0, float(z.max()))
        for k in ("sph_force", "sph_torque", "agg_acc", "agg_torque"):
            tols[k] = max(tol, cond)
        # a step changes a velocity by h a and a spin by h N / I, so those
        # carry the same relative error times the size of that change over
        # the size of the velocity (spin) itself; a sphere's predicted
        # velocity adds the spin's error times its lever |R b|
        # (a system at rest is compared relative to the change itself)
        h = o.dt
        dv = h * mx(AF)
        dw = h * mx(AT / a["I"].min(axis=1))
        dvi = dv + dw * mx(np.linalg.norm(s["b"], axis=1))
        w_ora = space_spin(a["q"], a["wb"])
        for k, d, ora, gpu in (("agg_vel", dv, a["vA"], g["agg_vel"]),
                               ("agg_spin", dw, w_ora, g["agg_spin"]),
                               ("sph_vel", dvi, s["v"], g["sph_vel"])):
            scale = max(mx(np.abs(ora)), d)
            if scale > 0.0:
                errs[k] = rel_err(gpu, ora, scale=scale)
                tols[k] = max(tol, cond * d / scale)
    if with_pairs:
        keys = oracle_keys(o)
        assert np.array_equal(g["pair_keys"], keys), "contact lists differ"
        if keys.size:
            errs["pair_hist"] = rel_err(g["pair_hist"], op["hist"])
            tols["pair_hist"] = max(tol, hist_tolerance(s["r"], op["diag"][:, 4]))
    print("parity (error / bound):",
          ", ".join(f"{k} {v:.2e}/{tols[k]:.1e}" for k, v in errs.items()), flush=True)
    bad = {k: (v, tols[k]) for k, v in errs.items() if not v <= tols[k]}
    assert not bad, f"parity above its bound: {bad}"
    return errs
