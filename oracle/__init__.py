"""ctypes access to the plain FP64 CPU oracle (``oracle.c``).

TEST INFRASTRUCTURE ONLY: the tests, the smoke check and the CPU-baseline leg
of the benchmark use this; the product path never does.  The oracle shares no
code with the GPU library.
"""
from __future__ import annotations

import ctypes as C
import os
from typing import Dict, Optional

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
_LIB = None

_PD = C.POINTER(C.c_double)
_PI64 = C.POINTER(C.c_int64)
_PI32 = C.POINTER(C.c_int32)
_PU64 = C.POINTER(C.c_uint64)


class Params(C.Structure):
    _fields_ = [
        ("dt", C.c_double), ("G", C.c_double), ("soft_frac", C.c_double),
        ("k_n", C.c_double), ("k_t", C.c_double),
        ("eps_n", C.c_double), ("eps_t", C.c_double),
        ("mu_s", C.c_double), ("mu_r", C.c_double), ("mu_t", C.c_double),
        ("k_r", C.c_double), ("k_q", C.c_double),
        ("periodic", C.c_int32), ("box", C.c_double * 3),
        ("spin_dw", C.c_double), ("torque_at_centre", C.c_int32),
        ("g", C.c_double * 3), ("n_walls", C.c_int32), ("wall", (C.c_double * 4) * 6),
        ("shake_amp", (C.c_double * 3) * 6), ("shake_omega", C.c_double),
        ("shake_phase", C.c_double),
        ("gravity_tree", C.c_int32), ("theta", C.c_double), ("tree_leaf", C.c_int32),
        ("tree_order", C.c_int32),
    ]


def lib():
    global _LIB
    if _LIB is None:
        path = os.path.join(HERE, "liboracle.so")
        if not os.path.exists(path):
            from . import build as _b
            _b.build()
        L = C.CDLL(path)
        L.ora_create.restype = C.c_void_p
        L.ora_create.argtypes = [C.POINTER(Params)]
        L.ora_destroy.argtypes = [C.c_void_p]
        L.ora_add.restype = C.c_int
        L.ora_add.argtypes = [C.c_void_p, C.c_int64, _PI32, _PD, _PD, _PD, _PD, _PD, C.c_int32]
        L.ora_step.restype = C.c_int
        L.ora_step.argtypes = [C.c_void_p, C.c_int64]
        L.ora_get_counts.argtypes = [C.c_void_p, _PI64, _PI64, _PI64]
        L.ora_get_aggregates.argtypes = [C.c_void_p] + [_PD] * 9
        L.ora_get_spheres.argtypes = [C.c_void_p] + [_PD] * 5
        L.ora_get_pairs.argtypes = [C.c_void_p, _PI64, _PI64, _PD, _PD, _PD]
        L.ora_diagnostics.argtypes = [C.c_void_p, _PD]
        L.ora_eval_subset.argtypes = [C.c_void_p, _PI64, C.c_int64, _PD, _PD]
        L.ora_find_contacts.restype = C.c_int64
        L.ora_find_contacts.argtypes = [_PD, _PD, _PI32, C.c_int64, _PD, _PU64, C.c_int64]
        L.ora_gravity.argtypes = [_PD, _PD, _PD, C.c_int64, C.c_double, C.c_double, _PI64,
                                  C.c_int64, _PD]
        L.ora_tree_gravity.argtypes = [_PD, _PD, _PD, C.c_int64, C.c_double, C.c_double,
                                       C.c_double, C.c_int32, C.c_int32, _PD]
        L.ora_set_perturber.argtypes = [C.c_void_p, C.c_double, _PD, _PD]
        L.ora_get_perturber.argtypes = [C.c_void_p, _PD, _PD, _PD]
        L.ora_rotate.argtypes = [_PD, _PD, _PD, _PD, C.c_double, _PD]
        L.ora_setup_body.restype = C.c_int
        L.ora_set_threads.restype = C.c_int32
        L.ora_contact_forces.restype = C.c_int64
        L.ora_contact_forces.argtypes = [C.POINTER(Params), C.c_int64, _PD, _PD, _PD, _PI32,
                                         C.c_int64, _PD, _PD, C.c_int64, _PU64, _PD, _PD, _PD,
                                         _PU64, _PD, C.c_int64]
        L.ora_set_threads.argtypes = [C.c_int32]
        L.ora_setup_body.argtypes = [C.c_int64, _PD, _PD, _PD, _PD, _PD, _PD, _PD, _PD]
        _LIB = L
    return _LIB


def _p(a, t=_PD):
    return None if a is None else a.ctypes.data_as(t)


def _f64(a, shape=None):
    a = np.ascontiguousarray(a, dtype=np.float64)
    if shape is not None:
        a = a.reshape(shape)
    return a


def make_params(d: Dict) -> Params:
    p = Params()
    for k in ("dt", "G", "soft_frac", "k_n", "k_t", "eps_n", "eps_t", "mu_s", "mu_r", "mu_t",
              "k_r", "k_q"):
        setattr(p, k, float(d[k]))
    p.periodic = int(d.get("periodic", 0))
    box = d.get("box", (0.0, 0.0, 0.0))
    for c in range(3):
        p.box[c] = float(box[c])
    p.spin_dw = float(d.get("spin_dw", 0.0))
    p.torque_at_centre = int(d.get("torque_at_centre", 0))
    g = d.get("g", (0.0, 0.0, 0.0))
    for c in range(3):
        p.g[c] = float(g[c])
    walls = d.get("walls", ())
    p.n_walls = len(walls)
    amp = d.get("shake_amp", ())
    for w, wl in enumerate(walls):
        for c in range(4):
            p.wall[w][c] = float(wl[c])
        for c in range(3):
            p.shake_amp[w][c] = float(amp[w][c]) if len(amp) else 0.0
    p.shake_omega = float(d.get("shake_omega", 0.0))
    p.shake_phase = float(d.get("shake_phase", 0.0))
    p.gravity_tree = int(d.get("gravity_tree", 0))
    p.theta = float(d.get("theta", 0.5))
    p.tree_leaf = int(d.get("tree_leaf", 16))
    p.tree_order = int(d.get("tree_order", 4))
    return p


class Oracle:
    """One simulated system held by the C oracle."""

    def __init__(self, params: Dict):
        self._params = make_params(params)
        self._h = lib().ora_create(C.byref(self._params))
        if not self._h:
            raise MemoryError("ora_create failed")

    @property
    def dt(self) -> float:
        return float(self._params.dt)

    def __del__(self):
        h = getattr(self, "_h", None)
        if h:
            lib().ora_destroy(h)
            self._h = None

    def add(self, counts, pos, radius, mass, agg_vel=None, agg_spin=None, evaluate=True):
        counts = np.ascontiguousarray(counts, dtype=np.int32)
        pos = _f64(pos)
        radius = _f64(radius)
        mass = _f64(mass)
        v = None if agg_vel is None else _f64(agg_vel)
        w = None if agg_spin is None else _f64(agg_spin)
        rc = lib().ora_add(self._h, counts.shape[0], _p(counts, _PI32), _p(pos), _p(radius),
                           _p(mass), _p(v), _p(w), int(bool(evaluate)))
        if rc != 0:
            raise ValueError("ora_add rejected the input")
        self.agg_counts = counts.copy()
        return self

    def add_workload(self, w, evaluate=True):
        return self.add(w.counts, w.pos, w.radius, w.mass, w.agg_vel, w.agg_spin, evaluate)

    def set_perturber(self, M, pos, vel):
        pos = _f64(pos)
        vel = _f64(vel)
        lib().ora_set_perturber(self._h, float(M), _p(pos), _p(vel))
        return self

    def perturber(self):
        r, v, a = np.zeros(3), np.zeros(3), np.zeros(3)
        lib().ora_get_perturber(self._h, _p(r), _p(v), _p(a))
        return r, v, a

    def step(self, n=1):
        if lib().ora_step(self._h, int(n)) != 0:
            raise RuntimeError("ora_step failed")

    def counts(self):
        a, s, p = C.c_int64(), C.c_int64(), C.c_int64()
        lib().ora_get_counts(self._h, C.byref(a), C.byref(s), C.byref(p))
        return a.value, s.value, p.value

    def aggregates(self) -> Dict[str, np.ndarray]:
        na, _, _ = self.counts()
        out = dict(M=np.zeros(na), rA=np.zeros((na, 3)), vA=np.zeros((na, 3)),
                   aA=np.zeros((na, 3)), NA=np.zeros((na, 3)), q=np.zeros((na, 4)),
                   wb=np.zeros((na, 3)), wA=np.zeros((na, 3)), I=np.zeros((na, 3)))
        lib().ora_get_aggregates(self._h, *[_p(out[k]) for k in
                                            ("M", "rA", "vA", "aA", "NA", "q", "wb", "wA", "I")])
        return out

    def spheres(self) -> Dict[str, np.ndarray]:
        _, ns, _ = self.counts()
        out = dict(r=np.zeros((ns, 3)), v=np.zeros((ns, 3)), F=np.zeros((ns, 3)),
                   tau=np.zeros((ns, 3)), b=np.zeros((ns, 3)))
        lib().ora_get_spheres(self._h, *[_p(out[k]) for k in ("r", "v", "F", "tau", "b")])
        return out

    def pairs(self) -> Dict[str, np.ndarray]:
        _, _, n = self.counts()
        out = dict(i=np.zeros(n, dtype=np.int64), j=np.zeros(n, dtype=np.int64),
                   hist=np.zeros((n, 7)), force=np.zeros((n, 9)), diag=np.zeros((n, 8)))
        lib().ora_get_pairs(self._h, _p(out["i"], _PI64), _p(out["j"], _PI64),
                            _p(out["hist"]), _p(out["force"]), _p(out["diag"]))
        return out

    def diagnostics(self) -> Dict[str, np.ndarray]:
        o = np.zeros(16)
        lib().ora_diagnostics(self._h, _p(o))
        return dict(P=o[0:3].copy(), L=o[3:6].copy(), Kt=o[6], Kr=o[7], Es=o[8], Ug=o[9],
                    max_overlap=o[10], R_bulk=o[11], com=o[12:15].copy(), Uu=o[15],
                    E=o[6] + o[7] + o[8] + o[9] + o[15])

    def eval_subset(self, idx):
        idx = np.ascontiguousarray(idx, dtype=np.int64)
        F = np.zeros((idx.shape[0], 3))
        T = np.zeros((idx.shape[0], 3))
        lib().ora_eval_subset(self._h, _p(idx, _PI64), idx.shape[0], _p(F), _p(T))
        return F, T


def find_contacts(pos, radius, agg, box=None) -> np.ndarray:
    """Brute-force canonical contact keys (i << 32 | j)."""
    pos = _f64(pos)
    radius = _f64(radius)
    agg = np.ascontiguousarray(agg, dtype=np.int32)
    n = radius.shape[0]
    bx = None if box is None else _f64(box)
    cap = 1 << 16
    while True:
        keys = np.zeros(cap, dtype=np.uint64)
        np_ = lib().ora_find_contacts(_p(pos), _p(radius), _p(agg, _PI32), n, _p(bx),
                                      _p(keys, _PU64), cap)
        if np_ <= cap:
            return keys[:np_]
        cap = int(np_)


def gravity(pos, mass, radius, G, soft_frac, idx=None) -> np.ndarray:
    pos = _f64(pos)
    mass = _f64(mass)
    radius = _f64(radius)
    n = mass.shape[0]
    idx = np.arange(n, dtype=np.int64) if idx is None else np.ascontiguousarray(idx, dtype=np.int64)
    F = np.zeros((idx.shape[0], 3))
    lib().ora_gravity(_p(pos), _p(mass), _p(radius), n, float(G), float(soft_frac),
                      _p(idx, _PI64), idx.shape[0], _p(F))
    return F


def tree_gravity(pos, mass, radius, G, soft_frac, theta=0.5, leaf=16, order=4) -> np.ndarray:
    """Tree gravity (multipoles to order 2 or 4) on every sphere."""
    pos = _f64(pos)
    mass = _f64(mass)
    radius = _f64(radius)
    n = mass.shape[0]
    F = np.zeros((n, 3))
    lib().ora_tree_gravity(_p(pos), _p(mass), _p(radius), n, float(G), float(soft_frac),
                           float(theta), int(leaf), int(order), _p(F))
    return F


def rotate(q, wb, I, N_space, h):
    q = _f64(q).copy()
    wb = _f64(wb).copy()
    I = _f64(I)
    N = _f64(N_space)
    err = np.zeros(1)
    lib().ora_rotate(_p(q), _p(wb), _p(I), _p(N), float(h), _p(err))
    return q, wb, float(err[0])


def setup_body(pos, radius, mass):
    pos = _f64(pos)
    radius = _f64(radius)
    mass = _f64(mass)
    n = radius.shape[0]
    M = np.zeros(1)
    r = np.zeros(3)
    I = np.zeros(3)
    q = np.zeros(4)
    b = np.zeros((n, 3))
    rc = lib().ora_setup_body(n, _p(pos), _p(radius), _p(mass), _p(M), _p(r), _p(I), _p(q), _p(b))
    if rc != 0:
        raise ValueError("setup rejected")
    return float(M[0]), r, I, q, b


def quat_matrix(q) -> np.ndarray:
    """Rotation matrix of a quaternion (w, x, y, z) -- a test helper written
    from the textbook formula, used to express body-frame results in space."""
    w, x, y, z = q
    return np.array([
        [1 - 2 * (y * y + z * z), 2 * (x * y - w * z), 2 * (x * z + w * y)],
        [2 * (x * y + w * z), 1 - 2 * (x * x + z * z), 2 * (y * z - w * x)],
        [2 * (x * z - w * y), 2 * (y * z + w * x), 1 - 2 * (x * x + y * y)],
    ])


def set_threads(n: int = 0) -> int:
    """Threads of the oracle's gravity target loops (OpenMP); the results do
    not depend on it.  n <= 0 only queries.  Returns the count in effect."""
    return int(lib().ora_set_threads(int(n)))


def contact_forces(params: Dict, pos, vel, radius, agg, agg_mass, agg_spin, old_keys=None,
                   old_hist=None) -> Dict[str, np.ndarray]:
    """Contact part of one evaluation on given sphere states: per-sphere
    contact force and torque, new canonical keys and their history."""
    prm = make_params(params)
    pos = _f64(pos)
    vel = _f64(vel)
    radius = _f64(radius)
    agg = np.ascontiguousarray(agg, dtype=np.int32)
    agg_mass = _f64(agg_mass)
    agg_spin = _f64(agg_spin)
    ok = np.zeros(0, np.uint64) if old_keys is None else np.ascontiguousarray(old_keys, np.uint64)
    oh = np.zeros((0, 7)) if old_hist is None else _f64(old_hist)
    n = radius.shape[0]
    cap = 64 * n
    F = np.zeros((n, 3))
    T = np.zeros((n, 3))
    keys = np.zeros(cap, np.uint64)
    hist = np.zeros((cap, 7))
    k = lib().ora_contact_forces(C.byref(prm), n, _p(pos), _p(vel), _p(radius), _p(agg, _PI32),
                                 agg_mass.shape[0], _p(agg_mass), _p(agg_spin), ok.shape[0],
                                 _p(ok, _PU64), _p(oh), _p(F), _p(T), _p(keys, _PU64), _p(hist),
                                 cap)
    return {"F": F, "tau": T, "keys": keys[:k].copy(), "hist": hist[:k].copy()}
