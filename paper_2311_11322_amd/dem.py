"""Thin ctypes binding of the C-ABI in ``include/dem.h`` (same names).

Argument marshalling only: every step of the method runs in the HIP
library.  PyTorch, when used, only provides device memory (through the
library's allocator callback) and the HIP stream.  Importing this module
loads ``libdem.so`` and fails loudly if it has not been built.
"""
from __future__ import annotations

import ctypes as C
import os
from typing import Dict, Iterable, Optional

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libdem.so")

DEM_OK = 0
DEM_ERR_INVALID_ARG = -1
DEM_ERR_OOM = -2
DEM_ERR_CAPACITY = -3
DEM_ERR_UNSTABLE = -4
DEM_ERR_DEVICE = -5
DEM_ERR_STATE = -6
DEM_STOPPED = 1
STATUS_NAMES = {0: "OK", -1: "INVALID_ARG", -2: "OOM", -3: "CAPACITY", -4: "UNSTABLE",
                -5: "DEVICE", -6: "STATE", 1: "STOPPED"}

PREC_FP64 = 0
PREC_FP32_FORCE = 1

_PD = C.POINTER(C.c_double)
_PU64 = C.POINTER(C.c_uint64)
_PI32 = C.POINTER(C.c_int32)
_PI64 = C.POINTER(C.c_int64)


class DemError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"{STATUS_NAMES.get(code, code)}: {msg}")
        self.code = code


class dem_params(C.Structure):
    _fields_ = [
        ("dt", C.c_double), ("G", C.c_double), ("softening_frac", C.c_double),
        ("k_n", C.c_double), ("k_t", C.c_double), ("eps_n", C.c_double), ("eps_t", C.c_double),
        ("mu_s", C.c_double), ("mu_r", C.c_double), ("mu_t", C.c_double),
        ("k_r", C.c_double), ("k_q", C.c_double),
        ("periodic", C.c_int32), ("box", C.c_double * 3),
        ("precision", C.c_int32), ("max_contacts_per_sphere", C.c_int32),
        ("max_overlap_frac", C.c_double),
        ("g", C.c_double * 3), ("n_walls", C.c_int32), ("walls", (C.c_double * 4) * 6),
        ("shake_amp", (C.c_double * 3) * 6), ("shake_omega", C.c_double),
        ("shake_phase", C.c_double),
        ("gravity_tree", C.c_int32), ("tree_theta", C.c_double), ("tree_leaf", C.c_int32),
        ("tree_order", C.c_int32),
    ]


_ALLOC_FN = C.CFUNCTYPE(C.c_void_p, C.c_size_t, C.c_void_p)
_FREE_FN = C.CFUNCTYPE(None, C.c_void_p, C.c_void_p)


class dem_allocator(C.Structure):
    _fields_ = [("alloc", _ALLOC_FN), ("free", _FREE_FN), ("ctx", C.c_void_p)]


class dem_tuning(C.Structure):
    _fields_ = [("gravity_tile", C.c_int32), ("cell_scale", C.c_double),
                ("member_scan", C.c_int32), ("member_read", C.c_int32), ("fused", C.c_int32),
                ("gravity_form", C.c_int32)]


class dem_forcing(C.Structure):
    _fields_ = [("spin_dw", C.c_double), ("pert_mass", C.c_double),
                ("pert_pos", C.c_double * 3), ("pert_vel", C.c_double * 3),
                ("stop_growth", C.c_double)]


class dem_state(C.Structure):
    _fields_ = [(n, _PD) for n in ("agg_pos", "agg_vel", "agg_acc", "agg_torque", "agg_quat",
                                  "agg_spin", "agg_spin_body", "agg_mass", "agg_inertia",
                                  "sph_pos", "sph_vel", "sph_force", "sph_torque", "sph_body")] + [
        ("pair_keys", _PU64), ("pair_hist", _PD), ("n_pairs", C.c_int64), ("step", C.c_int64)]


_AGG_FIELDS = {"agg_pos": 3, "agg_vel": 3, "agg_acc": 3, "agg_torque": 3, "agg_quat": 4,
               "agg_spin": 3, "agg_spin_body": 3, "agg_mass": 1, "agg_inertia": 3}
_SPH_FIELDS = {"sph_pos": 3, "sph_vel": 3, "sph_force": 3, "sph_torque": 3, "sph_body": 3}

_LIB = None


def lib():
    """The loaded HIP library.  Raises if it was never built."""
    global _LIB
    if _LIB is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError(f"{LIB_PATH} is missing: build it with "
                              "`python -m paper_2311_11322_amd.build_lib` (hipcc, gfx950)")
        # PyTorch carries its own HIP runtime beside the one the library
        # links.  With the library's runtime initialised first, PyTorch then
        # finds no GPU; the other order works.  So PyTorch, when it sees a
        # GPU, is initialised before the library is loaded.
        try:
            import torch
            if torch.cuda.is_available():
                torch.cuda.init()
        except ImportError:
            pass
        L = C.CDLL(LIB_PATH)
        vp = C.c_void_p
        L.dem_create.argtypes = [C.POINTER(dem_params), C.POINTER(dem_allocator), vp, C.POINTER(vp)]
        L.dem_add_aggregates.argtypes = [vp, C.c_int64, _PI32, _PD, _PD, _PD, _PD, _PD, _PI64]
        L.dem_step.argtypes = [vp, C.c_int64]
        L.dem_read_state.argtypes = [vp, C.POINTER(dem_state)]
        L.dem_get_counts.argtypes = [vp, _PI64, _PI64, _PI64]
        L.dem_set_forcing.argtypes = [vp, C.POINTER(dem_forcing)]
        L.dem_get_forcing.argtypes = [vp, C.POINTER(dem_forcing)]
        L.dem_restore_state.argtypes = [vp, C.POINTER(dem_state)]
        L.dem_reserve_contacts.argtypes = [vp, C.c_int32]
        L.dem_find_contacts.argtypes = [_PD, _PD, _PI32, C.c_int64, _PD, _PU64, C.c_int64, _PI64]
        L.dem_find_contacts_noalloc.argtypes = [vp, vp, vp, C.c_int64, _PD, vp, C.c_int64, _PI64,
                                                vp]
        L.dem_contact_forces.argtypes = [C.POINTER(dem_params), C.c_int64, _PD, _PD, _PD, _PI32,
                                         C.c_int64, _PD, _PD, C.c_int64, _PU64, _PD, _PD, _PD,
                                         _PU64, _PD, C.c_int64, _PI64]
        L.dem_destroy.argtypes = [vp]
        L.dem_last_error.argtypes = [vp]
        L.dem_last_error.restype = C.c_char_p
        L.dem_engine_create.argtypes = [C.c_size_t, vp, C.POINTER(vp)]
        L.dem_engine_attach.argtypes = [vp, vp]
        L.dem_engine_step.argtypes = [vp, C.c_int64]
        L.dem_engine_detach.argtypes = [vp, vp]
        L.dem_engine_destroy.argtypes = [vp]
        L.dem_sim_status.argtypes = [vp]
        L.dem_engine_set_profiling.argtypes = [vp, C.c_int32]
        L.dem_engine_get_profile.argtypes = [vp, _PD, C.c_int32, _PI64]
        L.dem_set_tuning.argtypes = [vp, C.POINTER(dem_tuning)]
        L.dem_gravity_tiles.argtypes = [C.c_int32, _PI32, C.c_int32]
        L.dem_gravity_tiles.restype = C.c_int32
        L.dem_set_profiling.argtypes = [vp, C.c_int32]
        L.dem_get_profile.argtypes = [vp, _PD, C.c_int32, _PI64]
        L.dem_profile_names.restype = C.c_char_p
        L.dem_footprint_bytes.argtypes = [C.POINTER(dem_params), C.c_int64, C.c_int64]
        L.dem_footprint_bytes.restype = C.c_size_t
        for name in ("dem_create", "dem_add_aggregates", "dem_step", "dem_read_state",
                     "dem_get_counts", "dem_set_forcing", "dem_restore_state",
                     "dem_reserve_contacts", "dem_find_contacts", "dem_destroy",
                     "dem_engine_create", "dem_engine_attach", "dem_engine_step",
                     "dem_engine_detach", "dem_engine_destroy", "dem_sim_status",
                     "dem_set_profiling", "dem_get_profile", "dem_set_tuning",
                     "dem_get_forcing", "dem_find_contacts_noalloc", "dem_contact_forces",
                     "dem_engine_set_profiling", "dem_engine_get_profile"):
            getattr(L, name).restype = C.c_int
        _LIB = L
    return _LIB


def _check(code: int, handle=None):
    if code != DEM_OK:
        msg = lib().dem_last_error(handle).decode()
        raise DemError(code, msg)


def _p(a, t=_PD):
    return None if a is None else a.ctypes.data_as(t)


def make_params(d: Dict, precision: int = PREC_FP64, max_contacts: int = 0,
                max_overlap_frac: float = 0.0) -> dem_params:
    p = dem_params()
    p.dt = float(d["dt"])
    p.G = float(d.get("G", 0.0))
    p.softening_frac = float(d.get("soft_frac", d.get("softening_frac", 0.5)))
    for k in ("k_n", "k_t", "eps_n", "eps_t", "mu_s", "mu_r", "mu_t"):
        setattr(p, k, float(d[k]))
    p.k_r = float(d.get("k_r", -1.0))
    p.k_q = float(d.get("k_q", -1.0))
    p.periodic = int(d.get("periodic", 0))
    box = d.get("box", (0.0, 0.0, 0.0))
    for c in range(3):
        p.box[c] = float(box[c])
    p.precision = int(d.get("precision", precision))
    p.max_contacts_per_sphere = int(d.get("max_contacts_per_sphere", max_contacts))
    p.max_overlap_frac = float(d.get("max_overlap_frac", max_overlap_frac))
    g = d.get("g", (0.0, 0.0, 0.0))
    for c in range(3):
        p.g[c] = float(g[c])
    walls = d.get("walls", ())
    if len(walls) > 6:
        raise ValueError("at most 6 walls")
    p.n_walls = len(walls)
    amp = d.get("shake_amp", ())
    for w, wl in enumerate(walls):
        for c in range(4):
            p.walls[w][c] = float(wl[c])
        for c in range(3):
            p.shake_amp[w][c] = float(amp[w][c]) if len(amp) else 0.0
    p.shake_omega = float(d.get("shake_omega", 0.0))
    p.shake_phase = float(d.get("shake_phase", 0.0))
    p.gravity_tree = int(d.get("gravity_tree", 0))
    p.tree_theta = float(d.get("theta", 0.5))
    p.tree_leaf = int(d.get("tree_leaf", 16))
    p.tree_order = int(d.get("tree_order", 4))
    return p


class TorchAllocator:
    """Device memory for the library from PyTorch's caching allocator."""

    def __init__(self, device: int = 0):
        import torch
        self._torch = torch
        self.device = device
        self._alloc = _ALLOC_FN(self._do_alloc)
        self._free = _FREE_FN(self._do_free)
        self.struct = dem_allocator(self._alloc, self._free, None)

    def _do_alloc(self, nbytes, ctx):
        try:
            return int(self._torch.cuda.caching_allocator_alloc(int(nbytes), self.device))
        except Exception:  # noqa: BLE001 - report OOM to the library as NULL
            return None

    def _do_free(self, ptr, ctx):
        self._torch.cuda.caching_allocator_delete(int(ptr))


def torch_stream():
    """The HIP stream handle of torch's current stream on cuda:0."""
    import torch
    return C.c_void_p(torch.cuda.current_stream().cuda_stream)


class Sim:
    """One system (a pile of rigid aggregates) held on the device."""

    def __init__(self, params: Dict, precision: int = PREC_FP64, max_contacts: int = 0,
                 max_overlap_frac: float = 0.0, allocator: Optional[TorchAllocator] = None,
                 stream=None):
        self.params = make_params(params, precision, max_contacts, max_overlap_frac)
        self._allocator = allocator
        h = C.c_void_p()
        _check(lib().dem_create(C.byref(self.params),
                                C.byref(allocator.struct) if allocator else None,
                                stream, C.byref(h)))
        self.h = h
        self.n_agg = 0
        self.n_sph = 0

    def close(self):
        if getattr(self, "h", None) and self.h.value:
            lib().dem_destroy(self.h)
            self.h = C.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:  # noqa: BLE001
            pass

    def add_aggregates(self, counts, pos, radius, mass, agg_vel=None, agg_spin=None):
        counts = np.ascontiguousarray(counts, dtype=np.int32)
        pos = np.ascontiguousarray(pos, dtype=np.float64)
        radius = np.ascontiguousarray(radius, dtype=np.float64)
        mass = np.ascontiguousarray(mass, dtype=np.float64)
        v = None if agg_vel is None else np.ascontiguousarray(agg_vel, dtype=np.float64)
        w = None if agg_spin is None else np.ascontiguousarray(agg_spin, dtype=np.float64)
        first = C.c_int64()
        _check(lib().dem_add_aggregates(self.h, counts.shape[0], _p(counts, _PI32), _p(pos),
                                        _p(radius), _p(mass), _p(v), _p(w), C.byref(first)),
               self.h)
        self.n_agg = int(counts.shape[0])
        self.n_sph = int(radius.shape[0])
        return self

    def add_workload(self, w):
        return self.add_aggregates(w.counts, w.pos, w.radius, w.mass, w.agg_vel, w.agg_spin)

    def step(self, n: int = 1) -> int:
        """Advance n steps; returns DEM_OK, or DEM_STOPPED when the stop rule
        of the forcing fired (the state is then that at the start of the
        stopping step).  Failures raise DemError."""
        code = lib().dem_step(self.h, int(n))
        if code == DEM_STOPPED:
            return code
        _check(code, self.h)
        return code

    def counts(self):
        a, s, p = C.c_int64(), C.c_int64(), C.c_int64()
        _check(lib().dem_get_counts(self.h, C.byref(a), C.byref(s), C.byref(p)), self.h)
        return a.value, s.value, p.value

    def read_state(self, fields: Optional[Iterable[str]] = None, pairs: bool = False) -> Dict:
        na, ns, np_ = self.counts()
        names = list(_AGG_FIELDS) + list(_SPH_FIELDS) if fields is None else list(fields)
        st = dem_state()
        out = {}
        for n in names:
            if n in _AGG_FIELDS:
                k = _AGG_FIELDS[n]
                a = np.zeros((na, k) if k > 1 else na)
            else:
                a = np.zeros((ns, _SPH_FIELDS[n]))
            out[n] = a
            setattr(st, n, _p(a))
        if pairs:
            keys = np.zeros(max(np_, 1), dtype=np.uint64)
            hist = np.zeros((max(np_, 1), 7))
            st.pair_keys = _p(keys, _PU64)
            st.pair_hist = _p(hist)
        _check(lib().dem_read_state(self.h, C.byref(st)), self.h)
        if pairs:
            out["pair_keys"] = keys[:st.n_pairs].copy()
            out["pair_hist"] = hist[:st.n_pairs].copy()
        out["n_pairs"] = int(st.n_pairs)
        out["step"] = int(st.step)
        return out

    def checkpoint(self) -> Dict:
        return self.read_state(["agg_pos", "agg_vel", "agg_acc", "agg_torque", "agg_quat",
                                "agg_spin_body"], pairs=True)

    def restore(self, ck: Dict):
        st = dem_state()
        keep = {}
        for n in ("agg_pos", "agg_vel", "agg_acc", "agg_torque", "agg_quat", "agg_spin_body"):
            a = np.ascontiguousarray(ck[n], dtype=np.float64)
            keep[n] = a
            setattr(st, n, _p(a))
        keys = np.ascontiguousarray(ck["pair_keys"], dtype=np.uint64)
        hist = np.ascontiguousarray(ck["pair_hist"], dtype=np.float64)
        st.pair_keys = _p(keys, _PU64)
        st.pair_hist = _p(hist)
        st.n_pairs = int(keys.shape[0])
        st.step = int(ck.get("step", 0))
        _check(lib().dem_restore_state(self.h, C.byref(st)), self.h)

    def set_forcing(self, spin_dw: float = 0.0, pert_mass: float = 0.0, pert_pos=(0, 0, 0),
                    pert_vel=(0, 0, 0), stop_growth: float = 0.0):
        f = dem_forcing(float(spin_dw), float(pert_mass), (C.c_double * 3)(*map(float, pert_pos)),
                        (C.c_double * 3)(*map(float, pert_vel)), float(stop_growth))
        _check(lib().dem_set_forcing(self.h, C.byref(f)), self.h)

    def get_forcing(self) -> Dict:
        f = dem_forcing()
        _check(lib().dem_get_forcing(self.h, C.byref(f)), self.h)
        return {"spin_dw": f.spin_dw, "pert_mass": f.pert_mass,
                "pert_pos": np.array(f.pert_pos[:]), "pert_vel": np.array(f.pert_vel[:]),
                "stop_growth": f.stop_growth}

    def reserve_contacts(self, per_sphere: int):
        _check(lib().dem_reserve_contacts(self.h, int(per_sphere)), self.h)

    def status(self) -> int:
        return int(lib().dem_sim_status(self.h))

    def set_tuning(self, gravity_tile: int = 0, cell_scale: float = 1.0, member_scan: int = 0,
                   member_read: int = 0, fused: int = 0, gravity_form: int = 0):
        t = dem_tuning(int(gravity_tile), float(cell_scale), int(member_scan), int(member_read),
                       int(fused), int(gravity_form))
        _check(lib().dem_set_tuning(self.h, C.byref(t)), self.h)

    def set_profiling(self, on: bool, graph_order: bool = False):
        """Per-kernel timing: launches one after another with events between
        kernels, or (graph_order=True) launches ordered as in the step graph, gravity
        beside the contact kernels, with events around the gravity stage only."""
        _check(lib().dem_set_profiling(self.h, (2 if graph_order else 1) if on else 0), self.h)

    def profile(self) -> Dict[str, float]:
        """Accumulated per-kernel milliseconds and the steps they cover."""
        names = lib().dem_profile_names().decode().split(";")
        ms = np.zeros(len(names))
        n = C.c_int64()
        _check(lib().dem_get_profile(self.h, _p(ms), len(names), C.byref(n)), self.h)
        out = dict(zip(names, ms.tolist()))
        out["_steps"] = int(n.value)
        return out


class Engine:
    """Steps many systems together (one graph per step covering all)."""

    def __init__(self, hbm_budget_bytes: int, stream=None):
        h = C.c_void_p()
        _check(lib().dem_engine_create(int(hbm_budget_bytes), stream, C.byref(h)))
        self.h = h
        self.sims = []

    def attach(self, sim: Sim):
        _check(lib().dem_engine_attach(self.h, sim.h), sim.h)
        self.sims.append(sim)

    def detach(self, sim: Sim):
        _check(lib().dem_engine_detach(self.h, sim.h), sim.h)
        self.sims.remove(sim)

    def step(self, n: int = 1) -> int:
        """Advance every attached system; returns the first failure code
        (failed systems stop, the rest continue)."""
        return int(lib().dem_engine_step(self.h, int(n)))

    def set_profiling(self, on: bool):
        _check(lib().dem_engine_set_profiling(self.h, int(bool(on))))

    def profile(self) -> Dict[str, float]:
        """Accumulated per-kernel milliseconds of the engine's steps."""
        names = lib().dem_profile_names().decode().split(";")
        ms = np.zeros(len(names))
        n = C.c_int64()
        _check(lib().dem_engine_get_profile(self.h, _p(ms), len(names), C.byref(n)))
        out = dict(zip(names, ms.tolist()))
        out["_steps"] = int(n.value)
        return out

    def close(self):
        if getattr(self, "h", None) and self.h.value:
            lib().dem_engine_destroy(self.h)
            self.h = C.c_void_p()
            self.sims = []

    def __del__(self):
        try:
            self.close()
        except Exception:  # noqa: BLE001
            pass


def find_contacts(pos, radius, agg, box=None) -> np.ndarray:
    """Device contact search (stateless); canonical keys (i << 32 | j)."""
    pos = np.ascontiguousarray(pos, dtype=np.float64)
    radius = np.ascontiguousarray(radius, dtype=np.float64)
    agg = np.ascontiguousarray(agg, dtype=np.int32)
    n = radius.shape[0]
    bx = None if box is None else np.ascontiguousarray(box, dtype=np.float64)
    cap = 64 * n
    keys = np.zeros(cap, dtype=np.uint64)
    nout = C.c_int64()
    _check(lib().dem_find_contacts(_p(pos), _p(radius), _p(agg, _PI32), n, _p(bx),
                                   _p(keys, _PU64), cap, C.byref(nout)))
    return keys[:nout.value].copy()


def contact_forces(params: Dict, pos, vel, radius, agg, agg_mass, agg_spin, old_keys=None,
                   old_hist=None, precision: int = PREC_FP64) -> Dict:
    """Contact forces of given sphere states on the device (same-input hook):
    per-sphere force and torque, the new contact keys and their history."""
    prm = make_params(params, precision)
    pos = np.ascontiguousarray(pos, dtype=np.float64)
    vel = np.ascontiguousarray(vel, dtype=np.float64)
    radius = np.ascontiguousarray(radius, dtype=np.float64)
    agg = np.ascontiguousarray(agg, dtype=np.int32)
    agg_mass = np.ascontiguousarray(agg_mass, dtype=np.float64)
    agg_spin = np.ascontiguousarray(agg_spin, dtype=np.float64)
    ok = np.zeros(0, np.uint64) if old_keys is None else np.ascontiguousarray(old_keys, np.uint64)
    oh = np.zeros((0, 7)) if old_hist is None else np.ascontiguousarray(old_hist, np.float64)
    n = radius.shape[0]
    cap = 16 * n
    F = np.zeros((n, 3))
    T = np.zeros((n, 3))
    keys = np.zeros(cap, np.uint64)
    hist = np.zeros((cap, 7))
    nout = C.c_int64()
    _check(lib().dem_contact_forces(C.byref(prm), n, _p(pos), _p(vel), _p(radius), _p(agg, _PI32),
                                    agg_mass.shape[0], _p(agg_mass), _p(agg_spin), ok.shape[0],
                                    _p(ok, _PU64), _p(oh), _p(F), _p(T), _p(keys, _PU64),
                                    _p(hist), cap, C.byref(nout)))
    k = nout.value
    return {"F": F, "tau": T, "keys": keys[:k].copy(), "hist": hist[:k].copy()}


def find_contacts_noalloc(pos, radius, agg, box=None, out=None, stream=None):
    """The allocation-free device search on device tensors (torch, cuda:0):
    ``pos`` [n, 3] float64, ``radius`` [n] float64, ``agg`` [n] int32, all
    contiguous; ``out`` a device uint64/int64 tensor receiving the keys (up
    to its length).  Returns the total number of contacts.  Argument
    marshalling only; nothing here allocates device memory."""
    n = int(radius.shape[0])
    for t in (pos, radius, agg):
        if not t.is_contiguous():
            raise ValueError("device arrays must be contiguous")
    bx = None if box is None else np.ascontiguousarray(box, dtype=np.float64)
    cap = 0 if out is None else int(out.numel())
    nout = C.c_int64()
    st = torch_stream() if stream is None else stream
    _check(lib().dem_find_contacts_noalloc(
        C.c_void_p(pos.data_ptr()), C.c_void_p(radius.data_ptr()), C.c_void_p(agg.data_ptr()),
        n, _p(bx), None if out is None else C.c_void_p(out.data_ptr()), cap, C.byref(nout), st))
    return int(nout.value)


def gravity_tiles(precision: int = PREC_FP64):
    """Gravity tile sizes the library supports for a precision (default first)."""
    buf = (C.c_int32 * 8)()
    n = lib().dem_gravity_tiles(int(precision), buf, 8)
    return [int(buf[k]) for k in range(n)]


def footprint_bytes(params: Dict, n_agg: int, n_sph: int, precision: int = PREC_FP64,
                    max_contacts: int = 0) -> int:
    p = make_params(params, precision, max_contacts)
    return int(lib().dem_footprint_bytes(C.byref(p), int(n_agg), int(n_sph)))
