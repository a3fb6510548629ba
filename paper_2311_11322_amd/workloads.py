"""Seeded synthetic inputs shaped like the paper's workloads.

This module only *places* spheres and draws random numbers.  It contains none
of the method's arithmetic (no forces, no integration, no aggregate set-up),
so both the GPU library and the FP64 oracle may consume what it produces.

Workload shapes (all radii U[0.8, 1.2], density 1, aggregates built as random
touching clusters of equal-density spheres):

* ``periodic_box``  -- aggregates of 1-8 spheres placed by random sequential
  addition (RSA) in a periodic cube at a target packing fraction, velocities
  N(0, sigma) per component (the contact-only workload; no gravity).
* ``collapse_cloud`` -- aggregates of 2-8 spheres placed by RSA in a ball at
  initial packing fraction phi0 = 0.15, at rest, with self-gravity (the
  gravitational-collapse workload of Sec. 3.3 / Table 1 of the paper).
* ``contact_seeded`` -- as either of the above, but every aggregate after the
  first is put in contact with an already-placed aggregate with a small
  overlap, so that a single step exercises every branch of the contact model.
* ``pile_batch`` -- many independent piles with log-uniform sphere counts
  (the batched spin-up workload).

Every generator takes an explicit seed and uses ``numpy.random.default_rng``.
"""
from __future__ import annotations

import dataclasses
import math
from typing import Dict, List, Optional

import numpy as np

# Contact constants shared by all workloads (spring constant, restitution and
# friction coefficients are user parameters of the soft-sphere model, Sec. 2.1).
CONTACT_PARAMS: Dict[str, float] = dict(
    k_n=1.0e5,
    k_t=(2.0 / 7.0) * 1.0e5,
    eps_n=0.5,
    eps_t=0.5,
    mu_s=0.5,
    mu_r=0.1,
    mu_t=0.1,
    k_r=(2.0 / 7.0) * 1.0e5,
    k_q=(2.0 / 7.0) * 1.0e5,
)

# Smallest allowed surface gap between spheres of different aggregates when a
# workload is placed (keeps every candidate pair far from the contact
# threshold, so the FP64 contact decision is never a rounding coin-flip).
MIN_GAP = 1.0e-6


@dataclasses.dataclass
class Workload:
    """One synthetic system, in the layout the C-ABI takes.

    Spheres are grouped by aggregate: aggregate ``a`` owns spheres
    ``offsets[a] : offsets[a] + counts[a]`` of ``pos``/``radius``/``mass``.
    """

    name: str
    counts: np.ndarray      # int32 [n_agg]
    pos: np.ndarray         # float64 [n_sph, 3], space frame
    radius: np.ndarray      # float64 [n_sph]
    mass: np.ndarray        # float64 [n_sph]
    agg_vel: np.ndarray     # float64 [n_agg, 3]
    agg_spin: np.ndarray    # float64 [n_agg, 3], space frame
    params: Dict[str, float]
    n_steps: int
    pile_of_agg: Optional[np.ndarray] = None   # int32 [n_agg] for batches
    notes: str = ""

    @property
    def n_agg(self) -> int:
        return int(self.counts.shape[0])

    @property
    def n_sph(self) -> int:
        return int(self.pos.shape[0])

    def offsets(self) -> np.ndarray:
        off = np.zeros(self.n_agg + 1, dtype=np.int64)
        np.cumsum(self.counts, out=off[1:])
        return off

    def agg_of_sphere(self) -> np.ndarray:
        return np.repeat(np.arange(self.n_agg, dtype=np.int32), self.counts)


# --------------------------------------------------------------------------
# random primitives
# --------------------------------------------------------------------------

def _unit_vectors(rng: np.random.Generator, n: int) -> np.ndarray:
    v = rng.normal(size=(n, 3))
    return v / np.linalg.norm(v, axis=1, keepdims=True)


def _random_rotation(rng: np.random.Generator) -> np.ndarray:
    """Uniformly random proper rotation matrix (from a normalised 4-vector)."""
    q = rng.normal(size=4)
    q /= np.linalg.norm(q)
    w, x, y, z = q
    return np.array([
        [1 - 2 * (y * y + z * z), 2 * (x * y - w * z), 2 * (x * z + w * y)],
        [2 * (x * y + w * z), 1 - 2 * (x * x + z * z), 2 * (y * z - w * x)],
        [2 * (x * z - w * y), 2 * (y * z + w * x), 1 - 2 * (x * x + y * y)],
    ])


def random_cluster(rng: np.random.Generator, n: int,
                   rmin: float = 0.8, rmax: float = 1.2):
    """A random touching cluster of ``n`` spheres.

    Each new sphere is placed tangent to a uniformly chosen existing member in
    a uniform random direction; a placement that would overlap another member
    is rejected and redrawn.  Returns (offsets from the first sphere, radii).
    """
    radii = rng.uniform(rmin, rmax, n)
    pos = np.zeros((n, 3))
    for k in range(1, n):
        for _ in range(10000):
            a = int(rng.integers(k))
            u = _unit_vectors(rng, 1)[0]
            p = pos[a] + (radii[a] + radii[k]) * u
            d = np.linalg.norm(pos[:k] - p, axis=1)
            lim = radii[:k] + radii[k]
            ok = d >= lim * (1.0 - 1e-12)
            ok[a] = True
            if ok.all():
                pos[k] = p
                break
        else:  # pragma: no cover - geometrically impossible for n <= 8
            raise RuntimeError("could not grow cluster")
    return pos, radii


def sphere_mass(radius: np.ndarray, density: float = 1.0) -> np.ndarray:
    return density * (4.0 / 3.0) * math.pi * radius ** 3


# --------------------------------------------------------------------------
# spatial occupancy grid used only for placement rejection tests
# --------------------------------------------------------------------------

class _Grid:
    """Dense cell grid with fixed slots, for O(1) neighbour lookups while
    placing.  ``periodic`` wraps cell indices."""

    SLOTS = 24

    def __init__(self, lo, hi, cell, periodic=False, box=None):
        self.lo = np.asarray(lo, dtype=np.float64)
        self.cell = float(cell)
        self.periodic = periodic
        self.box = None if box is None else np.asarray(box, dtype=np.float64)
        if periodic:
            self.n = np.maximum((self.box // self.cell).astype(np.int64), 1)
            self.cell_v = self.box / self.n
        else:
            span = np.asarray(hi, dtype=np.float64) - self.lo
            self.n = np.maximum(np.ceil(span / self.cell).astype(np.int64) + 1, 1)
            self.cell_v = np.full(3, self.cell)
        self.slots = -np.ones(tuple(self.n) + (self.SLOTS,), dtype=np.int64)
        self.fill = np.zeros(tuple(self.n), dtype=np.int32)
        self.count = 0
        self._P = np.zeros((1024, 3))
        self._R = np.zeros(1024)

    def _cells(self, p):
        c = np.floor((p - self.lo) / self.cell_v).astype(np.int64)
        if self.periodic:
            c %= self.n
        return c

    def neighbours(self, p: np.ndarray) -> np.ndarray:
        """Indices of stored spheres in the cells touching points ``p``."""
        c = self._cells(p)
        lo = c.min(axis=0) - 1
        hi = c.max(axis=0) + 1
        if self.periodic:
            idx = [np.arange(lo[k], hi[k] + 1) % self.n[k] for k in range(3)]
            idx = [np.unique(ix) for ix in idx]
            sub = self.slots[np.ix_(idx[0], idx[1], idx[2])]
        else:
            lo = np.maximum(lo, 0)
            hi = np.minimum(hi, self.n - 1)
            sub = self.slots[lo[0]:hi[0] + 1, lo[1]:hi[1] + 1, lo[2]:hi[2] + 1]
        s = sub.ravel()
        return s[s >= 0]

    def insert(self, p: np.ndarray, r: np.ndarray):
        c = self._cells(p)
        base = self.count
        k_new = p.shape[0]
        if base + k_new > self._P.shape[0]:
            cap = 2 * (base + k_new)
            self._P = np.concatenate([self._P, np.zeros((cap - self._P.shape[0], 3))])
            self._R = np.concatenate([self._R, np.zeros(cap - self._R.shape[0])])
        for k in range(k_new):
            cx, cy, cz = c[k]
            f = self.fill[cx, cy, cz]
            if f >= self.SLOTS:
                raise RuntimeError("placement grid cell overflow")
            self.slots[cx, cy, cz, f] = base + k
            self.fill[cx, cy, cz] = f + 1
        self._P[base:base + k_new] = p
        self._R[base:base + k_new] = r
        self.count = base + k_new

    def arrays(self):
        return self._P[:self.count], self._R[:self.count]

    def gaps(self, p: np.ndarray, r: np.ndarray):
        """Surface gaps between candidate spheres and stored neighbours.
        Returns (gap matrix [k, m], neighbour indices [m])."""
        nb = self.neighbours(p)
        if nb.size == 0:
            return np.zeros((p.shape[0], 0)), nb
        P, R = self.arrays()
        d = P[nb][None, :, :] - p[:, None, :]
        if self.periodic:
            d -= self.box * np.round(d / self.box)
        dist = np.sqrt((d * d).sum(axis=2))
        return dist - (R[nb][None, :] + r[:, None]), nb


def _place(rng, counts, clusters, container, contact_seeded, max_tries=20000,
           near_after=200):
    """Random sequential addition of whole aggregates (largest first).

    container: ("ball", R): aggregate centres uniform in the ball; or
    ("box", L): centres uniform in the periodic cube; or ("cuboid", (Lx, Ly,
    Lz, z_lo, z_hi, p_floor)): inside the walled box [0, Lx] x [0, Ly] x
    [0, Lz], every sphere at least MIN_GAP clear of the walls, centres drawn
    with z in [z_lo, z_hi], and with probability p_floor an aggregate lowered
    onto the floor so that its lowest sphere overlaps it by U[1e-5, 1e-3].
    If ``contact_seeded`` every
    aggregate after the first is put in contact, with overlap drawn from
    U[1e-5, 1e-3], with a sphere of an already-placed aggregate.  Otherwise,
    once ``near_after`` uniform draws for one aggregate have failed (close to
    the jamming limit of RSA), candidates are drawn next to a placed sphere at
    a surface gap of U[1e-5, 1e-3] instead.
    Returns positions grouped in the *original* aggregate order.
    """
    kind, size = container
    order = np.argsort(-counts, kind="stable")
    if kind == "box":
        L = float(size)
        grid = _Grid(np.zeros(3), None, 2.4, periodic=True, box=np.full(3, L))
    elif kind == "cuboid":
        Lx, Ly, Lz, z_lo, z_hi, p_floor = (float(v) for v in size)
        grid = _Grid(np.full(3, -3.0), np.array([Lx, Ly, Lz]) + 3.0,
                     max(2.4, 2.0 * float(max(c[1].max() for c in clusters)) + 0.1))
    else:
        R = float(size)
        grid = _Grid(np.full(3, -R - 3.0), np.full(3, R + 3.0), 2.4)
    placed_pos = [None] * len(counts)
    sph_owner: List[int] = []
    for n_done, a in enumerate(order):
        rel, rad = clusters[a]
        rel = rel - rel.mean(axis=0)
        for tries in range(max_tries):
            rot = _random_rotation(rng)
            body = rel @ rot.T
            floor_pick = kind == "cuboid" and p_floor > 0 and rng.uniform() < p_floor
            seeded = contact_seeded and n_done > 0 and not floor_pick
            near = (not seeded) and (not floor_pick) and n_done > 0 and tries >= near_after
            if seeded or near:
                # put member m against placed sphere t: overlapping it by
                # U[1e-5, 1e-3] (contact-seeded) or, when plain random draws
                # keep failing near jamming, at a gap of U[1e-5, 1e-3]
                P, Rr = grid.arrays()
                t = int(rng.integers(P.shape[0]))
                m = int(rng.integers(body.shape[0]))
                u = _unit_vectors(rng, 1)[0]
                delta0 = rng.uniform(1e-5, 1e-3)
                sep = Rr[t] + rad[m] + (-delta0 if seeded else delta0)
                centre = P[t] + sep * u - body[m]
                if not seeded:
                    t = -1
            else:
                t = -1
                if kind == "box":
                    centre = rng.uniform(0.0, L, 3)
                elif kind == "cuboid":
                    centre = np.array([rng.uniform(0.0, Lx), rng.uniform(0.0, Ly),
                                       rng.uniform(z_lo, z_hi)])
                    if floor_pick:
                        centre[2] -= (body[:, 2] - rad + centre[2]).min() + rng.uniform(1e-5, 1e-3)
                else:
                    v = _unit_vectors(rng, 1)[0]
                    centre = v * R * rng.uniform() ** (1.0 / 3.0)
            if kind == "box":
                # keep the aggregate whole; only its centre is wrapped
                centre = np.mod(centre, L)
            elif kind == "cuboid":
                p = centre + body
                lo = p - rad[:, None]
                hi = p + rad[:, None]
                if ((lo[:, :2] < MIN_GAP).any() or (hi[:, 0] > Lx - MIN_GAP).any()
                        or (hi[:, 1] > Ly - MIN_GAP).any() or (hi[:, 2] > Lz).any()):
                    continue
                lz = lo[:, 2]
                if ((lz >= -MIN_GAP) & (lz < MIN_GAP)).any() or (lz < -1.001e-3).any():
                    continue    # floor contacts are seeded overlaps, never near misses
            elif np.linalg.norm(centre) > R:
                continue        # centres of mass uniform in the ball
            p = centre + body
            gap, nb = grid.gaps(p, rad)
            if gap.size:
                if t >= 0:
                    # the seeded pair is the only allowed overlap
                    ok_mask = gap >= MIN_GAP
                    seeded = nb == t
                    ok_mask[m, seeded] = True
                    if not ok_mask.all():
                        continue
                elif (gap < MIN_GAP).any():
                    continue
            grid.insert(p, rad)
            sph_owner.extend([a] * len(rad))
            placed_pos[a] = p
            break
        else:
            raise RuntimeError(f"random sequential addition failed after {n_done} of "
                               f"{len(counts)} aggregates; lower the packing")
    pos = np.concatenate([placed_pos[a] for a in range(len(counts))])
    radius = np.concatenate([clusters[a][1] for a in range(len(counts))])
    return pos, radius


def _random_rotations(rng: np.random.Generator, n: int) -> np.ndarray:
    """n uniformly random proper rotation matrices [n, 3, 3]."""
    q = rng.normal(size=(n, 4))
    q /= np.linalg.norm(q, axis=1, keepdims=True)
    w, x, y, z = q.T
    return np.stack([
        np.stack([1 - 2 * (y * y + z * z), 2 * (x * y - w * z), 2 * (x * z + w * y)], -1),
        np.stack([2 * (x * y + w * z), 1 - 2 * (x * x + z * z), 2 * (y * z - w * x)], -1),
        np.stack([2 * (x * z - w * y), 2 * (y * z + w * x), 1 - 2 * (x * x + y * y)], -1),
    ], 1)


def _place_rounds(rng, counts, clusters, container, chunk=16384, max_rounds=2000,
                  near_after=40):
    """Random sequential addition in rounds (fast path for large systems).

    Each round draws random centres and orientations for the pending
    aggregates (largest first; several tries each when few are pending),
    drops tries that come closer than MIN_GAP to a placed sphere, then accepts
    tries in order unless their aggregate is already placed or they clash with
    a try accepted earlier in the same round.  Centres are uniform in the
    ball / periodic cube.  After ``near_after`` rounds (close to the jamming
    limit) tries are drawn next to placed spheres at a small gap instead.
    """
    from scipy.spatial import cKDTree
    kind, size = container
    L = float(size) if kind == "box" else None
    R = float(size) if kind == "ball" else None
    rel = [c[0] - c[0].mean(axis=0) for c in clusters]
    order = list(np.argsort(-counts, kind="stable"))
    placed = [None] * len(counts)
    P = np.zeros((0, 3))
    Rr = np.zeros(0)
    reach = 2.4 + MIN_GAP
    for _round in range(max_rounds):
        if not order:
            break
        batch = order[:chunk]
        tries = max(1, min(4096, chunk // len(batch)))
        agg_of = np.repeat(np.asarray(batch), tries)           # aggregate of each try
        nt = agg_of.shape[0]
        rots = _random_rotations(rng, nt)
        sizes = counts[agg_of]
        starts = np.concatenate([[0], np.cumsum(sizes)])
        near = _round >= near_after and P.shape[0] > 0
        if near:
            # near jamming: put a random member of each try at a surface gap of
            # U[1e-5, 1e-3] from a random placed sphere
            t = rng.integers(P.shape[0], size=nt)
            mem = (rng.uniform(size=nt) * sizes).astype(np.int64)
            u = rng.normal(size=(nt, 3))
            u /= np.linalg.norm(u, axis=1, keepdims=True)
            gap0 = rng.uniform(1e-5, 1e-3, nt)
            mrel = np.stack([rel[a][k] for a, k in zip(agg_of, mem)])
            mrad = np.array([clusters[a][1][k] for a, k in zip(agg_of, mem)])
            centres = (P[t] + (Rr[t] + mrad + gap0)[:, None] * u
                       - np.einsum("kij,kj->ki", rots, mrel))
        elif kind == "box":
            centres = rng.uniform(0.0, L, (nt, 3))
        else:
            v = rng.normal(size=(nt, 3))
            v /= np.linalg.norm(v, axis=1, keepdims=True)
            centres = v * (R * rng.uniform(size=(nt, 1)) ** (1.0 / 3.0))
        owner = np.repeat(np.arange(nt), sizes)                # try of each sphere
        body = np.concatenate([rel[a] for a in agg_of])
        crad = np.concatenate([clusters[a][1] for a in agg_of])
        cpos = np.einsum("kij,kj->ki", rots[owner], body) + centres[owner]
        qpos = np.mod(cpos, L) if kind == "box" else cpos
        bad = np.zeros(nt, dtype=bool)
        if kind == "ball":
            bad |= np.linalg.norm(centres, axis=1) > R
        if P.shape[0]:
            tree = cKDTree(np.mod(P, L) if kind == "box" else P, boxsize=L)
            dist, idx = tree.query(qpos, k=16, distance_upper_bound=reach)
            hit = np.isfinite(dist)
            lim = np.where(hit, crad[:, None] + Rr[np.minimum(idx, len(Rr) - 1)] + MIN_GAP, 0.0)
            clash = (hit & (dist < lim)).any(axis=1)
            bad[np.unique(owner[clash])] = True
        good_sph = ~bad[owner]
        conflicts = {}
        if good_sph.any():
            gidx = np.nonzero(good_sph)[0]
            ctree = cKDTree(qpos[gidx], boxsize=L)
            pairs = ctree.query_pairs(reach, output_type="ndarray")
            if pairs.size:
                a0, a1 = gidx[pairs[:, 0]], gidx[pairs[:, 1]]
                oa, ob = owner[a0], owner[a1]
                d = qpos[a1] - qpos[a0]
                if kind == "box":
                    d -= L * np.round(d / L)
                gap = np.sqrt((d * d).sum(1)) - crad[a0] - crad[a1]
                m = (oa != ob) & (gap < MIN_GAP)
                for x, y in zip(oa[m].tolist(), ob[m].tolist()):
                    conflicts.setdefault(x, []).append(y)
                    conflicts.setdefault(y, []).append(x)
        accepted = np.zeros(nt, dtype=bool)
        done = set()
        for k in np.nonzero(~bad)[0].tolist():
            a = int(agg_of[k])
            if a in done:
                continue
            if any(accepted[o] for o in conflicts.get(k, ())):
                continue
            accepted[k] = True
            done.add(a)
        new_p, new_r = [], []
        for k in np.nonzero(accepted)[0].tolist():
            a = int(agg_of[k])
            pos = cpos[starts[k]:starts[k + 1]]
            if kind == "box":
                pos = pos - centres[k] + np.mod(centres[k], L)
            placed[a] = pos
            new_p.append(pos)
            new_r.append(clusters[a][1])
        if new_p:
            P = np.concatenate([P] + new_p)
            Rr = np.concatenate([Rr] + new_r)
        order = [a for a in batch if a not in done] + order[chunk:]
    if order:
        raise RuntimeError("random sequential addition did not converge; lower the packing")
    pos = np.concatenate([placed[a] for a in range(len(counts))])
    radius = np.concatenate([clusters[a][1] for a in range(len(counts))])
    return pos, radius


# --------------------------------------------------------------------------
# public workloads
# --------------------------------------------------------------------------

def _box_side(counts_total_volume: float, phi: float) -> float:
    return (counts_total_volume / phi) ** (1.0 / 3.0)


def periodic_box(seed: int = 0, n_agg: int = 500, cmin: int = 1, cmax: int = 8,
                 phi: float = 0.2, vel_sigma: float = 0.05, spin_sigma: float = 0.0,
                 dt: float = 1e-4, n_steps: int = 200,
                 contact_seeded: bool = False) -> Workload:
    """Contact-only workload in a periodic cube (no gravity)."""
    rng = np.random.default_rng(seed)
    counts = rng.integers(cmin, cmax + 1, n_agg).astype(np.int32)
    clusters = [random_cluster(rng, int(c)) for c in counts]
    vol = sum(float(sphere_mass(c[1]).sum()) for c in clusters)
    L = _box_side(vol, phi)
    pos, radius = _place(rng, counts, clusters, ("box", L), contact_seeded)
    mass = sphere_mass(radius)
    agg_vel = rng.normal(0.0, vel_sigma, (n_agg, 3))
    agg_spin = rng.normal(0.0, spin_sigma, (n_agg, 3)) if spin_sigma > 0 else np.zeros((n_agg, 3))
    params = dict(CONTACT_PARAMS, dt=dt, G=0.0, soft_frac=0.5, periodic=1,
                  box=(L, L, L))
    return Workload("periodic_box", counts, pos, radius, mass, agg_vel, agg_spin,
                    params, n_steps,
                    notes=f"periodic cube L={L:.4f}, phi={phi}, seed={seed}"
                    + (", contact-seeded" if contact_seeded else ""))


def collapse_radius(sphere_volume: float, phi0: float) -> float:
    """Radius of the ball whose volume is sphere_volume / phi0."""
    return (3.0 * sphere_volume / (4.0 * math.pi * phi0)) ** (1.0 / 3.0)


def collapse_cloud(seed: int = 1, n_agg: int = 25000, cmin: int = 2, cmax: int = 8,
                   phi0: float = 0.15, dt: float = 5e-4, n_steps: int = 2000,
                   G: float = 1.0, soft_frac: float = 0.5,
                   vel_sigma: float = 0.0, spin_sigma: float = 0.0,
                   contact_seeded: bool = False) -> Workload:
    """Self-gravitating cloud of aggregates at rest in a ball.

    The ball radius is sized for an initial packing fraction phi0 (0.15),
    because random non-overlapping placement cannot reach the packing implied
    by 125k spheres inside radius 60.
    """
    rng = np.random.default_rng(seed)
    counts = rng.integers(cmin, cmax + 1, n_agg).astype(np.int32)
    clusters = [random_cluster(rng, int(c)) for c in counts]
    vol = sum(float(sphere_mass(c[1]).sum()) for c in clusters)
    R = collapse_radius(vol, phi0)
    if contact_seeded:
        pos, radius = _place(rng, counts, clusters, ("ball", R), True)
    else:
        pos, radius = _place_rounds(rng, counts, clusters, ("ball", R))
    mass = sphere_mass(radius)
    agg_vel = rng.normal(0.0, vel_sigma, (n_agg, 3)) if vel_sigma > 0 else np.zeros((n_agg, 3))
    agg_spin = rng.normal(0.0, spin_sigma, (n_agg, 3)) if spin_sigma > 0 else np.zeros((n_agg, 3))
    params = dict(CONTACT_PARAMS, dt=dt, G=G, soft_frac=soft_frac, periodic=0,
                  box=(0.0, 0.0, 0.0))
    return Workload("collapse_cloud", counts, pos, radius, mass, agg_vel, agg_spin,
                    params, n_steps,
                    notes=f"ball R={R:.3f}, phi0={phi0}, seed={seed}"
                    + (", contact-seeded" if contact_seeded else ""))


def _one_pile(args):
    k, prng_seed, n_agg, cmin, cmax, phi0, dt, n_steps, G, soft_frac, spin = args
    w = collapse_cloud(seed=prng_seed, n_agg=n_agg, cmin=cmin, cmax=cmax, phi0=phi0, dt=dt,
                       n_steps=n_steps, G=G, soft_frac=soft_frac)
    w.name = f"pile{k}"
    w.params["spin_dw"] = spin / dt      # spin increment per step, rad per time unit
    return w


def pile_batch(seed: int = 3, n_piles: int = 256, nmin: int = 500, nmax: int = 20000,
               cmin: int = 1, cmax: int = 8, phi0: float = 0.15, dt: float = 5e-4,
               n_steps: int = 800, spin_rate_per_step2: float = 1e-6,
               G: float = 1.0, soft_frac: float = 0.5, workers: int = 0,
               executor=None) -> List[Workload]:
    """Independent piles with log-uniform sphere counts in [nmin, nmax].

    Each pile is a cloud of aggregates packed at phi0 about the origin; the
    spin-up forcing (constant spin increment per step) is recorded in the
    params of every pile.  ``workers`` > 1 generates piles in parallel
    processes, or ``executor`` (an existing process pool) does (same result:
    every pile has its own seed).
    """
    rng = np.random.default_rng(seed)
    targets = np.floor(np.exp(rng.uniform(math.log(nmin), math.log(nmax), n_piles))).astype(int)
    jobs = []
    for k, nt in enumerate(targets):
        prng_seed = int(rng.integers(2 ** 31))
        n_agg = max(1, int(round(nt / (0.5 * (cmin + cmax)))))
        jobs.append((k, prng_seed, n_agg, cmin, cmax, phi0, dt, n_steps, G, soft_frac,
                     spin_rate_per_step2))
    if executor is not None:
        return list(executor.map(_one_pile, jobs, chunksize=1))
    if workers and workers > 1:
        from concurrent.futures import ProcessPoolExecutor
        with ProcessPoolExecutor(max_workers=workers) as ex:
            return list(ex.map(_one_pile, jobs, chunksize=1))
    return [_one_pile(j) for j in jobs]


def flyby_orbit(M_pile: float, M_pert: float, periapsis: float, ecc: float = 2.0,
                start_factor: float = 10.0, G: float = 1.0, incline: float = 0.0):
    """Initial position and velocity (relative to the pile's centre of mass)
    of a perturber on an inbound hyperbolic orbit of eccentricity ``ecc`` and
    the given periapsis, starting at ``start_factor`` x periapsis.  Two-body
    relation for the relative orbit, G (M_pile + M_pert)."""
    mu = G * (M_pile + M_pert)
    a = periapsis / (ecc - 1.0)                 # |semi-major axis| of the hyperbola
    p = a * (ecc * ecc - 1.0)                   # semi-latus rectum
    r = start_factor * periapsis
    nu = -math.acos((p / r - 1.0) / ecc)        # inbound branch
    h = math.sqrt(mu * p)
    pos = np.array([r * math.cos(nu), r * math.sin(nu), 0.0])
    vel = (mu / h) * np.array([-math.sin(nu), ecc + math.cos(nu), 0.0])
    if incline:
        c, s_ = math.cos(incline), math.sin(incline)
        rot = np.array([[1, 0, 0], [0, c, -s_], [0, s_, c]])
        pos, vel = rot @ pos, rot @ vel
    return pos, vel


def _spread3(v: np.ndarray) -> np.ndarray:
    """Bits of v (< 2^10) moved to every third position."""
    v = v.astype(np.uint64) & np.uint64(0x3FF)
    out = np.zeros_like(v)
    for b in range(10):
        out |= ((v >> np.uint64(b)) & np.uint64(1)) << np.uint64(3 * b)
    return out


def dense_lattice(seed: int = 6, n_side: int = 50, spacing: float = 1.999,
                  jitter: float = 2e-4, dt: float = 1e-4, vel_sigma: float = 0.01,
                  n_steps: int = 100, order: str = "slices") -> Workload:
    """Contact-dense periodic workload: unit spheres on a jittered cubic
    lattice whose spacing is slightly below a diameter, so every sphere
    overlaps its six neighbours; lattice neighbours along x are bonded in
    pairs (dumbbells), the rest are lone spheres.  Used to measure the
    contact path, where memory traffic rather than arithmetic dominates.

    ``order`` numbers the aggregates: "slices" pairs x-slice a with a + 1
    and goes through them slice pair by slice pair (a sphere's x-neighbours
    are then n_side^2 ids away); "morton" lists the same aggregates in
    Morton order of their lattice cells, as a spatially sorted input would
    be."""
    rng = np.random.default_rng(seed)
    g = np.arange(n_side) * spacing
    p = np.stack(np.meshgrid(g, g, g, indexing="ij"), -1).reshape(-1, 3)
    p = p + rng.uniform(-jitter, jitter, p.shape) + 0.5 * spacing
    ix = np.arange(n_side)
    # pair (x even, x odd) into dumbbells when n_side is even; lone otherwise
    order_kind = order
    counts, order = [], []
    idx = np.arange(p.shape[0]).reshape(n_side, n_side, n_side)
    for a in range(0, n_side - 1, 2):
        pairs = np.stack([idx[a].ravel(), idx[a + 1].ravel()], 1)
        order.append(pairs.ravel())
        counts += [2] * pairs.shape[0]
    if n_side % 2:
        order.append(idx[n_side - 1].ravel())
        counts += [1] * (n_side * n_side)
    counts = np.asarray(counts, dtype=np.int32)
    if order_kind == "morton":
        first = np.concatenate([[0], np.cumsum(counts)[:-1]])
        flat = np.concatenate(order)
        c = np.stack(np.unravel_index(flat[first], (n_side, n_side, n_side)), 1)
        key = _spread3(c[:, 0]) | (_spread3(c[:, 1]) << np.uint64(1)) | (_spread3(c[:, 2]) << np.uint64(2))
        agg_order = np.argsort(key, kind="stable")
        order = [flat[first[a]:first[a] + counts[a]] for a in agg_order]
        counts = counts[agg_order]
    elif order_kind != "slices":
        raise ValueError(f"unknown order {order_kind!r}")
    order = np.concatenate(order)
    pos = p[order]
    radius = np.ones(pos.shape[0])
    n_agg = len(counts)
    L = n_side * spacing
    params = dict(CONTACT_PARAMS, dt=dt, G=0.0, soft_frac=0.5, periodic=1, box=(L, L, L))
    return Workload("dense_lattice", counts, pos, radius,
                    sphere_mass(radius), rng.normal(0.0, vel_sigma, (n_agg, 3)),
                    np.zeros((n_agg, 3)), params, n_steps,
                    notes=f"periodic lattice {n_side}^3 spacing {spacing}, seed {seed}, "
                          f"{order_kind} order")


def subset(w: Workload, n_agg: int) -> Workload:
    """First ``n_agg`` aggregates of a workload (for reduced-size checks)."""
    off = w.offsets()
    ns = int(off[n_agg])
    return Workload(w.name + f"[:{n_agg}]", w.counts[:n_agg].copy(), w.pos[:ns].copy(),
                    w.radius[:ns].copy(), w.mass[:ns].copy(), w.agg_vel[:n_agg].copy(),
                    w.agg_spin[:n_agg].copy(), dict(w.params), w.n_steps, notes=w.notes)


# --------------------------------------------------------------------------
# symmetric shape fixtures (Fig. 1 of the paper), equal spheres of radius s
# --------------------------------------------------------------------------

def shape_fixture(name: str, s: float = 1.0) -> np.ndarray:
    """Sphere centres (relative to the centroid) of the paper's symmetric
    aggregate shapes built from touching equal spheres of radius ``s``."""
    if name == "sphere":
        p = np.zeros((1, 3))
    elif name == "dumbbell":
        p = np.array([[-s, 0, 0], [s, 0, 0]], dtype=float)
    elif name == "rod":
        p = np.array([[-3 * s, 0, 0], [-s, 0, 0], [s, 0, 0], [3 * s, 0, 0]], dtype=float)
    elif name == "cube":
        p = np.array([[x, y, z] for x in (-s, s) for y in (-s, s) for z in (-s, s)], dtype=float)
    elif name == "tetrahedron":
        a = 2 * s / math.sqrt(8.0)
        p = np.array([[a, a, a], [a, -a, -a], [-a, a, -a], [-a, -a, a]], dtype=float)
    elif name == "diamond":
        h = math.sqrt(3.0) * s
        p = np.array([[-s, 0, 0], [s, 0, 0], [0, h, 0], [0, -h, 0]], dtype=float)
    else:
        raise KeyError(name)
    return p - p.mean(axis=0)


SHAPES = ("sphere", "dumbbell", "diamond", "tetrahedron", "rod", "cube")


def fixture_system(shapes, centres, s=1.0, vel=None, spin=None, rot=None,
                   params=None, dt=1e-4, n_steps=1, density=1.0) -> Workload:
    """Build a workload from shape fixtures placed at ``centres``."""
    pos, counts = [], []
    for k, (nm, c) in enumerate(zip(shapes, centres)):
        p = shape_fixture(nm, s)
        if rot is not None and rot[k] is not None:
            p = p @ np.asarray(rot[k]).T
        pos.append(p + np.asarray(c, dtype=float))
        counts.append(p.shape[0])
    pos = np.concatenate(pos)
    radius = np.full(pos.shape[0], float(s))
    mass = sphere_mass(radius, density)
    n = len(counts)
    vel = np.zeros((n, 3)) if vel is None else np.asarray(vel, dtype=float).reshape(n, 3)
    spin = np.zeros((n, 3)) if spin is None else np.asarray(spin, dtype=float).reshape(n, 3)
    prm = dict(CONTACT_PARAMS, dt=dt, G=0.0, soft_frac=0.5, periodic=0, box=(0.0, 0.0, 0.0))
    if params:
        prm.update(params)
    return Workload("fixture", np.asarray(counts, dtype=np.int32), pos, radius, mass,
                    vel, spin, prm, n_steps)


# --------------------------------------------------------------------------
# walled workloads: box filling (Sec. 3.3) and the Brazil-nut effect (Sec. 4.3)
# --------------------------------------------------------------------------

MIXED_SHAPES = ("dumbbell", "diamond", "tetrahedron", "rod", "cube")


def open_box_walls(Lx: float, Ly: float):
    """Floor z = 0 and four side walls of the box [0, Lx] x [0, Ly]; open top.
    Each wall is (n_x, n_y, n_z, d) with the unit normal pointing inward."""
    return [(0.0, 0.0, 1.0, 0.0), (1.0, 0.0, 0.0, 0.0), (-1.0, 0.0, 0.0, -float(Lx)),
            (0.0, 1.0, 0.0, 0.0), (0.0, -1.0, 0.0, -float(Ly))]


def _shape_mix(rng, n_sph: int, shape: str):
    """Shape names whose member counts add up to n_sph: one shape, or a
    uniform mix of the symmetric shapes of 2-8 spheres (no free spheres)."""
    if shape != "mixed":
        k = shape_fixture(shape).shape[0]
        if n_sph % k:
            raise ValueError(f"{n_sph} spheres do not divide into {shape}s")
        return [shape] * (n_sph // k)
    sizes = {s: shape_fixture(s).shape[0] for s in MIXED_SHAPES}
    if n_sph % 2:
        raise ValueError("a mix of even-sized shapes needs an even sphere count")
    out, left = [], n_sph
    while left > 0:
        fit = [s for s in MIXED_SHAPES if sizes[s] <= left]
        s = fit[int(rng.integers(len(fit)))]
        out.append(s)
        left -= sizes[s]
    return out


def box_fill(seed: int = 8, n_sph: int = 6400, shape: str = "mixed", base: float = 40.0,
             height: float = 240.0, g: float = 2.0, dt: float = 5e-4, z_range=None,
             floor_seeded: float = 0.0, contact_seeded: bool = False,
             n_steps: int = 10000) -> Workload:
    """Box filling under a uniform field (the uniform-gravity profiling runs).

    Equal spheres of radius 1 (0.25 cm in the paper) bound into the paper's
    symmetric shapes -- one shape, or "mixed": shapes of 2-8 members and no
    free spheres -- with ``n_sph`` member spheres in all, placed at rest at
    random positions and orientations in the open-topped box of base
    ``base`` x ``base`` and height ``height`` radii (10 x 10 x 60 cm), under
    a field of magnitude g along -z.  Length unit: the sphere radius; time
    unit: the one that makes lunar gravity equal ``g`` (0.056 s for g = 2).
    ``z_range`` limits the centres' heights (a partly filled box);
    ``floor_seeded`` is the fraction of aggregates set down on the floor with
    an overlap (for single-step checks of wall contacts).
    """
    rng = np.random.default_rng(seed)
    names = _shape_mix(rng, n_sph, shape)
    clusters = []
    for nm in names:
        rel = shape_fixture(nm)
        clusters.append((rel, np.ones(rel.shape[0])))
    counts = np.array([c[0].shape[0] for c in clusters], dtype=np.int32)
    z_lo, z_hi = z_range if z_range is not None else (0.0, height)
    pos, radius = _place(rng, counts, clusters,
                         ("cuboid", (base, base, height, z_lo, z_hi, floor_seeded)),
                         contact_seeded)
    mass = sphere_mass(radius)
    n_agg = counts.shape[0]
    params = dict(CONTACT_PARAMS, dt=dt, G=0.0, soft_frac=0.5, periodic=0,
                  box=(0.0, 0.0, 0.0), g=(0.0, 0.0, -float(g)),
                  walls=open_box_walls(base, base))
    return Workload("box_fill", counts, pos, radius, mass, np.zeros((n_agg, 3)),
                    np.zeros((n_agg, 3)), params, n_steps,
                    notes=f"{shape} shapes, {n_sph} spheres, box {base}x{base}x{height}, "
                    f"g={g}, seed={seed}")


def brazil_nut(seed: int = 9, n_sph: int = 4000, shape: str = "mixed",
               intruder_radius: float = 6.0, base: float = 40.0, fill_height: float = 60.0,
               g: float = 2.0, amplitude: float = 4.0, froude: float = 3.0,
               dt: float = 5e-4, floor_seeded: float = 0.0, n_steps: int = 1000) -> Workload:
    """Brazil-nut set-up: a large spherical intruder resting on the floor of
    a box of base ``base`` x ``base`` (10 x 10 cm at 0.25 cm grains), grains
    of radius 1 bound into the symmetric shapes placed at rest around and
    above it up to ``fill_height``, under a field g along -z.  Every wall
    oscillates vertically with amplitude A = ``amplitude`` (1 cm) and omega
    from the Froude number A omega^2 / g (3 in the paper, 54.2 rad/s at Earth
    gravity), starting from rest at the lowest point: displacement
    A (1 + sin(omega t - pi/2)), so the floor starts at z = 0.  The intruder
    is aggregate 0.  ``floor_seeded`` is the fraction of grains set down on
    the floor with an overlap of U[1e-5, 1e-3] (for short checks).
    """
    rng = np.random.default_rng(seed)
    names = _shape_mix(rng, n_sph, shape)
    clusters = [(shape_fixture(nm), np.ones(shape_fixture(nm).shape[0])) for nm in names]
    counts = np.array([c[0].shape[0] for c in clusters], dtype=np.int32)
    R = float(intruder_radius)
    x0 = np.array([0.5 * base, 0.5 * base, R + 1e-3])
    # grains by RSA in the fill region, clear of the intruder
    pos, radius = _place_around(rng, counts, clusters, base, fill_height, x0, R, floor_seeded)
    pos = np.concatenate([x0[None, :], pos])
    radius = np.concatenate([[R], radius])
    counts = np.concatenate([[1], counts]).astype(np.int32)
    mass = sphere_mass(radius)
    omega = math.sqrt(froude * g / amplitude)
    walls = open_box_walls(base, base)
    walls[0] = (0.0, 0.0, 1.0, float(amplitude))      # floor at z = 0 at t = 0
    params = dict(CONTACT_PARAMS, dt=dt, G=0.0, soft_frac=0.5, periodic=0,
                  box=(0.0, 0.0, 0.0), g=(0.0, 0.0, -float(g)), walls=walls,
                  shake_amp=[(0.0, 0.0, float(amplitude))] * len(walls),
                  shake_omega=omega, shake_phase=-0.5 * math.pi)
    n_agg = counts.shape[0]
    return Workload("brazil_nut", counts, pos, radius, mass, np.zeros((n_agg, 3)),
                    np.zeros((n_agg, 3)), params, n_steps,
                    notes=f"{shape} grains, {n_sph} spheres, intruder R={R}, "
                    f"omega={omega:.4f}, seed={seed}")


def _place_around(rng, counts, clusters, base, height, x0, R, p_floor=0.0, max_tries=20000):
    """RSA of aggregates in [0, base]^2 x [0, height], every sphere at least
    MIN_GAP clear of the walls and of a fixed sphere (x0, R); with
    probability p_floor an aggregate is lowered onto the floor so that its
    lowest sphere overlaps it by U[1e-5, 1e-3]."""
    order = np.argsort(-counts, kind="stable")
    grid = _Grid(np.full(3, -3.0), np.array([base, base, height]) + 3.0, 2.4)
    placed = [None] * len(counts)
    for a in order:
        rel, rad = clusters[a]
        rel = rel - rel.mean(axis=0)
        for _ in range(max_tries):
            body = rel @ _random_rotation(rng).T
            c = np.array([rng.uniform(0, base), rng.uniform(0, base), rng.uniform(0, height)])
            if p_floor > 0 and rng.uniform() < p_floor:
                c[2] -= (body[:, 2] - rad + c[2]).min() + rng.uniform(1e-5, 1e-3)
            p = c + body
            lo = p - rad[:, None]
            hi = p + rad[:, None]
            lz = lo[:, 2]
            if ((lo[:, :2] < MIN_GAP).any() or (hi[:, :2] > base - MIN_GAP).any()
                    or (hi[:, 2] > height).any() or ((lz >= -MIN_GAP) & (lz < MIN_GAP)).any()
                    or (lz < -1.001e-3).any()):
                continue
            if (np.linalg.norm(p - x0, axis=1) - (R + rad) < MIN_GAP).any():
                continue
            gap, _ = grid.gaps(p, rad)
            if gap.size and (gap < MIN_GAP).any():
                continue
            grid.insert(p, rad)
            placed[a] = p
            break
        else:
            raise RuntimeError("placement failed; raise fill_height")
    pos = np.concatenate([placed[a] for a in range(len(counts))])
    radius = np.concatenate([clusters[a][1] for a in range(len(counts))])
    return pos, radius


def boulders(seed: int = 13, n_agg: int = 600, n_big: int = 6, big_radius: float = 4.0,
             phi: float = 0.2, dt: float = 1e-4, vel_sigma: float = 0.05,
             contact_seeded: bool = True, n_steps: int = 100) -> Workload:
    """Polydisperse periodic cube: ``n_big`` single-sphere boulders of radius
    ``big_radius`` among aggregates of 1-8 spheres of radius U[0.8, 1.2].
    Boulders are placed first (with ``contact_seeded`` every other one
    touches the previous one, overlap U[1e-5, 1e-3]); then the aggregates by
    random sequential addition, every other one of the first 10 per boulder
    (if seeded) set against a random boulder with the same kind of overlap.  The boulders come first in
    the sphere order."""
    rng = np.random.default_rng(seed)
    counts = rng.integers(1, 9, n_agg).astype(np.int32)
    clusters = [random_cluster(rng, int(c)) for c in counts]
    vol = sum(float(sphere_mass(c[1]).sum()) for c in clusters) + n_big * sphere_mass(
        np.array([big_radius]))[0]
    L = _box_side(vol, phi)

    def mi(d):
        return d - L * np.round(d / L)

    bpos = []
    while len(bpos) < n_big:
        if contact_seeded and len(bpos) % 2 == 1:
            u = _unit_vectors(rng, 1)[0]
            c = np.mod(bpos[-1] + (2 * big_radius - rng.uniform(1e-5, 1e-3)) * u, L)
            skip = len(bpos) - 1
        else:
            c = rng.uniform(0, L, 3)
            skip = -1
        ok = all(np.linalg.norm(mi(c - b)) - 2 * big_radius >= MIN_GAP
                 for k, b in enumerate(bpos) if k != skip)
        if ok:
            bpos.append(c)
    bpos = np.array(bpos)
    grid = _Grid(np.zeros(3), None, 2.4, periodic=True, box=np.full(3, L))
    placed = [None] * n_agg
    order = np.argsort(-counts, kind="stable")
    for n_done, a in enumerate(order):
        rel, rad = clusters[a]
        rel = rel - rel.mean(axis=0)
        for _ in range(20000):
            body = rel @ _random_rotation(rng).T
            seeded = contact_seeded and n_done < 10 * n_big and n_done % 2 == 0
            if seeded:
                t = int(rng.integers(n_big))
                m = int(rng.integers(body.shape[0]))
                u = _unit_vectors(rng, 1)[0]
                centre = bpos[t] + (big_radius + rad[m] - rng.uniform(1e-5, 1e-3)) * u - body[m]
            else:
                t = -1
                centre = rng.uniform(0, L, 3)
            centre = np.mod(centre, L)
            p = centre + body
            gb = np.linalg.norm(mi(p[:, None, :] - bpos[None, :, :]), axis=2) \
                - (rad[:, None] + big_radius)
            if t >= 0:
                gb[m, t] = max(gb[m, t], MIN_GAP) if gb[m, t] < 0 else -1.0
            if (gb < MIN_GAP).any():
                continue
            gap, _ = grid.gaps(p, rad)
            if gap.size and (gap < MIN_GAP).any():
                continue
            grid.insert(p, rad)
            placed[a] = p
            break
        else:
            raise RuntimeError("boulder placement failed; lower the packing")
    pos = np.concatenate([bpos] + [placed[a] for a in range(n_agg)])
    radius = np.concatenate([np.full(n_big, big_radius)] + [clusters[a][1] for a in range(n_agg)])
    counts = np.concatenate([np.ones(n_big, dtype=np.int32), counts]).astype(np.int32)
    mass = sphere_mass(radius)
    na = counts.shape[0]
    params = dict(CONTACT_PARAMS, dt=dt, G=0.0, soft_frac=0.5, periodic=1, box=(L, L, L))
    return Workload("boulders", counts, pos, radius, mass, rng.normal(0.0, vel_sigma, (na, 3)),
                    np.zeros((na, 3)), params, n_steps,
                    notes=f"{n_big} boulders R={big_radius}, periodic L={L:.3f}, seed={seed}")
