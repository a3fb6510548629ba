// step_contact.h -- per-element device functions of the contact search:
// cell binning (counting sort of Morton codes, rank by id inside a cell),
// and the search that skips pairs inside one aggregate (the 27 neighbouring
// cells of a sphere split among a group of lanes; big spheres searched
// apart).  Included by the staged kernels and by the fused per-pile step.
//
// Paper references: contacts between spheres of different aggregates only
// (Sec. 2.2); the contact model acts on spheres in contact (Sec. 2.1).
#pragma once
#include "dem_internal.h"

namespace dem {

namespace {

// Morton code of a sphere's cell on the pile's current grid.
__device__ __forceinline__ void sphere_cell(const PileDev& P, const Grid& g, double x, double y,
                                            double z, int c[3]) {
  c[0] = cell_coord(x, g.lo[0], g.inv_cell, g.nc[0], P.periodic, P.box);
  c[1] = cell_coord(y, g.lo[1], g.inv_cell, g.nc[1], P.periodic, P.box);
  c[2] = cell_coord(z, g.lo[2], g.inv_cell, g.nc[2], P.periodic, P.box);
}

// Cell key of sphere i and its count (integer atomics on the cell table).
__device__ __forceinline__ void bin_one(const PileDev& P, int i) {
  const Grid g = *P.grid;
  const int ns = P.ns;
  uint32_t key;
  if (P.n_big > 0 && P.s[i] > P.s_cut) {
    key = 1u << (3 * P.bits);               // the cell after the Morton cells
  } else {
    int c[3];
    sphere_cell(P, g, P.r[i], P.r[ns + i], P.r[2 * ns + i], c);
    key = cell_key(c[0], c[1], c[2], g.nbits);
  }
  P.key[i] = key;
  atomicAdd(&P.cell_cnt[key], 1u);
}

// Place sphere i into its cell's range (in atomic arrival order); the
// counts return to zero, ready for the next step.
__device__ __forceinline__ void scatter_one(const PileDev& P, int i) {
  const uint32_t key = P.key[i];
  const uint32_t k = atomicSub(&P.cell_cnt[key], 1u) - 1u;
  P.sidx_raw[P.cell_start[key] + k] = (uint32_t)i;
}

// Order one cell's spheres by id, independent of atomic arrival order: the
// sphere at raw slot k goes to its cell's start plus its rank (the number of
// smaller ids in the cell).  The same thread writes the sphere's sorted
// copies there -- packed records for the search and, in a pile with
// gravity, positions and radius for it -- and the inverse permutation.
__device__ __forceinline__ void cell_sort_one(const PileDev& P, int k) {
  const int ns = P.ns;
  const uint32_t* __restrict__ raw = P.sidx_raw;
  const uint32_t i = raw[k];
  const uint32_t key = P.key[i];
  const uint32_t s0 = P.cell_start[key], s1 = P.cell_start[key + 1];
  uint32_t r = 0;
  for (uint32_t t = s0; t < s1; ++t) r += raw[t] < i;
  const uint32_t d = s0 + r;
  P.sidx[d] = i;
  P.slot[i] = d;
  const double x = P.r[i], y = P.r[ns + i], z = P.r[2 * ns + i], s = P.s[i];
  if (P.G != 0.0) {                          // only gravity reads these copies
    P.xs[d] = x;
    P.xs[ns + d] = y;
    P.xs[2 * ns + d] = z;
    P.xs[3 * ns + d] = s;
  }
  P.xg[d] = SortedGeom{x, y, z, s};
  P.sid[d] = SortedId{P.agg[i], i};
}

// Contact test exactly as written d^2 = (dx*dx + dy*dy) + dz*dz < S*S, each
// product and sum rounded separately (no fused multiply-add), with the
// minimum-image correction per axis in a periodic cube.
__device__ __forceinline__ bool touching(double dx, double dy, double dz, double S, int periodic,
                                         double L) {
  if (periodic) {
    const double hL = 0.5 * L;
    if (dx > hL) dx -= L;
    else if (dx < -hL) dx += L;
    if (dy > hL) dy -= L;
    else if (dy < -hL) dy += L;
    if (dz > hL) dz -= L;
    else if (dz < -hL) dz += L;
  }
  const double d2 = rn_add(rn_add(rn_mul(dx, dx), rn_mul(dy, dy)), rn_mul(dz, dz));
  return d2 < rn_mul(S, S);
}

// Insertion sort of a short run of ids in global memory.
__device__ __forceinline__ void sort_run(uint32_t* __restrict__ a, uint32_t n) {
  for (uint32_t x = 1; x < n; ++x) {
    const uint32_t v = a[x];
    uint32_t y = x;
    while (y > 0 && a[y - 1] > v) {
      a[y] = a[y - 1];
      --y;
    }
    a[y] = v;
  }
}

// The search gives each sphere a group of L lanes of one wave; the lanes
// split the 27 neighbouring cells (and the walls) between them, so a
// sphere's dependent cell-range and candidate loads run L-wide.  Eight lanes
// keep the dependent chains short where few spheres cannot fill the chip;
// four lanes issue fewer instructions per sphere (the per-lane work of a
// sphere is shared by fewer lanes) where many can.
template <int L>
struct SearchLanes {
  static constexpr int kGroups = kBlock / L;   // spheres per block
  // neighbour cells per lane (d = lane, lane + L, ... < 27), and the lane
  // whose last slot is free for the big spheres' cell
  static constexpr int kSlots = (27 + L - 1) / L;
  static constexpr int kBigLane = 27 - (kSlots - 1) * L;
  static_assert(kBigLane > 0 && kBigLane < L, "one lane needs a free last slot");
};
constexpr int kLanesSmall = 8;            // launches of few spheres
constexpr int kLanesLarge = 4;            // launches of many
// Runs of up to this many contacts per sphere are gathered in LDS and
// rank-sorted into a per-slot cache by the find pass; longer runs are found
// again by the write pass, written in arrival order and sorted in place by
// the group's first lane.
constexpr int kRunLds = kRunCache;

// The search of the sphere at sorted slot k by its group of L lanes
// (lane = this lane's index in the group; the group's LDS: buf_up, buf_lo of
// kRunLds entries and fill[2]).  Every lane tests the spheres of its share
// of the 27 neighbouring cells that belong to another aggregate, and its
// share of the walls.
//
// Find mode stores the number of contacts with j > i (upper) and j < i
// (lower) under sphere id i and, when both runs fit kRunLds entries, the
// runs themselves sorted by id in the slot's cache.  Write mode (after the
// scan) checks the pile's contact capacity and copies each cached run to its
// offsets; a sphere whose runs did not fit is searched again and its runs
// written in arrival order, then sorted in place.
template <int Lanes>
__device__ __forceinline__ void search_slot(PileDev& P, int k, int lane, int write,
                                            uint32_t* buf_up, uint32_t* buf_lo, uint32_t* fill) {
  constexpr int kLanes = Lanes;
  constexpr int kSlots = SearchLanes<Lanes>::kSlots;
  constexpr int kBigLane = SearchLanes<Lanes>::kBigLane;
  const int ns = P.ns, nxt = P.parity ^ 1;
  const SortedGeom* __restrict__ xg = P.xg;
  const SortedId* __restrict__ sid = P.sid;
  const SortedId me = sid[k];
  const uint32_t i = me.id;
  if (P.n_big > 0 && k >= ns - P.n_big) return;   // big spheres: k_search_big
  uint32_t* cache_up = P.run_cache + (size_t)k * kRunLds;
  uint32_t* cache_lo = P.run_cache + ((size_t)ns + k) * kRunLds;

  uint32_t* up_out = nullptr;
  uint32_t* lo_out = nullptr;
  uint32_t run_up = 0, run_lo = 0;
  if (write) {
    const uint32_t tot_up = P.up_off[nxt][ns], tot_lo = P.lo_off[ns];
    if (tot_up > (uint32_t)P.cap_pairs || tot_lo > (uint32_t)P.cap_pairs) {
      if (lane == 0) atomicOr(&P.status, kStCapacity);
      return;
    }
    const uint32_t u0 = P.up_off[nxt][i], l0 = P.lo_off[i];
    up_out = P.pair_j[nxt] + u0;
    lo_out = P.lo_nbr + l0;
    run_up = P.up_off[nxt][i + 1] - u0;
    run_lo = P.lo_off[i + 1] - l0;
    if (run_up <= (uint32_t)kRunLds && run_lo <= (uint32_t)kRunLds) {
      // the find pass kept both runs, sorted
      for (uint32_t e = lane; e < run_up; e += kLanes) up_out[e] = cache_up[e];
      for (uint32_t e = lane; e < run_lo; e += kLanes) lo_out[e] = cache_lo[e];
      return;
    }
  }
  if (lane == 0) {
    fill[0] = 0u;
    fill[1] = 0u;
  }
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();

  const Grid g = *P.grid;
  const uint32_t* __restrict__ cstart = P.cell_start;
  const SortedGeom mg = xg[k];
  const double x = mg.x, y = mg.y, z = mg.z, si = mg.s;
  const int ai = me.agg;
  const int periodic = P.periodic;
  const double L = P.box;
  int c[3];
  sphere_cell(P, g, x, y, z, c);
  const int n = g.nc[0];                  // periodic piles: the same on every axis
  // neighbouring cells along an axis: c-1..c+1, or every cell when a
  // periodic axis has fewer than three (so no cell is visited twice)
  const bool all = periodic && n < 3;
  // this lane's cells: d = lane, lane + kLanes, ... (d < 27)
  uint32_t rs[kSlots], re[kSlots];
#pragma unroll
  for (int q = 0; q < kSlots; ++q) {
    const int d = lane + q * kLanes;
    const int ox = d % 3, oy = (d / 3) % 3, oz = d / 9;
    int cx, cy, cz;
    bool ok;
    if (all) {
      cx = ox;
      cy = oy;
      cz = oz;
      ok = cx < n && cy < n && cz < n;
    } else {
      cx = c[0] + ox - 1;
      cy = c[1] + oy - 1;
      cz = c[2] + oz - 1;
      if (periodic) {
        cx += cx < 0 ? n : (cx >= n ? -n : 0);
        cy += cy < 0 ? n : (cy >= n ? -n : 0);
        cz += cz < 0 ? n : (cz >= n ? -n : 0);
        ok = true;
      } else {
        ok = cx >= 0 && cx < g.nc[0] && cy >= 0 && cy < g.nc[1] && cz >= 0 && cz < g.nc[2];
      }
    }
    ok = ok && d < 27;
    const uint32_t key = ok ? cell_key(cx, cy, cz, g.nbits) : 0u;
    rs[q] = ok ? cstart[key] : 0u;
    re[q] = ok ? cstart[key + 1] : 0u;
  }
  if (lane == kBigLane && P.n_big > 0) {    // a free slot: the big spheres' cell
    const uint32_t bk = 1u << (3 * P.bits);
    rs[kSlots - 1] = cstart[bk];
    re[kSlots - 1] = cstart[bk + 1];
  }
  // find mode keeps the first kRunLds ids of each run in LDS; write mode
  // (runs too long for the cache) writes them straight to the runs
  auto emit = [&](uint32_t j) {
    const bool up = j > i;
    const uint32_t pos = atomicAdd(&fill[up ? 0 : 1], 1u);
    if (write) (up ? up_out : lo_out)[pos] = j;
    else if (pos < (uint32_t)kRunLds) (up ? buf_up : buf_lo)[pos] = j;
  };
#pragma unroll
  for (int q = 0; q < kSlots; ++q) {
    for (uint32_t t = rs[q]; t < re[q]; ++t) {
      const SortedId o = sid[t];
      if (o.agg == ai) continue;          // same aggregate (includes t == k)
      const SortedGeom cg = xg[t];
      if (!touching(cg.x - x, cg.y - y, cg.z - z, si + cg.s, periodic, L)) continue;
      emit(o.id);
    }
  }
  // walls are partners ns + w, after every sphere partner
  for (int wi_ = lane; wi_ < P.n_walls; wi_ += kLanes)
    if (wall_gap(P, wi_, P.grid->wall_d[wi_], x, y, z) < si) emit((uint32_t)(ns + wi_));

  __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
  __builtin_amdgcn_wave_barrier();
  if (write) {
    __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "agent");
    if (lane == 0) {
      sort_run(up_out, run_up);
      sort_run(lo_out, run_lo);
    }
    return;
  }
  const uint32_t nup = fill[0], nlo = fill[1];
  if (lane == 0) {
    P.cnt_up[i] = nup;
    P.cnt_lo[i] = nlo;
  }
  if (nup > (uint32_t)kRunLds || nlo > (uint32_t)kRunLds) return;
  // rank sort into the cache: ids in a run are distinct, so each entry's
  // rank is the number of smaller entries
  for (uint32_t e = lane; e < nup; e += kLanes) {
    const uint32_t v = buf_up[e];
    uint32_t r = 0;
    for (uint32_t f = 0; f < nup; ++f) r += buf_up[f] < v;
    cache_up[r] = v;
  }
  for (uint32_t e = lane; e < nlo; e += kLanes) {
    const uint32_t v = buf_lo[e];
    uint32_t r = 0;
    for (uint32_t f = 0; f < nlo; ++f) r += buf_lo[f] < v;
    cache_lo[r] = v;
  }
}

// The kb-th big sphere of the pile (at slot ns - n_big + kb), searched by
// nthreads threads of one block (tid the thread's index; LDS buf_up, buf_lo
// of kBigRun entries and fill[2]; every thread of the block calls this):
// they split the cells within reach of any other sphere and the big
// spheres' cell.  Find mode stores the run lengths; write mode gathers both
// runs in LDS, rank-sorts them and stores them at the scanned offsets.  A run
// longer than kBigRun is a capacity failure.
__device__ __forceinline__ void search_big_one(PileDev& P, int kb, int write, int tid,
                                               int nthreads, uint32_t* buf_up, uint32_t* buf_lo,
                                               uint32_t* fill) {
  // one read of the status for the whole block (another block of this pile
  // may set it meanwhile), so that every thread takes the same path
  if (tid == 0) fill[0] = P.status != 0 ? 1u : 0u;
  __syncthreads();
  const bool failed = fill[0] != 0u;
  __syncthreads();
  if (failed) return;
  const int ns = P.ns, nxt = P.parity ^ 1;
  const int k = ns - P.n_big + kb;
  const SortedId me = P.sid[k];
  const SortedGeom mg = P.xg[k];
  const uint32_t i = me.id;
  const double x = mg.x, y = mg.y, z = mg.z, si = mg.s;
  const int ai = me.agg;
  uint32_t run_up = 0, run_lo = 0;
  if (write) {
    const uint32_t tot_up = P.up_off[nxt][ns], tot_lo = P.lo_off[ns];
    run_up = P.up_off[nxt][i + 1] - P.up_off[nxt][i];
    run_lo = P.lo_off[i + 1] - P.lo_off[i];
    if (tot_up > (uint32_t)P.cap_pairs || tot_lo > (uint32_t)P.cap_pairs ||
        run_up > (uint32_t)kBigRun || run_lo > (uint32_t)kBigRun) {
      if (tid == 0) atomicOr(&P.status, kStCapacity);
      return;
    }
  }
  if (tid == 0) {
    fill[0] = 0u;
    fill[1] = 0u;
  }
  __syncthreads();
  const SortedGeom* __restrict__ xg = P.xg;
  const SortedId* __restrict__ sid = P.sid;
  const uint32_t* __restrict__ cstart = P.cell_start;
  const int periodic = P.periodic;
  const double L = P.box;
  const Grid& g = *P.grid;
  int c[3];
  sphere_cell(P, g, x, y, z, c);
  // reach in cells of any partner: (s_i + s_small) / cell, plus one for rounding
  const int R = (int)ceil((si + P.s_small) * g.inv_cell) + 1;
  int start[3], cnt[3];
  for (int a = 0; a < 3; ++a) {
    const int n = g.nc[a];
    if (periodic) {
      if (2 * R + 1 >= n) {
        start[a] = 0;
        cnt[a] = n;
      } else {
        start[a] = c[a] - R;
        cnt[a] = 2 * R + 1;
      }
    } else {
      const int lo = c[a] - R < 0 ? 0 : c[a] - R;
      const int hi = c[a] + R > n - 1 ? n - 1 : c[a] + R;
      start[a] = lo;
      cnt[a] = hi - lo + 1;
    }
  }
  auto test = [&](uint32_t t) {
    const SortedId o = sid[t];
    if (o.agg == ai) return;
    const SortedGeom cg = xg[t];
    if (!touching(cg.x - x, cg.y - y, cg.z - z, si + cg.s, periodic, L)) return;
    const bool up = o.id > i;
    const uint32_t pos = atomicAdd(&fill[up ? 0 : 1], 1u);
    if (write) (up ? buf_up : buf_lo)[pos] = o.id;
  };
  const int total = cnt[0] * cnt[1] * cnt[2];
  for (int u = tid; u < total; u += nthreads) {
    int cx = start[0] + u % cnt[0];
    int cy = start[1] + (u / cnt[0]) % cnt[1];
    int cz = start[2] + u / (cnt[0] * cnt[1]);
    if (periodic) {
      const int n = g.nc[0];
      cx += cx < 0 ? n : (cx >= n ? -n : 0);
      cy += cy < 0 ? n : (cy >= n ? -n : 0);
      cz += cz < 0 ? n : (cz >= n ? -n : 0);
    }
    const uint32_t key = cell_key(cx, cy, cz, g.nbits);
    for (uint32_t t = cstart[key], t1 = cstart[key + 1]; t < t1; ++t) test(t);
  }
  const uint32_t bk = 1u << (3 * P.bits);
  for (uint32_t t = cstart[bk] + tid; t < cstart[bk + 1]; t += nthreads) test(t);
  for (int wi_ = tid; wi_ < P.n_walls; wi_ += nthreads) {
    if (wall_gap(P, wi_, g.wall_d[wi_], x, y, z) < si) {
      const uint32_t pos = atomicAdd(&fill[0], 1u);
      if (write) buf_up[pos] = (uint32_t)(ns + wi_);
    }
  }
  __syncthreads();
  if (!write) {
    if (tid == 0) {
      P.cnt_up[i] = fill[0];
      P.cnt_lo[i] = fill[1];
    }
    return;
  }
  uint32_t* up_out = P.pair_j[nxt] + P.up_off[nxt][i];
  uint32_t* lo_out = P.lo_nbr + P.lo_off[i];
  for (uint32_t e = tid; e < run_up; e += nthreads) {
    const uint32_t v = buf_up[e];
    uint32_t r = 0;
    for (uint32_t f = 0; f < run_up; ++f) r += buf_up[f] < v;
    up_out[r] = v;
  }
  for (uint32_t e = tid; e < run_lo; e += nthreads) {
    const uint32_t v = buf_lo[e];
    uint32_t r = 0;
    for (uint32_t f = 0; f < run_lo; ++f) r += buf_lo[f] < v;
    lo_out[r] = v;
  }
}

}  // namespace

}  // namespace dem
