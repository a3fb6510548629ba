// kernels_contact.hip -- cell-list binning, contact search that skips pairs
// inside one aggregate, and the per-contact soft-sphere force with spring
// history (Sec. 2.1 and 2.2.5 of the paper; lever arm Eq. 8, contact-point
// torque Eq. 9).
//
// Binning is a counting sort on Morton cell codes: integer atomics build the
// per-cell counts, a batched exclusive scan turns them into cell ranges, and
// a per-cell insertion sort by sphere id makes the order deterministic.  The
// search scans the 27 neighbouring cells of every sphere; each sphere lists
// its contacts with higher ids (the canonical upper list) and with lower ids
// (the lower list) as count -> scan -> write, so the contact list comes out
// in canonical (i, j) order without a global sort and without float atomics.
#include "dem_internal.h"

namespace dem {

namespace {

// Morton code of a sphere's cell on the pile's current grid.
__device__ __forceinline__ void sphere_cell(const PileDev& P, const Grid& g, double x, double y,
                                            double z, int c[3]) {
  const int n = 1 << g.nb;
  c[0] = cell_coord(x, g.lo[0], g.inv_cell, n, P.periodic, P.box);
  c[1] = cell_coord(y, g.lo[1], g.inv_cell, n, P.periodic, P.box);
  c[2] = cell_coord(z, g.lo[2], g.inv_cell, n, P.periodic, P.box);
}

__global__ __launch_bounds__(kBlock) void k_bin(const PileDev* __restrict__ piles,
                                                const WorkItem* __restrict__ wl) {
  const WorkItem w = wl[blockIdx.x];
  const PileDev& P = piles[w.pile];
  const int i = w.base + threadIdx.x;
  if (i >= P.ns || P.status != 0) return;
  const Grid g = *P.grid;
  const int ns = P.ns;
  int c[3];
  sphere_cell(P, g, P.r[i], P.r[ns + i], P.r[2 * ns + i], c);
  const uint32_t key = morton3(c[0], c[1], c[2]);
  P.key[i] = key;
  atomicAdd(&P.cell_cnt[key], 1u);
}

// Place each sphere into its cell's range; the counts return to zero, ready
// for the next step.
__global__ __launch_bounds__(kBlock) void k_scatter(const PileDev* __restrict__ piles,
                                                    const WorkItem* __restrict__ wl) {
  const WorkItem w = wl[blockIdx.x];
  const PileDev& P = piles[w.pile];
  const int i = w.base + threadIdx.x;
  if (i >= P.ns || P.status != 0) return;
  const uint32_t key = P.key[i];
  const uint32_t k = atomicSub(&P.cell_cnt[key], 1u) - 1u;
  P.sidx[P.cell_start[key] + k] = (uint32_t)i;
}

// The first slot of each cell sorts the cell's sphere ids (cells hold a few
// spheres), making the binned order independent of atomic arrival order.
__global__ __launch_bounds__(kBlock) void k_cell_sort(const PileDev* __restrict__ piles,
                                                      const WorkItem* __restrict__ wl) {
  const WorkItem w = wl[blockIdx.x];
  const PileDev& P = piles[w.pile];
  const int k = w.base + threadIdx.x;
  if (k >= P.ns || P.status != 0) return;
  uint32_t* __restrict__ sidx = P.sidx;
  const uint32_t key = P.key[sidx[k]];
  if (k > 0 && P.key[sidx[k - 1]] == key) return;
  const uint32_t e = P.cell_start[key + 1];
  for (uint32_t a = (uint32_t)k + 1; a < e; ++a) {
    const uint32_t v = sidx[a];
    uint32_t b = a;
    while (b > (uint32_t)k && sidx[b - 1] > v) {
      sidx[b] = sidx[b - 1];
      --b;
    }
    sidx[b] = v;
  }
}

// Sorted copies of positions, radii and aggregate ids (spatially coherent
// reads in the search and in gravity) and the inverse permutation.
__global__ __launch_bounds__(kBlock) void k_sorted_copy(const PileDev* __restrict__ piles,
                                                        const WorkItem* __restrict__ wl) {
  const WorkItem w = wl[blockIdx.x];
  const PileDev& P = piles[w.pile];
  const int k = w.base + threadIdx.x;
  if (k >= P.ns || P.status != 0) return;
  const int ns = P.ns;
  const uint32_t i = P.sidx[k];
  P.slot[i] = (uint32_t)k;
  const double x = P.r[i], y = P.r[ns + i], z = P.r[2 * ns + i], s = P.s[i];
  P.xs[k] = x;
  P.xs[ns + k] = y;
  P.xs[2 * ns + k] = z;
  P.xs[3 * ns + k] = s;
  P.sagg[k] = P.agg[i];
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
  const double d2 = __dadd_rn(__dadd_rn(__dmul_rn(dx, dx), __dmul_rn(dy, dy)), __dmul_rn(dz, dz));
  return d2 < __dmul_rn(S, S);
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

// One thread per sorted slot.  Scans the 27 neighbouring cells and finds
// every j != i of another aggregate in contact, then the walls it touches.  Count mode stores the number
// of contacts with j > i (upper) and j < i (lower) under sphere id i; write
// mode stores the ids at the scanned offsets and sorts each run, after
// checking the pile's contact capacity.
__global__ __launch_bounds__(kBlock) void k_search(PileDev* __restrict__ piles,
                                                   const WorkItem* __restrict__ wl, int write) {
  const WorkItem w = wl[blockIdx.x];
  PileDev& P = piles[w.pile];
  const int k = w.base + threadIdx.x;
  if (k >= P.ns || P.status != 0) return;
  const int ns = P.ns, nxt = P.parity ^ 1;
  const Grid g = *P.grid;
  const uint32_t* __restrict__ sidx = P.sidx;
  const double* __restrict__ xs = P.xs;
  const int32_t* __restrict__ sagg = P.sagg;
  const uint32_t* __restrict__ cstart = P.cell_start;
  const uint32_t i = sidx[k];
  const double x = xs[k], y = xs[ns + k], z = xs[2 * ns + k], si = xs[3 * ns + k];
  const int ai = sagg[k];
  const int periodic = P.periodic;
  const double L = P.box;
  int c[3];
  sphere_cell(P, g, x, y, z, c);
  const int n = 1 << g.nb;
  uint32_t* up_out = nullptr;
  uint32_t* lo_out = nullptr;
  if (write) {
    const uint32_t tot_up = P.up_off[nxt][ns], tot_lo = P.lo_off[ns];
    if (tot_up > (uint32_t)P.cap_pairs || tot_lo > (uint32_t)P.cap_pairs) {
      atomicOr(&P.status, kStCapacity);
      return;
    }
    up_out = P.pair_j[nxt] + P.up_off[nxt][i];
    lo_out = P.lo_nbr + P.lo_off[i];
  }
  uint32_t nup = 0, nlo = 0;
  // neighbouring cells along an axis: c-1..c+1, or every cell when a
  // periodic axis has fewer than three (so no cell is visited twice)
  const int lo_d = (periodic && n < 3) ? 0 : -1;
  const int hi_d = (periodic && n < 3) ? n - 1 : 1;
  for (int dz = lo_d; dz <= hi_d; ++dz) {
    int cz = (periodic && n < 3) ? dz : c[2] + dz;
    if (periodic) cz &= n - 1;
    else if (cz < 0 || cz >= n) continue;
    for (int dy = lo_d; dy <= hi_d; ++dy) {
      int cy = (periodic && n < 3) ? dy : c[1] + dy;
      if (periodic) cy &= n - 1;
      else if (cy < 0 || cy >= n) continue;
      for (int dx = lo_d; dx <= hi_d; ++dx) {
        int cx = (periodic && n < 3) ? dx : c[0] + dx;
        if (periodic) cx &= n - 1;
        else if (cx < 0 || cx >= n) continue;
        const uint32_t key = morton3(cx, cy, cz);
        const uint32_t t1 = cstart[key + 1];
        for (uint32_t t = cstart[key]; t < t1; ++t) {
          if (sagg[t] == ai) continue;        // same aggregate (includes t == k)
          const double S = si + xs[3 * ns + t];
          if (!touching(xs[t] - x, xs[ns + t] - y, xs[2 * ns + t] - z, S, periodic, L)) continue;
          const uint32_t j = sidx[t];
          if (j > i) {
            if (write) up_out[nup] = j;
            ++nup;
          } else {
            if (write) lo_out[nlo] = j;
            ++nlo;
          }
        }
      }
    }
  }
  // walls are partners ns + w, after every sphere partner
  for (int wl_ = 0; wl_ < P.n_walls; ++wl_) {
    if (!(wall_gap(P, g, wl_, x, y, z) < si)) continue;
    if (write) up_out[nup] = (uint32_t)(ns + wl_);
    ++nup;
  }
  if (write) {
    sort_run(up_out, nup);
    sort_run(lo_out, nlo);
  } else {
    P.cnt_up[i] = nup;
    P.cnt_lo[i] = nlo;
  }
}

}  // namespace

void launch_bin(hipStream_t st, const PileDev* piles, const WorkItem* wl, int nblk) {
  hipLaunchKernelGGL(k_bin, dim3(nblk), dim3(kBlock), 0, st, piles, wl);
}
void launch_scatter(hipStream_t st, const PileDev* piles, const WorkItem* wl, int nblk) {
  hipLaunchKernelGGL(k_scatter, dim3(nblk), dim3(kBlock), 0, st, piles, wl);
}
void launch_cell_sort(hipStream_t st, const PileDev* piles, const WorkItem* wl, int nblk) {
  hipLaunchKernelGGL(k_cell_sort, dim3(nblk), dim3(kBlock), 0, st, piles, wl);
}
void launch_sorted_copy(hipStream_t st, const PileDev* piles, const WorkItem* wl, int nblk) {
  hipLaunchKernelGGL(k_sorted_copy, dim3(nblk), dim3(kBlock), 0, st, piles, wl);
}
void launch_search(hipStream_t st, const PileDev* piles, const WorkItem* wl, int nblk, int write) {
  hipLaunchKernelGGL(k_search, dim3(nblk), dim3(kBlock), 0, st, const_cast<PileDev*>(piles), wl,
                     write);
}

}  // namespace dem
