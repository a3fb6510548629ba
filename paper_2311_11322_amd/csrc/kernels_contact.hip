// kernels_contact.hip -- cell-list binning, contact search that skips pairs
// inside one aggregate, and the per-contact soft-sphere force with spring
// history (Sec. 2.1, 2.2.4 and 2.2.5 of the paper; lever arm Eq. 8, contact-point
// torque Eq. 9).
//
// Binning is a counting sort on Morton cell codes: integer atomics build the
// per-cell counts, a batched exclusive scan turns them into cell ranges, and
// ranking each sphere by id within its cell makes the order deterministic.
// The search scans the 27 neighbouring cells of every sphere (a group of
// lanes per sphere, blocks mapped to XCDs by region); each sphere lists
// its contacts with higher ids (the canonical upper list) and with lower ids
// (the lower list) as count -> scan -> write, so the contact list comes out
// in canonical (i, j) order without a global sort and without float atomics.
#include "step_contact.h"

namespace dem {

namespace {

__global__ __launch_bounds__(kBlock) void k_bin(const PileDev* __restrict__ piles,
                                                const WorkItem* __restrict__ wl) {
  const WorkItem w = wl[xcd_block(blockIdx.x, gridDim.x)];
  const PileDev& P = piles[w.pile];
  const int i = w.base + threadIdx.x;
  if (i >= P.ns || P.status != 0) return;
  bin_one(P, i);
}

// Place each sphere into its cell's range (in atomic arrival order); the
// counts return to zero, ready for the next step.
__global__ __launch_bounds__(kBlock) void k_scatter(const PileDev* __restrict__ piles,
                                                    const WorkItem* __restrict__ wl) {
  const WorkItem w = wl[xcd_block(blockIdx.x, gridDim.x)];
  const PileDev& P = piles[w.pile];
  const int i = w.base + threadIdx.x;
  if (i >= P.ns || P.status != 0) return;
  scatter_one(P, i);
}

// Order each cell's spheres by id, independent of atomic arrival order: the
// sphere at raw slot k goes to its cell's start plus its rank (the number of
// smaller ids in the cell).  The same thread writes the sphere's sorted
// copies there -- packed records for the search and, in a pile with
// gravity, positions and radius for it -- and the inverse permutation.
__global__ __launch_bounds__(kBlock) void k_cell_sort(const PileDev* __restrict__ piles,
                                                      const WorkItem* __restrict__ wl) {
  const WorkItem w = wl[xcd_block(blockIdx.x, gridDim.x)];
  const PileDev& P = piles[w.pile];
  const int k = w.base + threadIdx.x;
  if (k >= P.ns || P.status != 0) return;
  cell_sort_one(P, k);
}

// L lanes per sorted slot.  Every lane tests the spheres of its share of
// the 27 neighbouring cells that belong to another aggregate, and its share
// of the walls.
//
// Find mode stores the number of contacts with j > i (upper) and j < i
// (lower) under sphere id i and, when both runs fit kRunLds entries, the
// runs themselves sorted by id in the slot's cache.  Write mode (after the
// scan) checks the pile's contact capacity and copies each cached run to its
// offsets; a sphere whose runs did not fit is searched again and its runs
// written in arrival order, then sorted in place.  Launched with L blocks
// per work item.
template <int L>
__global__ __launch_bounds__(kBlock) void k_search(PileDev* __restrict__ piles,
                                                   const WorkItem* __restrict__ wl, int write) {
  constexpr int kGroups = SearchLanes<L>::kGroups;
  __shared__ uint32_t buf_up[kGroups][kRunLds];
  __shared__ uint32_t buf_lo[kGroups][kRunLds];
  __shared__ uint32_t fill[kGroups][2];
  const int blk = xcd_block(blockIdx.x, gridDim.x);
  const WorkItem w = wl[blk / L];
  PileDev& P = piles[w.pile];
  const int grp = threadIdx.x / L, lane = threadIdx.x % L;
  const int k = w.base + (blk % L) * kGroups + grp;
  if (k >= P.ns || P.status != 0) return;      // uniform over the lane group
  search_slot<L>(P, k, lane, write, buf_up[grp], buf_lo[grp], fill[grp]);
}

// One block per big sphere (the k-th, by id, sits at slot ns - n_big + k):
// its threads split the cells within reach of any other sphere and the big
// spheres' cell.  Find mode stores the run lengths; write mode gathers both
// runs in LDS, rank-sorts them and stores them at the scanned offsets.  A run
// longer than kBigRun is a capacity failure.
__global__ __launch_bounds__(kBlock) void k_search_big(PileDev* __restrict__ piles,
                                                       const WorkItem* __restrict__ wl,
                                                       int write) {
  __shared__ uint32_t buf_up[kBigRun];
  __shared__ uint32_t buf_lo[kBigRun];
  __shared__ uint32_t fill[2];
  const WorkItem w = wl[blockIdx.x];
  PileDev& P = piles[w.pile];
  search_big_one(P, w.base, write, threadIdx.x, kBlock, buf_up, buf_lo, fill);
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
void launch_search_big(hipStream_t st, const PileDev* piles, const WorkItem* wl, int nblk,
                       int write) {
  hipLaunchKernelGGL(k_search_big, dim3(nblk), dim3(kBlock), 0, st, const_cast<PileDev*>(piles),
                     wl, write);
}
void launch_search(hipStream_t st, const PileDev* piles, const WorkItem* wl, int nblk, int write) {
  // measured on MI355X: four lanes per sphere are faster from about 32k
  // spheres in a launch (1M-sphere lattice: find pass 0.142 vs 0.173 ms),
  // eight below it (6,400-sphere box fill: 0.009 vs 0.012 ms)
  PileDev* p = const_cast<PileDev*>(piles);
  if ((int64_t)nblk * kBlock >= kSearchLargeLaunch)
    hipLaunchKernelGGL(k_search<kLanesLarge>, dim3(nblk * kLanesLarge), dim3(kBlock), 0, st, p, wl,
                       write);
  else
    hipLaunchKernelGGL(k_search<kLanesSmall>, dim3(nblk * kLanesSmall), dim3(kBlock), 0, st, p, wl,
                       write);
}

}  // namespace dem
