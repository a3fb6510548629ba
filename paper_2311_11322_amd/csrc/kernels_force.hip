// kernels_force.hip -- soft-sphere contact force of every contact, with the
// spring history carried from the previous step (Sec. 2.1: spring-dashpot
// normal and tangential forces, static friction, rolling and twisting
// friction, history kept while the contact lasts; Sec. 2.2.4: forces act at
// the contact point, lever arm of Eq. 8, torque of Eq. 9).
//
// One thread per contact (i, j) of the canonical upper list (j > i, runs
// sorted by j).  The previous step's upper run of i is sorted too, so the
// history lookup is a short search.  The thread also maps j's lower-list
// entry for i to the contact's index, which the per-sphere gather uses.  A
// wall is partner ns + w: infinite mass, no spin, moving rigidly; its
// reaction goes nowhere.  Geometry (separation, distance, overlap) is always
// FP64; the force arithmetic runs in T (double, or float for the FP32-force
// form).
#include "step_force.h"

namespace dem {

namespace {

// Blocks of the force kernel per work item (a work item covers 256 spheres,
// and a pile has about three upper-list contacts per sphere).
constexpr int kPairSplit = 4;

// One thread per contact (i, j) of the new upper list, grid-stride over the
// pile's contacts.  The history lookup searches i's previous (sorted) upper
// run; the thread also records where (i, j) sits for j's lower list.
template <typename T>
__global__ __launch_bounds__(kBlock) void k_pairs(PileDev* __restrict__ piles,
                                                  const WorkItem* __restrict__ wl,
                                                  ContactParams cp) {
  const int blk = xcd_block(blockIdx.x, gridDim.x);
  const WorkItem w = wl[blk / kPairSplit];
  PileDev& P = piles[w.pile];
  if (P.status != 0) return;
  const PairCtx<T> c = pair_ctx<T>(P, cp);
  if (c.n_pairs > (uint32_t)P.cap_pairs) return;
  const uint32_t nbp = (uint32_t)((P.ns + kBlock - 1) / kBlock) * kPairSplit;
  const uint32_t first = ((uint32_t)(w.base / kBlock) * kPairSplit + blk % kPairSplit) * kBlock;
  bool bad = false;
  for (uint32_t p = first + threadIdx.x; p < c.n_pairs; p += nbp * kBlock)
    pair_one<T>(P, c, cp, p, bad);
  if (bad) atomicOr(&P.status, kStUnstable);
}

}  // namespace

void launch_pairs(hipStream_t st, const PileDev* piles, const WorkItem* wl, int nblk,
                  ContactParams cp, int precision) {
  PileDev* p = const_cast<PileDev*>(piles);
  if (precision == 1)
    hipLaunchKernelGGL(k_pairs<float>, dim3(nblk * kPairSplit), dim3(kBlock), 0, st, p, wl, cp);
  else
    hipLaunchKernelGGL(k_pairs<double>, dim3(nblk * kPairSplit), dim3(kBlock), 0, st, p, wl, cp);
}

}  // namespace dem
