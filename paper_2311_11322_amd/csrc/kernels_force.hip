// kernels_force.hip -- soft-sphere contact forces of every sphere, with the
// spring history carried from the previous step (Sec. 2.1: spring-dashpot
// normal and tangential forces, static friction, rolling and twisting
// friction, history kept while the contact lasts; Sec. 2.2.4: forces act at
// the contact point, lever arm of Eq. 8, torque of Eq. 9).
//
// One thread per sphere i sums the force and torque of its contacts in
// canonical order: the lower list (j, i), j < i, then the upper list (i, j),
// each by increasing j.  Each contact is evaluated by both of its spheres
// with the same operands in the same order, so the two sums see the same
// force and no per-contact force is stored or read back; the lower sphere
// writes the contact's new spring history.  A wall is partner ns + w:
// infinite mass, no spin, moving rigidly; its reaction goes nowhere.
// Geometry is always FP64; the force arithmetic runs in T (double, or float
// for the FP32-force form).
#include "step_force.h"

namespace dem {

namespace {

template <typename T>
__global__ __launch_bounds__(kBlock) void k_forces(PileDev* __restrict__ piles,
                                                   const WorkItem* __restrict__ wl,
                                                   ContactParams cp) {
  const WorkItem w = wl[xcd_block(blockIdx.x, gridDim.x)];
  PileDev& P = piles[w.pile];
  const int i = w.base + threadIdx.x;
  if (i >= P.ns || P.status != 0) return;
  const PairCtx<T> c = pair_ctx<T>(P, cp);
  if (c.n_pairs > (uint32_t)P.cap_pairs) return;
  bool bad = false;
  forces_one<T>(P, c, cp, (uint32_t)i, bad);
  if (bad) atomicOr(&P.status, kStUnstable);
}

}  // namespace

void launch_forces(hipStream_t st, const PileDev* piles, const WorkItem* wl, int nblk,
                   ContactParams cp, int precision) {
  PileDev* p = const_cast<PileDev*>(piles);
  if (precision == 1)
    hipLaunchKernelGGL(k_forces<float>, dim3(nblk), dim3(kBlock), 0, st, p, wl, cp);
  else
    hipLaunchKernelGGL(k_forces<double>, dim3(nblk), dim3(kBlock), 0, st, p, wl, cp);
}

}  // namespace dem
