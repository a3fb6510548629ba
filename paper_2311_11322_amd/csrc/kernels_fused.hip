// kernels_fused.hip -- the whole step of a pile in one workgroup.
//
// For piles small enough that the staged step (one launch per stage, each
// over every pile of a batch) is bound by launch latency, one workgroup of
// kFusedThreads threads runs every stage of its pile in order, separated by
// workgroup barriers: kick/drift/rotate, member reconstruction, cell grid,
// binning and counting sort, contact search, per-sphere contact forces,
// member reduction and end-of-step bookkeeping.  Many piles run as
// many workgroups of one launch.  Gravity, when the pile has it, stays with
// the batched tile kernels (it would not fit one compute unit): the launch
// then covers the stages before gravity (part 1) and a second launch those
// after it (part 2); without gravity one launch (part 3) is the whole step.
//
// Every element is handled by the same device functions as in the staged
// kernels (step_body.h, step_contact.h, step_force.h), so the arithmetic of
// each element is the same; only the pile's centre of mass and bulk radius
// are summed in another order (block partials of another shape).
#include "step_body.h"
#include "step_contact.h"
#include "step_force.h"

namespace dem {

namespace {

constexpr int kFusedThreads = 512;
constexpr int kFusedWaves = kFusedThreads / 64;
constexpr int kFusedLanes = kLanesSmall;          // lanes per sphere in the search
constexpr int kFusedGroups = kFusedThreads / kFusedLanes;

// The pile's status as another thread of the workgroup may have set it.
__device__ __forceinline__ int status_of(const PileDev& P) {
  return __hip_atomic_load(&P.status, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Between stages: a workgroup barrier.  All waves of the workgroup run on
// one compute unit and share its first-level cache, so the barrier's
// workgroup-scope release and acquire make every global write of a stage
// visible to the next; a device-scope fence would also write the second-level
// cache back to memory at every stage.  Values changed by atomics (the
// status) are read with atomic loads, from the second level.
__device__ __forceinline__ void stage_sync() { __syncthreads(); }

// Exclusive prefix sum of in[0, n) into out[0, n) and the total into out[n],
// by the whole workgroup: each thread scans one contiguous run, the run
// totals are scanned across the workgroup.  Integer sums: any order gives
// the same result.
__device__ void block_scan(const uint32_t* __restrict__ in, uint32_t* __restrict__ out, int n,
                           uint32_t* sh /* [kFusedWaves + 1] */) {
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int per = (n + kFusedThreads - 1) / kFusedThreads;
  const int b0 = min(n, tid * per), b1 = min(n, b0 + per);
  uint32_t sum = 0;
  for (int k = b0; k < b1; ++k) sum += in[k];
  uint32_t x = sum;                       // inclusive scan inside the wave
  for (int off = 1; off < 64; off <<= 1) {
    const uint32_t y = __shfl_up(x, off);
    if (lane >= off) x += y;
  }
  if (lane == 63) sh[wave] = x;
  __syncthreads();
  uint32_t before = 0, total = 0;
  for (int w = 0; w < kFusedWaves; ++w) {
    const uint32_t t = sh[w];
    if (w < wave) before += t;
    total += t;
  }
  uint32_t run = before + x - sum;
  for (int k = b0; k < b1; ++k) {
    const uint32_t v = in[k];
    out[k] = run;
    run += v;
  }
  if (tid == 0) out[n] = total;
  __syncthreads();                        // sh is reused by the next scan
}

// The search of every sphere (find or write pass): lane groups over the
// sorted slots, then the big spheres with the whole workgroup.
__device__ void search_all(PileDev& P, int write, uint32_t (*buf_up)[kRunLds],
                           uint32_t (*buf_lo)[kRunLds], uint32_t (*fill)[2], uint32_t* big_up,
                           uint32_t* big_lo, uint32_t* big_fill) {
  const int tid = threadIdx.x, grp = tid / kFusedLanes, lane = tid % kFusedLanes;
  for (int k = grp; k < P.ns; k += kFusedGroups)
    search_slot<kFusedLanes>(P, k, lane, write, buf_up[grp], buf_lo[grp], fill[grp]);
  for (int kb = 0; kb < P.n_big; ++kb) {
    stage_sync();                         // runs written; the previous sphere's LDS read
    search_big_one(P, kb, write, tid, kFusedThreads, big_up, big_lo, big_fill);
  }
}

template <typename T>
__global__ __launch_bounds__(kFusedThreads) void k_fused(PileDev* __restrict__ piles,
                                                         const int32_t* __restrict__ plist,
                                                         ContactParams cp, int mode, int part) {
  __shared__ uint32_t buf_up[kFusedGroups][kRunLds];
  __shared__ uint32_t buf_lo[kFusedGroups][kRunLds];
  __shared__ uint32_t fill[kFusedGroups][2];
  __shared__ uint32_t big_up[kBigRun];
  __shared__ uint32_t big_lo[kBigRun];
  __shared__ uint32_t big_fill[2];
  __shared__ double red[kFusedWaves][kBbox];
  __shared__ uint32_t scan_sh[kFusedWaves + 1];
  PileDev& P = piles[plist[blockIdx.x]];
  const int tid = threadIdx.x;
  bool ok = status_of(P) == 0;            // a failed pile stays frozen
  if (part & 1) {
    if (ok) {
      // kick, drift and rotate every aggregate
      for (int A = tid; A < P.na; A += kFusedThreads) integrate_one(P, A, cp, mode);
      stage_sync();
      // members, and the bounding box and mass moments of the pile
      double acc[kBbox], one[kBbox], cref[3];
      bbox_identity(acc);
      bbox_ref(P, cref);
      for (int i = tid; i < P.ns; i += kFusedThreads) {
        reconstruct_one(P, i, cref, one);
        bbox_combine(acc, one);
      }
      for (int off = 32; off > 0; off >>= 1) {
        double o[kBbox];
        for (int k = 0; k < kBbox; ++k) o[k] = __shfl_xor(acc[k], off);
        bbox_combine(acc, o);
      }
      if ((tid & 63) == 0)
        for (int k = 0; k < kBbox; ++k) red[tid >> 6][k] = acc[k];
      stage_sync();
      if (tid == 0) {
        for (int w = 1; w < kFusedWaves; ++w) bbox_combine(red[0], red[w]);
        grid_from_vals(P, red[0], mode, cp.dt);
      }
      stage_sync();
      ok = status_of(P) == 0;
    }
    if (ok) {
      // counting sort of the cell keys
      for (int i = tid; i < P.ns; i += kFusedThreads) bin_one(P, i);
      stage_sync();
      block_scan(P.cell_cnt, P.cell_start, (1 << (3 * P.bits)) + 1, scan_sh);
      stage_sync();
      for (int i = tid; i < P.ns; i += kFusedThreads) scatter_one(P, i);
      stage_sync();
      for (int k = tid; k < P.ns; k += kFusedThreads) cell_sort_one(P, k);
      stage_sync();
      // contact search: counts, offsets, runs
      search_all(P, 0, buf_up, buf_lo, fill, big_up, big_lo, big_fill);
      stage_sync();
      const int nxt = P.parity ^ 1;
      block_scan(P.cnt_up, P.up_off[nxt], P.ns, scan_sh);
      block_scan(P.cnt_lo, P.lo_off, P.ns, scan_sh);
      stage_sync();
      search_all(P, 1, buf_up, buf_lo, fill, big_up, big_lo, big_fill);
      stage_sync();
      ok = status_of(P) == 0;
    }
    if (ok) {
      // contact forces with the spring history
      const PairCtx<T> c = pair_ctx<T>(P, cp);
      bool bad = false;
      for (int i = tid; i < P.ns; i += kFusedThreads) forces_one<T>(P, c, cp, (uint32_t)i, bad);
      if (bad) atomicOr(&P.status, kStUnstable);
      stage_sync();
      ok = status_of(P) == 0;
    }
  }
  if (part & 2) {
    if (ok) {
      const int na = P.na, nxt = P.parity ^ 1;
      for (int A = tid; A < na; A += kFusedThreads) {
        double q[4], R[9];
        for (int k = 0; k < 4; ++k) q[k] = P.q[nxt][k * na + A];
        quat_rot(q, R);
        double FA[3] = {0.0, 0.0, 0.0}, NA[3] = {0.0, 0.0, 0.0};
        if (P.member_scan != 0) reduce_members_scan(P, A, R, FA, NA);
        else reduce_members_direct(P, A, R, FA, NA);
        reduce_tail(P, A, R, FA, NA, cp, mode);
      }
      stage_sync();
    }
    if (tid == 0) finish_one(P, mode, cp.dt);
  }
}

}  // namespace

void launch_fused(hipStream_t st, const PileDev* piles, const int32_t* plist, int n, ContactParams cp,
                  int mode, int part, int precision) {
  if (n <= 0) return;
  PileDev* p = const_cast<PileDev*>(piles);
  if (precision == 1)
    hipLaunchKernelGGL(k_fused<float>, dim3(n), dim3(kFusedThreads), 0, st, p, plist, cp, mode,
                       part);
  else
    hipLaunchKernelGGL(k_fused<double>, dim3(n), dim3(kFusedThreads), 0, st, p, plist, cp, mode,
                       part);
}

}  // namespace dem
