// kernels_scan.hip -- batched exclusive prefix sum of uint32 arrays.
//
// Many independent segments (the cell counts and contact counts of every
// pile) are scanned by the same two launches: per-chunk totals, then the
// chunk-local scans, each chunk adding up the totals before it in its
// segment; or, when every segment is short, by one launch with a block per
// segment.  out[n] of each segment receives its total.
// Integer arithmetic, so the result does not depend on the order of work.
#include "dem_internal.h"

namespace dem {

namespace {

// Exclusive scan of one value per thread across a 256-thread block; returns
// the exclusive prefix and writes the block total to *total.
__device__ __forceinline__ uint32_t block_exclusive(uint32_t v, uint32_t* total) {
  __shared__ uint32_t wsum[kBlock / 64];
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  uint32_t x = v;
  for (int off = 1; off < 64; off <<= 1) {
    const uint32_t y = __shfl_up(x, off);
    if (lane >= off) x += y;
  }
  if (lane == 63) wsum[wave] = x;
  __syncthreads();
  uint32_t before = 0, all = 0;
  for (int k = 0; k < kBlock / 64; ++k) {
    const uint32_t s = wsum[k];
    if (k < wave) before += s;
    all += s;
  }
  __syncthreads();
  *total = all;
  return before + x - v;
}

// One thread's kScanItems consecutive elements: two 16-byte accesses when the
// run lies inside the segment and the array is 16-byte aligned, else one
// guarded access per element (zeros past the end).
static_assert(kScanItems == 8, "runs are read as two 16-byte vectors");

__device__ __forceinline__ bool whole_run(const void* p, int64_t base, int64_t n) {
  return base + kScanItems <= n && (reinterpret_cast<uintptr_t>(p) & 15) == 0;
}

__device__ __forceinline__ void load_run(const uint32_t* __restrict__ in, int64_t base, int64_t n,
                                         uint32_t v[kScanItems]) {
  if (whole_run(in, base, n)) {
    const uint4 a = *reinterpret_cast<const uint4*>(in + base);
    const uint4 b = *reinterpret_cast<const uint4*>(in + base + 4);
    v[0] = a.x, v[1] = a.y, v[2] = a.z, v[3] = a.w;
    v[4] = b.x, v[5] = b.y, v[6] = b.z, v[7] = b.w;
  } else {
#pragma unroll
    for (int k = 0; k < kScanItems; ++k) v[k] = base + k < n ? in[base + k] : 0u;
  }
}

__device__ __forceinline__ void store_run(uint32_t* __restrict__ out, int64_t base, int64_t n,
                                          const uint32_t r[kScanItems]) {
  if (whole_run(out, base, n)) {
    *reinterpret_cast<uint4*>(out + base) = make_uint4(r[0], r[1], r[2], r[3]);
    *reinterpret_cast<uint4*>(out + base + 4) = make_uint4(r[4], r[5], r[6], r[7]);
  } else {
#pragma unroll
    for (int k = 0; k < kScanItems; ++k)
      if (base + k < n) out[base + k] = r[k];
  }
}

// Exclusive prefix of a run, starting from run0.
__device__ __forceinline__ void run_prefix(const uint32_t v[kScanItems], uint32_t run0,
                                           uint32_t r[kScanItems]) {
#pragma unroll
  for (int k = 0; k < kScanItems; ++k) {
    r[k] = run0;
    run0 += v[k];
  }
}

__global__ __launch_bounds__(kBlock) void k_scan_reduce(const ScanSeg* __restrict__ segs,
                                                        const ScanItem* __restrict__ items,
                                                        uint32_t* __restrict__ sums) {
  const ScanItem it = items[blockIdx.x];
  const ScanSeg sg = segs[it.seg];
  const int64_t base = (int64_t)it.chunk * kScanChunk + threadIdx.x * kScanItems;
  uint32_t v[kScanItems];
  load_run(sg.in, base, sg.n, v);
  uint32_t acc = 0;
#pragma unroll
  for (int k = 0; k < kScanItems; ++k) acc += v[k];
  uint32_t total;
  block_exclusive(acc, &total);
  if (threadIdx.x == 0) sums[blockIdx.x] = total;
}

// One block per chunk: the chunk's offset is the sum of the totals of the
// segment's earlier chunks (read by the whole block), then the chunk-local
// scan; the segment's last chunk also writes the total into out[n].
__global__ __launch_bounds__(kBlock) void k_scan_down(const ScanSeg* __restrict__ segs,
                                                      const ScanItem* __restrict__ items,
                                                      const uint32_t* __restrict__ sums) {
  const ScanItem it = items[blockIdx.x];
  const ScanSeg sg = segs[it.seg];
  uint32_t* __restrict__ out = sg.parity ? sg.out_pp[*sg.parity ^ 1] : sg.out_pp[0];
  // the chunk's elements and the earlier chunks' totals are loaded before
  // the first barrier, so the two loads are in flight together
  const int64_t base = (int64_t)it.chunk * kScanChunk + threadIdx.x * kScanItems;
  uint32_t v[kScanItems], r[kScanItems];
  load_run(sg.in, base, sg.n, v);
  uint32_t part = 0;
  for (int c = threadIdx.x; c < it.chunk; c += kBlock) part += sums[sg.item0 + c];
  uint32_t offset;
  block_exclusive(part, &offset);
  uint32_t acc = 0;
#pragma unroll
  for (int k = 0; k < kScanItems; ++k) acc += v[k];
  uint32_t total;
  run_prefix(v, block_exclusive(acc, &total) + offset, r);
  store_run(out, base, sg.n, r);
  if (it.chunk == sg.n_items - 1 && threadIdx.x == 0) out[sg.n] = offset + total;
}

// One block per segment scans the whole segment chunk by chunk, carrying the
// running total (one launch; for batches whose segments are all short).
__global__ __launch_bounds__(kBlock) void k_scan_single(const ScanSeg* __restrict__ segs) {
  const ScanSeg sg = segs[blockIdx.x];
  uint32_t* __restrict__ out = sg.parity ? sg.out_pp[*sg.parity ^ 1] : sg.out_pp[0];
  uint32_t carry = 0;
  for (int c = 0; c < sg.n_items; ++c) {
    const int64_t base = (int64_t)c * kScanChunk + threadIdx.x * kScanItems;
    uint32_t v[kScanItems], r[kScanItems];
    load_run(sg.in, base, sg.n, v);
    uint32_t acc = 0;
#pragma unroll
    for (int k = 0; k < kScanItems; ++k) acc += v[k];
    uint32_t total;
    run_prefix(v, block_exclusive(acc, &total) + carry, r);
    store_run(out, base, sg.n, r);
    carry += total;
  }
  if (threadIdx.x == 0) out[sg.n] = carry;
}

}  // namespace

void launch_scan(hipStream_t st, const ScanSeg* segs, int n_segs, const ScanItem* items,
                 int n_items, uint32_t* item_sums, int max_seg_items) {
  if (n_items <= 0) return;
  if (max_seg_items <= kScanSingleItems) {
    hipLaunchKernelGGL(k_scan_single, dim3(n_segs), dim3(kBlock), 0, st, segs);
    return;
  }
  hipLaunchKernelGGL(k_scan_reduce, dim3(n_items), dim3(kBlock), 0, st, segs, items, item_sums);
  hipLaunchKernelGGL(k_scan_down, dim3(n_items), dim3(kBlock), 0, st, segs, items, item_sums);
}

}  // namespace dem
