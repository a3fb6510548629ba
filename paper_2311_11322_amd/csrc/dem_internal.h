// dem_internal.h -- device-side layout of the DEM step (gfx950).
//
// Every kernel covers a *batch* of independent systems ("piles").  Each pile
// owns its device buffers; a device-resident table of PileDev entries holds
// their pointers, and static work lists map each launch block to
// (pile, first element).  A standalone system is a batch of one pile.
//
// Layout in HBM: structure-of-arrays, FP64, 3-vectors stored component-major
// ([3][n]) so that consecutive lanes read consecutive addresses.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace dem {

constexpr int kBlock = 256;        // threads per block (4 wave64)
constexpr int kHist = 7;           // spring history per contact: xi_t[3], xi_r[3], xi_q
constexpr int kScanItems = 8;      // elements per thread in the batched scan
constexpr int kScanChunk = kBlock * kScanItems;
constexpr int kScanSingleItems = 4;   // segments of at most this many chunks: one-launch scan
constexpr int kRunCache = 16;      // contact ids per run kept by the search's find pass
constexpr int kMaxBig = 64;        // big spheres per pile searched separately
constexpr int kBigRun = 2048;      // contacts per run of a big sphere (LDS sort)
constexpr int kMom = 40;           // per tree node: M, c[3], sum m e, sum m e^2, traceless
                                   // Q2[6], Q3[10], Q4[15], 3 unused
constexpr int kRaw = 32;           // per tree node: raw M2[6], M3[10], M4[15], 1 unused

// status bits of a pile (device-written)
constexpr int kStCapacity = 1;
constexpr int kStUnstable = 2;
constexpr int kStStopped = 4;      // the stop rule fired (bulk radius grown by stop_growth)

// per-block partials of the sphere set for the cell grid: bbox min[3],
// max[3], mass moments sum m, sum m r[3], and sum m |r - c|^2 about a
// reference point c (aggregate 0's centre) for the bulk radius
constexpr int kBbox = 11;

// modes of one pass through the step graph
constexpr int kModeStep = 0;       // kick, drift, rotate, evaluate, kick
constexpr int kModeInit = 1;       // evaluate at t0 only (no motion, no kick)

// Contact model constants shared by every pile of a batch.
struct ContactParams {
  double dt;
  double k_n, k_t, k_r, k_q;
  double mu_s, mu_r, mu_t;
  double damp_n, damp_t;     // -2 ln(eps) / sqrt(pi^2 + ln^2 eps): C = damp * sqrt(k mu)
  double max_overlap_frac;   // <= 0: no check
};

// Per-pile cell grid, written on the device every step.
struct Grid {
  double lo[3];              // origin of cell (0,0,0)
  double cell;               // cell side (>= largest sphere diameter)
  double inv_cell;
  double com[3];             // centre of mass of the pile (spin-up forcing)
  int32_t nc[3];             // cells per axis
  int32_t nbits[3];          // key bits per axis (sum 3 * bits)
  double t;                  // time of this evaluation
  double R_bulk;             // bulk radius sqrt(5/3 <|r - com|^2>_m) of this evaluation
  double wall_d[6];          // plane offset of each wall at time t
  double wall_v[6][3];       // velocity of each wall at time t
};

// Sorted-slot records read by the contact search: one 32 B load for the
// geometry and one 8 B load for the identity of each candidate.
struct alignas(32) SortedGeom {
  double x, y, z, s;
};
struct alignas(8) SortedId {
  int32_t agg;
  uint32_t id;
};

struct PileDev {
  // sizes (host-set)
  int32_t na, ns;
  int32_t cap_pairs;         // capacity of each contact list (upper and lower)
  int32_t bits;              // cell table is (1 << bits)^3 Morton codes
  int32_t periodic;
  int32_t g_tile;            // gravity tile (slots per tile)
  int32_t g_nt;              // gravity tiles
  int32_t g_form;            // 1: symmetric super-tile pairs; 2: per-target
  int32_t g_np;              // partial-sum rows per sphere: super-tiles, or source splits
  int32_t n_rblk;            // reconstruct blocks (bbox partials)
  int32_t n_periodic;        // cells per axis of a periodic pile
  int32_t member_scan;       // 1: reduction finds members by scanning all spheres
  int32_t member_read;       // 0 automatic, 1 direct, 2 staged through LDS
  double box;                // periodic cube side
  double G, soft_frac, spin_dw;
  double stop_growth;        // > 0: stop (kStStopped) once R_bulk >= stop_growth * R0
  double R0;                 // bulk radius the stop rule compares with (device-set at the
                             // first evaluation with the rule on)
  double cell_min;           // cell side lower bound: largest diameter of the non-big spheres
  // spheres with radius > s_cut ("big", at most kMaxBig) are not binned: they
  // sit in one extra cell after the Morton cells and are searched by a block
  // each; s_small is the largest radius of the others
  double s_cut, s_small;
  int32_t n_big;
  int32_t given;             // 1: sphere positions and velocities are given (no rigid bodies
                             // to reconstruct them from; stateless test hooks)
  int32_t fused;             // 1: the whole step runs in one workgroup (k_fused); the staged
                             // kernels launched over every pile skip it
  int32_t pad6;
  // uniform field and container walls (host-set)
  int32_t n_walls;
  int32_t pad3;
  double gfield[3];
  double wall[6][4];         // unit normal (into the domain), offset
  double wall_amp[6][3];     // rigid sinusoidal displacement amplitude
  double wall_omega, wall_phase;
  // tree gravity (host-set)
  int32_t tree;              // 1: tree instead of the direct sum
  int32_t tree_leaf;         // nodes of at most this many spheres act as pairs
  double theta;              // opening angle
  int32_t tree_order;        // highest multipole order: 2 or 4
  int32_t pad5;
  double* tmom;              // [sum_l 8^l][kMom] node moments, level l at (8^l - 1) / 7
  double* traw;              // [sum_l 8^l][kRaw] raw moments about each node's centre of mass
  double* tpart;             // [64][3][ns] tree sum per level-2 subtree, by sorted slot
  double* tbox;              // [ceil(ns / 64)][6] bounding box (min xyz, max xyz) of each group

  // device-updated bookkeeping
  int32_t parity;            // which half of each ping-pong pair is current
  int32_t status;            // kSt* bits; a failed pile is frozen
  int64_t step;              // steps completed
  int64_t fail_step;         // step index at which it failed
  uint32_t n_pairs;          // contacts of the last evaluation
  uint32_t pad0;

  // point-mass perturber, ping-pong by parity (state lives in the table)
  int32_t pert_on;
  int32_t pad1;
  double pert_M;
  double pert_r[2][3], pert_v[2][3], pert_a[2][3];
  double* ppart;             // [n_rblk][3] block sums of the perturber's pull

  // aggregate constants (written once by the set-up kernel)
  int32_t* first;            // [na] first member sphere
  int32_t* count;            // [na]
  double* M;                 // [na]
  double* I;                 // [3][na] principal moments
  // aggregate state, ping-pong [2]
  double* rA[2];             // [3][na]
  double* vA[2];
  double* aA[2];
  double* NA[2];
  double* q[2];              // [4][na]
  double* wb[2];             // [3][na]
  double* wA;                // [3][na] spin in space frame (this step)
  double* vpred;             // [3][na] predicted COM velocity (Eq. 3, first bracket)

  // sphere constants (set-up)
  double* b;                 // [3][ns] body offsets
  double* s;                 // [ns] radius
  double* m;                 // [ns] mass
  int32_t* agg;              // [ns] aggregate of each sphere
  // sphere per-step
  double* r;                 // [3][ns]
  double* v;                 // [3][ns]
  double* F;                 // [3][ns] contact force (gravity is added by the reduction)
  double* tau;               // [3][ns] contact torque about the centre
  uint32_t* key;             // [ns] Morton cell code
  uint32_t* sidx;            // [ns] sphere at sorted slot
  uint32_t* sidx_raw;        // [ns] sphere at slot, in atomic arrival order
  uint32_t* slot;            // [ns] sorted slot of sphere
  double* xs;                // [4][ns] sorted x, y, z, radius (gravity)
  SortedGeom* xg;            // [ns] sorted x, y, z, radius (search)
  SortedId* sid;             // [ns] sorted aggregate id and sphere id
  void* jrec;                // gravity records in sorted order (64 B FP64 / 32 B FP32)
  double* ganchor;           // [g_nt][4] FP64 anchor of each tile (relative coordinates)
  void* gpart;               // [g_np][3][ns] partial sums (sorted slots)
  double* gacc;              // [3][ns] gravity force G m_i sum_j (by sphere id)
  double* bpart;             // [n_rblk][kBbox] bbox min/max + mass moments
  Grid* grid;
  uint32_t* cell_cnt;        // [cells]
  uint32_t* cell_start;      // [cells + 1]
  uint32_t* run_cache;       // [2][ns][kRunCache] sorted upper / lower runs by slot
  uint32_t* cnt_up;          // [ns]
  uint32_t* cnt_lo;          // [ns]
  uint32_t* up_off[2];       // [ns + 1] CSR of contacts (i, j>i) by i
  uint32_t* lo_off;          // [ns + 1] CSR of contacts (j<i, i) by i
  uint32_t* pair_j[2];       // [cap]
  double* hist[2];           // [kHist][cap]
  uint32_t* lo_nbr;          // [cap] lower neighbour ids
};

// One block of a per-element kernel: pile p, elements base .. base+255.
struct WorkItem {
  int32_t pile;
  int32_t base;
};

// One block of the gravity kernel: the super-tile pair (ti, tj), ti <= tj,
// of a pile; in the per-target form, target tile ti and source split tj.
struct GravItem {
  int32_t pile;
  int32_t ti, tj;
  int32_t pad;
};

// One segment of the batched exclusive scan (out[n] receives the total).
// When parity is set, the output is out_pp[*parity ^ 1] (the next half of a
// ping-pong pair), else out_pp[0].
struct ScanSeg {
  const uint32_t* in;
  uint32_t* out_pp[2];
  const int32_t* parity;
  int32_t n;
  int32_t item0;             // first work item of this segment
  int32_t n_items;
  int32_t pad;
};

struct ScanItem {
  int32_t seg;
  int32_t chunk;             // chunk index inside the segment
};

// ---------------------------------------------------------------------------
// launchers (each defined next to its kernels)
// ---------------------------------------------------------------------------
void launch_setup(hipStream_t st, const PileDev* piles, const WorkItem* wl, int nblk,
                  const double* pos_in, const double* vel_in, const double* spin_in);
void launch_integrate(hipStream_t st, const PileDev* piles, const WorkItem* wl, int nblk,
                      ContactParams cp, int mode);
void launch_reconstruct(hipStream_t st, const PileDev* piles, const WorkItem* wl, int nblk);
void launch_grid(hipStream_t st, const PileDev* piles, int n_piles, int mode, double dt);
void launch_bin(hipStream_t st, const PileDev* piles, const WorkItem* wl, int nblk);
void launch_scatter(hipStream_t st, const PileDev* piles, const WorkItem* wl, int nblk);
void launch_cell_sort(hipStream_t st, const PileDev* piles, const WorkItem* wl, int nblk);
void launch_search(hipStream_t st, const PileDev* piles, const WorkItem* wl, int nblk, int write);
void launch_search_big(hipStream_t st, const PileDev* piles, const WorkItem* wl, int nblk,
                       int write);
void launch_forces(hipStream_t st, const PileDev* piles, const WorkItem* wl, int nblk,
                   ContactParams cp, int precision);
// Gravity: records and the per-slot combine cover every pile; the pair and
// per-target kernels run once per tile size present in the batch.
void launch_gravity_records(hipStream_t st, const PileDev* piles, const WorkItem* wl, int nblk,
                            int precision);
// multi: the items' piles have more tiles than kGravSlots (super-tiles of
// several tiles); otherwise every item is one tile pair.
void launch_gravity_tiles(hipStream_t st, const PileDev* piles, const GravItem* gl, int nitems,
                          int precision, bool softened, int tile, bool multi);
void launch_gravity_split(hipStream_t st, const PileDev* piles, const GravItem* gl, int nitems,
                          int precision, bool softened, int tile);
// Targets per lane of the per-target kernel for a precision and tile size
// (a target group is 64 x that many slots).
int gravity_split_ipt(int precision, int tile);
void launch_gravity_combine(hipStream_t st, const PileDev* piles, const WorkItem* wl, int nblk,
                            int precision);
// Supported tile sizes for a precision (default first); returns the count.
int gravity_tiles(int precision, int* tiles);
// Aggregates in one launch from which the member reduction stages its
// members through LDS (below it, direct member reads are faster: few waves,
// and the members stay in L2 between a wave's member iterations).
constexpr int64_t kReduceStageMin = 131072;
// Super-tiles of the pair form of the exact gravity sum (at most this many
// partial sums per sphere: a super-tile is ceil(tiles / kGravSlots) tiles),
// source splits of the per-target form, and the size of the pair form's
// partial sums above which a system takes the per-target form by default.
constexpr int kGravSlots = 256;
constexpr int kGravSplits = 16;
// Targets per lane of the per-target kernel at most (measured at 125k
// spheres: FP64 2, 4, 8 took 10.5, 10.8, 11.0 ms; FP32 4, 8, 16 took 6.7,
// 6.7, 6.4 ms).
constexpr int kSplitIpt64 = 2, kSplitIpt32 = 16;
constexpr int64_t kSymPartialMax = int64_t(64) << 30;
// Spheres in one search launch from which each sphere gets four lanes
// instead of eight.
constexpr int64_t kSearchLargeLaunch = 32768;
void launch_reduce(hipStream_t st, const PileDev* piles, const WorkItem* wl, int nblk,
                   ContactParams cp, int mode, bool stage);
void launch_finish(hipStream_t st, PileDev* piles, int n_piles, int mode, double dt);
// any_order[0], [1]: some tree pile of multipole order 2, 4
// leaf_levels: bit l set when level l is some pile's finest
void launch_tree(hipStream_t st, const PileDev* piles, WorkItem* const* wl_level,
                 const int* n_level, unsigned leaf_levels, const WorkItem* wl_sph, int n_sph_blk,
                 const bool* any_order);
void launch_fill_u32(hipStream_t st, uint32_t* p, uint32_t value, int64_t n);
// The whole step of each listed pile in one workgroup: part 1 the stages
// before gravity, part 2 those after it, part 3 all (no gravity).
void launch_fused(hipStream_t st, const PileDev* piles, const int32_t* plist, int n,
                  ContactParams cp, int mode, int part, int precision);
// Piles of at most this many spheres run the fused step unless tuned
// otherwise: one workgroup hides the latency of its dependent loads only for
// a few hundred spheres (measured on MI355X: 97 spheres 41 us vs 52 us
// staged, 303 spheres 67 vs 58 us, 962 spheres 148 vs 65 us per step).
constexpr int64_t kFusedAutoMax = 256;
void launch_scan(hipStream_t st, const ScanSeg* segs, int n_segs, const ScanItem* items,
                 int n_items, uint32_t* item_sums, int max_seg_items);

// ---------------------------------------------------------------------------
// small device helpers
// ---------------------------------------------------------------------------

__device__ __forceinline__ void cross3(const double a[3], const double b[3], double c[3]) {
  const double x = a[1] * b[2] - a[2] * b[1];
  const double y = a[2] * b[0] - a[0] * b[2];
  const double z = a[0] * b[1] - a[1] * b[0];
  c[0] = x;
  c[1] = y;
  c[2] = z;
}

__device__ __forceinline__ double dot3(const double a[3], const double b[3]) {
  return a[0] * b[0] + a[1] * b[1] + a[2] * b[2];
}

// Rotation matrix (body -> space, row-major) of quaternion (w, x, y, z),
// the unit-quaternion formula applied to q as given.
__device__ __forceinline__ void quat_rot(const double q[4], double R[9]) {
  const double w = q[0], x = q[1], y = q[2], z = q[3];
  R[0] = 1.0 - 2.0 * (y * y + z * z);
  R[1] = 2.0 * (x * y - w * z);
  R[2] = 2.0 * (x * z + w * y);
  R[3] = 2.0 * (x * y + w * z);
  R[4] = 1.0 - 2.0 * (x * x + z * z);
  R[5] = 2.0 * (y * z - w * x);
  R[6] = 2.0 * (x * z - w * y);
  R[7] = 2.0 * (y * z + w * x);
  R[8] = 1.0 - 2.0 * (x * x + y * y);
}

__device__ __forceinline__ void rot_apply(const double R[9], const double a[3], double c[3]) {
  c[0] = R[0] * a[0] + R[1] * a[1] + R[2] * a[2];
  c[1] = R[3] * a[0] + R[4] * a[1] + R[5] * a[2];
  c[2] = R[6] * a[0] + R[7] * a[1] + R[8] * a[2];
}

__device__ __forceinline__ void rot_apply_T(const double R[9], const double a[3], double c[3]) {
  c[0] = R[0] * a[0] + R[3] * a[1] + R[6] * a[2];
  c[1] = R[1] * a[0] + R[4] * a[1] + R[7] * a[2];
  c[2] = R[2] * a[0] + R[5] * a[1] + R[8] * a[2];
}

// Spread the low 10 bits of v to every third bit.
__device__ __forceinline__ uint32_t spread3(uint32_t v) {
  v &= 0x3ffu;
  v = (v | (v << 16)) & 0x030000ffu;
  v = (v | (v << 8)) & 0x0300f00fu;
  v = (v | (v << 4)) & 0x030c30c3u;
  v = (v | (v << 2)) & 0x09249249u;
  return v;
}

__device__ __forceinline__ uint32_t morton3(uint32_t x, uint32_t y, uint32_t z) {
  return spread3(x) | (spread3(y) << 1) | (spread3(z) << 2);
}

// Cell key for per-axis bit counts b: with m = min(b), the Morton code of
// the low m bits of each coordinate (a block of 2^m cells per axis), then the
// block's row-major index above it -- a bijection onto [0, 2^(bx+by+bz)),
// and the plain Morton code when the counts are equal.
__device__ __forceinline__ uint32_t cell_key(int cx, int cy, int cz, const int32_t nbits[3]) {
  const int m = min(nbits[0], min(nbits[1], nbits[2]));
  const uint32_t lo = (1u << m) - 1u;
  const uint32_t blk = ((uint32_t)cx >> m) + (((uint32_t)cy >> m) << (nbits[0] - m)) +
                       (((uint32_t)cz >> m) << (nbits[0] + nbits[1] - 2 * m));
  return morton3((uint32_t)cx & lo, (uint32_t)cy & lo, (uint32_t)cz & lo) | (blk << (3 * m));
}

// Cell coordinate of a position on one axis.  Periodic piles wrap the
// coordinate into [0, L) first (sphere centres are not wrapped; only the
// aggregate centres are).
__device__ __forceinline__ int cell_coord(double x, double lo, double inv_cell, int n,
                                          int periodic, double L) {
  if (periodic) {
    if (x >= L) x -= L;
    else if (x < 0.0) x += L;
  }
  // clamped before the conversion: a sphere far outside the grid falls into
  // its outermost cell
  const double c = fmin(fmax(floor((x - lo) * inv_cell), 0.0), (double)(n - 1));
  return (int)c;
}

// Workgroups are dispatched round-robin over the 8 XCDs, each with its own
// L2.  This bijection of [0, n) gives XCD x (blocks b with b % 8 == x) one
// contiguous range of logical blocks, so spatially adjacent work shares an
// L2 instead of being fetched by every XCD.
constexpr int kXcds = 8;
__device__ __forceinline__ int xcd_block(int b, int n) {
  const int x = b % kXcds, r = b / kXcds, q = n / kXcds, rem = n % kXcds;
  return x < rem ? x * (q + 1) + r : rem * (q + 1) + (x - rem) * q + r;
}

// A product and a sum, each rounded on its own: compiled without
// contraction, so no fused multiply-add forms across them where they are
// inlined (a plain a * b + c may become one).
__device__ __forceinline__ double rn_mul(double a, double b) {
#pragma clang fp contract(off)
  return a * b;
}
__device__ __forceinline__ double rn_add(double a, double b) {
#pragma clang fp contract(off)
  return a + b;
}

// Signed distance of a point from wall w at the evaluation time (plane
// offset d_t = Grid::wall_d[w]), rounded step by step (no fused
// multiply-add) so that the contact decision is reproducible:
// ((n_x x + n_y y) + n_z z) - d_t.
__device__ __forceinline__ double wall_gap(const PileDev& P, int w, double d_t, double x, double y,
                                           double z) {
  const double* n = P.wall[w];
  const double s = rn_add(rn_add(rn_mul(n[0], x), rn_mul(n[1], y)), rn_mul(n[2], z));
  return rn_add(s, -d_t);
}

}  // namespace dem
