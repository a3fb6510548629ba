// kernels_tree.hip -- tree gravity: multipoles to hexadecapole order on the
// pyramid of the pile's cubic cell grid (the paper's gravity is a tree code
// with expansions to that order, Sec. 2), softened pairs in the near field.
#include "gravity_common.h"

namespace dem {

namespace {

// ---------------------------------------------------------------------------
// Tree gravity: the pyramid of the pile's cubic cell grid.  Node (l, p) is the
// cube of side cell * 2^(bits - l) whose Morton prefix is p; with the spheres
// sorted by cell code its spheres are the contiguous slots
// [cell_start[p << 3(bits-l)], cell_start[(p+1) << 3(bits-l)]).
//
// Each node keeps (kMom doubles) its mass M, centre of mass c, sum m e and
// sum m e^2 (e the sphere's softening half-length), and the traceless parts
// Q_n of its raw moments M_n = sum m d^n (d = x - c) for n = 2, 3, 4; beside
// them (kRaw doubles) the raw M_n, which the upward pass translates.  A
// symmetric tensor of rank n is stored by its distinct components, the index
// tuples a <= b <= ... in lexicographic order: a component with i zeros, j
// ones and n - i - j twos sits at sym_index(n, i, j).
// ---------------------------------------------------------------------------

constexpr int kTreeSplit = 2;      // a group's walk is split over the 8^2 subtrees of level 2
constexpr int kTreeParts = 1 << (3 * kTreeSplit);
constexpr int kQ2 = 6, kQ3 = 12, kQ4 = 22;   // offsets of Q2, Q3, Q4 in a node's moments
constexpr int kR2 = 0, kR3 = 6, kR4 = 16;    // offsets of M2, M3, M4 in a node's raw moments

typedef const __attribute__((address_space(4))) double* ConstD;
typedef const __attribute__((address_space(4))) uint32_t* ConstU;

__device__ __forceinline__ size_t level_offset(int l) { return (((size_t)1 << (3 * l)) - 1) / 7; }

__host__ __device__ constexpr int sym_index(int n, int i, int j) {
  int s = 0;
  for (int q = i + 1; q <= n; ++q) s += n - q + 1;
  return s + (n - i - j);
}
__host__ __device__ constexpr int zeros(int a, int b, int c = -1, int d = -1) {
  return (a == 0) + (b == 0) + (c == 0) + (d == 0);
}
__host__ __device__ constexpr int ones(int a, int b, int c = -1, int d = -1) {
  return (a == 1) + (b == 1) + (c == 1) + (d == 1);
}
__host__ __device__ constexpr int i2(int a, int b) { return sym_index(2, zeros(a, b), ones(a, b)); }
__host__ __device__ constexpr int i3(int a, int b, int c) {
  return sym_index(3, zeros(a, b, c), ones(a, b, c));
}
__host__ __device__ constexpr int i4(int a, int b, int c, int d) {
  return sym_index(4, zeros(a, b, c, d), ones(a, b, c, d));
}
__device__ __forceinline__ double ipow(double v, int k) {
  double r = 1.0;
#pragma unroll
  for (int q = 0; q < 4; ++q)
    if (q < k) r *= v;
  return r;
}

// raw[...] += w d^n for n = 2, 3, 4 (every distinct component)
__device__ __forceinline__ void add_powers(double* raw, double w, const double d[3]) {
#pragma unroll
  for (int n = 2; n <= 4; ++n) {
    const int off = n == 2 ? kR2 : (n == 3 ? kR3 : kR4);
#pragma unroll
    for (int i = n; i >= 0; --i)
#pragma unroll
      for (int j = n - i; j >= 0; --j)
        raw[off + sym_index(n, i, j)] += w * ipow(d[0], i) * ipow(d[1], j) * ipow(d[2], n - i - j);
  }
}

// Traceless parts of the raw moments:
//   Q2 = M2 - tr/3 1,  Q3 = M3 - 1/5 (sum of 3 delta t),  t_c = M3_aac,
//   Q4 = M4 - 1/7 (sum of 6 delta U) + s/35 (sum of 3 delta delta),
//   U_cd = M4_aacd, s = U_aa.
__device__ __forceinline__ void traceless(const double* raw, double* q) {
  const double tr = raw[kR2 + i2(0, 0)] + raw[kR2 + i2(1, 1)] + raw[kR2 + i2(2, 2)];
#pragma unroll
  for (int a = 0; a < 3; ++a)
#pragma unroll
    for (int b = a; b < 3; ++b)
      q[kQ2 + i2(a, b)] = raw[kR2 + i2(a, b)] - (a == b ? tr / 3.0 : 0.0);
  double t[3];
#pragma unroll
  for (int c = 0; c < 3; ++c)
    t[c] = raw[kR3 + i3(0, 0, c)] + raw[kR3 + i3(1, 1, c)] + raw[kR3 + i3(2, 2, c)];
#pragma unroll
  for (int a = 0; a < 3; ++a)
#pragma unroll
    for (int b = a; b < 3; ++b)
#pragma unroll
      for (int c = b; c < 3; ++c)
        q[kQ3 + i3(a, b, c)] = raw[kR3 + i3(a, b, c)] -
                               0.2 * ((a == b ? t[c] : 0.0) + (a == c ? t[b] : 0.0) +
                                      (b == c ? t[a] : 0.0));
  double U[3][3];
#pragma unroll
  for (int a = 0; a < 3; ++a)
#pragma unroll
    for (int b = 0; b < 3; ++b)
      U[a][b] = raw[kR4 + i4(0, 0, a, b)] + raw[kR4 + i4(1, 1, a, b)] + raw[kR4 + i4(2, 2, a, b)];
  const double su = U[0][0] + U[1][1] + U[2][2];
#pragma unroll
  for (int a = 0; a < 3; ++a)
#pragma unroll
    for (int b = a; b < 3; ++b)
#pragma unroll
      for (int c = b; c < 3; ++c)
#pragma unroll
        for (int d = c; d < 3; ++d) {
          const double u6 = (a == b ? U[c][d] : 0.0) + (a == c ? U[b][d] : 0.0) +
                            (a == d ? U[b][c] : 0.0) + (b == c ? U[a][d] : 0.0) +
                            (b == d ? U[a][c] : 0.0) + (c == d ? U[a][b] : 0.0);
          const double dd3 = (double)((a == b && c == d) + (a == c && b == d) + (a == d && b == c));
          q[kQ4 + i4(a, b, c, d)] = raw[kR4 + i4(a, b, c, d)] - u6 / 7.0 + su * dd3 / 35.0;
        }
}

// An empty node stores only its zero mass: readers look at the mass first.
__device__ __forceinline__ void store_node(const PileDev& P, size_t node, double M,
                                           const double c[3], double me1, double me2,
                                           const double* raw) {
  double* o = P.tmom + node * kMom;
  if (M == 0.0) {
    o[0] = 0.0;
    return;
  }
  // stored as computed (the traceless parts straight to memory)
  double* r = P.traw + node * kRaw;
#pragma unroll
  for (int u = 0; u < kRaw; ++u) r[u] = u < 31 ? raw[u] : 0.0;
  o[0] = M;
  o[1] = c[0];
  o[2] = c[1];
  o[3] = c[2];
  o[4] = me1;
  o[5] = me2;
  traceless(raw, o);
  o[37] = o[38] = o[39] = 0.0;
}

// Finest level: moments of node p from the cell's spheres.
__device__ void tree_leaf(const PileDev& P, uint32_t p) {
  const int L = P.bits;
  const Rec64* __restrict__ rec = (const Rec64*)P.jrec;
  const uint32_t s0 = P.cell_start[p], s1 = P.cell_start[p + 1];
  double M = 0.0, mc[3] = {0.0, 0.0, 0.0}, me1 = 0.0, me2 = 0.0;
  for (uint32_t t = s0; t < s1; ++t) {
    const Rec64 r = rec[t];
    M += r.m;
    mc[0] += r.m * r.x;
    mc[1] += r.m * r.y;
    mc[2] += r.m * r.z;
    me1 += r.m * r.e;
    me2 += r.m * r.e * r.e;
  }
  double c[3] = {0.0, 0.0, 0.0}, raw[kRaw];
#pragma unroll
  for (int u = 0; u < kRaw; ++u) raw[u] = 0.0;
  if (M > 0.0) {
    for (int a = 0; a < 3; ++a) c[a] = mc[a] / M;
    for (uint32_t t = s0; t < s1; ++t) {
      const Rec64 r = rec[t];
      const double d[3] = {r.x - c[0], r.y - c[1], r.z - c[2]};
      add_powers(raw, r.m, d);
    }
  }
  store_node(P, level_offset(L) + p, M, c, me1, me2, raw);
}

// Raw moment of a child of mass m: rank 0 is m, rank 1 vanishes about its
// centre of mass.
__device__ __forceinline__ double child_raw(const double* cr, double m, int n, int i, int j) {
  if (n == 0) return m;
  if (n == 1) return 0.0;
  return cr[(n == 2 ? kR2 : (n == 3 ? kR3 : kR4)) + sym_index(n, i, j)];
}
__device__ __forceinline__ double binom(int n, int k) {
  return (k == 0 || k == n) ? 1.0 : (n == 2 ? 2.0 : (n == 3 ? 3.0 : (k == 2 ? 6.0 : 4.0)));
}

// Sum over the eight lanes of an aligned group, in the order
// ((c0 + c1) + (c2 + c3)) + ((c4 + c5) + (c6 + c7)), the same in every lane.
__device__ __forceinline__ double sum8(double v) {
  v += __shfl_xor(v, 1);
  v += __shfl_xor(v, 2);
  v += __shfl_xor(v, 4);
  return v;
}

// Level l < bits: node p from its eight children, child o in lane o of an
// aligned group of eight lanes.  Each child's raw moments are moved from its
// centre of mass to the node's (d -> d + delta: the binomial expansion of
// sum m (d + delta)^n, term by term per exponent), then the eight are summed.
__device__ void tree_up8(const PileDev& P, int l, uint32_t p, int o, bool valid) {
  const size_t child = level_offset(l + 1) + ((size_t)p << 3) + (size_t)o;
  double m = 0.0, co[3] = {0.0, 0.0, 0.0}, e1 = 0.0, e2 = 0.0;
  if (valid) {
    const double* q = P.tmom + child * kMom;
    m = q[0];
    if (m != 0.0) {
      co[0] = q[1];
      co[1] = q[2];
      co[2] = q[3];
      e1 = q[4];
      e2 = q[5];
    }
  }
  const double M = sum8(m);
  const double mc[3] = {sum8(m * co[0]), sum8(m * co[1]), sum8(m * co[2])};
  const double me1 = sum8(e1), me2 = sum8(e2);
  double c[3] = {0.0, 0.0, 0.0}, raw[kRaw];
#pragma unroll
  for (int u = 0; u < kRaw; ++u) raw[u] = 0.0;
  if (M > 0.0)
    for (int a = 0; a < 3; ++a) c[a] = mc[a] / M;
  if (m != 0.0) {
    double cr[kRaw];
    const double* src = P.traw + child * kRaw;
#pragma unroll
    for (int u = 0; u < kRaw; ++u) cr[u] = src[u];
    const double dl[3] = {co[0] - c[0], co[1] - c[1], co[2] - c[2]};
#pragma unroll
    for (int n = 2; n <= 4; ++n) {
      const int off = n == 2 ? kR2 : (n == 3 ? kR3 : kR4);
#pragma unroll
      for (int i = n; i >= 0; --i)
#pragma unroll
        for (int j = n - i; j >= 0; --j) {
          const int k = n - i - j;
          double v = 0.0;
#pragma unroll
          for (int i1 = 0; i1 <= i; ++i1)
#pragma unroll
            for (int j1 = 0; j1 <= j; ++j1)
#pragma unroll
              for (int k1 = 0; k1 <= k; ++k1) {
                const int n1 = i1 + j1 + k1;
                if (n1 == 1) continue;
                v += binom(i, i1) * binom(j, j1) * binom(k, k1) * child_raw(cr, m, n1, i1, j1) *
                     (ipow(dl[0], i - i1) * ipow(dl[1], j - j1) * ipow(dl[2], k - k1));
              }
          raw[off + sym_index(n, i, j)] = v;
        }
    }
  }
#pragma unroll
  for (int u = 0; u < 31; ++u) raw[u] = sum8(raw[u]);
  if (valid && o == 0) store_node(P, level_offset(l) + p, M, c, me1, me2, raw);
}

// Finest level of a pile: one thread per node from its spheres (a block
// covers 256 nodes).  A separate kernel from the levels above, whose eight
// lanes per node need many more registers.
__global__ __launch_bounds__(kBlock) void k_tree_leaf_level(const PileDev* __restrict__ piles,
                                                            const WorkItem* __restrict__ wl, int l) {
  const WorkItem w = wl[blockIdx.x];
  const PileDev& P = piles[w.pile];
  if (P.status != 0 || l != P.bits) return;
  const uint32_t p = (uint32_t)(w.base + threadIdx.x);
  if (p < (1u << (3 * l))) tree_leaf(P, p);
}

// Levels below a pile's finest: eight lanes per node from its children (a
// block covers 32 nodes).
__global__ __launch_bounds__(kBlock) void k_tree_up_level(const PileDev* __restrict__ piles,
                                                          const WorkItem* __restrict__ wl, int l) {
  const WorkItem w = wl[blockIdx.x];
  const PileDev& P = piles[w.pile];
  if (P.status != 0 || l >= P.bits) return;
  const uint32_t p = (uint32_t)w.base + (threadIdx.x >> 3);
  tree_up8(P, l, p, threadIdx.x & 7, p < (1u << (3 * l)));
}

// Pull per unit mass at R = x - c of a node's moments q (uniform over the
// wave), for a sphere of softening half-length ei.  With V_n = Q_n . R^(n-1)
// and S_n = V_n . R, the expansion gives
//   sum_n (2n-1)!!/n! [n V_n / R^(2n+1) - (2n+1) S_n R / R^(2n+3)]  (n = 0, 2.., ORDER)
// and the softening term 3/2 E R / R^5, E = sum m (ei + e)^2.
template <int ORDER>
__device__ __forceinline__ void node_pull(ConstD q, const double R[3], double ei, double c15,
                                          double c1875, double acc[3]) {
  const double r2 = R[0] * R[0] + R[1] * R[1] + R[2] * R[2];
  // inverse powers from the hardware rsqrt estimate y0 and e = 1 - r2 y0^2:
  // r^-2 = y0^2 (1 + e + e^2 + ...), r^-3 = y0^3 (1 + 3e/2 + 15e^2/8 + ...)
  const double y0 = __builtin_amdgcn_rsq(r2);
  const double y2 = y0 * y0;
  const double e = fma(-r2, y2, 1.0);
  const double ir2 = fma(y2, fma(e, e, e), y2);
  const double y3 = y2 * y0;
  const double ir3 = fma(y3 * e, fma(e, c1875, c15), y3);
  const double ir4 = ir2 * ir2, ir5 = ir3 * ir2;
  double V[3], rad;
  {
    // n = 2
#pragma unroll
    for (int a = 0; a < 3; ++a)
      V[a] = q[kQ2 + i2(a, 0)] * R[0] + q[kQ2 + i2(a, 1)] * R[1] + q[kQ2 + i2(a, 2)] * R[2];
    const double S2 = V[0] * R[0] + V[1] * R[1] + V[2] * R[2];
#pragma unroll
    for (int a = 0; a < 3; ++a) V[a] *= 3.0;
    rad = 7.5 * S2;
  }
  if (ORDER >= 4) {
    // the distinct products R_b R_c (b <= c) and R_b R_c R_d (b <= c <= d),
    // each times the number of index orders it stands for
    double w2[6], w3[10];
#pragma unroll
    for (int b = 0; b < 3; ++b)
#pragma unroll
      for (int c = b; c < 3; ++c) {
        w2[i2(b, c)] = R[b] * R[c];
#pragma unroll
        for (int d = c; d < 3; ++d) {
          const double mult = (b == c && c == d) ? 1.0 : ((b == c || c == d) ? 3.0 : 6.0);
          w3[i3(b, c, d)] = mult * (R[b] * R[c]) * R[d];
        }
      }
#pragma unroll
    for (int b = 0; b < 3; ++b)
#pragma unroll
      for (int c = b + 1; c < 3; ++c) w2[i2(b, c)] *= 2.0;
    double V3[3], V4[3];
#pragma unroll
    for (int a = 0; a < 3; ++a) {
      double v3 = 0.0, v4 = 0.0;
#pragma unroll
      for (int b = 0; b < 3; ++b)
#pragma unroll
        for (int c = b; c < 3; ++c) {
          v3 += q[kQ3 + i3(a, b, c)] * w2[i2(b, c)];
#pragma unroll
          for (int d = c; d < 3; ++d) v4 += q[kQ4 + i4(a, b, c, d)] * w3[i3(b, c, d)];
        }
      V3[a] = v3;
      V4[a] = v4;
    }
    const double S3 = V3[0] * R[0] + V3[1] * R[1] + V3[2] * R[2];
    const double S4 = V4[0] * R[0] + V4[1] * R[1] + V4[2] * R[2];
#pragma unroll
    for (int a = 0; a < 3; ++a) V[a] += ir2 * (7.5 * V3[a] + 17.5 * ir2 * V4[a]);
    rad += ir2 * (17.5 * S3 + 39.375 * ir2 * S4);
  }
  const double E = ei * ei * q[0] + 2.0 * ei * q[4] + q[5];
  const double radial = ir3 * (q[0] - 1.5 * E * ir2 + ir4 * rad);
#pragma unroll
  for (int a = 0; a < 3; ++a) acc[a] += ir5 * V[a] - radial * R[a];
}

__device__ __forceinline__ double wave_min(double v) {
  for (int off = 32; off > 0; off >>= 1) v = fmin(v, __shfl_xor(v, off));
  return v;
}
__device__ __forceinline__ double wave_max(double v) {
  for (int off = 32; off > 0; off >>= 1) v = fmax(v, __shfl_xor(v, off));
  return v;
}

// One wave per group of 64 consecutive sorted slots: the group's bounding box.
__global__ __launch_bounds__(kBlock) void k_tree_boxes(const PileDev* __restrict__ piles,
                                                       const WorkItem* __restrict__ wl) {
  const WorkItem w = wl[blockIdx.x];
  const PileDev& P = piles[w.pile];
  if (P.status != 0 || !P.tree || P.G == 0.0) return;
  const int ns = P.ns;
  const int g0 = w.base + (threadIdx.x & ~63);
  if (g0 >= ns) return;
  const int k = w.base + threadIdx.x;
  const bool active = k < ns;
  double x = 0.0, y = 0.0, z = 0.0;
  if (active) {
    const Rec64* r = (const Rec64*)P.jrec + k;
    x = r->x;
    y = r->y;
    z = r->z;
  }
  const double b[6] = {wave_min(active ? x : INFINITY), wave_min(active ? y : INFINITY),
                       wave_min(active ? z : INFINITY), wave_max(active ? x : -INFINITY),
                       wave_max(active ? y : -INFINITY), wave_max(active ? z : -INFINITY)};
  if ((threadIdx.x & 63) == 0)
    for (int a = 0; a < 6; ++a) P.tbox[(size_t)(g0 / 64) * 6 + a] = b[a];
}

// One wave per group of 64 consecutive sorted slots.  The wave walks the
// pyramid from the root with a stack of opened nodes in LDS.  Each pass takes
// up to eight opened nodes off the stack and classifies their 64 children at
// once, one per lane: a child whose cube centre is farther from the group's
// bounding box than side / theta acts through its multipoles, a child of at
// most tree_leaf spheres (or a finest cell) through softened pairs, any other
// child is opened and pushed.  ORDER is the highest multipole order; the
// piles of the other order return at once.
//
// Stack bound: a pass that starts with at most kTreeBatchMax entries pops
// up to 8 and pushes at most 64, ending with at most kTreeBatchMax + 56;
// above kTreeBatchMax a pass pops one node (depth-first), which can add at
// most 7 entries per pyramid level below it (at most 9 levels hold opened
// nodes), so the stack never holds more than kTreeBatchMax + 56 + 63 entries.
constexpr int kTreeBatchMax = 512;
constexpr int kTreeStack = kTreeBatchMax + 56 + 63 + 9;   // 640 node ids per wave
static_assert(kTreeStack >= kTreeBatchMax + 56 + 63, "tree stack bound");

// Every third bit of v (bits 0, 3, 6, ...) packed together: one axis of a
// Morton code of up to ten levels.
__device__ __forceinline__ uint32_t compact3(uint32_t v) {
  v &= 0x09249249u;
  v = (v ^ (v >> 2)) & 0x030c30c3u;
  v = (v ^ (v >> 4)) & 0x0300f00fu;
  v = (v ^ (v >> 8)) & 0xff0000ffu;
  v = (v ^ (v >> 16)) & 0x000003ffu;
  return v;
}

// node id: (1 << 3l) | p, the level in the position of the leading bit
__device__ __forceinline__ int node_level(uint32_t id) { return (31 - __clz(id)) / 3; }

// Softened pulls of the spheres in slots t .. t + N - 1 (uniform) on this
// lane's sphere k, in slot order: all N records are read first (scalar
// loads in flight together), the sphere itself is skipped without a branch.
template <int N>
__device__ __forceinline__ void leaf_pairs(ConstRec64 rec, uint32_t t, double x, double y, double z,
                                           double ei, int k, double c15, double c1875,
                                           double acc[3]) {
  double sx[N], sy[N], sz[N], sm[N], se[N];
#pragma unroll
  for (int u = 0; u < N; ++u) {
    sx[u] = rec[t + u].x;
    sy[u] = rec[t + u].y;
    sz[u] = rec[t + u].z;
    sm[u] = rec[t + u].m;
    se[u] = rec[t + u].e;
  }
#pragma unroll
  for (int u = 0; u < N; ++u) {
    const bool self = t + u == (uint32_t)k;
    const double dx = sx[u] - x, dy = sy[u] - y, dz = sz[u] - z, e = ei + se[u];
    const double r2 = dx * dx + dy * dy + dz * dz + e * e;
    const double c3 = (self ? 0.0 : sm[u]) * inv_cube<true>(self ? 1.0 : r2, c15);
    acc[0] += c3 * dx;
    acc[1] += c3 * dy;
    acc[2] += c3 * dz;
  }
}

// One workgroup of one wave per (group of 64 sorted slots, level-2 subtree).
// Dispatch order, heaviest first on every XCD: workgroups go round-robin to
// the 8 XCDs, each XCD takes an eighth of the groups (contiguous, so their
// trees share its L2), and within an XCD the waves are issued rank by rank:
// rank r of a group walks the subtree whose digits are those of the group's
// own level-2 cube XOR r, so the own cube (the near field, most of the work)
// goes first, then its siblings, then the far octants.  The grid holds
// kTreeParts waves for each of 8 * ceil(groups / 8) groups; padding returns.
template <int ORDER>
__global__ __launch_bounds__(64) void k_tree_walk(const PileDev* __restrict__ piles,
                                                  const WorkItem* __restrict__ wl, int n_items) {
  __shared__ uint32_t stack[kTreeStack];
  const int xcd = blockIdx.x % kXcds, j = blockIdx.x / kXcds;
  const int gx = gridDim.x / kXcds / kTreeParts;   // groups per XCD
  const int rank = j / gx, gi = xcd * gx + j % gx;
  if ((gi >> 2) >= n_items) return;
  WorkItem w = wl[gi >> 2];              // the group: a quarter of a work item's block
  w.base += (gi & 3) * 64;
  const PileDev& P = piles[w.pile];
  if (P.status != 0 || !P.tree || P.G == 0.0 || P.tree_order != ORDER) return;
  const int ns = P.ns, L = P.bits;
  if (w.base >= ns) return;
  int part = rank;                       // the level-2 subtree this wave walks (octal digits)
  static_assert(kTreeSplit == 2, "the rank order below reads two digits");
  {
    // the level-1 and level-2 digits of the cell of the group's first sphere
    // (a tree pile has at least two levels)
    const Rec64* r0 = (const Rec64*)P.jrec + w.base;
    const double xyz[3] = {r0->x, r0->y, r0->z};
    const Grid& g0 = *P.grid;
    int d1 = 0, d2 = 0;
    for (int a = 0; a < 3; ++a) {
      const int c = cell_coord(xyz[a], g0.lo[a], g0.inv_cell, 1 << L, 0, 0.0);
      d1 |= ((c >> (L - 1)) & 1) << a;
      d2 |= ((c >> (L - 2)) & 1) << a;
    }
    part = ((d1 << 3) | d2) ^ rank;
  }
  const int lane = threadIdx.x;
  const int k = w.base + lane;
  const bool active = k < ns;
  const ConstRec64 rec = (ConstRec64)P.jrec;
  const ConstU cstart = (ConstU)P.cell_start;
  const ConstD mom = (ConstD)P.tmom;
  const Grid& g = *P.grid;
  const double cell = g.cell, theta = P.theta;
  double x = 0.0, y = 0.0, z = 0.0, ei = 0.0;
  if (active) {
    const Rec64* r = (const Rec64*)P.jrec + k;
    x = r->x;
    y = r->y;
    z = r->z;
    ei = r->e;
  }
  const ConstD box = (ConstD)P.tbox + (size_t)(w.base / 64) * 6;
  const double bmin[3] = {box[0], box[1], box[2]};
  const double bmax[3] = {box[3], box[4], box[5]};
  double acc[3] = {0.0, 0.0, 0.0};
  double c15, c1875;
  series_coeffs(c15, c1875);
  int sp = 0;
  {
    // the root is never accepted (the group lies inside it and theta <= 1);
    // a root with few spheres is one set of pairs (part 0's wave), else it
    // is opened; above level 2 each wave follows only its own digits
    const uint32_t n0 = cstart[(size_t)1 << (3 * L)] - cstart[0];
    if (n0 <= (uint32_t)P.tree_leaf) {
      if (part == 0)
        for (uint32_t t = cstart[0]; t < cstart[(size_t)1 << (3 * L)]; ++t)
          leaf_pairs<1>(rec, t, x, y, z, ei, k, c15, c1875, acc);
    } else {
      if (lane == 0) stack[0] = 1u;    // the root: level 0, prefix 0
      sp = 1;
    }
  }
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  while (sp > 0) {
    const int nb = sp > kTreeBatchMax ? 1 : min(sp, 8);
    const int slot = lane >> 3;
    const bool valid = slot < nb;
    const uint32_t id = valid ? stack[sp - 1 - slot] : 1u;
    sp -= nb;
    // lane (slot, c) classifies child c of the slot-th node off the top
    const int lp = node_level(id);
    const uint32_t pp = id ^ (1u << (3 * lp));
    const int l = lp + 1;
    const int sh = 3 * (L - l);
    const uint32_t p = (pp << 3) | (uint32_t)(lane & 7);
    uint32_t t0 = 0, t1 = 0;
    int kind = 0;                        // 0 empty, 1 multipole, 2 pairs, 3 open
    if (valid) {
      t0 = cstart[(size_t)p << sh];
      t1 = cstart[(size_t)(p + 1) << sh];
      if (t1 > t0) {
        const double side = ldexp(cell, L - l);
        const uint32_t ix[3] = {compact3(p), compact3(p >> 1), compact3(p >> 2)};
        double dd[3];
        for (int a = 0; a < 3; ++a) {
          const double ctr = rn_add(g.lo[a], rn_mul((double)ix[a] + 0.5, side));
          dd[a] = fmax(fmax(rn_add(bmin[a], -ctr), rn_add(ctr, -bmax[a])), 0.0);
        }
        const double dist2 = rn_add(rn_add(rn_mul(dd[0], dd[0]), rn_mul(dd[1], dd[1])),
                                       rn_mul(dd[2], dd[2]));
        const double thr = side / theta;
        if (dist2 > rn_mul(thr, thr)) kind = 1;
        else if (t1 - t0 <= (uint32_t)P.tree_leaf || l == L) kind = 2;
        else kind = 3;
      }
      if (lp < kTreeSplit) {
        // above the split: only this wave's child; a child that is not
        // opened there is handled by the wave whose lower digits are zero
        const int digit = (part >> (3 * (kTreeSplit - 1 - lp))) & 7;
        const int lower = part & ((1 << (3 * (kTreeSplit - 1 - lp))) - 1);
        if ((lane & 7) != digit || (kind != 3 && lower != 0)) kind = 0;
      }
    }
    // multipoles: each accepted child's moments, read by the whole wave
    {
      const uint32_t nidx = (uint32_t)level_offset(l) + p;
      uint64_t mask = __ballot(kind == 1);
      while (mask) {
        const int b = __builtin_ctzll(mask);
        mask &= mask - 1;
        const uint32_t nb_idx = (uint32_t)__builtin_amdgcn_readlane((int)nidx, b);
        const ConstD q = mom + (size_t)nb_idx * kMom;
        const double R[3] = {x - q[1], y - q[2], z - q[3]};
        node_pull<ORDER>(q, R, ei, c15, c1875, acc);
      }
    }
    // pairs: each leaf child's spheres in slot order, read by the whole wave
    // (uniform addresses: scalar loads, four sources in flight)
    {
      uint64_t lm = __ballot(kind == 2);
      while (lm) {
        const int b = __builtin_ctzll(lm);
        lm &= lm - 1;
        const uint32_t s0 = (uint32_t)__builtin_amdgcn_readlane((int)t0, b);
        const uint32_t s1 = (uint32_t)__builtin_amdgcn_readlane((int)t1, b);
        uint32_t t = s0;
        for (; t + 4 <= s1; t += 4) leaf_pairs<4>(rec, t, x, y, z, ei, k, c15, c1875, acc);
        for (; t < s1; ++t) leaf_pairs<1>(rec, t, x, y, z, ei, k, c15, c1875, acc);
      }
    }
    // opened children go on the stack in lane order
    {
      const uint64_t om = __ballot(kind == 3);
      if (kind == 3) {
        const int rank = __builtin_popcountll(om & ((1ull << lane) - 1ull));
        stack[sp + rank] = (1u << (3 * l)) | p;
      }
      sp += __builtin_popcountll(om);
    }
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
  }
  // this subtree's part of the sum, by slot
  if (active)
    for (int a = 0; a < 3; ++a) P.tpart[((size_t)part * 3 + a) * ns + k] = acc[a];
}

// One thread per sorted slot: the subtree parts in order, G m_i, and the
// perturber's pull, exactly as the direct path's combine.
__global__ __launch_bounds__(kBlock) void k_tree_combine(const PileDev* __restrict__ piles,
                                                         const WorkItem* __restrict__ wl) {
  const WorkItem w = wl[blockIdx.x];
  const PileDev& P = piles[w.pile];
  if (P.status != 0 || !P.tree || P.G == 0.0) return;
  const int ns = P.ns;
  const int k = w.base + threadIdx.x;
  double pull[3] = {0.0, 0.0, 0.0};
  if (k < ns) {
    double acc[3] = {0.0, 0.0, 0.0};
    for (int o = 0; o < kTreeParts; ++o)
      for (int a = 0; a < 3; ++a) acc[a] += P.tpart[((size_t)o * 3 + a) * ns + k];
    const uint32_t i = P.sidx[k];
    const double gm = P.G * P.m[i];
    for (int a = 0; a < 3; ++a) acc[a] *= gm;
    if (P.pert_on) {
      const int nxt = P.parity ^ 1;
      const double d[3] = {P.pert_r[nxt][0] - P.xs[k], P.pert_r[nxt][1] - P.xs[ns + k],
                           P.pert_r[nxt][2] - P.xs[2 * ns + k]};
      const double r2 = d[0] * d[0] + d[1] * d[1] + d[2] * d[2];
      const double f = gm * P.pert_M / (r2 * sqrt(r2));
      for (int a = 0; a < 3; ++a) {
        pull[a] = f * d[a];
        acc[a] += pull[a];
      }
    }
    for (int a = 0; a < 3; ++a) P.gacc[a * ns + i] = acc[a];
  }
  if (!P.pert_on) return;
  for (int off = 32; off > 0; off >>= 1)
    for (int a = 0; a < 3; ++a) pull[a] += __shfl_xor(pull[a], off);
  __shared__ double red[4][3];
  const int wave = threadIdx.x >> 6;
  if ((threadIdx.x & 63) == 0)
    for (int a = 0; a < 3; ++a) red[wave][a] = pull[a];
  __syncthreads();
  if (threadIdx.x == 0)
    for (int a = 0; a < 3; ++a)
      P.ppart[(w.base / kBlock) * 3 + a] = ((red[0][a] + red[1][a]) + red[2][a]) + red[3][a];
}
}  // namespace

void launch_tree(hipStream_t st, const PileDev* piles, WorkItem* const* wl_level,
                 const int* n_level, unsigned leaf_levels, const WorkItem* wl_sph, int n_sph_blk,
                 const bool* any_order) {
  for (int l = 10; l >= 0; --l) {
    if (n_level[l] <= 0) continue;
    if (leaf_levels >> l & 1u)
      hipLaunchKernelGGL(k_tree_leaf_level, dim3(n_level[l]), dim3(kBlock), 0, st, piles,
                         wl_level[l], l);
    if ((leaf_levels >> (l + 1)) != 0u)   // some pile is deeper than l
      hipLaunchKernelGGL(k_tree_up_level, dim3(n_level[l]), dim3(kBlock), 0, st, piles,
                         wl_level[l], l);
  }
  // four groups per work item, padded to a multiple of the XCD count
  const int walk_blocks = ((n_sph_blk * 4 + kXcds - 1) / kXcds) * kXcds * kTreeParts;
  hipLaunchKernelGGL(k_tree_boxes, dim3(n_sph_blk), dim3(kBlock), 0, st, piles, wl_sph);
  if (any_order[0])
    hipLaunchKernelGGL(k_tree_walk<2>, dim3(walk_blocks), dim3(64), 0, st, piles, wl_sph,
                       n_sph_blk);
  if (any_order[1])
    hipLaunchKernelGGL(k_tree_walk<4>, dim3(walk_blocks), dim3(64), 0, st, piles, wl_sph,
                       n_sph_blk);
  hipLaunchKernelGGL(k_tree_combine, dim3(n_sph_blk), dim3(kBlock), 0, st, piles, wl_sph);
}

}  // namespace dem
