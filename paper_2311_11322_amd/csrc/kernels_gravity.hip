// kernels_gravity.hip -- softened all-pairs self-gravity (Eq. 4 of the
// paper, with Plummer softening eps_ij = soft_frac (s_i + s_j) / 2).
//
// Spheres are taken in cell-sorted (Morton) order and cut into tiles of B
// slots.  One wave computes one tile pair (I, J), I <= J, so every unordered
// pair of spheres is evaluated once (Newton's third law):
//  * each lane holds IPT targets of tile I in registers;
//  * the sources of tile J enter 64 at a time, one per lane, together with
//    a reaction accumulator, and rotate one lane per step (DPP wave_ror:1)
//    so that after 64 steps every source has met every target of the wave
//    and is back in its own lane holding its complete reaction sum;
//  * a diagonal pair (I, I) evaluates the ordered pairs i != j one way only,
//    with the sources walked by a uniform index (scalar loads).
// Each sphere receives exactly one partial sum per tile (its own tile's row
// or column), stored per tile; the combine kernel adds them in tile order,
// so the result is deterministic and independent of other piles.
//
// FP64 form: rsqrt from the hardware estimate y0 and one third-order
// correction folded into the cube: r^-3 = y0^3 (1 + 3e/2 + 15e^2/8),
// e = 1 - r^2 y0^2.  FP32-force form: coordinates relative to an FP64 anchor
// per tile (the first sphere of the tile); the tile-pair anchor offset is
// formed in FP64 once per block; FP32 partial sums per tile, FP64 across
// tiles.
#include "dem_internal.h"

namespace dem {

namespace {

struct alignas(64) Rec64 {
  double x, y, z, m, e, p0, p1, p2;
};
struct alignas(32) Rec32 {
  float x, y, z, m, e, p0, p1, p2;
};

// Records are read through the constant address space: with a uniform index
// these become scalar loads into SGPRs.
typedef const __attribute__((address_space(4))) Rec64* ConstRec64;
typedef const __attribute__((address_space(4))) Rec32* ConstRec32;

// One thread per sorted slot: the source record of the sphere in that slot.
__global__ __launch_bounds__(kBlock) void k_grav_records(const PileDev* __restrict__ piles,
                                                         const WorkItem* __restrict__ wl,
                                                         int precision) {
  const WorkItem w = wl[blockIdx.x];
  const PileDev& P = piles[w.pile];
  const int k = w.base + threadIdx.x;
  if (k >= P.ns || P.status != 0 || P.G == 0.0) return;
  const int ns = P.ns;
  const double x = P.xs[k], y = P.xs[ns + k], z = P.xs[2 * ns + k];
  const double e = 0.5 * P.soft_frac * P.xs[3 * ns + k];
  const double m = P.m[P.sidx[k]];
  if (precision == 1 && !P.tree) {
    const int a = (k / P.g_tile) * P.g_tile;
    const double ax = P.xs[a], ay = P.xs[ns + a], az = P.xs[2 * ns + a];
    Rec32 r;
    r.x = (float)(x - ax);
    r.y = (float)(y - ay);
    r.z = (float)(z - az);
    r.m = (float)m;
    r.e = (float)e;
    r.p0 = r.p1 = r.p2 = 0.f;
    ((Rec32*)P.jrec)[k] = r;
    if (k == a) {
      double* an = P.ganchor + (size_t)(k / P.g_tile) * 4;
      an[0] = ax;
      an[1] = ay;
      an[2] = az;
      an[3] = 0.0;
    }
  } else {
    Rec64 r;
    r.x = x;
    r.y = y;
    r.z = z;
    r.m = m;
    r.e = e;
    r.p0 = r.p1 = r.p2 = 0.0;
    ((Rec64*)P.jrec)[k] = r;
  }
}

// Rotate a value by one lane across the whole wave (DPP wave_ror:1): after
// 64 rotations every value is back in its own lane.
__device__ __forceinline__ float ror1(float v) {
  return __int_as_float(__builtin_amdgcn_mov_dpp(__float_as_int(v), 0x13C, 0xF, 0xF, true));
}
__device__ __forceinline__ double ror1(double v) {
  const long long b = __double_as_longlong(v);
  const int lo = __builtin_amdgcn_mov_dpp((int)(b & 0xffffffff), 0x13C, 0xF, 0xF, true);
  const int hi = __builtin_amdgcn_mov_dpp((int)(b >> 32), 0x13C, 0xF, 0xF, true);
  return __longlong_as_double(((long long)hi << 32) | (unsigned int)lo);
}

// Series coefficients of the rsqrt correction, read from memory so that the
// compiler keeps them in registers instead of re-materialising literals.
__constant__ double kSeries[2] = {1.5, 1.875};

// r^-3 of a softened squared distance, FP64.
template <bool SOFT>
__device__ __forceinline__ double inv_cube(double r2, double c15, double c1875) {
  const double y = __builtin_amdgcn_rsq(r2);
  const double y2 = y * y;
  const double e = fma(-r2, y2, 1.0);
  const double p = fma(e, c1875, c15);
  const double y3 = y2 * y;
  const double c3 = fma(y3 * e, p, y3);
  if (!SOFT) return r2 > 0.0 ? c3 : 0.0;
  return c3;
}

template <bool SOFT>
__device__ __forceinline__ float inv_cube(float r2, double, double) {
  const float y = __builtin_amdgcn_rsqf(r2);
  const float c3 = (y * y) * y;
  if (!SOFT) return r2 > 0.f ? c3 : 0.f;
  return c3;
}

template <typename T, int IPT, bool SOFT>
__global__ __launch_bounds__(64) void k_grav_tiles(const PileDev* __restrict__ piles,
                                                   const GravItem* __restrict__ gl) {
  constexpr int B = 64 * IPT;
  constexpr bool F32 = sizeof(T) == 4;
  const GravItem it = gl[blockIdx.x];
  const PileDev& P = piles[it.pile];
  if (P.status != 0) return;
  const int ns = P.ns, lane = threadIdx.x;
  const int i0 = it.ti * B, j0 = it.tj * B;
  const int j1 = min(j0 + B, ns);
  const bool diag = it.ti == it.tj;
  const double c15 = kSeries[0], c1875 = kSeries[1];

  // tile-pair anchor offset (FP32 form): d = (x_j - A_J) - ((x_i - A_I) - (A_J - A_I))
  T sx = 0, sy = 0, sz = 0;
  if (F32) {
    const double* aI = P.ganchor + (size_t)it.ti * 4;
    const double* aJ = P.ganchor + (size_t)it.tj * 4;
    sx = (T)(aJ[0] - aI[0]);
    sy = (T)(aJ[1] - aI[1]);
    sz = (T)(aJ[2] - aI[2]);
  }

  T xi[IPT], yi[IPT], zi[IPT], ei[IPT], mi[IPT], ax[IPT], ay[IPT], az[IPT];
#pragma unroll
  for (int u = 0; u < IPT; ++u) {
    const int k = i0 + u * 64 + lane;
    const int kk = k < ns ? k : ns - 1;
    if (F32) {
      const Rec32 r = ((const Rec32*)P.jrec)[kk];
      xi[u] = (T)r.x - sx;
      yi[u] = (T)r.y - sy;
      zi[u] = (T)r.z - sz;
      ei[u] = (T)r.e;
      mi[u] = k < ns ? (T)r.m : (T)0;
    } else {
      const Rec64 r = ((const Rec64*)P.jrec)[kk];
      xi[u] = (T)r.x;
      yi[u] = (T)r.y;
      zi[u] = (T)r.z;
      ei[u] = (T)r.e;
      mi[u] = k < ns ? (T)r.m : (T)0;
    }
    ax[u] = ay[u] = az[u] = (T)0;
  }

  T* __restrict__ part = (T*)P.gpart;
  if (diag) {
    // ordered pairs inside one tile, one way only; sources via scalar loads
    for (int j = j0; j < j1; ++j) {
      T xj, yj, zj, mj, ej;
      if (F32) {
        const ConstRec32 cr = (ConstRec32)P.jrec;
        xj = cr[j].x;
        yj = cr[j].y;
        zj = cr[j].z;
        mj = cr[j].m;
        ej = cr[j].e;
      } else {
        const ConstRec64 cr = (ConstRec64)P.jrec;
        xj = (T)cr[j].x;
        yj = (T)cr[j].y;
        zj = (T)cr[j].z;
        mj = (T)cr[j].m;
        ej = (T)cr[j].e;
      }
#pragma unroll
      for (int u = 0; u < IPT; ++u) {
        const T dx = xj - xi[u], dy = yj - yi[u], dz = zj - zi[u];
        const T t = ei[u] + ej;
        const T r2 = fma(dx, dx, fma(dy, dy, fma(dz, dz, t * t)));
        const T w = mj * inv_cube<SOFT>(r2, c15, c1875);
        ax[u] = fma(w, dx, ax[u]);
        ay[u] = fma(w, dy, ay[u]);
        az[u] = fma(w, dz, az[u]);
      }
    }
  } else {
    // sources of tile J travel around the wave 64 at a time, each carrying
    // its own reaction sum; after 64 one-lane rotations it is back home
    for (int jc = j0; jc < j1; jc += 64) {
      const int jx = jc + lane;
      const int jk = jx < j1 ? jx : j1 - 1;
      T xj, yj, zj, mj, ej;
      if (F32) {
        const Rec32 r = ((const Rec32*)P.jrec)[jk];
        xj = r.x;
        yj = r.y;
        zj = r.z;
        mj = jx < j1 ? r.m : 0.f;
        ej = r.e;
      } else {
        const Rec64 r = ((const Rec64*)P.jrec)[jk];
        xj = (T)r.x;
        yj = (T)r.y;
        zj = (T)r.z;
        mj = jx < j1 ? (T)r.m : (T)0;
        ej = (T)r.e;
      }
      T bx = 0, by = 0, bz = 0;
      for (int step = 0; step < 64; ++step) {
#pragma unroll
        for (int u = 0; u < IPT; ++u) {
          const T dx = xj - xi[u], dy = yj - yi[u], dz = zj - zi[u];
          const T t = ei[u] + ej;
          const T r2 = fma(dx, dx, fma(dy, dy, fma(dz, dz, t * t)));
          const T c3 = inv_cube<SOFT>(r2, c15, c1875);
          const T wi = mj * c3, wj = mi[u] * c3;
          ax[u] = fma(wi, dx, ax[u]);
          ay[u] = fma(wi, dy, ay[u]);
          az[u] = fma(wi, dz, az[u]);
          bx = fma(wj, dx, bx);
          by = fma(wj, dy, by);
          bz = fma(wj, dz, bz);
        }
        xj = ror1(xj);
        yj = ror1(yj);
        zj = ror1(zj);
        mj = ror1(mj);
        ej = ror1(ej);
        bx = ror1(bx);
        by = ror1(by);
        bz = ror1(bz);
      }
      if (jx < j1) {
        part[((size_t)it.ti * 3 + 0) * ns + jx] = -bx;
        part[((size_t)it.ti * 3 + 1) * ns + jx] = -by;
        part[((size_t)it.ti * 3 + 2) * ns + jx] = -bz;
      }
    }
  }
  // targets of tile I store under "other tile" J (J = I on the diagonal)
#pragma unroll
  for (int u = 0; u < IPT; ++u) {
    const int k = i0 + u * 64 + lane;
    if (k < ns) {
      part[((size_t)it.tj * 3 + 0) * ns + k] = ax[u];
      part[((size_t)it.tj * 3 + 1) * ns + k] = ay[u];
      part[((size_t)it.tj * 3 + 2) * ns + k] = az[u];
    }
  }
}

// One thread per sorted slot: add the per-tile partials in tile order (FP64)
// and store the gravity force G m_i sum under the sphere's id.  With a
// perturber, its unsoftened pull G m_i M d/|d|^3 is added (FP64) and each
// block stores the sum of its spheres' pulls (the reaction, reduced in block
// order at the end of the step).
template <typename T>
__global__ __launch_bounds__(kBlock) void k_grav_combine(const PileDev* __restrict__ piles,
                                                         const WorkItem* __restrict__ wl) {
  const WorkItem w = wl[blockIdx.x];
  const PileDev& P = piles[w.pile];
  if (P.status != 0 || P.G == 0.0 || P.tree) return;
  const int k = w.base + threadIdx.x;
  const int ns = P.ns, nt = P.g_nt;
  double pull[3] = {0.0, 0.0, 0.0};
  if (k < ns) {
    const T* __restrict__ part = (const T*)P.gpart;
    double g[3] = {0.0, 0.0, 0.0};
    for (int t = 0; t < nt; ++t)
      for (int c = 0; c < 3; ++c) g[c] += (double)part[((size_t)t * 3 + c) * ns + k];
    const uint32_t i = P.sidx[k];
    const double gm = P.G * P.m[i];
    for (int c = 0; c < 3; ++c) g[c] *= gm;
    if (P.pert_on) {
      const int nxt = P.parity ^ 1;
      const double d[3] = {P.pert_r[nxt][0] - P.xs[k], P.pert_r[nxt][1] - P.xs[ns + k],
                           P.pert_r[nxt][2] - P.xs[2 * ns + k]};
      const double r2 = d[0] * d[0] + d[1] * d[1] + d[2] * d[2];
      const double f = gm * P.pert_M / (r2 * sqrt(r2));
      for (int c = 0; c < 3; ++c) {
        pull[c] = f * d[c];
        g[c] += pull[c];
      }
    }
    for (int c = 0; c < 3; ++c) P.gacc[c * ns + i] = g[c];
  }
  if (!P.pert_on) return;
  // block sum of the pulls (fixed order: wave butterflies, then waves 0..3)
  for (int off = 32; off > 0; off >>= 1)
    for (int c = 0; c < 3; ++c) pull[c] += __shfl_xor(pull[c], off);
  __shared__ double red[4][3];
  const int wave = threadIdx.x >> 6;
  if ((threadIdx.x & 63) == 0)
    for (int c = 0; c < 3; ++c) red[wave][c] = pull[c];
  __syncthreads();
  if (threadIdx.x == 0)
    for (int c = 0; c < 3; ++c)
      P.ppart[(w.base / kBlock) * 3 + c] = ((red[0][c] + red[1][c]) + red[2][c]) + red[3][c];
}


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

constexpr int kTreeStack = 96;     // nodes waiting per wave (depth <= 7 * 10 + 1)
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

__device__ __forceinline__ void store_node(const PileDev& P, size_t node, double M,
                                           const double c[3], double me1, double me2,
                                           const double* raw) {
  double q[kMom];
#pragma unroll
  for (int u = 0; u < kMom; ++u) q[u] = 0.0;
  q[0] = M;
  q[1] = c[0];
  q[2] = c[1];
  q[3] = c[2];
  q[4] = me1;
  q[5] = me2;
  traceless(raw, q);
  double* o = P.tmom + node * kMom;
#pragma unroll
  for (int u = 0; u < kMom; ++u) o[u] = q[u];
  double* r = P.traw + node * kRaw;
#pragma unroll
  for (int u = 0; u < kRaw; ++u) r[u] = u < 31 ? raw[u] : 0.0;
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

// Level l < bits: node p from its eight children in order.  Each child's raw
// moments are moved from its centre of mass to the node's (d -> d + delta:
// the binomial expansion of sum m (d + delta)^n, term by term per exponent).
__device__ void tree_up(const PileDev& P, int l, uint32_t p) {
  const size_t first = level_offset(l + 1) + ((size_t)p << 3);
  const double* ch = P.tmom + first * kMom;
  const double* chr = P.traw + first * kRaw;
  double M = 0.0, mc[3] = {0.0, 0.0, 0.0}, me1 = 0.0, me2 = 0.0;
  for (int o = 0; o < 8; ++o) {
    const double m = ch[o * kMom];
    M += m;
    for (int a = 0; a < 3; ++a) mc[a] += m * ch[o * kMom + 1 + a];
    me1 += ch[o * kMom + 4];
    me2 += ch[o * kMom + 5];
  }
  double c[3] = {0.0, 0.0, 0.0}, raw[kRaw];
#pragma unroll
  for (int u = 0; u < kRaw; ++u) raw[u] = 0.0;
  if (M > 0.0) {
    for (int a = 0; a < 3; ++a) c[a] = mc[a] / M;
    for (int o = 0; o < 8; ++o) {
      const double* q = ch + o * kMom;
      const double m = q[0];
      if (m == 0.0) continue;
      const double* cr = chr + o * kRaw;
      const double dl[3] = {q[1] - c[0], q[2] - c[1], q[3] - c[2]};
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
                  v += binom(i, i1) * binom(j, j1) * binom(k, k1) *
                       child_raw(cr, m, n1, i1, j1) *
                       (ipow(dl[0], i - i1) * ipow(dl[1], j - j1) * ipow(dl[2], k - k1));
                }
            raw[off + sym_index(n, i, j)] += v;
          }
      }
    }
  }
  store_node(P, level_offset(l) + p, M, c, me1, me2, raw);
}

// One thread per node of level l of every tree pile: finest-level moments
// from spheres where l is the pile's depth, else from the level below.
__global__ __launch_bounds__(kBlock) void k_tree_level(const PileDev* __restrict__ piles,
                                                       const WorkItem* __restrict__ wl, int l) {
  const WorkItem w = wl[blockIdx.x];
  const PileDev& P = piles[w.pile];
  if (P.status != 0 || l > P.bits) return;
  const uint32_t p = (uint32_t)(w.base + threadIdx.x);
  if (p >= (1u << (3 * l))) return;
  if (l == P.bits) tree_leaf(P, p);
  else tree_up(P, l, p);
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
    // R_b R_c for b <= c, off-diagonal ones doubled (they occur twice)
    double w2[6];
#pragma unroll
    for (int b = 0; b < 3; ++b)
#pragma unroll
      for (int c = b; c < 3; ++c) w2[i2(b, c)] = (b == c ? 1.0 : 2.0) * R[b] * R[c];
    double V3[3], V4[3];
#pragma unroll
    for (int a = 0; a < 3; ++a) {
      double v3 = 0.0, v4 = 0.0;
#pragma unroll
      for (int b = 0; b < 3; ++b) {
        double tab = 0.0;
#pragma unroll
        for (int c = 0; c < 3; ++c)
#pragma unroll
          for (int d = c; d < 3; ++d) tab += q[kQ4 + i4(a, b, c, d)] * w2[i2(c, d)];
        v4 += tab * R[b];
      }
#pragma unroll
      for (int b = 0; b < 3; ++b)
#pragma unroll
        for (int c = b; c < 3; ++c) v3 += q[kQ3 + i3(a, b, c)] * w2[i2(b, c)];
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

// A double held by lane c, in every lane.
__device__ __forceinline__ double bcast(double v, int c) {
  const long long b = __double_as_longlong(v);
  const int lo = __builtin_amdgcn_readlane((int)(b & 0xffffffff), c);
  const int hi = __builtin_amdgcn_readlane((int)(b >> 32), c);
  return __longlong_as_double(((long long)hi << 32) | (unsigned int)lo);
}

// One wave per group of 64 consecutive sorted slots.  The wave walks the
// pyramid from the root with a stack in LDS; every decision is uniform over
// the wave: a node whose cube centre is farther from the group's bounding box
// than side / theta acts through its multipoles, a node of at most tree_leaf
// spheres (or a finest cell) through softened pairs, any other node is
// opened.  ORDER is the highest multipole order; the piles of the other
// order return at once.
template <int ORDER>
__global__ __launch_bounds__(kBlock) void k_tree_walk(const PileDev* __restrict__ piles,
                                                      const WorkItem* __restrict__ wl) {
  __shared__ uint64_t stack[kBlock / 64][kTreeStack];
  const int blk = xcd_block(blockIdx.x, gridDim.x);
  const WorkItem w = wl[blk / kTreeParts];
  const int part = blk % kTreeParts;     // the level-2 subtree this block walks (octal digits)
  const PileDev& P = piles[w.pile];
  if (P.status != 0 || !P.tree || P.G == 0.0 || P.tree_order != ORDER) return;
  const int ns = P.ns, L = P.bits;
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int k = w.base + threadIdx.x;
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
  const double bmin[3] = {wave_min(active ? x : INFINITY), wave_min(active ? y : INFINITY),
                          wave_min(active ? z : INFINITY)};
  const double bmax[3] = {wave_max(active ? x : -INFINITY), wave_max(active ? y : -INFINITY),
                          wave_max(active ? z : -INFINITY)};
  double acc[3] = {0.0, 0.0, 0.0};
  const double c15 = kSeries[0], c1875 = kSeries[1];
  const bool any = w.base + wave * 64 < ns;
  // softened pairs with the spheres of slots [t0, t1) (uniform)
  auto pairs = [&](uint32_t t0, uint32_t t1) {
    for (uint32_t t = t0; t < t1; ++t) {
      const double dx = rec[t].x - x, dy = rec[t].y - y, dz = rec[t].z - z, e = ei + rec[t].e;
      const double r2 = dx * dx + dy * dy + dz * dz + e * e;
      const double c3 = (t == (uint32_t)k) ? 0.0 : rec[t].m * inv_cube<true>(r2, c15, c1875);
      acc[0] += c3 * dx;
      acc[1] += c3 * dy;
      acc[2] += c3 * dz;
    }
  };
  int sp = 0;
  if (any) {
    // the root is never accepted (the group lies inside it and theta <= 1);
    // a root with few spheres is one set of pairs (part 0's block), else it
    // is opened; above level 2 each block follows only its own digits
    const uint32_t n0 = cstart[(size_t)1 << (3 * L)] - cstart[0];
    if (n0 <= (uint32_t)P.tree_leaf) {
      if (part == 0) pairs(cstart[0], cstart[(size_t)1 << (3 * L)]);
    } else {
      stack[wave][sp++] = 0;             // (level 0, prefix 0)
    }
  }
  while (sp > 0) {
    const uint64_t nd = stack[wave][--sp];
    // the stack is the wave's: make the node id uniform
    const int lp = __builtin_amdgcn_readfirstlane((int)(nd >> 32));
    const uint32_t pp = (uint32_t)__builtin_amdgcn_readfirstlane((int)(uint32_t)nd);
    // lanes 0..7 classify the eight children of the opened node at once
    const int l = lp + 1;
    const int sh = 3 * (L - l);
    const double side = ldexp(cell, L - l);
    const uint32_t p = (pp << 3) | (uint32_t)(lane & 7);
    uint32_t t0 = 0, t1 = 0;
    int kind = 0;                        // 0 empty, 1 multipole, 2 pairs, 3 open
    if (lane < 8) {
      t0 = P.cell_start[(size_t)p << sh];
      t1 = P.cell_start[(size_t)(p + 1) << sh];
      if (t1 > t0) {
        uint32_t ix[3] = {0u, 0u, 0u};
        for (int b = 0; b < l; ++b)
          for (int a = 0; a < 3; ++a) ix[a] |= ((p >> (3 * b + a)) & 1u) << b;
        double dd[3];
        for (int a = 0; a < 3; ++a) {
          const double ctr = __dadd_rn(g.lo[a], __dmul_rn((double)ix[a] + 0.5, side));
          dd[a] = fmax(fmax(__dadd_rn(bmin[a], -ctr), __dadd_rn(ctr, -bmax[a])), 0.0);
        }
        const double dist2 = __dadd_rn(__dadd_rn(__dmul_rn(dd[0], dd[0]), __dmul_rn(dd[1], dd[1])),
                                       __dmul_rn(dd[2], dd[2]));
        const double thr = side / theta;
        if (dist2 > __dmul_rn(thr, thr)) kind = 1;
        else if (t1 - t0 <= (uint32_t)P.tree_leaf || l == L) kind = 2;
        else kind = 3;
      }
      if (lp < kTreeSplit) {
        // above the split: only this block's child; a child that is not
        // opened there is handled by the block whose lower digits are zero
        const int digit = (part >> (3 * (kTreeSplit - 1 - lp))) & 7;
        const int lower = part & ((1 << (3 * (kTreeSplit - 1 - lp))) - 1);
        if (lane != digit || (kind != 3 && lower != 0)) kind = 0;
      }
    }
    // multipoles: each accepted child's moments, read by the whole wave
    for (int c = 0; c < 8; ++c) {
      if (__builtin_amdgcn_readlane(kind, c) == 1) {
        const ConstD q = mom + (level_offset(l) + ((pp << 3) | (uint32_t)c)) * kMom;
        const double R[3] = {x - q[1], y - q[2], z - q[3]};
        node_pull<ORDER>(q, R, ei, c15, c1875, acc);
      }
    }
    // pairs: the leaf children's spheres, concatenated and loaded 64 at a time
    // (one per lane), then broadcast one by one
    {
      uint32_t pre[8], cnt[8], beg[8], total = 0;
      for (int c = 0; c < 8; ++c) {
        const bool leafc = __builtin_amdgcn_readlane(kind, c) == 2;
        beg[c] = (uint32_t)__builtin_amdgcn_readlane((int)t0, c);
        cnt[c] = leafc ? (uint32_t)__builtin_amdgcn_readlane((int)t1, c) - beg[c] : 0u;
        pre[c] = total;
        total += cnt[c];
      }
      for (uint32_t b0 = 0; b0 < total; b0 += 64) {
        const uint32_t f = b0 + (uint32_t)lane;
        uint32_t ts = 0;
        for (int c = 0; c < 8; ++c)
          if (f >= pre[c] && f < pre[c] + cnt[c]) ts = beg[c] + (f - pre[c]);
        double sx = 0.0, sy = 0.0, sz = 0.0, sm = 0.0, se = 0.0;
        if (f < total) {
          const Rec64* r = (const Rec64*)P.jrec + ts;
          sx = r->x;
          sy = r->y;
          sz = r->z;
          sm = r->m;
          se = r->e;
        }
        const int nb = (int)min(64u, total - b0);
        for (int j = 0; j < nb; ++j) {
          const uint32_t tj = (uint32_t)__builtin_amdgcn_readlane((int)ts, j);
          const double dx = bcast(sx, j) - x, dy = bcast(sy, j) - y, dz = bcast(sz, j) - z;
          const double e = ei + bcast(se, j);
          const double r2 = dx * dx + dy * dy + dz * dz + e * e;
          const double c3 = (tj == (uint32_t)k) ? 0.0 : bcast(sm, j) * inv_cube<true>(r2, c15, c1875);
          acc[0] += c3 * dx;
          acc[1] += c3 * dy;
          acc[2] += c3 * dz;
        }
      }
    }
    // opened children go on the stack, the lowest popped first
    for (int c = 7; c >= 0; --c) {
      if (__builtin_amdgcn_readlane(kind, c) == 3) {
        if (lane == 0) stack[wave][sp] = ((uint64_t)l << 32) | (uint64_t)((pp << 3) | (uint32_t)c);
        ++sp;
      }
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

int gravity_tiles(int precision, int* tiles) {
  // default first: the fastest at 125k spheres on MI355X (measured)
  if (precision == 1) {
    tiles[0] = 64 * 16;
    tiles[1] = 64 * 8;
    tiles[2] = 64 * 4;
  } else {
    tiles[0] = 64 * 8;
    tiles[1] = 64 * 4;
    tiles[2] = 64 * 2;
  }
  return 3;
}

void launch_gravity_records(hipStream_t st, const PileDev* piles, const WorkItem* wl, int nblk,
                            int precision) {
  hipLaunchKernelGGL(k_grav_records, dim3(nblk), dim3(kBlock), 0, st, piles, wl, precision);
}

template <typename T, int IPT>
static void tiles_launch(hipStream_t st, const PileDev* piles, const GravItem* gl, int n, bool soft) {
  if (soft)
    hipLaunchKernelGGL((k_grav_tiles<T, IPT, true>), dim3(n), dim3(64), 0, st, piles, gl);
  else
    hipLaunchKernelGGL((k_grav_tiles<T, IPT, false>), dim3(n), dim3(64), 0, st, piles, gl);
}

void launch_gravity_tiles(hipStream_t st, const PileDev* piles, const GravItem* gl, int nitems,
                          int precision, bool softened, int tile) {
  if (nitems <= 0) return;
  const int ipt = tile / 64;
  if (precision == 1) {
    if (ipt == 4) tiles_launch<float, 4>(st, piles, gl, nitems, softened);
    else if (ipt == 16) tiles_launch<float, 16>(st, piles, gl, nitems, softened);
    else tiles_launch<float, 8>(st, piles, gl, nitems, softened);
  } else {
    if (ipt == 2) tiles_launch<double, 2>(st, piles, gl, nitems, softened);
    else if (ipt == 8) tiles_launch<double, 8>(st, piles, gl, nitems, softened);
    else tiles_launch<double, 4>(st, piles, gl, nitems, softened);
  }
}

void launch_gravity_combine(hipStream_t st, const PileDev* piles, const WorkItem* wl, int nblk,
                            int precision) {
  if (precision == 1)
    hipLaunchKernelGGL(k_grav_combine<float>, dim3(nblk), dim3(kBlock), 0, st, piles, wl);
  else
    hipLaunchKernelGGL(k_grav_combine<double>, dim3(nblk), dim3(kBlock), 0, st, piles, wl);
}

void launch_tree(hipStream_t st, const PileDev* piles, WorkItem* const* wl_level,
                 const int* n_level, const WorkItem* wl_sph, int n_sph_blk, const bool* any_order) {
  for (int l = 10; l >= 0; --l)
    if (n_level[l] > 0)
      hipLaunchKernelGGL(k_tree_level, dim3(n_level[l]), dim3(kBlock), 0, st, piles, wl_level[l], l);
  if (any_order[0])
    hipLaunchKernelGGL(k_tree_walk<2>, dim3(n_sph_blk * kTreeParts), dim3(kBlock), 0, st, piles,
                       wl_sph);
  if (any_order[1])
    hipLaunchKernelGGL(k_tree_walk<4>, dim3(n_sph_blk * kTreeParts), dim3(kBlock), 0, st, piles,
                       wl_sph);
  hipLaunchKernelGGL(k_tree_combine, dim3(n_sph_blk), dim3(kBlock), 0, st, piles, wl_sph);
}

}  // namespace dem
