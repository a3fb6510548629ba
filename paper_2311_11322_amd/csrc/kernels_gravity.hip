// kernels_gravity.hip -- softened all-pairs self-gravity (Eq. 4 of the
// paper, with Plummer softening eps_ij = soft_frac (s_i + s_j) / 2).
//
// Spheres are taken in cell-sorted (Morton) order and cut into tiles of B
// slots, and the tiles into at most kGravSlots super-tiles of `span`
// consecutive tiles.  One wave computes one super-tile pair (SI, SJ),
// SI <= SJ, tile pair by tile pair (I, J), I <= J, so every unordered pair
// of spheres is evaluated once (Newton's third law):
//  * each lane holds IPT targets of tile I in registers, and their sums
//    over all J of SJ;
//  * the sources of tile J enter 64 at a time, one per lane, together with
//    a reaction accumulator, and rotate one lane per step (DPP wave_ror:1)
//    so that after 64 steps every source has met every target of the wave
//    and is back in its own lane holding its complete reaction sum, which
//    that lane adds to the source's running sum over the tiles of SI;
//  * a diagonal pair (I, I) evaluates the ordered pairs i != j one way only,
//    with the sources walked by a uniform index (scalar loads).
// Each sphere receives exactly one partial sum per super-tile (as a target
// of SJ's row or a source of SI's column), summed in a fixed order and
// stored per super-tile; the combine kernel adds them in super-tile order,
// so the result is deterministic and independent of other piles, and the
// partial sums take at most kGravSlots x 3 values per sphere.  With no more
// tiles than kGravSlots a super-tile is one tile.
//
// FP64 form: rsqrt from the hardware estimate y0 and one first-order
// correction folded into the cube: r^-3 = y0^3 (1 + 3e/2), e = 1 - r^2 y0^2.
// FP32-force form: coordinates relative to an FP64 anchor per tile (the
// first sphere of the tile); the anchor offset of a tile pair, formed in
// FP64, moves one tile into the other's frame; FP32 partial sums per
// super-tile, FP64 across them.
#include "gravity_common.h"

namespace dem {

namespace {

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

// FP64 with 8 targets per lane runs at two waves per SIMD whatever the
// schedule; saying so lets the compiler issue the eight inverse square roots
// together (measured 1.5 % faster at 125k spheres than its three-wave
// schedule).
template <typename T, int IPT, bool SOFT, bool MULTI>
__global__ __launch_bounds__(64) __attribute__((amdgpu_waves_per_eu(
    1, (sizeof(T) == 8 && IPT == 8) ? 2 : 8))) void k_grav_tiles(const PileDev* __restrict__ piles,
                                                   const GravItem* __restrict__ gl) {
  constexpr int B = 64 * IPT;
  constexpr bool F32 = sizeof(T) == 4;
  const GravItem it = gl[blockIdx.x];
  const PileDev& P = piles[it.pile];
  if (P.status != 0) return;
  const int ns = P.ns, nt = P.g_nt, lane = threadIdx.x;
  // tiles per super-tile (the launch for piles of at most kGravSlots tiles
  // takes one, fixed at compile time)
  const int span = MULTI ? (nt + kGravSlots - 1) / kGravSlots : 1;
  const int si = it.ti, sj = it.tj;
  const int I0 = si * span, I1 = MULTI ? min(I0 + span, nt) : I0 + 1;
  const int J0 = sj * span, J1 = MULTI ? min(J0 + span, nt) : J0 + 1;
  const bool diag_item = si == sj;
  double c15;
  series_coeffs(c15);
  T* __restrict__ part = (T*)P.gpart;

  for (int I = I0; I < I1; ++I) {
    const int i0 = I * B;
    T xi[IPT], yi[IPT], zi[IPT], ei[IPT], mi[IPT], ax[IPT], ay[IPT], az[IPT];
#pragma unroll
    for (int u = 0; u < IPT; ++u) ax[u] = ay[u] = az[u] = (T)0;
    // targets of tile I, in the FP32 form less an anchor offset
    auto load_targets = [&](T tx, T ty, T tz) {
#pragma unroll
      for (int u = 0; u < IPT; ++u) {
        const int k = i0 + u * 64 + lane;
        const int kk = k < ns ? k : ns - 1;
        if (F32) {
          const Rec32 r = ((const Rec32*)P.jrec)[kk];
          xi[u] = (T)r.x - tx;
          yi[u] = (T)r.y - ty;
          zi[u] = (T)r.z - tz;
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
      }
    };
    if (MULTI) load_targets((T)0, (T)0, (T)0);
    for (int J = diag_item ? I : J0; J < J1; ++J) {
      // FP32 form: anchor offset A_J - A_I, formed in FP64; it moves the
      // targets into J's frame when an item is one tile pair, and the
      // sources into I's frame when the targets stay for several J
      T sx = 0, sy = 0, sz = 0;
      if (F32) {
        const double* aI = P.ganchor + (size_t)I * 4;
        const double* aJ = P.ganchor + (size_t)J * 4;
        sx = (T)(aJ[0] - aI[0]);
        sy = (T)(aJ[1] - aI[1]);
        sz = (T)(aJ[2] - aI[2]);
      }
      if (!MULTI) load_targets(sx, sy, sz);
      const int j0 = J * B, j1 = min(j0 + B, ns);
      if (J == I) {
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
            // j == i gives d = 0 and contributes nothing (r^-3 = 0 when unsoftened)
            const T dx = xj - xi[u], dy = yj - yi[u], dz = zj - zi[u];
            const T t = ei[u] + ej;
            const T r2 = fma(dx, dx, fma(dy, dy, fma(dz, dz, t * t)));
            const T w = mj * inv_cube<SOFT>(r2, c15);
            ax[u] = fma(w, dx, ax[u]);
            ay[u] = fma(w, dy, ay[u]);
            az[u] = fma(w, dz, az[u]);
          }
        }
        continue;
      }
      // sources of tile J travel around the wave 64 at a time, each carrying
      // its own reaction sum; after 64 one-lane rotations it is back home
      for (int jc = j0; jc < j1; jc += 64) {
        const int jx = jc + lane;
        const int jk = jx < j1 ? jx : j1 - 1;
        T xj, yj, zj, mj, ej;
        if (F32) {
          const Rec32 r = ((const Rec32*)P.jrec)[jk];
          xj = MULTI ? r.x + sx : r.x;
          yj = MULTI ? r.y + sy : r.y;
          zj = MULTI ? r.z + sz : r.z;
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
            const T c3 = inv_cube<SOFT>(r2, c15);
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
        // add to the source's reaction sum over the tiles of SI so far (which
        // this same lane stored)
        if (jx < j1) {
          T* qx = part + ((size_t)si * 3 + 0) * ns + jx;
          T* qy = part + ((size_t)si * 3 + 1) * ns + jx;
          T* qz = part + ((size_t)si * 3 + 2) * ns + jx;
          const bool first = !MULTI || I == I0;
          *qx = first ? -bx : *qx - bx;
          *qy = first ? -by : *qy - by;
          *qz = first ? -bz : *qz - bz;
        }
      }
    }
    // targets of tile I store under super-tile sj; on a diagonal item that
    // slot already holds the reactions from the tiles before I
    const bool add = MULTI && diag_item && I > I0;
#pragma unroll
    for (int u = 0; u < IPT; ++u) {
      const int k = i0 + u * 64 + lane;
      if (k < ns) {
        T* px = part + ((size_t)sj * 3 + 0) * ns + k;
        T* py = part + ((size_t)sj * 3 + 1) * ns + k;
        T* pz = part + ((size_t)sj * 3 + 2) * ns + k;
        *px = add ? *px + ax[u] : ax[u];
        *py = add ? *py + ay[u] : ay[u];
        *pz = add ? *pz + az[u] : az[u];
      }
    }
  }
}

// The per-target form (O(N) partial sums): one wave per (target group,
// source split s), a target group being 64 x IPT consecutive slots inside
// one tile (IPT per lane, fewer than a tile holds, so that the launch has
// enough waves).  Split s covers a run of consecutive source tiles; the
// wave's lanes hold the group's targets and walk every source of the run by
// a uniform index (scalar loads), evaluating each ordered pair once from the
// target's side, so no reaction is carried and each sphere receives one
// partial per split.  Twice the pair evaluations of the pair form, for 16
// partial sums per sphere.
template <typename T, int IPT, bool SOFT>
__global__ __launch_bounds__(64) void k_grav_split(const PileDev* __restrict__ piles,
                                                   const GravItem* __restrict__ gl) {
  constexpr int G = 64 * IPT;
  constexpr bool F32 = sizeof(T) == 4;
  const GravItem it = gl[blockIdx.x];
  const PileDev& P = piles[it.pile];
  if (P.status != 0) return;
  const int ns = P.ns, nt = P.g_nt, B = P.g_tile, lane = threadIdx.x;
  const int span = (nt + kGravSplits - 1) / kGravSplits;  // source tiles per split
  const int t0 = it.tj * span, t1 = min(t0 + span, nt);
  const int i0 = it.ti * G;
  const int ti = i0 / B;                                   // the targets' tile
  double c15;
  series_coeffs(c15);

  T xi[IPT], yi[IPT], zi[IPT], ei[IPT], ax[IPT], ay[IPT], az[IPT];
#pragma unroll
  for (int u = 0; u < IPT; ++u) {
    const int k = i0 + u * 64 + lane;
    const int kk = k < ns ? k : ns - 1;
    if (F32) {
      const Rec32 r = ((const Rec32*)P.jrec)[kk];
      xi[u] = (T)r.x;
      yi[u] = (T)r.y;
      zi[u] = (T)r.z;
      ei[u] = (T)r.e;
    } else {
      const Rec64 r = ((const Rec64*)P.jrec)[kk];
      xi[u] = (T)r.x;
      yi[u] = (T)r.y;
      zi[u] = (T)r.z;
      ei[u] = (T)r.e;
    }
    ax[u] = ay[u] = az[u] = (T)0;
  }
  for (int tj = t0; tj < t1; ++tj) {
    // FP32 form: targets relative to source tile J's anchor,
    // (x_i - A_I) - (A_J - A_I), the offset formed in FP64
    T xs[IPT], ys[IPT], zs[IPT];
    T sx = 0, sy = 0, sz = 0;
    if (F32) {
      const double* aI = P.ganchor + (size_t)ti * 4;
      const double* aJ = P.ganchor + (size_t)tj * 4;
      sx = (T)(aJ[0] - aI[0]);
      sy = (T)(aJ[1] - aI[1]);
      sz = (T)(aJ[2] - aI[2]);
    }
#pragma unroll
    for (int u = 0; u < IPT; ++u) {
      xs[u] = xi[u] - sx;
      ys[u] = yi[u] - sy;
      zs[u] = zi[u] - sz;
    }
    const int j0 = tj * B, j1 = min(j0 + B, ns);
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
      // the sphere itself contributes nothing: d = 0 (and r^-3 = 0 when
      // unsoftened)
#pragma unroll
      for (int u = 0; u < IPT; ++u) {
        const T dx = xj - xs[u], dy = yj - ys[u], dz = zj - zs[u];
        const T t = ei[u] + ej;
        const T r2 = fma(dx, dx, fma(dy, dy, fma(dz, dz, t * t)));
        const T w = mj * inv_cube<SOFT>(r2, c15);
        ax[u] = fma(w, dx, ax[u]);
        ay[u] = fma(w, dy, ay[u]);
        az[u] = fma(w, dz, az[u]);
      }
    }
  }
  T* __restrict__ part = (T*)P.gpart;
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

// One thread per sorted slot: add the partials in order -- per super-tile
// (pair form) or per source split (per-target form) -- in FP64, and store the
// gravity force G m_i sum under the sphere's id.  With a
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
  const int ns = P.ns, nt = P.g_np;
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
static void tiles_launch(hipStream_t st, const PileDev* piles, const GravItem* gl, int n, bool soft,
                         bool multi) {
  if (multi) {
    if (soft)
      hipLaunchKernelGGL((k_grav_tiles<T, IPT, true, true>), dim3(n), dim3(64), 0, st, piles, gl);
    else
      hipLaunchKernelGGL((k_grav_tiles<T, IPT, false, true>), dim3(n), dim3(64), 0, st, piles, gl);
  } else {
    if (soft)
      hipLaunchKernelGGL((k_grav_tiles<T, IPT, true, false>), dim3(n), dim3(64), 0, st, piles, gl);
    else
      hipLaunchKernelGGL((k_grav_tiles<T, IPT, false, false>), dim3(n), dim3(64), 0, st, piles, gl);
  }
}

void launch_gravity_tiles(hipStream_t st, const PileDev* piles, const GravItem* gl, int nitems,
                          int precision, bool softened, int tile, bool multi) {
  if (nitems <= 0) return;
  const int ipt = tile / 64;
  if (precision == 1) {
    if (ipt == 4) tiles_launch<float, 4>(st, piles, gl, nitems, softened, multi);
    else if (ipt == 16) tiles_launch<float, 16>(st, piles, gl, nitems, softened, multi);
    else tiles_launch<float, 8>(st, piles, gl, nitems, softened, multi);
  } else {
    if (ipt == 2) tiles_launch<double, 2>(st, piles, gl, nitems, softened, multi);
    else if (ipt == 8) tiles_launch<double, 8>(st, piles, gl, nitems, softened, multi);
    else tiles_launch<double, 4>(st, piles, gl, nitems, softened, multi);
  }
}

template <typename T, int IPT>
static void split_launch(hipStream_t st, const PileDev* piles, const GravItem* gl, int n, bool soft) {
  if (soft)
    hipLaunchKernelGGL((k_grav_split<T, IPT, true>), dim3(n), dim3(64), 0, st, piles, gl);
  else
    hipLaunchKernelGGL((k_grav_split<T, IPT, false>), dim3(n), dim3(64), 0, st, piles, gl);
}

int gravity_split_ipt(int precision, int tile) {
  // targets per lane of the per-target kernel: at most kSplitIpt64 (FP64) or
  // kSplitIpt32 (FP32), and never more than one tile holds
  const int cap = precision == 1 ? kSplitIpt32 : kSplitIpt64;
  return std::min(tile / 64, cap);
}

void launch_gravity_split(hipStream_t st, const PileDev* piles, const GravItem* gl, int nitems,
                          int precision, bool softened, int tile) {
  if (nitems <= 0) return;
  const int ipt = gravity_split_ipt(precision, tile);
  if (precision == 1) {
    if (ipt == 4) split_launch<float, 4>(st, piles, gl, nitems, softened);
    else if (ipt == 16) split_launch<float, 16>(st, piles, gl, nitems, softened);
    else split_launch<float, 8>(st, piles, gl, nitems, softened);
  } else {
    if (ipt == 2) split_launch<double, 2>(st, piles, gl, nitems, softened);
    else if (ipt == 8) split_launch<double, 8>(st, piles, gl, nitems, softened);
    else split_launch<double, 4>(st, piles, gl, nitems, softened);
  }
}

void launch_gravity_combine(hipStream_t st, const PileDev* piles, const WorkItem* wl, int nblk,
                            int precision) {
  if (precision == 1)
    hipLaunchKernelGGL(k_grav_combine<float>, dim3(nblk), dim3(kBlock), 0, st, piles, wl);
  else
    hipLaunchKernelGGL(k_grav_combine<double>, dim3(nblk), dim3(kBlock), 0, st, piles, wl);
}

}  // namespace dem
