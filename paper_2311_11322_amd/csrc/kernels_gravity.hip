// kernels_gravity.hip -- softened all-pairs self-gravity (Eq. 4 of the
// paper, with Plummer softening eps_ij = soft_frac (s_i + s_j) / 2).
//
// The sum runs over spheres in cell-sorted order.  Each block owns up to
// IPT*256 consecutive target slots and one contiguous range of source slots
// (a j-split); every lane keeps IPT targets in registers.  The source loop
// index is uniform across the block, so source records are fetched with
// scalar loads and broadcast to the lanes from SGPRs (no LDS traffic).
// Each split writes its partial acceleration sum sum_j m_j d_ij / r^3; the
// aggregate reduction adds the splits in a fixed order and multiplies by
// G m_i, so the result is deterministic.
//
// FP64 form: the reciprocal square root comes from the hardware estimate
// refined by one third-order step y (1 + e/2 + 3e^2/8), e = 1 - r^2 y^2,
// which brings it to full double precision.
#include "dem_internal.h"

namespace dem {

namespace {

struct alignas(64) Rec64 {
  double x, y, z, m, e, p0, p1, p2;
};

// Source records are read through the constant address space: the loop
// index is uniform, so these become scalar loads into SGPRs.
typedef const __attribute__((address_space(4))) Rec64* ConstRec64;

__device__ __forceinline__ double rsqrt_f64(double r2) {
  const double y = __builtin_amdgcn_rsq(r2);
  const double e = fma(-r2, y * y, 1.0);
  const double p = fma(e, 0.375, 0.5);
  return fma(y * e, p, y);
}

template <int IPT, bool SOFT>
__global__ __launch_bounds__(kBlock) void k_gravity64(const PileDev* __restrict__ piles,
                                                      const GravItem* __restrict__ gl) {
  const GravItem it = gl[blockIdx.x];
  const PileDev& P = piles[it.pile];
  if (P.status != 0) return;
  const int ns = P.ns;
  const Rec64* __restrict__ rec = (const Rec64*)P.jrec;
  ConstRec64 crec = (ConstRec64)P.jrec;
  double xi[IPT], yi[IPT], zi[IPT], ei[IPT], ax[IPT], ay[IPT], az[IPT];
#pragma unroll
  for (int u = 0; u < IPT; ++u) {
    const int k = it.ibase + u * kBlock + threadIdx.x;
    const int kk = k < ns ? k : ns - 1;
    xi[u] = rec[kk].x;
    yi[u] = rec[kk].y;
    zi[u] = rec[kk].z;
    ei[u] = rec[kk].e;
    ax[u] = ay[u] = az[u] = 0.0;
  }
  const int j1 = it.j1;
#pragma unroll 2
  for (int j = it.j0; j < j1; ++j) {
    const double xj = crec[j].x, yj = crec[j].y, zj = crec[j].z, mj = crec[j].m, ej = crec[j].e;
#pragma unroll
    for (int u = 0; u < IPT; ++u) {
      const double dx = xj - xi[u], dy = yj - yi[u], dz = zj - zi[u];
      const double t = ei[u] + ej;
      const double r2 = fma(dx, dx, fma(dy, dy, fma(dz, dz, t * t)));
      double inv = rsqrt_f64(r2);
      if (!SOFT) inv = r2 > 0.0 ? inv : 0.0;
      const double w = (mj * inv) * (inv * inv);
      ax[u] = fma(w, dx, ax[u]);
      ay[u] = fma(w, dy, ay[u]);
      az[u] = fma(w, dz, az[u]);
    }
  }
  double* __restrict__ out = P.gpart + (size_t)it.split * 3 * ns;
#pragma unroll
  for (int u = 0; u < IPT; ++u) {
    const int k = it.ibase + u * kBlock + threadIdx.x;
    if (k < ns) {
      out[k] = ax[u];
      out[ns + k] = ay[u];
      out[2 * ns + k] = az[u];
    }
  }
}

}  // namespace

// Targets per lane of the gravity kernel (the host sizes its work list with it).
int gravity_ipt(int precision) { return 2; }

void launch_gravity(hipStream_t st, const PileDev* piles, const GravItem* gl, int nitems,
                    int precision, bool softened) {
  if (nitems <= 0) return;
  if (softened)
    hipLaunchKernelGGL((k_gravity64<2, true>), dim3(nitems), dim3(kBlock), 0, st, piles, gl);
  else
    hipLaunchKernelGGL((k_gravity64<2, false>), dim3(nitems), dim3(kBlock), 0, st, piles, gl);
}

}  // namespace dem
