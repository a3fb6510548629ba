// step_force.h -- the soft-sphere contact force of one contact, with the
// spring history carried from the previous step (Sec. 2.1: spring-dashpot
// normal and tangential forces, static friction, rolling and twisting
// friction, history kept while the contact lasts; Sec. 2.2.4: forces act at
// the contact point, lever arm of Eq. 8, torque of Eq. 9).  Included by the
// staged force kernel and by the fused per-pile step.
//
// Geometry (separation, distance, overlap) is always FP64; the force
// arithmetic runs in T (double, or float for the FP32-force form).  A wall
// is partner ns + w: infinite mass, no spin, moving rigidly; its reaction
// goes nowhere.
#pragma once
#include "dem_internal.h"

namespace dem {

namespace {

template <typename T>
struct V3 {
  T x, y, z;
};

template <typename T>
__device__ __forceinline__ V3<T> mk(T x, T y, T z) {
  return V3<T>{x, y, z};
}
template <typename T>
__device__ __forceinline__ V3<T> operator+(V3<T> a, V3<T> b) {
  return mk(a.x + b.x, a.y + b.y, a.z + b.z);
}
template <typename T>
__device__ __forceinline__ V3<T> operator-(V3<T> a, V3<T> b) {
  return mk(a.x - b.x, a.y - b.y, a.z - b.z);
}
template <typename T>
__device__ __forceinline__ V3<T> operator*(T s, V3<T> a) {
  return mk(s * a.x, s * a.y, s * a.z);
}
template <typename T>
__device__ __forceinline__ T dotv(V3<T> a, V3<T> b) {
  return a.x * b.x + a.y * b.y + a.z * b.z;
}
template <typename T>
__device__ __forceinline__ V3<T> crossv(V3<T> a, V3<T> b) {
  return mk(a.y * b.z - a.z * b.y, a.z * b.x - a.x * b.z, a.x * b.y - a.y * b.x);
}
template <typename T>
__device__ __forceinline__ T normv(V3<T> a) {
  return sqrt(dotv(a, a));
}

// Rescale a spring so that k |xi| does not exceed the friction limit.
template <typename T>
__device__ __forceinline__ V3<T> cap_spring(V3<T> xi, T k, T limit, bool* capped) {
  const T mag = normv(xi);
  if (k * mag > limit) {
    *capped = true;
    return (limit / (k * mag)) * xi;
  }
  *capped = false;
  return xi;
}

// What every contact of a pile's step reads from its table entry.
template <typename T>
struct PairCtx {
  int ns, na, cap;
  const uint32_t* __restrict__ new_j;
  const uint32_t* __restrict__ own;
  const uint32_t* __restrict__ old_off;
  const uint32_t* __restrict__ old_j;
  const double* __restrict__ old_h;
  double* __restrict__ new_h;
  uint32_t n_pairs;
  int periodic;
  double L;
  T h, kn, kt, kr, kq;
};

template <typename T>
__device__ __forceinline__ PairCtx<T> pair_ctx(const PileDev& P, const ContactParams& cp) {
  PairCtx<T> c;
  const int cur = P.parity, nxt = cur ^ 1;
  c.ns = P.ns;
  c.na = P.na;
  c.cap = P.cap_pairs;
  c.new_j = P.pair_j[nxt];
  c.own = P.pair_i;
  c.old_off = P.up_off[cur];
  c.old_j = P.pair_j[cur];
  c.old_h = P.hist[cur];
  c.new_h = P.hist[nxt];
  c.n_pairs = P.up_off[nxt][P.ns];
  c.periodic = P.periodic;
  c.L = P.box;
  c.h = (T)cp.dt;
  c.kn = (T)cp.k_n;
  c.kt = (T)cp.k_t;
  c.kr = (T)cp.k_r;
  c.kq = (T)cp.k_q;
  return c;
}

// Contact p (i, j) of the new upper list: history lookup in i's previous
// (sorted) upper run, contact force and torques, new history; records, for
// j's lower list, where the contact sits.  Sets bad on a non-finite force or
// an overlap beyond the limit.
template <typename T>
__device__ __forceinline__ void pair_one(const PileDev& P, const PairCtx<T>& c,
                                         const ContactParams& cp, uint32_t p, bool& bad) {
  const int ns = c.ns, na = c.na, cap = c.cap;
  const uint32_t* __restrict__ new_j = c.new_j;
  const uint32_t* __restrict__ own = c.own;
  const uint32_t* __restrict__ old_off = c.old_off;
  const uint32_t* __restrict__ old_j = c.old_j;
  const double* __restrict__ old_h = c.old_h;
  double* __restrict__ new_h = c.new_h;
  const int periodic = c.periodic;
  const double L = c.L;
  const T h = c.h, kn = c.kn, kt = c.kt, kr = c.kr, kq = c.kq;
    const uint32_t i = own[p];
    const uint32_t j = new_j[p];
    const double rix = P.r[i], riy = P.r[ns + i], riz = P.r[2 * ns + i];
    const double si = P.s[i];
    const int Ai = P.agg[i];
    const V3<T> vi = mk<T>(P.v[i], P.v[ns + i], P.v[2 * ns + i]);
    const V3<T> wi = mk<T>(P.wA[Ai], P.wA[na + Ai], P.wA[2 * na + Ai]);
    const double Mi = P.M[Ai];
    // geometry in FP64; partner velocity, spin and the reduced mass
    double delta_d, li_d, lj_d, mu, Rij_d, s_min;
    V3<T> n, vj, wj;
    if (j >= (uint32_t)ns) {
      // a wall: infinite mass, no spin; the contact point is the foot of
      // the perpendicular and the normal points from the sphere into the wall
      const int wi_ = (int)(j - (uint32_t)ns);
      const Grid& g = *P.grid;
      const double gap = wall_gap(P, wi_, g.wall_d[wi_], rix, riy, riz);
      n = mk<T>((T)-P.wall[wi_][0], (T)-P.wall[wi_][1], (T)-P.wall[wi_][2]);
      delta_d = si - gap;
      li_d = gap;
      lj_d = 0.0;
      mu = Mi;
      Rij_d = si;
      s_min = si;
      vj = mk<T>((T)g.wall_v[wi_][0], (T)g.wall_v[wi_][1], (T)g.wall_v[wi_][2]);
      wj = mk<T>((T)0, (T)0, (T)0);
    } else {
      double dx = P.r[j] - rix, dy = P.r[ns + j] - riy, dz = P.r[2 * ns + j] - riz;
      if (periodic) {
        const double hL = 0.5 * L;
        if (dx > hL) dx -= L;
        else if (dx < -hL) dx += L;
        if (dy > hL) dy -= L;
        else if (dy < -hL) dy += L;
        if (dz > hL) dz -= L;
        else if (dz < -hL) dz += L;
      }
      // |d| from d^2 = (dx*dx + dy*dy) + dz*dz rounded step by step, as the
      // contact search forms it (no fused multiply-add)
      const double dist = sqrt(
          __dadd_rn(__dadd_rn(__dmul_rn(dx, dx), __dmul_rn(dy, dy)), __dmul_rn(dz, dz)));
      const double sj = P.s[j];
      delta_d = (si + sj) - dist;
      li_d = (si * si - sj * sj + dist * dist) / (2.0 * dist);
      lj_d = dist - li_d;
      const double inv_d = 1.0 / dist;
      n = mk<T>(dx * inv_d, dy * inv_d, dz * inv_d);
      const int Aj = P.agg[j];
      vj = mk<T>(P.v[j], P.v[ns + j], P.v[2 * ns + j]);
      wj = mk<T>(P.wA[Aj], P.wA[na + Aj], P.wA[2 * na + Aj]);
      const double Mj = P.M[Aj];
      mu = Mi * Mj / (Mi + Mj);
      Rij_d = si * sj / (si + sj);
      s_min = fmin(si, sj);
    }
    const T delta = (T)delta_d;
    const T li = (T)li_d;
    const T lj = (T)lj_d;

    // history of this contact from the previous step, if it existed
    uint32_t o = old_off[i];
    const uint32_t o1 = old_off[i + 1];
    while (o < o1 && old_j[o] < j) ++o;
    T hs[kHist];
    if (o < o1 && old_j[o] == j) {
      for (int c = 0; c < kHist; ++c) hs[c] = (T)old_h[(size_t)c * cap + o];
    } else {
      for (int c = 0; c < kHist; ++c) hs[c] = (T)0;
    }

    // velocity of each body's material point at the contact point
    const V3<T> arm_i = li * n;
    const V3<T> arm_j = ((T)-1) * (lj * n);
    const V3<T> u = (vj + crossv(wj, arm_j)) - (vi + crossv(wi, arm_i));
    const T un = dotv(u, n);
    const V3<T> ut = u - un * n;
    // dashpots from the restitution coefficients, aggregate reduced mass
    const T Cn = (T)(cp.damp_n * sqrt(cp.k_n * mu));
    const T Ct = (T)(cp.damp_t * sqrt(cp.k_t * mu));
    const T fn = -kn * delta + Cn * un;              // along n, on i
    T fN = kn * delta - Cn * un;                     // repulsive load for the caps
    fN = fN > (T)0 ? fN : (T)0;

    // sliding: spring on the tangent plane, static-friction cap
    V3<T> xt = mk(hs[0], hs[1], hs[2]);
    xt = xt - dotv(xt, n) * n;
    xt = xt + h * ut;
    bool slid;
    xt = cap_spring(xt, kt, (T)cp.mu_s * fN, &slid);
    const V3<T> FT = slid ? kt * xt : kt * xt + Ct * ut;

    // rolling and twisting: springs on the relative spin of the two bodies
    const T Rij = (T)Rij_d;
    const V3<T> dw = wj - wi;
    V3<T> xr = mk(hs[3], hs[4], hs[5]);
    xr = (xr - dotv(xr, n) * n) + (h * Rij) * crossv(dw, n);
    bool tmp;
    xr = cap_spring(xr, kr, (T)cp.mu_r * fN, &tmp);
    const V3<T> tau_r = Rij * crossv(n, kr * xr);
    T xq = hs[6] + h * Rij * dotv(dw, n);
    const T xq_lim = (T)cp.mu_t * fN;
    if (kq * fabs(xq) > xq_lim) xq = xq * (xq_lim / (kq * fabs(xq)));
    const V3<T> tau_q = (Rij * kq * xq) * n;

    const V3<T> F = fn * n + FT;
    const V3<T> ti = crossv(arm_i, F) + tau_r + tau_q;
    const V3<T> tj = crossv(arm_j, ((T)-1) * F) - tau_r - tau_q;

    P.pF[p] = F.x;
    P.pF[cap + p] = F.y;
    P.pF[2 * cap + p] = F.z;
    P.pTi[p] = ti.x;
    P.pTi[cap + p] = ti.y;
    P.pTi[2 * cap + p] = ti.z;
    P.pTj[p] = tj.x;
    P.pTj[cap + p] = tj.y;
    P.pTj[2 * cap + p] = tj.z;
    const T hn[kHist] = {xt.x, xt.y, xt.z, xr.x, xr.y, xr.z, xq};
    for (int c = 0; c < kHist; ++c) new_h[(size_t)c * cap + p] = (double)hn[c];

    if (!isfinite((double)F.x) || !isfinite((double)F.y) || !isfinite((double)F.z)) bad = true;
    if (cp.max_overlap_frac > 0.0 && delta_d > cp.max_overlap_frac * s_min) bad = true;

    // j's lower list holds i: point that entry at this contact
    if (j < (uint32_t)ns) {
      for (uint32_t e = P.lo_off[j], e1 = P.lo_off[j + 1]; e < e1; ++e) {
        if (P.lo_nbr[e] == i) {
          P.lo_pair[e] = p;
          break;
        }
      }
    }
}

}  // namespace

}  // namespace dem
