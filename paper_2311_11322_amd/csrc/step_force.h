// step_force.h -- the soft-sphere contact forces of one sphere, with the
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

// Every floating-point operation of the contact model is rounded on its own
// (no fused multiply-add): a contact is evaluated by both of its spheres, in
// different places of the code, and both must see the same force.
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
#pragma clang fp contract(off)
  return mk(a.x + b.x, a.y + b.y, a.z + b.z);
}
template <typename T>
__device__ __forceinline__ V3<T> operator-(V3<T> a, V3<T> b) {
#pragma clang fp contract(off)
  return mk(a.x - b.x, a.y - b.y, a.z - b.z);
}
template <typename T>
__device__ __forceinline__ V3<T> operator*(T s, V3<T> a) {
#pragma clang fp contract(off)
  return mk(s * a.x, s * a.y, s * a.z);
}
template <typename T>
__device__ __forceinline__ T dotv(V3<T> a, V3<T> b) {
#pragma clang fp contract(off)
  return a.x * b.x + a.y * b.y + a.z * b.z;
}
template <typename T>
__device__ __forceinline__ V3<T> crossv(V3<T> a, V3<T> b) {
#pragma clang fp contract(off)
  return mk(a.y * b.z - a.z * b.y, a.z * b.x - a.x * b.z, a.x * b.y - a.y * b.x);
}
template <typename T>
__device__ __forceinline__ T normv(V3<T> a) {
  return sqrt(dotv(a, a));
}

// Rescale a spring so that k |xi| does not exceed the friction limit.
template <typename T>
__device__ __forceinline__ V3<T> cap_spring(V3<T> xi, T k, T limit, bool* capped) {
#pragma clang fp contract(off)
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
  const uint32_t* __restrict__ up_off;
  const uint32_t* __restrict__ new_j;
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
  c.up_off = P.up_off[nxt];
  c.new_j = P.pair_j[nxt];
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

// What the force needs of one sphere of a contact: centre, radius, its
// aggregate's mass, the sphere's velocity and the aggregate's spin.
template <typename T>
struct Body {
  double x, y, z, s, M;
  V3<T> v, w;
};

template <typename T>
__device__ __forceinline__ Body<T> load_body(const PileDev& P, uint32_t i, int ns, int na) {
  Body<T> b;
  b.x = P.r[i];
  b.y = P.r[ns + i];
  b.z = P.r[2 * ns + i];
  b.s = P.s[i];
  const int A = P.agg[i];
  b.v = mk<T>(P.v[i], P.v[ns + i], P.v[2 * ns + i]);
  b.w = mk<T>(P.wA[A], P.wA[na + A], P.wA[2 * na + A]);
  b.M = P.M[A];
  return b;
}

// Spring history of contact (a, b) from the previous step: searched in a's
// previous (sorted) upper run from position o on; o is left at the first
// entry not below b, so a caller walking a's new (sorted) run can go on
// from there.  Zero for a new contact.
template <typename T>
__device__ __forceinline__ void find_hist(const PairCtx<T>& c, uint32_t& o, uint32_t o1,
                                          uint32_t b, T hs[kHist]) {
  while (o < o1 && c.old_j[o] < b) ++o;
  if (o < o1 && c.old_j[o] == b) {
    for (int k = 0; k < kHist; ++k) hs[k] = (T)c.old_h[(size_t)k * c.cap + o];
  } else {
    for (int k = 0; k < kHist; ++k) hs[k] = (T)0;
  }
}

// The same search in b's partner a's previous upper run [o, o1) when no merge
// pointer is carried (the lower contacts): the first four keys are loaded
// together, so the usual short run costs one round of loads, not a chain.
template <typename T>
__device__ __forceinline__ void find_hist_run(const PairCtx<T>& c, uint32_t o, uint32_t o1,
                                              uint32_t b, T hs[kHist]) {
  const uint32_t n = o1 - o;
  uint32_t kk[4];
#pragma unroll
  for (int u = 0; u < 4; ++u) kk[u] = (uint32_t)u < n ? c.old_j[o + u] : 0xffffffffu;
  int pos = -1;
#pragma unroll
  for (int u = 3; u >= 0; --u)
    if (kk[u] == b) pos = u;
  uint32_t p = o + (uint32_t)pos;
  if (pos < 0 && n > 4u) {
    p = o + 4u;
    while (p < o1 && c.old_j[p] < b) ++p;
    if (!(p < o1 && c.old_j[p] == b)) p = o1;
  } else if (pos < 0) {
    p = o1;
  }
  if (p < o1) {
    for (int k = 0; k < kHist; ++k) hs[k] = (T)c.old_h[(size_t)k * c.cap + p];
  } else {
    for (int k = 0; k < kHist; ++k) hs[k] = (T)0;
  }
}

// Force on a, torques on a and b about their centres, and the new spring
// history of one contact (a, b), a < b.
template <typename T>
struct ContactOut {
  V3<T> F, Ta, Tb;
  T hn[kHist];
  double delta, s_min;
};

// The contact model for normal n (from a towards b), overlap delta, lever
// arms la, lb along n, reduced mass mu, effective radius Rab, and the two
// bodies' velocities and spins at their centres.
template <typename T>
__device__ __forceinline__ void contact_model(const PairCtx<T>& c, const ContactParams& cp,
                                              V3<T> n, double delta_d, double la_d, double lb_d,
                                              double mu, double Rab_d, V3<T> va, V3<T> wa,
                                              V3<T> vb, V3<T> wb, const T hs[kHist],
                                              ContactOut<T>& out) {
#pragma clang fp contract(off)
  const T h = c.h, kn = c.kn, kt = c.kt, kr = c.kr, kq = c.kq;
  const T delta = (T)delta_d;
  const T li = (T)la_d;
  const T lj = (T)lb_d;
  // velocity of each body's material point at the contact point
  const V3<T> arm_i = li * n;
  const V3<T> arm_j = ((T)-1) * (lj * n);
  const V3<T> u = (vb + crossv(wb, arm_j)) - (va + crossv(wa, arm_i));
  const T un = dotv(u, n);
  const V3<T> ut = u - un * n;
  // dashpots from the restitution coefficients, aggregate reduced mass
  const T Cn = (T)(cp.damp_n * sqrt(cp.k_n * mu));
  const T Ct = (T)(cp.damp_t * sqrt(cp.k_t * mu));
  const T fn = -kn * delta + Cn * un;              // along n, on a
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
  const T Rij = (T)Rab_d;
  const V3<T> dw = wb - wa;
  V3<T> xr = mk(hs[3], hs[4], hs[5]);
  xr = (xr - dotv(xr, n) * n) + (h * Rij) * crossv(dw, n);
  bool tmp;
  xr = cap_spring(xr, kr, (T)cp.mu_r * fN, &tmp);
  const V3<T> tau_r = Rij * crossv(n, kr * xr);
  T xq = hs[6] + h * Rij * dotv(dw, n);
  const T xq_lim = (T)cp.mu_t * fN;
  if (kq * fabs(xq) > xq_lim) xq = xq * (xq_lim / (kq * fabs(xq)));
  const V3<T> tau_q = (Rij * kq * xq) * n;

  out.F = fn * n + FT;
  out.Ta = crossv(arm_i, out.F) + tau_r + tau_q;
  out.Tb = crossv(arm_j, ((T)-1) * out.F) - tau_r - tau_q;
  out.hn[0] = xt.x;
  out.hn[1] = xt.y;
  out.hn[2] = xt.z;
  out.hn[3] = xr.x;
  out.hn[4] = xr.y;
  out.hn[5] = xr.z;
  out.hn[6] = xq;
}

// Contact of spheres a < b: separation by the minimum image, distance
// formed as the contact search forms it, contact point at la from a.
template <typename T>
__device__ __forceinline__ void sphere_contact(const PairCtx<T>& c, const ContactParams& cp,
                                               const Body<T>& a, const Body<T>& b,
                                               const T hs[kHist], ContactOut<T>& out) {
#pragma clang fp contract(off)
  double dx = b.x - a.x, dy = b.y - a.y, dz = b.z - a.z;
  if (c.periodic) {
    const double L = c.L, hL = 0.5 * L;
    if (dx > hL) dx -= L;
    else if (dx < -hL) dx += L;
    if (dy > hL) dy -= L;
    else if (dy < -hL) dy += L;
    if (dz > hL) dz -= L;
    else if (dz < -hL) dz += L;
  }
  // |d| from d^2 = (dx*dx + dy*dy) + dz*dz rounded step by step (no fused
  // multiply-add)
  const double dist =
      sqrt(rn_add(rn_add(rn_mul(dx, dx), rn_mul(dy, dy)), rn_mul(dz, dz)));
  const double si = a.s, sj = b.s;
  const double delta_d = (si + sj) - dist;
  const double li_d = (si * si - sj * sj + dist * dist) / (2.0 * dist);
  const double lj_d = dist - li_d;
  const double inv_d = 1.0 / dist;
  const V3<T> n = mk<T>(dx * inv_d, dy * inv_d, dz * inv_d);
  const double mu = a.M * b.M / (a.M + b.M);
  const double Rij_d = si * sj / (si + sj);
  contact_model<T>(c, cp, n, delta_d, li_d, lj_d, mu, Rij_d, a.v, a.w, b.v, b.w, hs, out);
  out.delta = delta_d;
  out.s_min = fmin(si, sj);
}

// Contact of sphere a with wall w: infinite mass, no spin; the contact
// point is the foot of the perpendicular and the normal points from the
// sphere into the wall.
template <typename T>
__device__ __forceinline__ void wall_contact(const PileDev& P, const PairCtx<T>& c,
                                             const ContactParams& cp, const Body<T>& a, int w,
                                             const T hs[kHist], ContactOut<T>& out) {
#pragma clang fp contract(off)
  const Grid& g = *P.grid;
  const double gap = wall_gap(P, w, g.wall_d[w], a.x, a.y, a.z);
  const V3<T> n = mk<T>((T)-P.wall[w][0], (T)-P.wall[w][1], (T)-P.wall[w][2]);
  const double delta_d = a.s - gap;
  const V3<T> vw = mk<T>((T)g.wall_v[w][0], (T)g.wall_v[w][1], (T)g.wall_v[w][2]);
  const V3<T> zero = mk<T>((T)0, (T)0, (T)0);
  contact_model<T>(c, cp, n, delta_d, gap, 0.0, a.M, a.s, a.v, a.w, vw, zero, hs, out);
  out.delta = delta_d;
  out.s_min = a.s;
}

// Sphere i: the force and torque of all its contacts, summed in canonical
// contact order -- contacts (j, i) with j < i by increasing j, then (i, j)
// by increasing j (walls last) -- into F and tau; the new spring history of
// its upper contacts (i, j).  A contact is evaluated by both of its spheres,
// with the same operands in the same order, so both see the same force; its
// lower sphere writes the history and checks it (sets bad on a non-finite
// force or an overlap beyond the limit).  Contacts are taken two at a time,
// so that the partner and history loads of both are in flight together; the
// sums still follow the canonical order.
template <typename T>
__device__ __forceinline__ void forces_one(const PileDev& P, const PairCtx<T>& c,
                                           const ContactParams& cp, uint32_t i, bool& bad) {
  const int ns = c.ns, na = c.na, cap = c.cap;
  const Body<T> me = load_body<T>(P, i, ns, na);
  double f[3] = {0.0, 0.0, 0.0}, t[3] = {0.0, 0.0, 0.0};
  auto acc_lo = [&](const ContactOut<T>& r) {
    f[0] -= (double)r.F.x;
    f[1] -= (double)r.F.y;
    f[2] -= (double)r.F.z;
    t[0] += (double)r.Tb.x;
    t[1] += (double)r.Tb.y;
    t[2] += (double)r.Tb.z;
  };
  uint32_t e = P.lo_off[i];
  const uint32_t e1 = P.lo_off[i + 1];
  for (; e + 1 < e1; e += 2) {
    const uint32_t j0 = P.lo_nbr[e], j1 = P.lo_nbr[e + 1];
    const Body<T> o0 = load_body<T>(P, j0, ns, na);
    const Body<T> o1 = load_body<T>(P, j1, ns, na);
    T h0[kHist], h1[kHist];
    const uint32_t a0 = c.old_off[j0], a1 = c.old_off[j1];
    const uint32_t b0 = c.old_off[j0 + 1], b1 = c.old_off[j1 + 1];
    find_hist_run<T>(c, a0, b0, i, h0);
    find_hist_run<T>(c, a1, b1, i, h1);
    ContactOut<T> r0, r1;
    sphere_contact<T>(c, cp, o0, me, h0, r0);
    acc_lo(r0);
    sphere_contact<T>(c, cp, o1, me, h1, r1);
    acc_lo(r1);
  }
  if (e < e1) {
    const uint32_t j = P.lo_nbr[e];
    const Body<T> o = load_body<T>(P, j, ns, na);
    T hs[kHist];
    find_hist_run<T>(c, c.old_off[j], c.old_off[j + 1], i, hs);
    ContactOut<T> r;
    sphere_contact<T>(c, cp, o, me, hs, r);
    acc_lo(r);
  }
  uint32_t q = c.old_off[i];
  const uint32_t q1 = c.old_off[i + 1];
  auto up_done = [&](uint32_t p, const ContactOut<T>& r) {
    for (int k = 0; k < kHist; ++k) c.new_h[(size_t)k * cap + p] = (double)r.hn[k];
    if (!isfinite((double)r.F.x) || !isfinite((double)r.F.y) || !isfinite((double)r.F.z))
      bad = true;
    if (cp.max_overlap_frac > 0.0 && r.delta > cp.max_overlap_frac * r.s_min) bad = true;
    f[0] += (double)r.F.x;
    f[1] += (double)r.F.y;
    f[2] += (double)r.F.z;
    t[0] += (double)r.Ta.x;
    t[1] += (double)r.Ta.y;
    t[2] += (double)r.Ta.z;
  };
  uint32_t p = c.up_off[i];
  const uint32_t p1 = c.up_off[i + 1];
  for (; p + 1 < p1; p += 2) {
    const uint32_t j0 = c.new_j[p], j1 = c.new_j[p + 1];
    if (j1 >= (uint32_t)ns) break;                // a wall: one at a time
    const Body<T> o0 = load_body<T>(P, j0, ns, na);
    const Body<T> o1 = load_body<T>(P, j1, ns, na);
    T h0[kHist], h1[kHist];
    find_hist<T>(c, q, q1, j0, h0);
    find_hist<T>(c, q, q1, j1, h1);
    ContactOut<T> r0, r1;
    sphere_contact<T>(c, cp, me, o0, h0, r0);
    up_done(p, r0);
    sphere_contact<T>(c, cp, me, o1, h1, r1);
    up_done(p + 1, r1);
  }
  for (; p < p1; ++p) {
    const uint32_t j = c.new_j[p];
    T hs[kHist];
    find_hist<T>(c, q, q1, j, hs);
    ContactOut<T> r;
    if (j >= (uint32_t)ns) {
      wall_contact<T>(P, c, cp, me, (int)(j - (uint32_t)ns), hs, r);
    } else {
      const Body<T> o = load_body<T>(P, j, ns, na);
      sphere_contact<T>(c, cp, me, o, hs, r);
    }
    up_done(p, r);
  }
  for (int k = 0; k < 3; ++k) {
    P.F[k * ns + i] = f[k];
    P.tau[k * ns + i] = t[k];
  }
}

}  // namespace

}  // namespace dem
