// step_body.h -- per-element device functions of the rigid-body part of a
// step: the fifth-order rotation step, kick/drift/rotate of one aggregate,
// member reconstruction, the per-pile cell grid from reduced partials, the
// member reduction (GetAccelAndTorque, which adds each sphere's gravity force
// to its contact force) and the end-of-step bookkeeping.  Included by the staged kernels and by the fused
// per-pile step, so both do the same arithmetic.
//
// Paper references: leapfrog for centres of mass and a fifth-order
// Runge-Kutta step for orientation and spin (Sec. 2.1-2.2); predicted member
// velocity (Eq. 3); aggregate acceleration and torque (Eqs. 5-7, 9).
#pragma once
#include "dem_internal.h"

namespace dem {

namespace {

// ---------------------------------------------------------------------------
// rotation: Euler's equations with quaternion kinematics, Cash-Karp RK5
// ---------------------------------------------------------------------------

// y = (q0..q3, w1..w3); body-frame principal moments I; torque N fixed in
// the space frame.  dq/dt = q (x) (0, w) / 2; I dw/dt = R^T N - w x (I w).
__device__ __forceinline__ void euler_deriv(const double y[7], const double I[3],
                                            const double N[3], double f[7]) {
  double R[9], Nb[3];
  quat_rot(y, R);
  rot_apply_T(R, N, Nb);
  const double w = y[0], x = y[1], yy = y[2], z = y[3];
  const double o1 = y[4], o2 = y[5], o3 = y[6];
  f[0] = 0.5 * (-x * o1 - yy * o2 - z * o3);
  f[1] = 0.5 * (w * o1 + yy * o3 - z * o2);
  f[2] = 0.5 * (w * o2 + z * o1 - x * o3);
  f[3] = 0.5 * (w * o3 + x * o2 - yy * o1);
  f[4] = (Nb[0] - (I[2] - I[1]) * o2 * o3) / I[0];
  f[5] = (Nb[1] - (I[0] - I[2]) * o3 * o1) / I[1];
  f[6] = (Nb[2] - (I[1] - I[0]) * o1 * o2) / I[2];
}

// Cash & Karp (1990) fifth-order weights and stage matrix.
__constant__ double ck_a[6][5] = {
    {0.0, 0.0, 0.0, 0.0, 0.0},
    {1.0 / 5.0, 0.0, 0.0, 0.0, 0.0},
    {3.0 / 40.0, 9.0 / 40.0, 0.0, 0.0, 0.0},
    {3.0 / 10.0, -9.0 / 10.0, 6.0 / 5.0, 0.0, 0.0},
    {-11.0 / 54.0, 5.0 / 2.0, -70.0 / 27.0, 35.0 / 27.0, 0.0},
    {1631.0 / 55296.0, 175.0 / 512.0, 575.0 / 13824.0, 44275.0 / 110592.0, 253.0 / 4096.0}};
__constant__ double ck_b[6] = {37.0 / 378.0, 0.0, 250.0 / 621.0, 125.0 / 594.0, 0.0,
                               512.0 / 1771.0};

__device__ void rk5_rotate(double y[7], const double I[3], const double N[3], double h) {
  double k[6][7];
  for (int st = 0; st < 6; ++st) {
    double ys[7];
    for (int c = 0; c < 7; ++c) {
      double acc = 0.0;
      for (int j = 0; j < st; ++j) acc += ck_a[st][j] * k[j][c];
      ys[c] = y[c] + h * acc;
    }
    euler_deriv(ys, I, N, k[st]);
  }
  for (int c = 0; c < 7; ++c) {
    double acc = 0.0;
    for (int st = 0; st < 6; ++st) acc += ck_b[st] * k[st][c];
    y[c] = y[c] + h * acc;
  }
  const double inv = 1.0 / sqrt(y[0] * y[0] + y[1] * y[1] + y[2] * y[2] + y[3] * y[3]);
  for (int c = 0; c < 4; ++c) y[c] *= inv;
}

// One aggregate.  Step mode: v_A += h/2 a_A, r_A += h v_A (wrapped in a
// periodic cube), one RK5 step of (q, w_b) with the last torque.  Writes the
// next state, the space-frame spin w_A = R w_b and the predicted
// centre-of-mass velocity v_A + h/2 a_A (first bracket of Eq. 3).  Init mode
// copies the state unchanged (evaluation at t0).
__device__ __forceinline__ void integrate_one(PileDev& P, int A, const ContactParams& cp,
                                              int mode) {
  const int na = P.na, cur = P.parity, nxt = cur ^ 1;
  const double h = cp.dt;
  double v[3], r[3], a[3], y[7];
  for (int k = 0; k < 3; ++k) {
    v[k] = P.vA[cur][k * na + A];
    r[k] = P.rA[cur][k * na + A];
    a[k] = P.aA[cur][k * na + A];
  }
  for (int k = 0; k < 4; ++k) y[k] = P.q[cur][k * na + A];
  for (int k = 0; k < 3; ++k) y[4 + k] = P.wb[cur][k * na + A];
  if (mode == kModeStep) {
    for (int k = 0; k < 3; ++k) {
      v[k] += 0.5 * h * a[k];
      r[k] += h * v[k];
    }
    if (P.periodic) {
      const double L = P.box;
      for (int k = 0; k < 3; ++k) {
        if (r[k] >= L) r[k] -= L;
        if (r[k] < 0.0) r[k] += L;
      }
    }
    const double I[3] = {P.I[A], P.I[na + A], P.I[2 * na + A]};
    const double N[3] = {P.NA[cur][A], P.NA[cur][na + A], P.NA[cur][2 * na + A]};
    rk5_rotate(y, I, N, h);
  }
  double R[9], ws[3];
  quat_rot(y, R);
  rot_apply(R, &y[4], ws);
  const double hh = (mode == kModeStep) ? 0.5 * h : 0.0;
  for (int k = 0; k < 3; ++k) {
    P.vA[nxt][k * na + A] = v[k];
    P.rA[nxt][k * na + A] = r[k];
    P.wA[k * na + A] = ws[k];
    P.vpred[k * na + A] = v[k] + hh * a[k];
    P.wb[nxt][k * na + A] = y[4 + k];
  }
  for (int k = 0; k < 4; ++k) P.q[nxt][k * na + A] = y[k];
  if (A == 0 && P.pert_on) {
    // the perturber is one more body of the same leapfrog
    for (int k = 0; k < 3; ++k) {
      double pv = P.pert_v[cur][k], pr = P.pert_r[cur][k];
      if (mode == kModeStep) {
        pv += 0.5 * h * P.pert_a[cur][k];
        pr += h * pv;
      }
      P.pert_v[nxt][k] = pv;
      P.pert_r[nxt][k] = pr;
    }
  }
}

// Partials of an empty set of spheres: bbox min / max and mass moments.
__device__ __forceinline__ void bbox_identity(double vals[kBbox]) {
  for (int k = 0; k < 3; ++k) {
    vals[k] = INFINITY;
    vals[3 + k] = -INFINITY;
  }
  for (int k = 6; k < kBbox; ++k) vals[k] = 0.0;
}

// Combine partials b into a (min, max, sums).
__device__ __forceinline__ void bbox_combine(double a[kBbox], const double b[kBbox]) {
  for (int k = 0; k < 3; ++k) a[k] = fmin(a[k], b[k]);
  for (int k = 3; k < 6; ++k) a[k] = fmax(a[k], b[k]);
  for (int k = 6; k < kBbox; ++k) a[k] += b[k];
}

// Reference point of the second moment: aggregate 0's new centre (the
// origin for a pile of given positions).
__device__ __forceinline__ void bbox_ref(const PileDev& P, double cref[3]) {
  const int na = P.na, nxt = P.parity ^ 1;
  for (int k = 0; k < 3; ++k) cref[k] = (na > 0 && !P.given) ? P.rA[nxt][k * na] : 0.0;
}

// Member reconstruction of sphere i (SetSpacePos / SetSpaceVel, Eq. 3):
// r_i = r_A + R b_i, v_i = vpred_A + w_A x (R b_i); a pile without
// aggregates, or with given sphere states, keeps the positions and
// velocities it was given.  Its bounding-box and mass-moment contributions
// (second moment about cref) go into vals.
__device__ __forceinline__ void reconstruct_one(const PileDev& P, int i, const double cref[3],
                                                double vals[kBbox]) {
  const int ns = P.ns, na = P.na, nxt = P.parity ^ 1;
  if (na == 0 || P.given) {
    // positions given directly (stateless hooks): bbox only
    for (int k = 0; k < 3; ++k) {
      const double x = P.r[k * ns + i];
      vals[k] = x;
      vals[3 + k] = x;
      vals[7 + k] = x;
    }
    vals[6] = 1.0;
    vals[10] = 0.0;
    return;
  }
  const int A = P.agg[i];
  double q[4], R[9];
  for (int k = 0; k < 4; ++k) q[k] = P.q[nxt][k * na + A];
  quat_rot(q, R);
  const double bb[3] = {P.b[i], P.b[ns + i], P.b[2 * ns + i]};
  double d[3], wxd[3];
  rot_apply(R, bb, d);
  const double wa[3] = {P.wA[A], P.wA[na + A], P.wA[2 * na + A]};
  cross3(wa, d, wxd);
  const double mi = P.m[i];
  double d2 = 0.0;
  for (int k = 0; k < 3; ++k) {
    const double x = P.rA[nxt][k * na + A] + d[k];
    P.r[k * ns + i] = x;
    P.v[k * ns + i] = P.vpred[k * na + A] + wxd[k];
    vals[k] = x;
    vals[3 + k] = x;
    vals[7 + k] = mi * x;
    d2 += (x - cref[k]) * (x - cref[k]);
  }
  vals[6] = mi;
  vals[10] = mi * d2;
}

// The pile's cell grid, centre of mass, bulk radius and stop rule, wall
// offsets and velocities, from the reduced partials of all its spheres.
// Cells are at least one largest-sphere diameter; an open pile's grid spans
// its bounding box, or only the part of it within three rms radii of the
// centre of mass when that is smaller.
__device__ __forceinline__ void grid_from_vals(PileDev& P, double vals[kBbox], int mode,
                                               double dt) {
  // written in place: a local Grid (its wall arrays indexed by a count
  // known only at run time) would live in scratch memory
  Grid& g = *P.grid;
  bool finite = true;
  for (int k = 0; k < kBbox; ++k) finite = finite && isfinite(vals[k]);
  if (!finite) {
    atomicOr(&P.status, kStUnstable);
    return;
  }
  for (int k = 0; k < 3; ++k) g.com[k] = vals[7 + k] / vals[6];
  // second moment about the centre of mass, from the one about aggregate 0's
  // centre c: <|r - com|^2>_m = <|r - c|^2>_m - |com - c|^2
  double s2;
  {
    double c[3] = {0.0, 0.0, 0.0};
    const int na = P.na, nxt = P.parity ^ 1;
    if (na > 0 && !P.given)
      for (int k = 0; k < 3; ++k) c[k] = P.rA[nxt][k * na];
    s2 = vals[10] / vals[6];
    for (int k = 0; k < 3; ++k) s2 -= (g.com[k] - c[k]) * (g.com[k] - c[k]);
    s2 = fmax(s2, 0.0);
  }
  g.R_bulk = sqrt(s2 * (5.0 / 3.0));
  if (P.periodic) {
    for (int k = 0; k < 3; ++k) {
      g.nc[k] = P.n_periodic;
      g.nbits[k] = P.bits;
    }
    g.lo[0] = g.lo[1] = g.lo[2] = 0.0;
    g.cell = P.box / (double)P.n_periodic;
  } else {
    double lo[3], hi[3];
    for (int k = 0; k < 3; ++k) {
      lo[k] = vals[k];
      hi[k] = vals[3 + k];
    }
    if (!P.tree && !P.given && P.na > 0) {
      // a few spheres thrown far from the rest would make every cell of a
      // bounding-box grid large and crowd the rest into a few cells; the
      // grid covers three rms radii about the centre of mass instead, and a
      // sphere beyond it falls into an outermost cell (clamping keeps two
      // spheres in contact within one cell of each other on every axis, so
      // the 27-cell search still finds every contact)
      const double h = 3.0 * sqrt(s2) + P.cell_min;
      for (int k = 0; k < 3; ++k) {
        lo[k] = fmax(lo[k], g.com[k] - h);
        hi[k] = fmax(lo[k], fmin(hi[k], g.com[k] + h));
      }
    }
    // cube cells; the key's 3 * bits bits go one at a time to the axis whose
    // cells are currently the longest, so an elongated pile (a tall box)
    // gets more cells along its long axis
    double ext[3];
    for (int k = 0; k < 3; ++k) {
      g.lo[k] = lo[k];
      ext[k] = hi[k] - lo[k];
    }
    // per-axis bit counts kept in scalars (an array indexed by the chosen
    // axis would live in scratch memory)
    int b0 = 0, b1 = 0, b2 = 0;
    for (int t = 0; t < 3 * P.bits; ++t) {
      if (P.tree) {                      // the tree's pyramid needs a cubic code
        const int a = t % 3;
        b0 += a == 0;
        b1 += a == 1;
        b2 += a == 2;
        continue;
      }
      // the axis with the longest cells among those below 10 bits (the
      // first one on a tie)
      int a = -1;
      double best = -1.0;
      const double l0 = ldexp(ext[0], -b0), l1 = ldexp(ext[1], -b1), l2 = ldexp(ext[2], -b2);
      if (b0 < 10 && l0 > best) {
        best = l0;
        a = 0;
      }
      if (b1 < 10 && l1 > best) {
        best = l1;
        a = 1;
      }
      if (b2 < 10 && l2 > best) a = 2;
      b0 += a == 0;
      b1 += a == 1;
      b2 += a == 2;
    }
    const int b[3] = {b0, b1, b2};
    double fit = 0.0;
    for (int k = 0; k < 3; ++k) {
      g.nbits[k] = b[k];
      g.nc[k] = 1 << b[k];
      fit = fmax(fit, ldexp(ext[k] * (1.0 + 1e-12), -b[k]));
    }
    g.cell = fmax(P.cell_min, fit + 1e-300);
  }
  g.inv_cell = 1.0 / g.cell;
  if (P.stop_growth > 0.0) {
    // the stop rule: the first evaluation sets the reference radius; an
    // evaluation at or beyond stop_growth times it stops the pile (its step
    // is not committed, like a failure)
    if (!(P.R0 > 0.0)) {
      P.R0 = g.R_bulk;
    } else if (g.R_bulk >= P.stop_growth * P.R0) {
      atomicOr(&P.status, kStStopped);
    }
  }
  // time of this evaluation: the end of the step being taken, or the
  // current time for an evaluation in place; walls displaced rigidly by
  // A sin(omega t + phase), moving at A omega cos(omega t + phase)
  g.t = (double)(P.step + (mode == kModeStep ? 1 : 0)) * dt;
  for (int w = 0; w < 6; ++w) {
    g.wall_d[w] = 0.0;
    for (int k = 0; k < 3; ++k) g.wall_v[w][k] = 0.0;
  }
  if (P.n_walls > 0) {
    const double ph = rn_add(rn_mul(P.wall_omega, g.t), P.wall_phase);
    double sn, cs;
    sincos(ph, &sn, &cs);
    for (int w = 0; w < P.n_walls; ++w) {
      const double* n = P.wall[w];
      const double* A = P.wall_amp[w];
      const double shift =
          rn_add(rn_add(rn_mul(n[0], A[0]), rn_mul(n[1], A[1])), rn_mul(n[2], A[2]));
      g.wall_d[w] = rn_add(n[3], rn_mul(shift, sn));
      for (int k = 0; k < 3; ++k) g.wall_v[w][k] = rn_mul(rn_mul(A[k], P.wall_omega), cs);
    }
  }
}

// Force on sphere i: its contact force plus, in a pile with gravity, its
// gravity force (added last, after the contacts).
__device__ __forceinline__ void sphere_force(const PileDev& P, int i, double f[3]) {
  const int ns = P.ns;
  for (int k = 0; k < 3; ++k) f[k] = P.F[k * ns + i];
  if (P.G != 0.0)
    for (int k = 0; k < 3; ++k) f[k] += P.gacc[k * ns + i];
}

// One member's share of F_A and N_A: f_i and (R b_i) x f_i + tau_i.
__device__ __forceinline__ void add_member(const double R[9], const double f[3],
                                           const double bb[3], const double tau[3], double FA[3],
                                           double NA[3]) {
  double d[3], dxf[3];
  rot_apply(R, bb, d);
  cross3(d, f, dxf);
  for (int k = 0; k < 3; ++k) {
    FA[k] += f[k];
    NA[k] += dxf[k] + tau[k];
  }
}

// Members of aggregate A added in member order, read directly.
__device__ __forceinline__ void reduce_members_direct(const PileDev& P, int A, const double R[9],
                                                      double FA[3], double NA[3]) {
  const int ns = P.ns;
  // unrolled so that two members' loads are in flight (same order of sums)
#pragma unroll 2
  for (int i = P.first[A], i1 = i + P.count[A]; i < i1; ++i) {
    double f[3];
    sphere_force(P, i, f);
    const double bb[3] = {P.b[i], P.b[ns + i], P.b[2 * ns + i]};
    const double tau[3] = {P.tau[i], P.tau[ns + i], P.tau[2 * ns + i]};
    add_member(R, f, bb, tau, FA, NA);
  }
}

// The paper's original member search (ablation): every sphere of the pile
// tested for membership, in order.
__device__ __forceinline__ void reduce_members_scan(const PileDev& P, int A, const double R[9],
                                                    double FA[3], double NA[3]) {
  const int ns = P.ns;
  for (int i = 0; i < ns; ++i) {
    if (P.agg[i] != A) continue;
    double f[3];
    sphere_force(P, i, f);
    const double bb[3] = {P.b[i], P.b[ns + i], P.b[2 * ns + i]};
    const double tau[3] = {P.tau[i], P.tau[ns + i], P.tau[2 * ns + i]};
    add_member(R, f, bb, tau, FA, NA);
  }
}

// a_A = F_A / M + g, N_A; in step mode the closing half kick and the spin-up
// increment about +z through the pile's centre of mass.
__device__ __forceinline__ void reduce_tail(const PileDev& P, int A, const double R[9],
                                            const double FA[3], const double NA[3],
                                            const ContactParams& cp, int mode) {
  const int na = P.na, nxt = P.parity ^ 1;
  const double M = P.M[A];
  double a[3];
  for (int k = 0; k < 3; ++k) {
    a[k] = FA[k] / M + P.gfield[k];      // a uniform field adds no torque
    P.aA[nxt][k * na + A] = a[k];
    P.NA[nxt][k * na + A] = NA[k];
  }
  if (mode == kModeStep) {
    double v[3];
    for (int k = 0; k < 3; ++k) v[k] = P.vA[nxt][k * na + A] + 0.5 * cp.dt * a[k];
    if (P.spin_dw != 0.0) {
      // spin-up: w += dw z-hat about the pile's centre of mass
      const Grid g = *P.grid;
      const double dw = P.spin_dw;
      const double rel[3] = {P.rA[nxt][A] - g.com[0], P.rA[nxt][na + A] - g.com[1],
                             P.rA[nxt][2 * na + A] - g.com[2]};
      const double z[3] = {0.0, 0.0, dw};
      double dv[3], dwb[3];
      cross3(z, rel, dv);
      for (int k = 0; k < 3; ++k) v[k] += dv[k];
      rot_apply_T(R, z, dwb);
      for (int k = 0; k < 3; ++k) P.wb[nxt][k * na + A] += dwb[k];
    }
    for (int k = 0; k < 3; ++k) P.vA[nxt][k * na + A] = v[k];
  }
}

// Per pile: commit the step (flip the ping-pong halves) unless the pile
// failed during it, in which case its state stays at the failing step's
// start and the step index is recorded; the perturber's reaction and kick.
__device__ __forceinline__ void finish_one(PileDev& P, int mode, double dt) {
  if (P.status != 0) {
    if (P.fail_step < 0) P.fail_step = P.step;
    return;
  }
  const int nxt = P.parity ^ 1;
  if (P.pert_on) {
    // reaction on the perturber: minus the pull on every sphere, summed over
    // the per-block partials in block order; then its closing half kick
    double f[3] = {0.0, 0.0, 0.0};
    for (int b = 0; b < P.n_rblk; ++b)
      for (int k = 0; k < 3; ++k) f[k] += P.ppart[b * 3 + k];
    for (int k = 0; k < 3; ++k) {
      const double a = -f[k] / P.pert_M;
      P.pert_a[nxt][k] = a;
      if (mode == kModeStep) P.pert_v[nxt][k] += 0.5 * dt * a;
    }
  }
  P.n_pairs = P.up_off[nxt][P.ns];
  P.parity = nxt;
  if (mode == kModeStep) P.step += 1;
}

}  // namespace

}  // namespace dem
