// kernels_body.hip -- rigid-body kernels: aggregate set-up, kick/drift/rotate,
// member reconstruction, reduction onto aggregates, end-of-step bookkeeping.
//
// Paper references: aggregate mass and centre of mass (Eqs. 1-2); the
// appendix table of aggregate functions (CountPart, GetCOM, GetAxesAndSpin,
// SetBodyPos, SetMassDEM, SetSpacePos/Spin/Vel, GetAccelAndTorque); leapfrog
// for centres of mass and a fifth-order Runge-Kutta step for orientation and
// spin (Sec. 2.1-2.2); predicted member velocity (Eq. 3); aggregate
// acceleration and torque (Eqs. 5-7, 9).
#include "step_body.h"

namespace dem {

namespace {

// ---------------------------------------------------------------------------
// set-up of one aggregate
// ---------------------------------------------------------------------------

// Symmetric 3x3 eigen-decomposition by cyclic Jacobi plane rotations.  a is
// overwritten (eigenvalues on the diagonal); columns of V are eigenvectors.
__device__ void jacobi_eig3(double a[3][3], double V[3][3]) {
  for (int i = 0; i < 3; ++i)
    for (int j = 0; j < 3; ++j) V[i][j] = (i == j) ? 1.0 : 0.0;
  const int P[3] = {0, 0, 1}, Q[3] = {1, 2, 2};
  for (int sweep = 0; sweep < 50; ++sweep) {
    const double off = a[0][1] * a[0][1] + a[0][2] * a[0][2] + a[1][2] * a[1][2];
    const double dia = a[0][0] * a[0][0] + a[1][1] * a[1][1] + a[2][2] * a[2][2];
    if (off == 0.0 || off <= 1e-34 * dia) break;
    for (int k = 0; k < 3; ++k) {
      const int p = P[k], q = Q[k];
      const double apq = a[p][q];
      if (apq == 0.0) continue;
      const double zeta = (a[q][q] - a[p][p]) / (2.0 * apq);
      const double t = (zeta >= 0.0 ? 1.0 : -1.0) / (fabs(zeta) + sqrt(1.0 + zeta * zeta));
      const double c = 1.0 / sqrt(1.0 + t * t);
      const double s = t * c;
      a[p][p] -= t * apq;
      a[q][q] += t * apq;
      a[p][q] = a[q][p] = 0.0;
      const int r = 3 - p - q;
      const double arp = a[r][p], arq = a[r][q];
      a[r][p] = a[p][r] = c * arp - s * arq;
      a[r][q] = a[q][r] = s * arp + c * arq;
      for (int i = 0; i < 3; ++i) {
        const double vip = V[i][p], viq = V[i][q];
        V[i][p] = c * vip - s * viq;
        V[i][q] = s * vip + c * viq;
      }
    }
  }
}

// Unit quaternion of a proper rotation matrix (largest-component branch).
__device__ void rot_to_quat(const double R[3][3], double q[4]) {
  const double t0 = R[0][0] + R[1][1] + R[2][2];
  double w, x, y, z;
  if (t0 >= R[0][0] && t0 >= R[1][1] && t0 >= R[2][2]) {
    const double f = 2.0 * sqrt(1.0 + t0);
    w = 0.25 * f;
    x = (R[2][1] - R[1][2]) / f;
    y = (R[0][2] - R[2][0]) / f;
    z = (R[1][0] - R[0][1]) / f;
  } else if (R[0][0] >= R[1][1] && R[0][0] >= R[2][2]) {
    const double f = 2.0 * sqrt(1.0 + R[0][0] - R[1][1] - R[2][2]);
    w = (R[2][1] - R[1][2]) / f;
    x = 0.25 * f;
    y = (R[0][1] + R[1][0]) / f;
    z = (R[0][2] + R[2][0]) / f;
  } else if (R[1][1] >= R[2][2]) {
    const double f = 2.0 * sqrt(1.0 + R[1][1] - R[0][0] - R[2][2]);
    w = (R[0][2] - R[2][0]) / f;
    x = (R[0][1] + R[1][0]) / f;
    y = 0.25 * f;
    z = (R[1][2] + R[2][1]) / f;
  } else {
    const double f = 2.0 * sqrt(1.0 + R[2][2] - R[0][0] - R[1][1]);
    w = (R[1][0] - R[0][1]) / f;
    x = (R[0][2] + R[2][0]) / f;
    y = (R[1][2] + R[2][1]) / f;
    z = 0.25 * f;
  }
  const double inv = 1.0 / sqrt(w * w + x * x + y * y + z * z);
  q[0] = w * inv;
  q[1] = x * inv;
  q[2] = y * inv;
  q[3] = z * inv;
}

// One thread per aggregate: CountPart/GetCOM (Eqs. 1-2), the inertia tensor
// about the centre of mass with each sphere's own 2/5 m s^2, its principal
// axes (GetAxesAndSpin) as a proper rotation and quaternion, body offsets
// (SetBodyPos) and the body-frame spin.  pos_in/vel_in/spin_in are the
// caller's row-major arrays copied to the device.
__global__ __launch_bounds__(kBlock) void k_setup(const PileDev* __restrict__ piles,
                                                  const WorkItem* __restrict__ wl,
                                                  const double* __restrict__ pos_in,
                                                  const double* __restrict__ vel_in,
                                                  const double* __restrict__ spin_in) {
  const WorkItem w = wl[xcd_block(blockIdx.x, gridDim.x)];
  const PileDev& P = piles[w.pile];
  const int A = w.base + threadIdx.x;
  if (A >= P.na) return;
  const int i0 = P.first[A], n = P.count[A];
  double M = 0.0, c[3] = {0.0, 0.0, 0.0};
  for (int i = i0; i < i0 + n; ++i) M += P.m[i];
  for (int i = i0; i < i0 + n; ++i)
    for (int k = 0; k < 3; ++k) c[k] += P.m[i] * pos_in[3 * i + k];
  for (int k = 0; k < 3; ++k) c[k] /= M;
  double T[3][3] = {{0, 0, 0}, {0, 0, 0}, {0, 0, 0}};
  for (int i = i0; i < i0 + n; ++i) {
    const double d[3] = {pos_in[3 * i] - c[0], pos_in[3 * i + 1] - c[1], pos_in[3 * i + 2] - c[2]};
    const double mi = P.m[i];
    const double tr = d[0] * d[0] + d[1] * d[1] + d[2] * d[2] + 0.4 * P.s[i] * P.s[i];
    for (int a = 0; a < 3; ++a)
      for (int b = 0; b < 3; ++b) T[a][b] += mi * ((a == b ? tr : 0.0) - d[a] * d[b]);
  }
  double V[3][3];
  jacobi_eig3(T, V);
  // right-handed axes
  const double c0[3] = {V[0][0], V[1][0], V[2][0]}, c1[3] = {V[0][1], V[1][1], V[2][1]},
               c2[3] = {V[0][2], V[1][2], V[2][2]};
  double x01[3];
  cross3(c0, c1, x01);
  if (dot3(x01, c2) < 0.0)
    for (int a = 0; a < 3; ++a) V[a][2] = -V[a][2];
  double q[4], R[9];
  rot_to_quat(V, q);
  quat_rot(q, R);
  for (int i = i0; i < i0 + n; ++i) {
    const double d[3] = {pos_in[3 * i] - c[0], pos_in[3 * i + 1] - c[1], pos_in[3 * i + 2] - c[2]};
    double bb[3];
    rot_apply_T(R, d, bb);
    for (int k = 0; k < 3; ++k) P.b[k * P.ns + i] = bb[k];
  }
  const int cur = P.parity;
  P.M[A] = M;
  for (int k = 0; k < 3; ++k) {
    P.I[k * P.na + A] = T[k][k];
    double x = c[k];
    if (P.periodic) {
      const double L = P.box;
      x = x - L * floor(x / L);
      if (x >= L) x -= L;
    }
    P.rA[cur][k * P.na + A] = x;
    P.vA[cur][k * P.na + A] = vel_in ? vel_in[3 * A + k] : 0.0;
    P.aA[cur][k * P.na + A] = 0.0;
    P.NA[cur][k * P.na + A] = 0.0;
  }
  double ws[3] = {0.0, 0.0, 0.0}, wbv[3];
  if (spin_in)
    for (int k = 0; k < 3; ++k) ws[k] = spin_in[3 * A + k];
  rot_apply_T(R, ws, wbv);
  for (int k = 0; k < 3; ++k) P.wb[cur][k * P.na + A] = wbv[k];
  for (int k = 0; k < 4; ++k) P.q[cur][k * P.na + A] = q[k];
}

// One thread per aggregate.  Step mode: v_A += h/2 a_A, r_A += h v_A (wrapped
// in a periodic cube), one RK5 step of (q, w_b) with the last torque.  Writes
// the next state, the space-frame spin w_A = R w_b and the predicted
// centre-of-mass velocity v_A + h/2 a_A (first bracket of Eq. 3).  Init mode
// copies the state unchanged (evaluation at t0).
__global__ __launch_bounds__(kBlock) void k_integrate(PileDev* __restrict__ piles,
                                                      const WorkItem* __restrict__ wl,
                                                      ContactParams cp, int mode) {
  const WorkItem w = wl[xcd_block(blockIdx.x, gridDim.x)];
  PileDev& P = piles[w.pile];
  const int A = w.base + threadIdx.x;
  if (A >= P.na || P.status != 0) return;
  integrate_one(P, A, cp, mode);
}

// ---------------------------------------------------------------------------
// member reconstruction (SetSpacePos / SetSpaceSpin / SetSpaceVel, Eq. 3)
// ---------------------------------------------------------------------------

// One thread per sphere: r_i = r_A + R b_i and v_i = vpred_A + w_A x (R b_i)
// (a pile without aggregates, or with given sphere states, keeps the
// positions and velocities it was given).  Each block
// also writes the bounding box and mass moments of its spheres
// for the per-pile cell grid.
__global__ __launch_bounds__(kBlock) void k_reconstruct(const PileDev* __restrict__ piles,
                                                        const WorkItem* __restrict__ wl) {
  const WorkItem w = wl[xcd_block(blockIdx.x, gridDim.x)];
  const PileDev& P = piles[w.pile];
  if (P.status != 0) return;
  const int i = w.base + threadIdx.x;
  double vals[kBbox];
  bbox_identity(vals);
  double cref[3];
  bbox_ref(P, cref);
  if (i < P.ns) reconstruct_one(P, i, cref, vals);
  // block reduction (wave shuffles, then across the 4 waves through LDS)
  __shared__ double red[4][kBbox];
  for (int off = 32; off > 0; off >>= 1) {
    for (int k = 0; k < 3; ++k) vals[k] = fmin(vals[k], __shfl_xor(vals[k], off));
    for (int k = 3; k < 6; ++k) vals[k] = fmax(vals[k], __shfl_xor(vals[k], off));
    for (int k = 6; k < kBbox; ++k) vals[k] += __shfl_xor(vals[k], off);
  }
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  if (lane == 0)
    for (int k = 0; k < kBbox; ++k) red[wave][k] = vals[k];
  __syncthreads();
  if (threadIdx.x == 0) {
    double* out = P.bpart + (size_t)(w.base / kBlock) * kBbox;
    for (int k = 0; k < kBbox; ++k) {
      double x = red[0][k];
      for (int j = 1; j < 4; ++j) {
        const double y = red[j][k];
        x = (k < 3) ? fmin(x, y) : (k < 6 ? fmax(x, y) : x + y);
      }
      out[k] = x;
    }
  }
}

// One block of kGridThreads per pile: the reconstruction's block partials
// combined (each thread its share in block order, then across the block)
// into the pile's bounding box and mass moments, and from them the cell grid,
// centre of mass and bulk radius (grid_from_vals).
constexpr int kGridThreads = 256;
__global__ __launch_bounds__(kGridThreads) void k_grid(PileDev* __restrict__ piles, int mode,
                                                       double dt) {
  PileDev& P = piles[blockIdx.x];
  if (P.status != 0 || P.fused) return;
  double vals[kBbox] = {INFINITY, INFINITY, INFINITY, -INFINITY, -INFINITY, -INFINITY,
                        0.0, 0.0, 0.0, 0.0, 0.0};
  // unrolled so that several partials' loads are in flight (same order)
#pragma unroll 4
  for (int b = threadIdx.x; b < P.n_rblk; b += kGridThreads) {
    const double* p = P.bpart + (size_t)b * kBbox;
    for (int k = 0; k < 3; ++k) vals[k] = fmin(vals[k], p[k]);
    for (int k = 3; k < 6; ++k) vals[k] = fmax(vals[k], p[k]);
    for (int k = 6; k < kBbox; ++k) vals[k] += p[k];
  }
  for (int off = 32; off > 0; off >>= 1) {
    for (int k = 0; k < 3; ++k) vals[k] = fmin(vals[k], __shfl_xor(vals[k], off));
    for (int k = 3; k < 6; ++k) vals[k] = fmax(vals[k], __shfl_xor(vals[k], off));
    for (int k = 6; k < kBbox; ++k) vals[k] += __shfl_xor(vals[k], off);
  }
  __shared__ double red[kGridThreads / 64][kBbox];
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  if (lane == 0)
    for (int k = 0; k < kBbox; ++k) red[wave][k] = vals[k];
  __syncthreads();
  if (threadIdx.x != 0) return;
  for (int k = 0; k < kBbox; ++k) {
    double x = red[0][k];
    for (int j = 1; j < kGridThreads / 64; ++j) {
      const double y = red[j][k];
      x = (k < 3) ? fmin(x, y) : (k < 6 ? fmax(x, y) : x + y);
    }
    vals[k] = x;
  }
  grid_from_vals(P, vals, mode, dt);
}

// ---------------------------------------------------------------------------
// GetAccelAndTorque (Eqs. 5-7, 9) and the closing half kick
// ---------------------------------------------------------------------------

// One thread per aggregate: F_A = sum F_i (F_i a member's contact force,
// plus its gravity force in a pile with gravity), a_A = F_A / M + g,
// N_A = sum [ (R b_i) x F_i + tau_i ] over the members in order, and in step
// mode v_A += h/2 a_A followed by the spin-up increment about +z through the
// pile's centre.  Members are added in member order, read in one of two
// ways with the same arithmetic:
// * direct (launches of few aggregates): each lane reads its members;
// * staged (many aggregates): lanes ~5 spheres apart would re-fetch each
//   line once per member, the lines leaving L2 between a wave's member
//   iterations, so a wave's 64 aggregates -- one contiguous run of
//   spheres -- pass through the wave's LDS slice 64 spheres at a time (one
//   coalesced load per array) and each lane adds the members in the slice.
// The launch chooses (stage: at least kReduceStageMin aggregates) unless the
// pile's tuning fixes one way.
__global__ __launch_bounds__(kBlock) void k_reduce(const PileDev* __restrict__ piles,
                                                   const WorkItem* __restrict__ wl,
                                                   ContactParams cp, int mode, int stage) {
  __shared__ double sh_all[kBlock / 64][9][64];
  const WorkItem w = wl[xcd_block(blockIdx.x, gridDim.x)];
  const PileDev& P = piles[w.pile];
  const int na = P.na, ns = P.ns, nxt = P.parity ^ 1;
  const int wv = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int a0 = w.base + wv * 64;               // the wave's first aggregate
  if (a0 >= na || P.status != 0) return;         // uniform over the wave
  const int A = a0 + lane;
  const bool own = A < na;
  double (*sh)[64] = sh_all[wv];
  double R[9];
  if (own) {
    double q[4];
    for (int k = 0; k < 4; ++k) q[k] = P.q[nxt][k * na + A];
    quat_rot(q, R);
  }
  double FA[3] = {0.0, 0.0, 0.0}, NA[3] = {0.0, 0.0, 0.0};
  if (P.member_scan != 0) {
    // ablation of the paper's original routines: every sphere of the pile
    // tested for membership, in order
    if (own) reduce_members_scan(P, A, R, FA, NA);
  } else if (P.member_read == 1 || (P.member_read == 0 && !stage)) {
    if (own) reduce_members_direct(P, A, R, FA, NA);
  } else {
    const int a_last = min(a0 + 64, na) - 1;
    const int s0 = P.first[a0], s1 = P.first[a_last] + P.count[a_last];
    const int m0 = own ? P.first[A] : 0, m1 = own ? m0 + P.count[A] : 0;
    // Loads through the global address space: a generic load would also
    // count against the LDS wait counter that the slice reads wait on.  The
    // next slice's nine loads are in flight while the lanes add this one.
    typedef const __attribute__((address_space(1))) double* GlobalD;
    const GlobalD gF = (GlobalD)P.F, gb = (GlobalD)P.b, gt = (GlobalD)P.tau;
    const GlobalD gg = (GlobalD)P.gacc;
    const bool grav = P.G != 0.0;
    double v[9];
    auto fetch = [&](int c) {
      const int t = c + lane;
      if (t < s1)
        for (int k = 0; k < 3; ++k) {
          v[k] = gF[k * ns + t];
          if (grav) v[k] += gg[k * ns + t];     // gravity after the contacts
          v[3 + k] = gb[k * ns + t];
          v[6 + k] = gt[k * ns + t];
        }
    };
    fetch(s0);
    for (int c0 = s0; c0 < s1; c0 += 64) {
      if (c0 + lane < s1)
        for (int k = 0; k < 9; ++k) sh[k][lane] = v[k];
      if (c0 + 64 < s1) fetch(c0 + 64);
      __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
      __builtin_amdgcn_wave_barrier();
      __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
      for (int i = max(m0, c0), i1 = min(m1, c0 + 64); i < i1; ++i) {
        const int l = i - c0;
        const double f[3] = {sh[0][l], sh[1][l], sh[2][l]};
        const double bb[3] = {sh[3][l], sh[4][l], sh[5][l]};
        const double tau[3] = {sh[6][l], sh[7][l], sh[8][l]};
        add_member(R, f, bb, tau, FA, NA);
      }
      // every lane has read the slice before the next pass overwrites it
      __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
      __builtin_amdgcn_wave_barrier();
      __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    }
  }
  if (!own) return;
  reduce_tail(P, A, R, FA, NA, cp, mode);
}

// One thread per pile: commit the step (flip the ping-pong halves) unless
// the pile failed during it, in which case its state stays at the failing
// step's start and the step index is recorded.
__global__ void k_finish(PileDev* __restrict__ piles, int n_piles, int mode, double dt) {
  const int p = blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= n_piles) return;
  PileDev& P = piles[p];
  if (P.fused) return;                       // k_fused finishes it
  finish_one(P, mode, dt);
}

__global__ void k_fill_u32(uint32_t* __restrict__ p, uint32_t value, int64_t n) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = value;
}

}  // namespace

void launch_setup(hipStream_t st, const PileDev* piles, const WorkItem* wl, int nblk,
                  const double* pos_in, const double* vel_in, const double* spin_in) {
  hipLaunchKernelGGL(k_setup, dim3(nblk), dim3(kBlock), 0, st, piles, wl, pos_in, vel_in, spin_in);
}

void launch_integrate(hipStream_t st, const PileDev* piles, const WorkItem* wl, int nblk,
                      ContactParams cp, int mode) {
  hipLaunchKernelGGL(k_integrate, dim3(nblk), dim3(kBlock), 0, st, const_cast<PileDev*>(piles), wl,
                     cp, mode);
}

void launch_reconstruct(hipStream_t st, const PileDev* piles, const WorkItem* wl, int nblk) {
  hipLaunchKernelGGL(k_reconstruct, dim3(nblk), dim3(kBlock), 0, st, piles, wl);
}

void launch_grid(hipStream_t st, const PileDev* piles, int n_piles, int mode, double dt) {
  hipLaunchKernelGGL(k_grid, dim3(n_piles), dim3(kGridThreads), 0, st, const_cast<PileDev*>(piles),
                     mode, dt);
}

void launch_reduce(hipStream_t st, const PileDev* piles, const WorkItem* wl, int nblk,
                   ContactParams cp, int mode, bool stage) {
  hipLaunchKernelGGL(k_reduce, dim3(nblk), dim3(kBlock), 0, st, piles, wl, cp, mode, (int)stage);
}

void launch_finish(hipStream_t st, PileDev* piles, int n_piles, int mode, double dt) {
  hipLaunchKernelGGL(k_finish, dim3((n_piles + 63) / 64), dim3(64), 0, st, piles, n_piles, mode,
                     dt);
}

void launch_fill_u32(hipStream_t st, uint32_t* p, uint32_t value, int64_t n) {
  if (n <= 0) return;
  hipLaunchKernelGGL(k_fill_u32, dim3((unsigned)((n + kBlock - 1) / kBlock)), dim3(kBlock), 0, st,
                     p, value, n);
}

}  // namespace dem
