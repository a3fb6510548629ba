/*
 * oracle.h -- plain FP64 CPU reference of one soft-sphere DEM step for rigid
 * aggregates of bonded spheres (Marohnic et al., arXiv 2311.11322).
 *
 * TEST INFRASTRUCTURE ONLY.  This code exists to check the GPU library
 * against the paper; only the test-suite, the smoke check and the CPU
 * baseline leg of the benchmark may load it.  It shares no source with the
 * GPU library and is deliberately simple: scalar loops, brute-force O(N^2)
 * pair search and gravity, no blocking, no fusion, no reordering.
 *
 * All floating point is IEEE double, compiled without FMA contraction.
 */
#ifndef DEM_ORACLE_H
#define DEM_ORACLE_H
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct {
    double dt;          /* fixed leapfrog step h (Sec. 2.1)                       */
    double G;           /* gravitational constant; 0 disables self-gravity         */
    double soft_frac;   /* Plummer softening eps_ij = soft_frac*(s_i+s_j)/2        */
    double k_n, k_t;    /* normal / tangential spring constants (Sec. 2.1)         */
    double eps_n, eps_t;/* normal / tangential restitution -> dashpot constants    */
    double mu_s, mu_r, mu_t; /* sliding, rolling, twisting friction coefficients   */
    double k_r, k_q;    /* rolling / twisting spring constants                     */
    int32_t periodic;   /* 1: periodic cube of side box[0..2]                      */
    double box[3];
    double spin_dw;     /* spin-up forcing: spin increment per step about +z      */
    int32_t torque_at_centre; /* negative control only: apply contact forces at
                                 sphere centres instead of the contact point       */
    /* box-filling and shaking workloads: uniform acceleration on every body,
     * and up to 6 planar walls n.x = d (unit n pointing into the domain),
     * displaced rigidly by A_w sin(omega t + phase) */
    double g[3];
    int32_t n_walls;
    double wall[6][4];
    double shake_amp[6][3];
    double shake_omega, shake_phase;
    /* tree gravity instead of the direct sum: opening angle theta, leaf size */
    int32_t gravity_tree;
    double theta;
    int32_t tree_leaf;
    int32_t tree_order;  /* 2: monopole + quadrupole; 4: up to hexadecapole */
} ora_params;

typedef struct ora_sim ora_sim;

ora_sim* ora_create(const ora_params* p);
void     ora_destroy(ora_sim* s);

/* Add all aggregates at once.  Spheres are grouped by aggregate.  evaluate=1
 * performs the initial force evaluation at t0 (needed before the first step);
 * evaluate=0 skips it (for sampled checks at sizes where O(N^2) is too slow).
 * Returns 0 on success, <0 on invalid input. */
int ora_add(ora_sim* s, int64_t n_agg, const int32_t* counts,
            const double* pos, const double* radius, const double* mass,
            const double* agg_vel, const double* agg_spin, int32_t evaluate);

int ora_step(ora_sim* s, int64_t n_steps);

/* State read-out (caller-owned buffers, NULL to skip a field). */
void ora_get_counts(const ora_sim* s, int64_t* n_agg, int64_t* n_sph, int64_t* n_pairs);
void ora_get_aggregates(const ora_sim* s, double* M, double* rA, double* vA, double* aA,
                        double* NA, double* q, double* wb, double* wA, double* I);
void ora_get_spheres(const ora_sim* s, double* r, double* v, double* F, double* tau,
                     double* body);
/* Per-pair output of the last evaluation, canonical (i<j, lexicographic);
 * a contact of sphere i with wall w has j = n_sph + w.
 * hist: 7 per pair (xi_t[3], xi_r[3], xi_q).  force: F on i[3], tau_i[3],
 * tau_j[3].  diag: f_N, |F_T|, |F_r|, |F_q|, delta, l_i, l_j, sliding flag. */
void ora_get_pairs(const ora_sim* s, int64_t* pi, int64_t* pj, double* hist,
                   double* force, double* diag);

/* Point-mass perturber (tidal flyby): unsoftened, mass M, integrated by the
 * same leapfrog; every sphere feels G m_i M (r_p - r_i)/|r_p - r_i|^3 and the
 * perturber the sum of the reactions.  Set before ora_add (its t0
 * acceleration comes from the initial evaluation).  get returns pos, vel. */
void ora_set_perturber(ora_sim* s, double M, const double* pos, const double* vel);
void ora_get_perturber(const ora_sim* s, double* pos, double* vel, double* acc);

/* Diagnostics of the current state: out[0..2] linear momentum, out[3..5]
 * angular momentum about the origin, out[6] translational KE, out[7]
 * rotational KE, out[8] normal spring energy, out[9] gravitational energy,
 * out[10] max overlap, out[11] bulk radius, out[12..14] centre of mass,
 * out[15] potential of the uniform field. */
void ora_diagnostics(ora_sim* s, double* out);

/* Forces and torques on a subset of spheres at the current state, evaluated
 * one sphere at a time by brute force (contacts with zero spring history,
 * as at t0, plus direct-sum gravity).  Used for sampled checks at full size. */
void ora_eval_subset(const ora_sim* s, const int64_t* idx, int64_t n_idx,
                     double* F, double* tau);

/* Stateless brute-force contact search: all i<j with agg_i != agg_j and
 * d^2 < (s_i+s_j)^2; box == NULL for open space.  Writes i*2^32+j keys in
 * lexicographic order.  Returns the number of pairs (may exceed cap; only
 * the first cap are written). */
int64_t ora_find_contacts(const double* pos, const double* radius, const int32_t* agg,
                          int64_t n, const double* box, uint64_t* keys, int64_t cap);

/* Direct-sum softened gravity force on the listed targets. */
void ora_gravity(const double* pos, const double* mass, const double* radius, int64_t n,
                 double G, double soft_frac, const int64_t* idx, int64_t n_idx, double* F);

/* Tree gravity (multipoles about each node's centre of mass up to the
 * quadrupole, order 2, or the hexadecapole, order 4; with order >= 2 also the
 * eps^2 term of the softened kernel's expansion, which is of the
 * quadrupole's order).  The paper takes its expansions to hexadecapole order
 * (Sec. 2) and gives no other detail of its tree.
 * The tree: a cube grid over the bounding box of the centres -- bits =
 * ceil(ceil(log2 2n) / 3) levels (2..10), finest cell side
 * max(2 * largest radius, 1.000000000001 * largest extent / 2^bits) -- with
 * spheres ordered by (Morton code of their finest cell, index); node (l, p)
 * holds the spheres whose code has prefix p at level l.  Targets go in
 * groups of 64 consecutive spheres in that order.  A node is taken as a
 * multipole when the distance from its cube's centre to the group's bounding
 * box exceeds side / theta, else as direct (softened) pairs when it holds at
 * most `leaf` spheres or is a finest cell, else it is opened. */
void ora_tree_gravity(const double* pos, const double* mass, const double* radius, int64_t n,
                      double G, double soft_frac, double theta, int32_t leaf, int32_t order,
                      double* F);

/* One fixed Cash-Karp step of the torque-coupled Euler equations for a single
 * body (exposed for the rotation pins).  q[4], wb[3] updated in place; err
 * receives the embedded 4th/5th-order difference norm. */
void ora_rotate(double* q, double* wb, const double* I, const double* N_space, double h,
                double* err);

/* Aggregate set-up of one body (exposed for the inertia pins):
 * M, COM r[3], principal moments I[3], quaternion q[4], body offsets b[3n]. */
int ora_setup_body(int64_t n, const double* pos, const double* radius, const double* mass,
                   double* M, double* r, double* I, double* q, double* b);

/* Contact part of one evaluation on given sphere states (same-input check
 * of the contact model): brute-force search, history carried from the given
 * previous contacts, every contact's force, per-sphere sums in canonical
 * order.  pos, vel [n][3]; agg ids in 0..n_agg-1; agg_mass [n_agg],
 * agg_spin [n_agg][3] space frame; old_keys canonical and sorted (wall w of
 * sphere i: i << 32 | (n + w)), old_hist [n_old][7]; walls at t = 0.
 * Outputs F, tau [n][3], keys [cap], hist [cap][7]; returns the count. */
int64_t ora_contact_forces(const ora_params* p, int64_t n, const double* pos, const double* vel,
                           const double* radius, const int32_t* agg, int64_t n_agg,
                           const double* agg_mass, const double* agg_spin, int64_t n_old,
                           const uint64_t* old_keys, const double* old_hist, double* F,
                           double* tau, uint64_t* keys, double* hist, int64_t cap);

/* Threads used by the gravity target loops (OpenMP); results do not depend
 * on it.  n <= 0 only queries.  Returns the count in effect. */
int32_t ora_set_threads(int32_t n);

#ifdef __cplusplus
}
#endif
#endif
