/*
 * dem.h -- C-ABI of the MI355X soft-sphere DEM step for rigid aggregates of
 * bonded spheres (Marohnic et al., arXiv 2311.11322).
 *
 * The library (libdem.so, HIP for gfx950) integrates systems ("piles") of
 * rigid aggregates.  Each step: leapfrog kick and drift of aggregate centres
 * of mass, a fifth-order Runge-Kutta step of Euler's rigid-body equations
 * (Sec. 2.1-2.2 of the paper), reconstruction of member positions and
 * predicted velocities (Eq. 3 and the SetSpace* functions of the appendix
 * table), contact search that skips pairs inside one aggregate, spring-
 * dashpot contacts with tangential/rolling/twisting spring history applied
 * at the contact point (Sec. 2.1, Eqs. 8-9), softened direct-sum self-gravity
 * (Eq. 4) and the reduction onto aggregates (Eqs. 5-7, 9; GetAccelAndTorque).
 *
 * Conventions for every call:
 *  - Every function returns dem_status; nothing aborts or throws across the
 *    ABI.  On error, dem_last_error(sim) describes it.
 *  - Pointers documented as host arrays are read (or written) before the
 *    call returns; the caller keeps ownership.
 *  - Arrays of 3-vectors are row-major [n][3] (x, y, z), quaternions [n][4]
 *    (w, x, y, z) mapping body frame to space frame.
 *  - Sphere ids are input positions (0-based, grouped by aggregate);
 *    aggregate ids are consecutive in call order.  Both are persistent and
 *    define the canonical contact order: pairs (i, j), i < j, sorted
 *    lexicographically, keyed as (uint64)i << 32 | j.
 *  - Device memory is owned by the library and obtained through the
 *    caller's allocator (NULL: hipMalloc/hipFree).  All device work is
 *    issued on the stream given at creation (NULL: the null stream).
 */
#ifndef DEM_H
#define DEM_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    DEM_OK = 0,
    DEM_ERR_INVALID_ARG = -1,  /* bad pointer, size, non-finite value, radius or mass <= 0 */
    DEM_ERR_OOM = -2,          /* allocation failed, or an engine's memory budget is exceeded */
    DEM_ERR_CAPACITY = -3,     /* contact capacity exceeded; state rolled back to the failing step's start */
    DEM_ERR_UNSTABLE = -4,     /* non-finite force or overlap > max_overlap_frac*radius; rolled back */
    DEM_ERR_DEVICE = -5,       /* a HIP call failed */
    DEM_ERR_STATE = -6,        /* call out of order (e.g. adding aggregates after stepping) */
    DEM_STOPPED = 1            /* not an error: the system's stop rule fired (dem_forcing);
                                  its state is that at the start of the stopping step */
} dem_status;

typedef enum {
    DEM_PREC_FP64 = 0,         /* every force in FP64 */
    DEM_PREC_FP32_FORCE = 1    /* pair forces and gravity in FP32 on relative coordinates;
                                  positions, velocities, quaternions, accumulation in FP64 */
} dem_precision;

/* Model parameters.  Spring and damping constants are user parameters of
 * the soft-sphere model (Sec. 2.1); the time step is fixed (Sec. 2.1). */
typedef struct {
    double dt;                 /* leapfrog step h > 0 */
    double G;                  /* gravitational constant; 0 disables self-gravity */
    double softening_frac;     /* Plummer eps_ij = softening_frac*(s_i+s_j)/2 (>= 0) */
    double k_n, k_t;           /* normal and tangential spring constants (> 0) */
    double eps_n, eps_t;       /* restitution coefficients in (0, 1]; set the dashpots */
    double mu_s, mu_r, mu_t;   /* sliding, rolling, twisting friction coefficients (>= 0) */
    double k_r, k_q;           /* rolling and twisting spring constants; < 0 means k_t */
    int32_t periodic;          /* 1: periodic cube box[0..2] (same side on all axes) */
    double box[3];
    int32_t precision;         /* dem_precision */
    int32_t max_contacts_per_sphere; /* contact capacity: the system holds up to this many
                                        contacts per sphere on average; <= 0: 8 */
    double max_overlap_frac;   /* > 0: overlap above this fraction of the smaller radius is
                                  an instability (DEM_ERR_UNSTABLE); <= 0: no check */
    /* Container and uniform field of the box-filling and shaking workloads
     * (Sec. 3.3 performance-scaling runs, Sec. 4.3 Brazil-nut runs).  g is added to the
     * acceleration of every body.  Wall w is the plane n.x = d with
     * walls[w] = {n_x, n_y, n_z, d}, n a unit normal pointing into the domain,
     * displaced rigidly by shake_amp[w] * sin(shake_omega * t + shake_phase)
     * at time t = step * dt.  A wall is a contact partner of infinite mass
     * and no spin under the same contact model as a sphere pair; the contact
     * of sphere i with wall w has the key i * 2^32 + (n_sph + w).  Walls need
     * an open system (periodic == 0). */
    double g[3];
    int32_t n_walls;           /* 0 .. 6 */
    double walls[6][4];
    double shake_amp[6][3];
    double shake_omega, shake_phase;
    /* Tree gravity instead of the exact direct sum (the paper's own gravity
     * is a tree code with multipoles to hexadecapole order, Sec. 2): a node
     * of the pyramid of the pile's cubic cell grid acts on a group of 64
     * spheres through its multipoles about its centre of mass, to order
     * tree_order (2: quadrupole, 4: hexadecapole), plus the eps^2 term of the
     * softened kernel's expansion, when its cube's centre is farther from the
     * group's bounding box than side / tree_theta; through softened pairs
     * when it holds at most tree_leaf spheres; FP64 in both precisions.
     * Needs an open system; 0 < tree_theta <= 1, 1 <= tree_leaf <= 4096,
     * tree_order 2 or 4. */
    int32_t gravity_tree;
    double tree_theta;
    int32_t tree_leaf;
    int32_t tree_order;
} dem_params;

typedef struct {
    void* (*alloc)(size_t bytes, void* ctx);  /* returns device memory or NULL */
    void (*free)(void* ptr, void* ctx);
    void* ctx;
} dem_allocator;

/* Optional forcing of one system.  Spin-up (Sec. 4.1: a constant spin
 * increment per step about +z through the system's centre of mass) and a
 * tidal perturber (Sec. 4.2: a point mass passing the system), which is an
 * unsoftened point mass integrated by the same leapfrog: every sphere feels
 * G m_i M (r_p - r_i)/|r_p - r_i|^3 and the perturber the sum of the
 * reactions.  Requires G > 0. */
typedef struct {
    double spin_dw;            /* spin increment per step (rad per time unit); 0: off */
    double pert_mass;          /* perturber mass; 0: no perturber */
    double pert_pos[3];        /* perturber position */
    double pert_vel[3];        /* perturber velocity */
    double stop_growth;        /* > 0: stop rule of a spin-up run (Sec. 4.1: the pile has
                                  failed once its bulk radius has grown by 5 %, i.e. 1.05):
                                  the first evaluation after dem_set_forcing records the bulk
                                  radius R0 = sqrt(5/3 <|r_i - r_com|^2>_m) of the sphere
                                  centres; the first step whose evaluation finds
                                  R >= stop_growth * R0 is not committed and the system stops
                                  (dem_step / dem_sim_status report DEM_STOPPED, the step
                                  index in dem_state.step).  Setting the forcing again
                                  re-arms the rule and lets a stopped system go on. */
} dem_forcing;

/* State read-out / restore.  Caller-owned host buffers sized by
 * dem_get_counts; a NULL field is skipped.  Sphere fields describe the last
 * force evaluation. */
typedef struct {
    double* agg_pos;           /* [n_agg][3] centre of mass r_A */
    double* agg_vel;           /* [n_agg][3] centre-of-mass velocity v_A */
    double* agg_acc;           /* [n_agg][3] last evaluated a_A */
    double* agg_torque;        /* [n_agg][3] last evaluated torque N_A (space frame) */
    double* agg_quat;          /* [n_agg][4] orientation (body -> space) */
    double* agg_spin;          /* [n_agg][3] spin, space frame (read only) */
    double* agg_spin_body;     /* [n_agg][3] spin, body frame */
    double* agg_mass;          /* [n_agg] total mass M (Eq. 1) (read only) */
    double* agg_inertia;       /* [n_agg][3] principal moments (read only) */
    double* sph_pos;           /* [n_sph][3] space-frame centres (read only) */
    double* sph_vel;           /* [n_sph][3] predicted velocities, Eq. 3 (read only) */
    double* sph_force;         /* [n_sph][3] contact + gravity force (read only) */
    double* sph_torque;        /* [n_sph][3] contact torque about the centre (read only) */
    double* sph_body;          /* [n_sph][3] body-frame offsets (read only) */
    uint64_t* pair_keys;       /* [n_pairs] canonical contact keys */
    double* pair_hist;         /* [n_pairs][7] spring history xi_t[3], xi_r[3], xi_q */
    int64_t n_pairs;           /* out: contacts written; in (restore): contacts given */
    int64_t step;              /* out: steps taken; in (restore): step counter */
} dem_state;

typedef struct dem_sim dem_sim;
typedef struct dem_engine dem_engine;

/* Create an empty system.  Validates parameters (dt > 0, springs > 0,
 * restitution in (0, 1], frictions >= 0, positive box if periodic). */
dem_status dem_create(const dem_params* params, const dem_allocator* alloc,
                      void* hip_stream, dem_sim** out);

/* Add rigid aggregates (Sec. 2.2: spheres fixed into rigid bodies, each with
 * a unique index).  May be called only once per system, before dem_step.
 * Spheres are grouped by aggregate: aggregate a owns the next
 * spheres_per_agg[a] entries.  sphere_pos is space-frame [n_sph][3];
 * agg_vel ([n_agg][3], centre-of-mass velocity) and agg_spin ([n_agg][3],
 * space frame) may be NULL (zero).  Performs the aggregate set-up on the
 * device (Eqs. 1-2, inertia and principal axes, body offsets, aggregate mass
 * per member) and the initial force evaluation at t0.  first_agg_id (may be
 * NULL) receives the id of the first aggregate (always 0).
 * Errors: INVALID_ARG for an empty aggregate, non-finite value, radius or
 * mass <= 0; STATE if called
 * twice or after stepping; CAPACITY if the initial contacts do not fit. */
dem_status dem_add_aggregates(dem_sim* sim, int64_t n_agg, const int32_t* spheres_per_agg,
                              const double* sphere_pos, const double* sphere_radius,
                              const double* sphere_mass, const double* agg_vel,
                              const double* agg_spin, int64_t* first_agg_id);

/* Advance n_steps fixed steps (replays of one captured HIP graph).  Returns
 * after the work is complete.  On CAPACITY / UNSTABLE (and on DEM_STOPPED,
 * the stop rule of dem_forcing) the state is that at the start of the
 * failing step and dem_state.step tells which step it is.
 * STATE if the system is attached to an engine or has no aggregates. */
dem_status dem_step(dem_sim* sim, int64_t n_steps);

/* Copy the state to host buffers (synchronises the stream). */
dem_status dem_read_state(dem_sim* sim, dem_state* out);

/* Counts: aggregates, spheres, contacts of the last evaluation. */
dem_status dem_get_counts(const dem_sim* sim, int64_t* n_agg, int64_t* n_sph, int64_t* n_pairs);

/* Set the forcing.  A perturber set before dem_add_aggregates gets its t0
 * acceleration from the initial evaluation; set later, its acceleration
 * starts at zero until the next evaluation. */
dem_status dem_set_forcing(dem_sim* sim, const dem_forcing* forcing);
/* Current forcing, with the perturber's position and velocity now. */
dem_status dem_get_forcing(dem_sim* sim, dem_forcing* out);

/* Restore aggregate state, contact list and spring history from a checkpoint
 * written by dem_read_state (fields agg_pos, agg_vel, agg_acc, agg_torque,
 * agg_quat, agg_spin_body, pair_keys, pair_hist, n_pairs, step).  Resuming
 * reproduces the uninterrupted run bit for bit.  A perturber is not part of
 * the checkpoint (dem_get_forcing / dem_set_forcing carry its position and
 * velocity). */
dem_status dem_restore_state(dem_sim* sim, const dem_state* in);

/* Grow the contact capacity (per sphere, each side) after DEM_ERR_CAPACITY. */
dem_status dem_reserve_contacts(dem_sim* sim, int32_t max_contacts_per_sphere);

/* Stateless contact search on the device (test hook): all i<j with
 * agg[i] != agg[j] and d^2 < (s_i+s_j)^2, d^2 = (dx*dx + dy*dy) + dz*dz with
 * the minimum-image rule when box != NULL (cube of side box[0]).  Host arrays
 * in; canonical keys out (up to cap); *n_out gets the total count.
 * n = 0 is an empty search (*n_out = 0, the arrays may be NULL).
 * CAPACITY if more than 64 contacts per sphere are found. */
dem_status dem_find_contacts(const double* pos, const double* radius, const int32_t* agg,
                             int64_t n, const double* box, uint64_t* pairs_out, int64_t cap,
                             int64_t* n_out);

/* Contact forces of given sphere states (test hook, so that a checker can
 * evaluate the contact model on exactly the same FP64 input): one evaluation
 * of the contact part of a step -- search skipping pairs of one aggregate,
 * spring history carried from the given previous contacts, the contact force
 * of every contact (Sec. 2.1, 2.2.4, 2.2.5; Eqs. 8-9) and the per-sphere sums
 * in canonical order -- without motion, gravity or the aggregate reduction.
 * Walls of params are evaluated at t = 0; params->G is ignored.  Host arrays:
 *   pos, vel  [n][3] sphere centres and velocities (the predicted velocities
 *             of Eq. 3)
 *   radius    [n]; agg [n] aggregate of each sphere, 0 .. n_agg-1
 *   agg_mass  [n_agg] aggregate masses (the reduced mass of a contact is
 *             formed from them); agg_spin [n_agg][3] space-frame spins
 *   old_keys  [n_old] canonical sorted keys of the previous contacts (a wall
 *             w of a sphere i is i << 32 | (n + w)); old_hist [n_old][7]
 *   force, torque  out [n][3]: contact force on each sphere and contact
 *             torque about its centre
 *   keys_out, hist_out  out [cap] and [cap][7]: the new contacts and their
 *             updated history (the first cap); *n_out gets the count.
 * Precision and contact capacity (default 16 per sphere) from params.
 * Errors: INVALID_ARG (sizes, non-finite values, unsorted keys), CAPACITY,
 * UNSTABLE (non-finite force). */
dem_status dem_contact_forces(const dem_params* params, int64_t n, const double* pos,
                              const double* vel, const double* radius, const int32_t* agg,
                              int64_t n_agg, const double* agg_mass, const double* agg_spin,
                              int64_t n_old, const uint64_t* old_keys, const double* old_hist,
                              double* force, double* torque, uint64_t* keys_out,
                              double* hist_out, int64_t cap, int64_t* n_out);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid allocation): the
 * stateless contact search of dem_find_contacts on arrays already in device
 * memory, allocating nothing.  Every scratch buffer of the search (cell
 * table, sorted copies, contact runs, work lists) lives in one static device
 * array of 40 MiB, which each GPU the library runs on holds until the process
 * ends; it is found on the current device.
 *   pos     device [n][3] row-major sphere centres
 *   radius  device [n] radii (> 0, finite)
 *   agg     device [n] aggregate ids; pairs with equal ids never count
 *   box     host pointer to the periodic cube side (box[0]), or NULL (open)
 *   pairs_out device [cap] canonical keys i << 32 | j, in order; the first
 *           cap are written
 *   n_out   host; total number of contacts
 *   hip_stream  stream the work is issued on (NULL: the null stream); the
 *           call returns after the work is complete
 * Limits: n <= 65536 spheres and at most 1,048,576 contacts (CAPACITY
 * beyond, with *n_out the total found).  INVALID_ARG for larger n, a
 * non-positive or non-finite radius, a non-finite position or box.
 * Calls on one GPU share its scratch array: calls that overlap in time on
 * the same GPU (other threads or streams) race and must not be made. */
dem_status dem_find_contacts_noalloc(const double* pos, const double* radius,
                                     const int32_t* agg, int64_t n, const double* box,
                                     uint64_t* pairs_out, int64_t cap, int64_t* n_out,
                                     void* hip_stream);

dem_status dem_destroy(dem_sim* sim);

/* Description of the last error on this system (or the last global error if
 * sim is NULL).  Never NULL. */
const char* dem_last_error(const dem_sim* sim);

/* ---- batching and serving -------------------------------------------------
 * An engine steps many independent systems together: every kernel of a step
 * covers all attached systems in one launch, one HIP graph per step.  State
 * and contact history stay in each system's own device buffers. */

/* hbm_budget_bytes: total device footprint the attached systems may use. */
dem_status dem_engine_create(size_t hbm_budget_bytes, void* hip_stream, dem_engine** out);
/* Attach a system that has aggregates.  OOM if its footprint exceeds the free
 * budget; INVALID_ARG if its contact parameters or time step differ from
 * those already attached. */
dem_status dem_engine_attach(dem_engine* eng, dem_sim* sim);
/* Advance every attached system by n_steps.  A system that fails (or whose
 * stop rule fires) stops, rolled back to that step's start, while the others
 * continue; the return value is the first failure code (a stopped system is
 * not a failure), and dem_sim_status tells which. */
dem_status dem_engine_step(dem_engine* eng, int64_t n_steps);
dem_status dem_engine_detach(dem_engine* eng, dem_sim* sim);
dem_status dem_engine_destroy(dem_engine* eng);
/* Per-kernel timing of an engine's steps, as dem_set_profiling /
 * dem_get_profile for one system with enabled = 1 (eager launches with a HIP
 * event between consecutive kernels while enabled is nonzero; totals in
 * milliseconds in the order of dem_profile_names). */
dem_status dem_engine_set_profiling(dem_engine* eng, int32_t enabled);
dem_status dem_engine_get_profile(const dem_engine* eng, double* kernel_ms, int32_t n_max,
                                  int64_t* n_steps);
/* Status of one system after an engine step (DEM_OK, DEM_STOPPED or the
 * failure code). */
dem_status dem_sim_status(const dem_sim* sim);

/* Launch-shape tuning of one system, set before dem_add_aggregates (the
 * buffers are sized from it).  gravity_tile: spheres per gravity tile, one of
 * the sizes dem_gravity_tiles lists for the system's precision (0: default);
 * cell_scale >= 1 multiplies the contact cell side (at least the largest
 * sphere diameter).  Results do not depend on cell_scale; gravity_tile changes
 * the summation order of gravity (rounding only).  An engine may hold systems
 * with different tunings. */
typedef struct {
    int32_t gravity_tile;
    double cell_scale;
    int32_t member_scan;       /* 1: GetAccelAndTorque finds each aggregate's members by a
                                  full scan of the sphere list, as the paper's original
                                  routines did (Sec. 3.1); 0: contiguous member segments
                                  (the paper's improvement).  Same results, different cost. */
    int32_t member_read;       /* how the member segments are read (member_scan 0):
                                  0 automatic -- staged through LDS, a wave's run of spheres
                                  at a time, in launches of at least 131,072 aggregates,
                                  else each aggregate's members directly; 1 directly;
                                  2 staged.  Same order and arithmetic, so the same
                                  results; different cost. */
    int32_t fused;             /* 0 automatic -- the whole step of the system in one
                                  workgroup (one launch per step for a batch of such systems;
                                  with gravity, two launches around the batched gravity
                                  kernels) when it has at most 256 spheres; 1 always; 2 never
                                  (one launch per stage).  Never with tree gravity.  The same
                                  arithmetic per element; the centre of mass and bulk radius
                                  are summed in another order (spin-up, stop rule). */
    int32_t gravity_form;      /* form of the exact softened sum (Eq. 4): 0 automatic --
                                  pairs unless their partial sums would exceed 64 GiB;
                                  1 pairs: each unordered pair once, on super-tiles of
                                  ceil(tiles / 256) tiles, one partial sum per sphere and
                                  super-tile (at most 256 x 3 values per sphere); 2 per
                                  target: each ordered pair from its target's side, one
                                  partial per sphere and source split (16 splits), about
                                  1.7x the time.  Same sum in another order (rounding). */
} dem_tuning;
dem_status dem_set_tuning(dem_sim* sim, const dem_tuning* tuning);
/* Gravity tile sizes supported for a precision: writes up to n_max of them
 * to tiles (default first) and returns how many there are. */
int32_t dem_gravity_tiles(int32_t precision, int32_t* tiles, int32_t n_max);

/* Per-kernel timing (measurement aid for benchmarks).  enabled = 1: dem_step
 * launches the step's kernels one by one (no graph) with a HIP event before
 * and after each, on the system's stream, and accumulates the elapsed time of
 * every kernel family.  enabled = 2: dem_step launches the kernels (no graph)
 * in the order and on the streams of the step graph -- gravity on a second
 * stream beside the contact kernels -- with a HIP event before and after the
 * gravity stage only, on the stream that runs it; only the gravity total is
 * kept.  0 turns timing off; other values are INVALID_ARG.  dem_get_profile
 * copies up to n_max totals in milliseconds (order given by
 * dem_profile_names, a ';'-separated list) and the number of steps they
 * cover.  Setting the mode clears the totals. */
dem_status dem_set_profiling(dem_sim* sim, int32_t enabled);
dem_status dem_get_profile(const dem_sim* sim, double* kernel_ms, int32_t n_max,
                           int64_t* n_steps);
const char* dem_profile_names(void);

/* Device bytes a system of this size uses (for admission control). */
size_t dem_footprint_bytes(const dem_params* params, int64_t n_agg, int64_t n_sph);

#ifdef __cplusplus
}
#endif
#endif
