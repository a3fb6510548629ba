/*
 * oracle.c -- plain FP64 CPU reference of the soft-sphere DEM step for rigid
 * aggregates of bonded spheres (Marohnic et al., arXiv 2311.11322).
 *
 * TEST INFRASTRUCTURE ONLY: loaded by the tests, the smoke check and the CPU
 * baseline of the benchmark, never by the product path.  Shares no source
 * with the GPU library.
 *
 * What each function follows:
 *   setup_body      Eqs. 1-2 (mass, centre of mass); the inertia tensor and
 *                   principal axes of GetAxesAndSpin; body-frame offsets of
 *                   SetBodyPos; aggregate mass per member of SetMassDEM
 *                   (appendix table of aggregate functions).
 *   kick / drift    fixed-step leapfrog for centres of mass (Sec. 2.1).
 *   rotate          Euler's rigid-body equations integrated by a fifth-order
 *                   Runge-Kutta step (Sec. 2.2); Cash-Karp coefficients,
 *                   torque held at its last evaluated value, one step per h.
 *   reconstruct     SetSpacePos / SetSpaceSpin / SetSpaceVel; the predicted
 *                   member velocity of Eq. 3 (Sec. 2.2.2).
 *   find_pairs      brute force over all i<j, skipping pairs inside one
 *                   aggregate (members are rigidly bonded, Sec. 2.2).
 *   pair_force      spring-dashpot normal force, tangential spring with
 *                   history and a static-friction cap, rolling and twisting
 *                   friction (Sec. 2.1, 2.2.5); contact point (Sec. 2.2.4) from the lever
 *                   arm of Eq. 8; forces applied at that point (Eq. 9).
 *   gravity         direct sum of Eq. 4 with Plummer softening.
 *   reduce          Eqs. 5-7 and 9: aggregate acceleration and torque about
 *                   the centre of mass (GetAccelAndTorque).
 *
 * Readings of passages that are silent or garbled are listed in the design
 * notes of the repository and restated next to the code that takes them.
 */
#include "oracle.h"

#include <math.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define PI 3.14159265358979323846

struct ora_sim {
    ora_params p;
    int64_t na, ns;
    /* aggregates */
    int64_t *first, *count;
    double *M, *rA, *vA, *aA, *NA, *q, *wb, *I, *wA;
    /* spheres, grouped by aggregate */
    int64_t *agg;
    double *b, *s, *m;
    double *r, *v, *F, *tau;
    /* contacts, canonical order (i<j, lexicographic) */
    int64_t np, cap;
    int64_t *pi, *pj;
    double *hist;   /* 7 per pair */
    double *pforce; /* 9 per pair */
    double *pdiag;  /* 8 per pair */
    /* time of the current evaluation (walls move with it) */
    double t_eval;
    int64_t steps;
    /* point-mass perturber */
    int pert_on;
    double pert_M, pert_r[3], pert_v[3], pert_a[3];
};

/* ------------------------------------------------------------------ */
/* small vector helpers                                                */
/* ------------------------------------------------------------------ */

static void cross(const double* a, const double* b, double* c)
{
    double x = a[1] * b[2] - a[2] * b[1];
    double y = a[2] * b[0] - a[0] * b[2];
    double z = a[0] * b[1] - a[1] * b[0];
    c[0] = x; c[1] = y; c[2] = z;
}

static double dot(const double* a, const double* b)
{
    return a[0] * b[0] + a[1] * b[1] + a[2] * b[2];
}

static double norm3(const double* a) { return sqrt(dot(a, a)); }

/* Rotation matrix (body -> space) of quaternion q = (w, x, y, z), taken as
 * given (no normalisation): the standard unit-quaternion formula. */
static void quat_to_R(const double* q, double R[3][3])
{
    double w = q[0], x = q[1], y = q[2], z = q[3];
    R[0][0] = 1.0 - 2.0 * (y * y + z * z);
    R[0][1] = 2.0 * (x * y - w * z);
    R[0][2] = 2.0 * (x * z + w * y);
    R[1][0] = 2.0 * (x * y + w * z);
    R[1][1] = 1.0 - 2.0 * (x * x + z * z);
    R[1][2] = 2.0 * (y * z - w * x);
    R[2][0] = 2.0 * (x * z - w * y);
    R[2][1] = 2.0 * (y * z + w * x);
    R[2][2] = 1.0 - 2.0 * (x * x + y * y);
}

static void mat_vec(double R[3][3], const double* a, double* c)
{
    double x = R[0][0] * a[0] + R[0][1] * a[1] + R[0][2] * a[2];
    double y = R[1][0] * a[0] + R[1][1] * a[1] + R[1][2] * a[2];
    double z = R[2][0] * a[0] + R[2][1] * a[1] + R[2][2] * a[2];
    c[0] = x; c[1] = y; c[2] = z;
}

static void mat_T_vec(double R[3][3], const double* a, double* c)
{
    double x = R[0][0] * a[0] + R[1][0] * a[1] + R[2][0] * a[2];
    double y = R[0][1] * a[0] + R[1][1] * a[1] + R[2][1] * a[2];
    double z = R[0][2] * a[0] + R[1][2] * a[1] + R[2][2] * a[2];
    c[0] = x; c[1] = y; c[2] = z;
}

/* ------------------------------------------------------------------ */
/* aggregate set-up                                                     */
/* ------------------------------------------------------------------ */

/* Eigen-decomposition of a symmetric 3x3 matrix by cyclic Jacobi rotations
 * (textbook method).  On return A holds the eigenvalues on its diagonal and
 * the columns of V the eigenvectors. */
static void jacobi3(double A[3][3], double V[3][3])
{
    int i, j, k, sweep;
    for (i = 0; i < 3; i++)
        for (j = 0; j < 3; j++) V[i][j] = (i == j) ? 1.0 : 0.0;
    for (sweep = 0; sweep < 64; sweep++) {
        double off = fabs(A[0][1]) + fabs(A[0][2]) + fabs(A[1][2]);
        double scale = fabs(A[0][0]) + fabs(A[1][1]) + fabs(A[2][2]);
        if (off <= 1e-300 || off <= 1e-17 * scale) break;
        for (i = 0; i < 2; i++) {
            for (j = i + 1; j < 3; j++) {
                double apq = A[i][j];
                if (apq == 0.0) continue;
                /* rotation angle that zeroes A[i][j] */
                double theta = (A[j][j] - A[i][i]) / (2.0 * apq);
                double t = (theta >= 0.0 ? 1.0 : -1.0) / (fabs(theta) + sqrt(theta * theta + 1.0));
                double c = 1.0 / sqrt(t * t + 1.0);
                double sn = t * c;
                /* A <- J^T A J with J the (i,j) plane rotation */
                for (k = 0; k < 3; k++) {
                    double aki = A[k][i], akj = A[k][j];
                    A[k][i] = c * aki - sn * akj;
                    A[k][j] = sn * aki + c * akj;
                }
                for (k = 0; k < 3; k++) {
                    double aik = A[i][k], ajk = A[j][k];
                    A[i][k] = c * aik - sn * ajk;
                    A[j][k] = sn * aik + c * ajk;
                }
                for (k = 0; k < 3; k++) {
                    double vki = V[k][i], vkj = V[k][j];
                    V[k][i] = c * vki - sn * vkj;
                    V[k][j] = sn * vki + c * vkj;
                }
            }
        }
    }
}

/* Quaternion of a proper rotation matrix (Shepperd's method: branch on the
 * largest of the four squared components). */
static void R_to_quat(double R[3][3], double* q)
{
    double tr = R[0][0] + R[1][1] + R[2][2];
    double w, x, y, z;
    if (tr >= R[0][0] && tr >= R[1][1] && tr >= R[2][2]) {
        double t = sqrt(1.0 + tr) * 2.0;           /* 4w */
        w = 0.25 * t;
        x = (R[2][1] - R[1][2]) / t;
        y = (R[0][2] - R[2][0]) / t;
        z = (R[1][0] - R[0][1]) / t;
    } else if (R[0][0] >= R[1][1] && R[0][0] >= R[2][2]) {
        double t = sqrt(1.0 + R[0][0] - R[1][1] - R[2][2]) * 2.0; /* 4x */
        w = (R[2][1] - R[1][2]) / t;
        x = 0.25 * t;
        y = (R[0][1] + R[1][0]) / t;
        z = (R[0][2] + R[2][0]) / t;
    } else if (R[1][1] >= R[2][2]) {
        double t = sqrt(1.0 + R[1][1] - R[0][0] - R[2][2]) * 2.0; /* 4y */
        w = (R[0][2] - R[2][0]) / t;
        x = (R[0][1] + R[1][0]) / t;
        y = 0.25 * t;
        z = (R[1][2] + R[2][1]) / t;
    } else {
        double t = sqrt(1.0 + R[2][2] - R[0][0] - R[1][1]) * 2.0; /* 4z */
        w = (R[1][0] - R[0][1]) / t;
        x = (R[0][2] + R[2][0]) / t;
        y = (R[1][2] + R[2][1]) / t;
        z = 0.25 * t;
    }
    double nq = sqrt(w * w + x * x + y * y + z * z);
    q[0] = w / nq; q[1] = x / nq; q[2] = y / nq; q[3] = z / nq;
}

/* Set-up of one aggregate of n member spheres.
 *  Eq. 1: M = sum m_i.   Eq. 2: r_A = sum m_i r_i / M.
 *  Inertia tensor about the centre of mass, including each sphere's own
 *  moment 2/5 m s^2 (needed so a lone sphere has a finite inertia), then its
 *  principal axes (GetAxesAndSpin) as a proper rotation R, the quaternion of
 *  R, and the body-frame offsets b_i = R^T (r_i - r_A) (SetBodyPos). */
int ora_setup_body(int64_t n, const double* pos, const double* radius, const double* mass,
                   double* M_out, double* r_out, double* I_out, double* q_out, double* b_out)
{
    int64_t i;
    int a, c;
    double M = 0.0, r[3] = {0.0, 0.0, 0.0};
    if (n <= 0) return -1;
    for (i = 0; i < n; i++) M += mass[i];
    for (i = 0; i < n; i++)
        for (c = 0; c < 3; c++) r[c] += mass[i] * pos[3 * i + c];
    for (c = 0; c < 3; c++) r[c] /= M;

    double T[3][3] = {{0, 0, 0}, {0, 0, 0}, {0, 0, 0}};
    for (i = 0; i < n; i++) {
        double d[3] = {pos[3 * i] - r[0], pos[3 * i + 1] - r[1], pos[3 * i + 2] - r[2]};
        double d2 = dot(d, d) + 0.4 * radius[i] * radius[i];
        for (a = 0; a < 3; a++)
            for (c = 0; c < 3; c++)
                T[a][c] += mass[i] * ((a == c ? d2 : 0.0) - d[a] * d[c]);
    }
    double V[3][3];
    jacobi3(T, V);
    /* make the axes a proper rotation */
    double col0[3] = {V[0][0], V[1][0], V[2][0]};
    double col1[3] = {V[0][1], V[1][1], V[2][1]};
    double col2[3] = {V[0][2], V[1][2], V[2][2]};
    double x01[3];
    cross(col0, col1, x01);
    if (dot(x01, col2) < 0.0)
        for (a = 0; a < 3; a++) V[a][2] = -V[a][2];
    double q[4], R[3][3];
    R_to_quat(V, q);
    quat_to_R(q, R);
    for (i = 0; i < n; i++) {
        double d[3] = {pos[3 * i] - r[0], pos[3 * i + 1] - r[1], pos[3 * i + 2] - r[2]};
        mat_T_vec(R, d, &b_out[3 * i]);
    }
    *M_out = M;
    for (c = 0; c < 3; c++) { r_out[c] = r[c]; I_out[c] = T[c][c]; }
    for (c = 0; c < 4; c++) q_out[c] = q[c];
    return 0;
}

/* ------------------------------------------------------------------ */
/* rotation: Euler's equations, one Cash-Karp RK5 step                 */
/* ------------------------------------------------------------------ */

/* Right-hand side for y = (q[4], wb[3]):
 *   dq/dt   = 1/2 q (x) (0, wb)                (quaternion kinematics)
 *   I dwb/dt = N_body - wb x (I wb),  N_body = R(q)^T N_space
 * with I diagonal (principal axes) and the space-frame torque held fixed. */
static void euler_rhs(const double* y, const double* I, const double* N_space, double* dy)
{
    double R[3][3], Nb[3];
    double w = y[0], x = y[1], yy = y[2], z = y[3];
    double o1 = y[4], o2 = y[5], o3 = y[6];
    quat_to_R(y, R);
    mat_T_vec(R, N_space, Nb);
    dy[0] = 0.5 * (-x * o1 - yy * o2 - z * o3);
    dy[1] = 0.5 * (w * o1 + yy * o3 - z * o2);
    dy[2] = 0.5 * (w * o2 + z * o1 - x * o3);
    dy[3] = 0.5 * (w * o3 + x * o2 - yy * o1);
    dy[4] = (Nb[0] - (I[2] - I[1]) * o2 * o3) / I[0];
    dy[5] = (Nb[1] - (I[0] - I[2]) * o3 * o1) / I[1];
    dy[6] = (Nb[2] - (I[1] - I[0]) * o1 * o2) / I[2];
}

/* Cash & Karp (1990) embedded Runge-Kutta coefficients. */
static const double CK_A[6][5] = {
    {0.0, 0.0, 0.0, 0.0, 0.0},
    {1.0 / 5.0, 0.0, 0.0, 0.0, 0.0},
    {3.0 / 40.0, 9.0 / 40.0, 0.0, 0.0, 0.0},
    {3.0 / 10.0, -9.0 / 10.0, 6.0 / 5.0, 0.0, 0.0},
    {-11.0 / 54.0, 5.0 / 2.0, -70.0 / 27.0, 35.0 / 27.0, 0.0},
    {1631.0 / 55296.0, 175.0 / 512.0, 575.0 / 13824.0, 44275.0 / 110592.0, 253.0 / 4096.0},
};
static const double CK_B5[6] = {37.0 / 378.0, 0.0, 250.0 / 621.0, 125.0 / 594.0, 0.0, 512.0 / 1771.0};
static const double CK_B4[6] = {2825.0 / 27648.0, 0.0, 18575.0 / 48384.0, 13525.0 / 55296.0,
                                277.0 / 14336.0, 1.0 / 4.0};

void ora_rotate(double* q, double* wb, const double* I, const double* N_space, double h,
                double* err)
{
    double y0[7], k[6][7], yt[7];
    int st, c, j;
    for (c = 0; c < 4; c++) y0[c] = q[c];
    for (c = 0; c < 3; c++) y0[4 + c] = wb[c];
    for (st = 0; st < 6; st++) {
        for (c = 0; c < 7; c++) {
            double acc = 0.0;
            for (j = 0; j < st; j++) acc += CK_A[st][j] * k[j][c];
            yt[c] = y0[c] + h * acc;
        }
        euler_rhs(yt, I, N_space, k[st]);
    }
    double e2 = 0.0;
    for (c = 0; c < 7; c++) {
        double s5 = 0.0, s4 = 0.0;
        for (st = 0; st < 6; st++) {
            s5 += CK_B5[st] * k[st][c];
            s4 += CK_B4[st] * k[st][c];
        }
        double y5 = y0[c] + h * s5;
        double y4 = y0[c] + h * s4;
        e2 += (y5 - y4) * (y5 - y4);
        yt[c] = y5;
    }
    /* renormalise the quaternion after the step */
    double nq = sqrt(yt[0] * yt[0] + yt[1] * yt[1] + yt[2] * yt[2] + yt[3] * yt[3]);
    for (c = 0; c < 4; c++) q[c] = yt[c] / nq;
    for (c = 0; c < 3; c++) wb[c] = yt[4 + c];
    if (err) *err = sqrt(e2);
}

/* ------------------------------------------------------------------ */
/* simulation handle                                                    */
/* ------------------------------------------------------------------ */

ora_sim* ora_create(const ora_params* p)
{
    ora_sim* s = (ora_sim*)calloc(1, sizeof(ora_sim));
    if (!s) return NULL;
    s->p = *p;
    return s;
}

static void free_pairs(ora_sim* s)
{
    free(s->pi); free(s->pj); free(s->hist); free(s->pforce); free(s->pdiag);
    s->pi = s->pj = NULL; s->hist = s->pforce = s->pdiag = NULL;
    s->np = s->cap = 0;
}

void ora_destroy(ora_sim* s)
{
    if (!s) return;
    free(s->first); free(s->count); free(s->M); free(s->rA); free(s->vA); free(s->aA);
    free(s->NA); free(s->q); free(s->wb); free(s->I); free(s->wA);
    free(s->agg); free(s->b); free(s->s); free(s->m);
    free(s->r); free(s->v); free(s->F); free(s->tau);
    free_pairs(s);
    free(s);
}

/* ------------------------------------------------------------------ */
/* per-step pieces                                                     */
/* ------------------------------------------------------------------ */

/* SetSpacePos / SetSpaceSpin / SetSpaceVel.  Member positions are rebuilt
 * from the rigid body every step: r_i = r_A + R b_i.  Spin in space frame
 * w_A = R w_b.  Velocity, Eq. 3: the predicted centre-of-mass velocity
 * v_A(n+1/2) + h/2 a_A(n), plus w_A(n+1) x (r_i - r_A). */
static void reconstruct(ora_sim* s, double half_h_accel)
{
    int64_t A, i;
    int c;
    for (A = 0; A < s->na; A++) {
        double R[3][3];
        quat_to_R(&s->q[4 * A], R);
        mat_vec(R, &s->wb[3 * A], &s->wA[3 * A]);
        double vpred[3];
        for (c = 0; c < 3; c++) vpred[c] = s->vA[3 * A + c] + half_h_accel * s->aA[3 * A + c];
        for (i = s->first[A]; i < s->first[A] + s->count[A]; i++) {
            double d[3], wxd[3];
            mat_vec(R, &s->b[3 * i], d);
            cross(&s->wA[3 * A], d, wxd);
            for (c = 0; c < 3; c++) {
                s->r[3 * i + c] = s->rA[3 * A + c] + d[c];
                s->v[3 * i + c] = vpred[c] + wxd[c];
            }
        }
    }
}

/* Separation vector d = r_j - r_i, with the minimum-image rule in a periodic
 * cube (one branchy correction per axis; sphere positions are not wrapped,
 * only aggregate centres are). */
static void separation(const ora_params* p, const double* ri, const double* rj, double* d)
{
    int c;
    for (c = 0; c < 3; c++) {
        double x = rj[c] - ri[c];
        if (p->periodic) {
            double L = p->box[c];
            if (x > 0.5 * L) x -= L;
            else if (x < -0.5 * L) x += L;
        }
        d[c] = x;
    }
}

/* Contact test: strict d^2 < (s_i + s_j)^2, d^2 summed as (x*x + y*y) + z*z. */
static int in_contact(const double* d, double si, double sj)
{
    double d2 = (d[0] * d[0] + d[1] * d[1]) + d[2] * d[2];
    double S = si + sj;
    return d2 < S * S;
}

static void push_pair(ora_sim* s, int64_t i, int64_t j)
{
    if (s->np == s->cap) {
        int64_t nc = s->cap ? 2 * s->cap : 1024;
        s->pi = (int64_t*)realloc(s->pi, nc * sizeof(int64_t));
        s->pj = (int64_t*)realloc(s->pj, nc * sizeof(int64_t));
        s->hist = (double*)realloc(s->hist, nc * 7 * sizeof(double));
        s->pforce = (double*)realloc(s->pforce, nc * 9 * sizeof(double));
        s->pdiag = (double*)realloc(s->pdiag, nc * 8 * sizeof(double));
        s->cap = nc;
    }
    s->pi[s->np] = i;
    s->pj[s->np] = j;
    s->np++;
}

/* Wall w at time t: signed distance of point x from the plane n.x = d
 * displaced by A sin(omega t + phase), summed as ((n0 x0 + n1 x1) + n2 x2)
 * - (d + n.A sin(.)); and the wall's velocity. */
static double wall_distance(const ora_params* p, int w, double t, const double* x, double* vel)
{
    const double* n = p->wall[w];
    const double* A = p->shake_amp[w];
    double ph = p->shake_omega * t + p->shake_phase;
    double sn = sin(ph), cs = cos(ph);
    double shift = (n[0] * A[0] + n[1] * A[1]) + n[2] * A[2];
    int c;
    if (vel)
        for (c = 0; c < 3; c++) vel[c] = A[c] * p->shake_omega * cs;
    return ((n[0] * x[0] + n[1] * x[1]) + n[2] * x[2]) - (n[3] + shift * sn);
}

/* Brute-force search over all i<j (lexicographic order); spheres of the
 * same aggregate never form a contact.  Walls follow the spheres as
 * partners n_sph + w: sphere i touches wall w iff its centre is closer to the
 * plane than its radius (strict). */
static void find_pairs(ora_sim* s)
{
    int64_t i, j;
    int w;
    s->np = 0;
    for (i = 0; i < s->ns; i++) {
        for (j = i + 1; j < s->ns; j++) {
            double d[3];
            if (s->agg[i] == s->agg[j]) continue;
            separation(&s->p, &s->r[3 * i], &s->r[3 * j], d);
            if (in_contact(d, s->s[i], s->s[j])) push_pair(s, i, j);
        }
        for (w = 0; w < s->p.n_walls; w++) {
            if (wall_distance(&s->p, w, s->t_eval, &s->r[3 * i], NULL) < s->s[i])
                push_pair(s, i, s->ns + w);
        }
    }
}

/* Dashpot constant of a linear spring k with reduced mass mu giving
 * restitution eps: C = -2 ln(eps) sqrt(k mu / (pi^2 + ln^2 eps)). */
static double dashpot(double k, double mu, double eps)
{
    double le = log(eps);
    return -2.0 * le * sqrt(k * mu / (PI * PI + le * le));
}

/* Force of one contact (i, j), i < j, evaluated with spring history h_old
 * (xi_t[3], xi_r[3], xi_q); writes the updated history, the force on i and
 * the torques about the two sphere centres, and diagnostics.
 *
 *  Geometry: d = r_j - r_i, n = d/|d| (i toward j), overlap delta = S - |d|.
 *  Lever arm (Eq. 8): l_i = (s_i^2 - s_j^2 + |d|^2) / (2|d|), l_j = |d| - l_i;
 *  the contact point is r_i + l_i n = r_j - l_j n.
 *  Contact-point velocities: v_ci = v_i + w_A(i) x (l_i n),
 *                            v_cj = v_j + w_A(j) x (-l_j n);  u = v_cj - v_ci.
 *  Reduced mass from the *aggregate* masses (SetMassDEM stores the aggregate
 *  mass on members for the contact routines).
 *  Normal: F_N = (-k_n delta + C_n u_n) n on i (no clamp; the friction caps
 *  use the repulsive load f_N = max(0, k_n delta - C_n u_n)).
 *  Tangential: xi_t projected onto the tangent plane, advanced by h u_t; if
 *  k_t|xi_t| exceeds mu_s f_N it is scaled back onto the cap and the force is
 *  the capped spring alone, else F_T = k_t xi_t + C_t u_t.
 *  Rolling / twisting: spring-sliders on the relative spin of the two bodies
 *  with lever R_ij = s_i s_j/(s_i+s_j), capped at mu_r f_N and mu_t f_N.
 *  Forces act at the contact point, so tau_i = (l_i n) x F + couples and
 *  tau_j = (-l_j n) x (-F) - couples. */
static void pair_force(const ora_sim* s, int64_t i, int64_t j, const double* h_old,
                       double* h_new, double* out9, double* diag8)
{
    const ora_params* p = &s->p;
    const double h = p->dt;
    const int wall = j >= s->ns;
    int c;
    double d[3], n[3], dist, delta, li, lj, si = s->s[i], sj, Rij, mu;
    double vj[3], wj_zero[3] = {0.0, 0.0, 0.0};
    const double* wj;
    int64_t Ai = s->agg[i];
    const double* wi = &s->wA[3 * Ai];
    if (wall) {
        /* sphere against a plane: the partner is the wall (infinite mass, no
         * spin); the contact point is the foot of the perpendicular, so the
         * lever arm is the centre's distance from the plane, and the normal
         * points from the sphere into the wall */
        int w = (int)(j - s->ns);
        dist = wall_distance(p, w, s->t_eval, &s->r[3 * i], vj);
        for (c = 0; c < 3; c++) n[c] = -p->wall[w][c];
        delta = si - dist;
        li = dist;
        lj = 0.0;
        sj = 0.0;
        wj = wj_zero;
        mu = s->M[Ai];
        Rij = si;
    } else {
        separation(p, &s->r[3 * i], &s->r[3 * j], d);
        dist = sqrt(dot(d, d));
        for (c = 0; c < 3; c++) n[c] = d[c] / dist;
        sj = s->s[j];
        delta = (si + sj) - dist;
        li = (si * si - sj * sj + dist * dist) / (2.0 * dist);
        lj = dist - li;
        int64_t Aj = s->agg[j];
        wj = &s->wA[3 * Aj];
        for (c = 0; c < 3; c++) vj[c] = s->v[3 * j + c];
        double MA = s->M[Ai], MB = s->M[Aj];
        mu = MA * MB / (MA + MB);
        Rij = si * sj / (si + sj);
    }

    double arm_i[3], arm_j[3], t1[3], t2[3], u[3];
    for (c = 0; c < 3; c++) { arm_i[c] = li * n[c]; arm_j[c] = -lj * n[c]; }
    cross(wi, arm_i, t1);
    cross(wj, arm_j, t2);
    for (c = 0; c < 3; c++)
        u[c] = (vj[c] + t2[c]) - (s->v[3 * i + c] + t1[c]);
    double un = dot(u, n);
    double ut[3];
    for (c = 0; c < 3; c++) ut[c] = u[c] - un * n[c];

    double Cn = dashpot(p->k_n, mu, p->eps_n);
    double Ct = dashpot(p->k_t, mu, p->eps_t);

    double fn_signed = -p->k_n * delta + Cn * un;      /* along n, on i */
    double fN = p->k_n * delta - Cn * un;
    if (fN < 0.0) fN = 0.0;

    /* tangential spring */
    double xt[3];
    double xt_n = dot(&h_old[0], n);
    for (c = 0; c < 3; c++) xt[c] = h_old[c] - xt_n * n[c];
    for (c = 0; c < 3; c++) xt[c] += h * ut[c];
    double FT[3];
    double xt_mag = norm3(xt);
    int sliding = 0;
    if (p->k_t * xt_mag > p->mu_s * fN) {
        double sc = p->mu_s * fN / (p->k_t * xt_mag);
        for (c = 0; c < 3; c++) { xt[c] *= sc; FT[c] = p->k_t * xt[c]; }
        sliding = 1;
    } else {
        for (c = 0; c < 3; c++) FT[c] = p->k_t * xt[c] + Ct * ut[c];
    }

    /* rolling (lever R_ij = s_i s_j/(s_i+s_j); s_i against a wall) */
    double dw[3], dwxn[3], xr[3];
    for (c = 0; c < 3; c++) dw[c] = wj[c] - wi[c];
    cross(dw, n, dwxn);
    double xr_n = dot(&h_old[3], n);
    for (c = 0; c < 3; c++) xr[c] = h_old[3 + c] - xr_n * n[c] + h * Rij * dwxn[c];
    double xr_mag = norm3(xr);
    if (p->k_r * xr_mag > p->mu_r * fN) {
        double sc = p->mu_r * fN / (p->k_r * xr_mag);
        for (c = 0; c < 3; c++) xr[c] *= sc;
    }
    double Fr[3], tau_r[3];
    for (c = 0; c < 3; c++) Fr[c] = p->k_r * xr[c];
    cross(n, Fr, tau_r);
    for (c = 0; c < 3; c++) tau_r[c] *= Rij;

    /* twisting */
    double xq = h_old[6] + h * Rij * dot(dw, n);
    if (p->k_q * fabs(xq) > p->mu_t * fN) {
        double sc = p->mu_t * fN / (p->k_q * fabs(xq));
        xq *= sc;
    }
    double Fq = p->k_q * xq;
    double tau_q[3];
    for (c = 0; c < 3; c++) tau_q[c] = Rij * Fq * n[c];

    /* total contact force on i, applied at the contact point */
    double F[3], ti[3], tj[3], mF[3];
    for (c = 0; c < 3; c++) { F[c] = fn_signed * n[c] + FT[c]; mF[c] = -F[c]; }
    if (p->torque_at_centre) {
        for (c = 0; c < 3; c++) { ti[c] = 0.0; tj[c] = 0.0; }
    } else {
        cross(arm_i, F, ti);
        cross(arm_j, mF, tj);
    }
    for (c = 0; c < 3; c++) {
        ti[c] += tau_r[c] + tau_q[c];
        tj[c] -= tau_r[c] + tau_q[c];
    }

    for (c = 0; c < 3; c++) { h_new[c] = xt[c]; h_new[3 + c] = xr[c]; }
    h_new[6] = xq;
    for (c = 0; c < 3; c++) { out9[c] = F[c]; out9[3 + c] = ti[c]; out9[6 + c] = tj[c]; }
    if (diag8) {
        diag8[0] = fN;
        diag8[1] = norm3(FT);
        diag8[2] = norm3(Fr);
        diag8[3] = fabs(Fq);
        diag8[4] = delta;
        diag8[5] = li;
        diag8[6] = lj;
        diag8[7] = (double)sliding;
    }
}

/* Softened pair gravity on i from j (Eq. 4 with Plummer softening
 * eps_ij = soft_frac (s_i + s_j)/2), added to F. */
static void gravity_pair(double G, double soft_frac, const double* ri, const double* rj,
                         double mi, double mj, double si, double sj, double* F)
{
    double d[3] = {rj[0] - ri[0], rj[1] - ri[1], rj[2] - ri[2]};
    double eps = soft_frac * 0.5 * (si + sj);
    double r2 = dot(d, d) + eps * eps;
    double inv3 = 1.0 / (r2 * sqrt(r2));
    double f = G * mi * mj * inv3;
    F[0] += f * d[0];
    F[1] += f * d[1];
    F[2] += f * d[2];
}

/* Targets are independent: with OpenMP they are shared among threads, each
 * target's sum still taken over j in index order, so the result does not
 * depend on the thread count. */
void ora_gravity(const double* pos, const double* mass, const double* radius, int64_t n,
                 double G, double soft_frac, const int64_t* idx, int64_t n_idx, double* F)
{
    int64_t k;
#pragma omp parallel for schedule(static)
    for (k = 0; k < n_idx; k++) {
        int64_t i = idx[k], j;
        double acc[3] = {0.0, 0.0, 0.0};
        for (j = 0; j < n; j++) {
            if (j == i) continue;
            gravity_pair(G, soft_frac, &pos[3 * i], &pos[3 * j], mass[i], mass[j],
                         radius[i], radius[j], acc);
        }
        F[3 * k] = acc[0]; F[3 * k + 1] = acc[1]; F[3 * k + 2] = acc[2];
    }
}

/* ---- tree gravity ---------------------------------------------------- */

typedef struct {
    uint32_t prefix;
    int64_t s, e;          /* range in the sorted order */
    double M, c[3];        /* mass, centre of mass */
    double Ms1, Ms2;       /* sum m s, sum m s^2 (s = sphere radius) */
    /* raw moments about the centre of mass: sum m d_i d_j (d_k (d_l)) */
    double M2[3][3], M3[3][3][3], M4[3][3][3][3];
} tnode;

typedef struct {
    const double *r, *m, *rad;
    double G, soft_frac, theta;
    int leaf, bits, mp_order;  /* highest multipole order kept */
    double lo[3], cell;
    int64_t* order;        /* sorted index -> sphere */
    uint32_t* key;         /* sorted keys */
    tnode* lev[11];
    int64_t nlev[11];
    /* current group */
    int64_t g0, g1;
    double bmin[3], bmax[3];
    double* acc;           /* [3][group size] */
} tree;

static uint32_t dilate3(uint32_t v)
{
    uint32_t r = 0;
    int b;
    for (b = 0; b < 10; b++) r |= ((v >> b) & 1u) << (3 * b);
    return r;
}


static const uint32_t* g_sort_keys;
static int cmp_sorted(const void* a, const void* b)
{
    int64_t x = *(const int64_t*)a, y = *(const int64_t*)b;
    if (g_sort_keys[x] != g_sort_keys[y]) return g_sort_keys[x] < g_sort_keys[y] ? -1 : 1;
    return x < y ? -1 : (x > y ? 1 : 0);
}

static void node_moments(const tree* t, tnode* nd)
{
    int64_t k;
    int c;
    double M = 0.0, mc[3] = {0.0, 0.0, 0.0};
    for (k = nd->s; k < nd->e; k++) {
        int64_t i = t->order[k];
        M += t->m[i];
        for (c = 0; c < 3; c++) mc[c] += t->m[i] * t->r[3 * i + c];
    }
    nd->M = M;
    for (c = 0; c < 3; c++) nd->c[c] = mc[c] / M;
    nd->Ms1 = nd->Ms2 = 0.0;
    memset(nd->M2, 0, sizeof(nd->M2));
    memset(nd->M3, 0, sizeof(nd->M3));
    memset(nd->M4, 0, sizeof(nd->M4));
    for (k = nd->s; k < nd->e; k++) {
        int64_t i = t->order[k];
        double d[3], m = t->m[i];
        int a, b, e, f;
        for (c = 0; c < 3; c++) d[c] = t->r[3 * i + c] - nd->c[c];
        nd->Ms1 += m * t->rad[i];
        nd->Ms2 += m * t->rad[i] * t->rad[i];
        for (a = 0; a < 3; a++)
            for (b = 0; b < 3; b++) {
                nd->M2[a][b] += m * d[a] * d[b];
                for (e = 0; e < 3; e++) {
                    nd->M3[a][b][e] += m * d[a] * d[b] * d[e];
                    for (f = 0; f < 3; f++) nd->M4[a][b][e][f] += m * d[a] * d[b] * d[e] * d[f];
                }
            }
    }
}

static const tnode* find_node(const tree* t, int l, uint32_t prefix)
{
    int64_t lo = 0, hi = t->nlev[l];
    while (lo < hi) {
        int64_t mid = (lo + hi) / 2;
        if (t->lev[l][mid].prefix < prefix) lo = mid + 1;
        else hi = mid;
    }
    if (lo < t->nlev[l] && t->lev[l][lo].prefix == prefix) return &t->lev[l][lo];
    return NULL;
}

/* Force per unit target mass of a node at R = x - c, from the expansion
 * 1/|R - d| = sum_n (2n-1)!!/n! [d^n]_traceless . R^n / R^(2n+1).  With
 * S_n = Q_n . R^n (Q_n the traceless part of the raw moment M_n) and
 * V_n = Q_n . R^(n-1) = grad S_n / n, the pull is
 * G sum_n c_n [n V_n / R^(2n+1) - (2n+1) S_n R / R^(2n+3)], c_n = (2n-1)!!/n!;
 * the dipole vanishes about the centre of mass.  Orders n <= the tree's order.
 *
 * The pairs are Plummer-softened, 1/sqrt(|R - d|^2 + eps^2): the eps^2 term
 * of that expansion, -eps^2 / (2 R^3), is of the quadrupole's order and is
 * kept, with E = sum_j m_j eps_ij^2 = (f/2)^2 (s_i^2 M + 2 s_i sum m s + sum m s^2)
 * for eps_ij = f (s_i + s_j)/2; its pull is +3/2 G E R / R^5. */
static void m2p(const tnode* nd, const double* x, double si, const tree* t, double* acc)
{
    const int order = t->mp_order;
    double R[3] = {x[0] - nd->c[0], x[1] - nd->c[1], x[2] - nd->c[2]};
    double r2 = R[0] * R[0] + R[1] * R[1] + R[2] * R[2];
    double r = sqrt(r2);
    double S[5] = {0, 0, 0, 0, 0}, V[5][3];
    int a, b, e, f, n;
    memset(V, 0, sizeof(V));
    S[0] = nd->M;
    if (order >= 2) {
        double tr = nd->M2[0][0] + nd->M2[1][1] + nd->M2[2][2];
        for (a = 0; a < 3; a++) {
            double v = 0.0;
            for (b = 0; b < 3; b++) v += nd->M2[a][b] * R[b];
            V[2][a] = v - tr * R[a] / 3.0;
            S[2] += v * R[a];
        }
        S[2] -= tr * r2 / 3.0;
    }
    if (order >= 3) {
        double tv[3], tR = 0.0;
        for (a = 0; a < 3; a++) {
            tv[a] = nd->M3[0][0][a] + nd->M3[1][1][a] + nd->M3[2][2][a];
            tR += tv[a] * R[a];
        }
        for (a = 0; a < 3; a++) {
            double v = 0.0;
            for (b = 0; b < 3; b++)
                for (e = 0; e < 3; e++) v += nd->M3[a][b][e] * R[b] * R[e];
            V[3][a] = v - (2.0 * R[a] * tR + r2 * tv[a]) / 5.0;
            S[3] += v * R[a];
        }
        S[3] -= 3.0 / 5.0 * r2 * tR;
    }
    if (order >= 4) {
        double U[3][3], UR[3] = {0, 0, 0}, URR = 0.0, sU = 0.0;
        for (a = 0; a < 3; a++)
            for (b = 0; b < 3; b++)
                U[a][b] = nd->M4[0][0][a][b] + nd->M4[1][1][a][b] + nd->M4[2][2][a][b];
        for (a = 0; a < 3; a++) {
            for (b = 0; b < 3; b++) UR[a] += U[a][b] * R[b];
            URR += UR[a] * R[a];
            sU += U[a][a];
        }
        for (a = 0; a < 3; a++) {
            double v = 0.0;
            for (b = 0; b < 3; b++)
                for (e = 0; e < 3; e++)
                    for (f = 0; f < 3; f++) v += nd->M4[a][b][e][f] * R[b] * R[e] * R[f];
            V[4][a] = v - 3.0 / 7.0 * (R[a] * URR + r2 * UR[a]) + 3.0 / 35.0 * r2 * R[a] * sU;
            S[4] += v * R[a];
        }
        S[4] += -6.0 / 7.0 * r2 * URR + 3.0 / 35.0 * r2 * r2 * sU;
    }
    {
        const double cn[5] = {1.0, 0.0, 1.5, 2.5, 4.375};
        double irn = 1.0 / r;               /* 1 / R^(2n+1), n = 0 */
        for (n = 0; n <= order && n <= 4; n++) {
            if (n > 0) irn /= r2;
            if (n == 1) continue;
            for (a = 0; a < 3; a++)
                acc[a] += t->G * cn[n] * (n * V[n][a] * irn - (2 * n + 1) * S[n] * R[a] * irn / r2);
        }
        if (order >= 2) {
            double hf = 0.5 * t->soft_frac;
            double E = hf * hf * (si * si * nd->M + 2.0 * si * nd->Ms1 + nd->Ms2);
            double ir5 = 1.0 / (r2 * r2 * r);
            for (a = 0; a < 3; a++) acc[a] += t->G * 1.5 * E * R[a] * ir5;
        }
    }
}

static void visit(tree* t, int l, uint32_t prefix)
{
    const tnode* nd = find_node(t, l, prefix);
    int c, o;
    int64_t g, k;
    if (!nd) return;
    /* geometric centre of the node's cube, distance to the group's box */
    double side = ldexp(t->cell, t->bits - l);
    double ctr[3], dd[3], dist2, thr;
    uint32_t ix[3] = {0, 0, 0};
    int b;
    for (b = 0; b < l; b++)
        for (c = 0; c < 3; c++) ix[c] |= ((prefix >> (3 * b + c)) & 1u) << b;
    for (c = 0; c < 3; c++) {
        ctr[c] = t->lo[c] + ((double)ix[c] + 0.5) * side;
        double u = t->bmin[c] - ctr[c], v = ctr[c] - t->bmax[c];
        dd[c] = u > v ? u : v;
        if (dd[c] < 0.0) dd[c] = 0.0;
    }
    dist2 = (dd[0] * dd[0] + dd[1] * dd[1]) + dd[2] * dd[2];
    thr = side / t->theta;
    if (dist2 > thr * thr) {
        for (g = t->g0; g < t->g1; g++) {
            int64_t i = t->order[g];
            double a[3] = {0.0, 0.0, 0.0};
            m2p(nd, &t->r[3 * i], t->rad[i], t, a);
            for (c = 0; c < 3; c++) t->acc[3 * (g - t->g0) + c] += t->m[i] * a[c];
        }
        return;
    }
    if (nd->e - nd->s <= t->leaf || l == t->bits) {
        for (g = t->g0; g < t->g1; g++) {
            int64_t i = t->order[g];
            double f[3] = {0.0, 0.0, 0.0};
            for (k = nd->s; k < nd->e; k++) {
                int64_t j = t->order[k];
                if (j == i) continue;
                gravity_pair(t->G, t->soft_frac, &t->r[3 * i], &t->r[3 * j], t->m[i], t->m[j],
                             t->rad[i], t->rad[j], f);
            }
            for (c = 0; c < 3; c++) t->acc[3 * (g - t->g0) + c] += f[c];
        }
        return;
    }
    for (o = 0; o < 8; o++) visit(t, l + 1, (prefix << 3) | (uint32_t)o);
}

void ora_tree_gravity(const double* pos, const double* mass, const double* radius, int64_t n,
                      double G, double soft_frac, double theta, int32_t leaf, int32_t order,
                      double* F)
{
    tree t;
    int64_t i, k;
    int c, l;
    double hi[3], ext = 0.0, smax = 0.0;
    uint32_t* key_of = (uint32_t*)malloc(n * sizeof(uint32_t));
    memset(&t, 0, sizeof(t));
    t.r = pos; t.m = mass; t.rad = radius; t.G = G; t.soft_frac = soft_frac;
    t.theta = theta; t.leaf = leaf; t.mp_order = order;
    /* depth: about two finest cells per sphere, 2..10 levels */
    {
        int lg = 0;
        while ((int64_t)1 << lg < 2 * n) lg++;
        t.bits = (lg + 2) / 3;
        if (t.bits < 2) t.bits = 2;
        if (t.bits > 10) t.bits = 10;
    }
    for (c = 0; c < 3; c++) { t.lo[c] = pos[c]; hi[c] = pos[c]; }
    for (i = 0; i < n; i++) {
        for (c = 0; c < 3; c++) {
            if (pos[3 * i + c] < t.lo[c]) t.lo[c] = pos[3 * i + c];
            if (pos[3 * i + c] > hi[c]) hi[c] = pos[3 * i + c];
        }
        if (radius[i] > smax) smax = radius[i];
    }
    for (c = 0; c < 3; c++) if (hi[c] - t.lo[c] > ext) ext = hi[c] - t.lo[c];
    t.cell = ldexp(ext * (1.0 + 1e-12), -t.bits) + 1e-300;
    if (t.cell < 2.0 * smax) t.cell = 2.0 * smax;
    {
        double inv = 1.0 / t.cell;
        int nc = 1 << t.bits;
        for (i = 0; i < n; i++) {
            int cc[3];
            for (c = 0; c < 3; c++) {
                int v = (int)floor((pos[3 * i + c] - t.lo[c]) * inv);
                cc[c] = v < 0 ? 0 : (v > nc - 1 ? nc - 1 : v);
            }
            key_of[i] = dilate3((uint32_t)cc[0]) | (dilate3((uint32_t)cc[1]) << 1) |
                        (dilate3((uint32_t)cc[2]) << 2);
        }
    }
    t.order = (int64_t*)malloc(n * sizeof(int64_t));
    t.key = (uint32_t*)malloc(n * sizeof(uint32_t));
    for (i = 0; i < n; i++) t.order[i] = i;
    g_sort_keys = key_of;
    qsort(t.order, n, sizeof(int64_t), cmp_sorted);
    for (k = 0; k < n; k++) t.key[k] = key_of[t.order[k]];
    /* nodes of every level: runs of equal prefix */
    for (l = 0; l <= t.bits; l++) {
        int sh = 3 * (t.bits - l);
        int64_t runs = 0;
        for (k = 0; k < n; k++)
            if (k == 0 || (t.key[k] >> sh) != (t.key[k - 1] >> sh)) runs++;
        t.lev[l] = (tnode*)malloc((size_t)runs * sizeof(tnode));
        t.nlev[l] = 0;
        for (k = 0; k < n;) {
            uint32_t p = t.key[k] >> sh;
            int64_t e = k;
            while (e < n && (t.key[e] >> sh) == p) e++;
            tnode* nd = &t.lev[l][t.nlev[l]++];
            nd->prefix = p; nd->s = k; nd->e = e;
            node_moments(&t, nd);
            k = e;
        }
    }
    t.acc = (double*)malloc(3 * 64 * sizeof(double));
    for (t.g0 = 0; t.g0 < n; t.g0 += 64) {
        t.g1 = t.g0 + 64 < n ? t.g0 + 64 : n;
        for (c = 0; c < 3; c++) { t.bmin[c] = INFINITY; t.bmax[c] = -INFINITY; }
        for (k = t.g0; k < t.g1; k++) {
            i = t.order[k];
            for (c = 0; c < 3; c++) {
                if (pos[3 * i + c] < t.bmin[c]) t.bmin[c] = pos[3 * i + c];
                if (pos[3 * i + c] > t.bmax[c]) t.bmax[c] = pos[3 * i + c];
            }
        }
        memset(t.acc, 0, 3 * 64 * sizeof(double));
        visit(&t, 0, 0u);
        for (k = t.g0; k < t.g1; k++) {
            i = t.order[k];
            for (c = 0; c < 3; c++) F[3 * i + c] = t.acc[3 * (k - t.g0) + c];
        }
    }
    for (l = 0; l <= t.bits; l++) free(t.lev[l]);
    free(t.acc); free(t.order); free(t.key); free(key_of);
}

/* Unsoftened pull of the perturber on sphere i (added to F). */
static void perturber_pull(const ora_sim* s, int64_t i, double* F)
{
    double d[3] = {s->pert_r[0] - s->r[3 * i], s->pert_r[1] - s->r[3 * i + 1],
                   s->pert_r[2] - s->r[3 * i + 2]};
    double r2 = dot(d, d);
    double f = s->p.G * s->m[i] * s->pert_M / (r2 * sqrt(r2));
    F[0] += f * d[0];
    F[1] += f * d[1];
    F[2] += f * d[2];
}

void ora_set_perturber(ora_sim* s, double M, const double* pos, const double* vel)
{
    int c;
    s->pert_on = M > 0.0;
    s->pert_M = M;
    for (c = 0; c < 3; c++) { s->pert_r[c] = pos[c]; s->pert_v[c] = vel[c]; s->pert_a[c] = 0.0; }
}

void ora_get_perturber(const ora_sim* s, double* pos, double* vel, double* acc)
{
    int c;
    for (c = 0; c < 3; c++) {
        if (pos) pos[c] = s->pert_r[c];
        if (vel) vel[c] = s->pert_v[c];
        if (acc) acc[c] = s->pert_a[c];
    }
}

/* Binary search for (i, j) in the previous step's canonical pair list. */
static int64_t find_old(const int64_t* opi, const int64_t* opj, int64_t onp, int64_t i, int64_t j)
{
    int64_t lo = 0, hi = onp;
    while (lo < hi) {
        int64_t mid = (lo + hi) / 2;
        if (opi[mid] < i || (opi[mid] == i && opj[mid] < j)) lo = mid + 1;
        else hi = mid;
    }
    if (lo < onp && opi[lo] == i && opj[lo] == j) return lo;
    return -1;
}

/* Contacts at the current positions and velocities: brute-force search,
 * spring history carried from the previous list (opi, opj, ohist of onp
 * pairs; none when onp is 0), the force of every contact, and the per-sphere
 * sums in canonical order (F and tau are overwritten). */
static void contact_pass(ora_sim* s, const int64_t* opi, const int64_t* opj, const double* ohist,
                         int64_t onp)
{
    int64_t k, i;
    int c;
    find_pairs(s);
    for (i = 0; i < 3 * s->ns; i++) { s->F[i] = 0.0; s->tau[i] = 0.0; }
    /* pairs in lexicographic order: each sphere accumulates its contacts in
     * that order */
    for (k = 0; k < s->np; k++) {
        double h_old[7] = {0, 0, 0, 0, 0, 0, 0};
        int64_t ii = s->pi[k], jj = s->pj[k];
        if (onp > 0) {
            int64_t o = find_old(opi, opj, onp, ii, jj);
            if (o >= 0) memcpy(h_old, &ohist[7 * o], 7 * sizeof(double));
        }
        pair_force(s, ii, jj, h_old, &s->hist[7 * k], &s->pforce[9 * k], &s->pdiag[8 * k]);
    }
    /* per-sphere accumulation in canonical order (pairs sorted by (i, j)) */
    for (k = 0; k < s->np; k++) {
        int64_t ii = s->pi[k], jj = s->pj[k];
        const double* f = &s->pforce[9 * k];
        for (c = 0; c < 3; c++) {
            s->F[3 * ii + c] += f[c];
            s->tau[3 * ii + c] += f[3 + c];
            if (jj < s->ns) {             /* a wall takes the reaction */
                s->F[3 * jj + c] -= f[c];
                s->tau[3 * jj + c] += f[6 + c];
            }
        }
    }
}

/* Full force evaluation at the current positions and predicted velocities:
 * contacts (with history carried for pairs that persist), gravity, and the
 * reduction onto aggregates (Eqs. 5-7, 9). */
static void evaluate(ora_sim* s, int carry_history)
{
    int64_t i, A;
    int c;
    /* keep the previous contact list for the history carry */
    int64_t onp = s->np;
    int64_t* opi = NULL;
    int64_t* opj = NULL;
    double* ohist = NULL;
    if (carry_history && onp > 0) {
        opi = (int64_t*)malloc(onp * sizeof(int64_t));
        opj = (int64_t*)malloc(onp * sizeof(int64_t));
        ohist = (double*)malloc(onp * 7 * sizeof(double));
        memcpy(opi, s->pi, onp * sizeof(int64_t));
        memcpy(opj, s->pj, onp * sizeof(int64_t));
        memcpy(ohist, s->hist, onp * 7 * sizeof(double));
    }
    contact_pass(s, opi, opj, ohist, ohist ? onp : 0);
    free(opi); free(opj); free(ohist);
    /* self-gravity, Eq. 4, every j != i including members of the same
     * aggregate (their forces cancel in Eqs. 5-6) */
    if (s->p.G != 0.0 && s->p.gravity_tree) {
        double* Fg = (double*)malloc(3 * s->ns * sizeof(double));
        ora_tree_gravity(s->r, s->m, s->s, s->ns, s->p.G, s->p.soft_frac, s->p.theta,
                         s->p.tree_leaf, s->p.tree_order, Fg);
        for (i = 0; i < 3 * s->ns; i++) s->F[i] += Fg[i];
        free(Fg);
    } else if (s->p.G != 0.0) {
        /* one target per iteration (threads share the targets; each sum runs
         * over j in index order, so the thread count changes nothing) */
#pragma omp parallel for schedule(static)
        for (i = 0; i < s->ns; i++) {
            double acc[3] = {0.0, 0.0, 0.0};
            int64_t j;
            int c;
            for (j = 0; j < s->ns; j++) {
                if (j == i) continue;
                gravity_pair(s->p.G, s->p.soft_frac, &s->r[3 * i], &s->r[3 * j], s->m[i], s->m[j],
                             s->s[i], s->s[j], acc);
            }
            for (c = 0; c < 3; c++) s->F[3 * i + c] += acc[c];
        }
    }
    /* perturber: pull on every sphere (after self-gravity), reaction on it */
    if (s->pert_on) {
        double Fp[3] = {0.0, 0.0, 0.0};
        for (i = 0; i < s->ns; i++) {
            double f[3] = {0.0, 0.0, 0.0};
            perturber_pull(s, i, f);
            for (c = 0; c < 3; c++) { s->F[3 * i + c] += f[c]; Fp[c] -= f[c]; }
        }
        for (c = 0; c < 3; c++) s->pert_a[c] = Fp[c] / s->pert_M;
    }
    /* GetAccelAndTorque: a_A = (1/M) sum F_i  (Eqs. 5, 7);
     * N_A = sum [(r_i - r_A) x F_i + tau_i]  (Eqs. 6, 9: the contact part of
     * tau_i moves each contact force to its contact point). */
    for (A = 0; A < s->na; A++) {
        double FA[3] = {0, 0, 0}, NA[3] = {0, 0, 0};
        double R[3][3];
        quat_to_R(&s->q[4 * A], R);
        for (i = s->first[A]; i < s->first[A] + s->count[A]; i++) {
            double d[3], dxF[3];
            mat_vec(R, &s->b[3 * i], d);
            cross(d, &s->F[3 * i], dxF);
            for (c = 0; c < 3; c++) {
                FA[c] += s->F[3 * i + c];
                NA[c] += dxF[c] + s->tau[3 * i + c];
            }
        }
        /* a uniform field adds g to every body and no torque */
        for (c = 0; c < 3; c++) {
            s->aA[3 * A + c] = FA[c] / s->M[A] + s->p.g[c];
            s->NA[3 * A + c] = NA[c];
        }
    }
}

static int finite_all(const double* a, int64_t n)
{
    int64_t i;
    for (i = 0; i < n; i++) if (!isfinite(a[i])) return 0;
    return 1;
}

int ora_add(ora_sim* s, int64_t n_agg, const int32_t* counts, const double* pos,
            const double* radius, const double* mass, const double* agg_vel,
            const double* agg_spin, int32_t evaluate_now)
{
    int64_t A, i, ns = 0;
    int c;
    if (s->na != 0 || n_agg <= 0) return -1;
    for (A = 0; A < n_agg; A++) {
        if (counts[A] <= 0) return -1;
        ns += counts[A];
    }
    if (!finite_all(pos, 3 * ns) || !finite_all(radius, ns) || !finite_all(mass, ns)) return -1;
    for (i = 0; i < ns; i++) if (radius[i] <= 0.0 || mass[i] <= 0.0) return -1;
    s->na = n_agg;
    s->ns = ns;
    s->first = (int64_t*)malloc(n_agg * sizeof(int64_t));
    s->count = (int64_t*)malloc(n_agg * sizeof(int64_t));
    s->M = (double*)calloc(n_agg, sizeof(double));
    s->rA = (double*)calloc(3 * n_agg, sizeof(double));
    s->vA = (double*)calloc(3 * n_agg, sizeof(double));
    s->aA = (double*)calloc(3 * n_agg, sizeof(double));
    s->NA = (double*)calloc(3 * n_agg, sizeof(double));
    s->q = (double*)calloc(4 * n_agg, sizeof(double));
    s->wb = (double*)calloc(3 * n_agg, sizeof(double));
    s->I = (double*)calloc(3 * n_agg, sizeof(double));
    s->wA = (double*)calloc(3 * n_agg, sizeof(double));
    s->agg = (int64_t*)malloc(ns * sizeof(int64_t));
    s->b = (double*)calloc(3 * ns, sizeof(double));
    s->s = (double*)malloc(ns * sizeof(double));
    s->m = (double*)malloc(ns * sizeof(double));
    s->r = (double*)calloc(3 * ns, sizeof(double));
    s->v = (double*)calloc(3 * ns, sizeof(double));
    s->F = (double*)calloc(3 * ns, sizeof(double));
    s->tau = (double*)calloc(3 * ns, sizeof(double));
    int64_t off = 0;
    for (A = 0; A < n_agg; A++) {
        s->first[A] = off;
        s->count[A] = counts[A];
        for (i = off; i < off + counts[A]; i++) {
            s->agg[i] = A;
            s->s[i] = radius[i];
            s->m[i] = mass[i];
        }
        ora_setup_body(counts[A], &pos[3 * off], &radius[off], &mass[off], &s->M[A],
                       &s->rA[3 * A], &s->I[3 * A], &s->q[4 * A], &s->b[3 * off]);
        /* centre-of-mass velocity and space-frame spin as given; body spin
         * w_b = R^T w */
        double R[3][3];
        quat_to_R(&s->q[4 * A], R);
        for (c = 0; c < 3; c++) s->vA[3 * A + c] = agg_vel ? agg_vel[3 * A + c] : 0.0;
        if (agg_spin) mat_T_vec(R, &agg_spin[3 * A], &s->wb[3 * A]);
        if (s->p.periodic) {
            for (c = 0; c < 3; c++) {
                double L = s->p.box[c];
                double x = s->rA[3 * A + c];
                x = x - L * floor(x / L);
                if (x >= L) x -= L;
                s->rA[3 * A + c] = x;
            }
        }
        off += counts[A];
    }
    /* initial evaluation at t0: unpredicted velocities (a_A = 0 so the Eq. 3
     * extrapolation term vanishes) and empty contact history */
    reconstruct(s, 0.0);
    if (evaluate_now) evaluate(s, 0);
    return 0;
}

/* Spin-up forcing: a constant spin increment dw about +z through the pile's
 * centre of mass, applied to every aggregate after the second kick. */
static void spin_up(ora_sim* s)
{
    int64_t A;
    int c;
    double dw = s->p.spin_dw;
    if (dw == 0.0) return;
    double Mt = 0.0, com[3] = {0, 0, 0};
    for (A = 0; A < s->na; A++) {
        Mt += s->M[A];
        for (c = 0; c < 3; c++) com[c] += s->M[A] * s->rA[3 * A + c];
    }
    for (c = 0; c < 3; c++) com[c] /= Mt;
    for (A = 0; A < s->na; A++) {
        double rel[3], dv[3], R[3][3], dws[3] = {0.0, 0.0, dw}, dwb[3];
        double z[3] = {0.0, 0.0, dw};
        for (c = 0; c < 3; c++) rel[c] = s->rA[3 * A + c] - com[c];
        cross(z, rel, dv);
        for (c = 0; c < 3; c++) s->vA[3 * A + c] += dv[c];
        quat_to_R(&s->q[4 * A], R);
        mat_T_vec(R, dws, dwb);
        for (c = 0; c < 3; c++) s->wb[3 * A + c] += dwb[c];
    }
}

static void step_once(ora_sim* s)
{
    const double h = s->p.dt;
    int64_t A;
    int c;
    /* kick (half step) and drift of the centres of mass (leapfrog) */
    for (A = 0; A < s->na; A++) {
        for (c = 0; c < 3; c++) {
            s->vA[3 * A + c] += 0.5 * h * s->aA[3 * A + c];
            s->rA[3 * A + c] += h * s->vA[3 * A + c];
        }
        if (s->p.periodic) {
            for (c = 0; c < 3; c++) {
                double L = s->p.box[c];
                if (s->rA[3 * A + c] >= L) s->rA[3 * A + c] -= L;
                if (s->rA[3 * A + c] < 0.0) s->rA[3 * A + c] += L;
            }
        }
    }
    if (s->pert_on) {
        for (c = 0; c < 3; c++) {
            s->pert_v[c] += 0.5 * h * s->pert_a[c];
            s->pert_r[c] += h * s->pert_v[c];
        }
    }
    /* orientation and spin: one RK5 step with the last torque */
    for (A = 0; A < s->na; A++)
        ora_rotate(&s->q[4 * A], &s->wb[3 * A], &s->I[3 * A], &s->NA[3 * A], h, NULL);
    /* member positions and predicted velocities (Eq. 3) */
    reconstruct(s, 0.5 * h);
    s->t_eval = (double)(s->steps + 1) * h;
    evaluate(s, 1);
    s->steps++;
    /* second half kick */
    for (A = 0; A < s->na; A++)
        for (c = 0; c < 3; c++) s->vA[3 * A + c] += 0.5 * h * s->aA[3 * A + c];
    if (s->pert_on)
        for (c = 0; c < 3; c++) s->pert_v[c] += 0.5 * h * s->pert_a[c];
    spin_up(s);
}

int ora_step(ora_sim* s, int64_t n_steps)
{
    int64_t k;
    if (s->na == 0) return -1;
    for (k = 0; k < n_steps; k++) step_once(s);
    return 0;
}

void ora_get_counts(const ora_sim* s, int64_t* n_agg, int64_t* n_sph, int64_t* n_pairs)
{
    if (n_agg) *n_agg = s->na;
    if (n_sph) *n_sph = s->ns;
    if (n_pairs) *n_pairs = s->np;
}

void ora_get_aggregates(const ora_sim* s, double* M, double* rA, double* vA, double* aA,
                        double* NA, double* q, double* wb, double* wA, double* I)
{
    int64_t n = s->na;
    if (M) memcpy(M, s->M, n * sizeof(double));
    if (rA) memcpy(rA, s->rA, 3 * n * sizeof(double));
    if (vA) memcpy(vA, s->vA, 3 * n * sizeof(double));
    if (aA) memcpy(aA, s->aA, 3 * n * sizeof(double));
    if (NA) memcpy(NA, s->NA, 3 * n * sizeof(double));
    if (q) memcpy(q, s->q, 4 * n * sizeof(double));
    if (wb) memcpy(wb, s->wb, 3 * n * sizeof(double));
    if (wA) memcpy(wA, s->wA, 3 * n * sizeof(double));
    if (I) memcpy(I, s->I, 3 * n * sizeof(double));
}

void ora_get_spheres(const ora_sim* s, double* r, double* v, double* F, double* tau,
                     double* body)
{
    int64_t n = s->ns;
    if (r) memcpy(r, s->r, 3 * n * sizeof(double));
    if (v) memcpy(v, s->v, 3 * n * sizeof(double));
    if (F) memcpy(F, s->F, 3 * n * sizeof(double));
    if (tau) memcpy(tau, s->tau, 3 * n * sizeof(double));
    if (body) memcpy(body, s->b, 3 * n * sizeof(double));
}

void ora_get_pairs(const ora_sim* s, int64_t* pi, int64_t* pj, double* hist, double* force,
                   double* diag)
{
    int64_t n = s->np;
    if (pi) memcpy(pi, s->pi, n * sizeof(int64_t));
    if (pj) memcpy(pj, s->pj, n * sizeof(int64_t));
    if (hist) memcpy(hist, s->hist, 7 * n * sizeof(double));
    if (force) memcpy(force, s->pforce, 9 * n * sizeof(double));
    if (diag) memcpy(diag, s->pdiag, 8 * n * sizeof(double));
}

void ora_diagnostics(ora_sim* s, double* out)
{
    int64_t A, i, j, k;
    int c;
    double P[3] = {0, 0, 0}, L[3] = {0, 0, 0}, Kt = 0, Kr = 0, Es = 0, Ug = 0, maxov = 0;
    for (A = 0; A < s->na; A++) {
        double R[3][3], Iw[3], Ls[3], rxp[3], p[3];
        const double* w = &s->wb[3 * A];
        for (c = 0; c < 3; c++) p[c] = s->M[A] * s->vA[3 * A + c];
        for (c = 0; c < 3; c++) P[c] += p[c];
        cross(&s->rA[3 * A], p, rxp);
        quat_to_R(&s->q[4 * A], R);
        for (c = 0; c < 3; c++) Iw[c] = s->I[3 * A + c] * w[c];
        mat_vec(R, Iw, Ls);
        for (c = 0; c < 3; c++) L[c] += rxp[c] + Ls[c];
        Kt += 0.5 * s->M[A] * dot(&s->vA[3 * A], &s->vA[3 * A]);
        Kr += 0.5 * dot(w, Iw);
    }
    for (k = 0; k < s->np; k++) {
        double delta = s->pdiag[8 * k + 4];
        Es += 0.5 * s->p.k_n * delta * delta;
        if (delta > maxov) maxov = delta;
    }
    if (s->p.G != 0.0) {
        for (i = 0; i < s->ns; i++) {
            for (j = i + 1; j < s->ns; j++) {
                double d[3] = {s->r[3 * j] - s->r[3 * i], s->r[3 * j + 1] - s->r[3 * i + 1],
                               s->r[3 * j + 2] - s->r[3 * i + 2]};
                double eps = s->p.soft_frac * 0.5 * (s->s[i] + s->s[j]);
                Ug -= s->p.G * s->m[i] * s->m[j] / sqrt(dot(d, d) + eps * eps);
            }
        }
    }
    /* bulk radius: uniform-sphere equivalent of the mass-weighted mean
     * square distance of sphere centres from the centre of mass */
    double Mt = 0, com[3] = {0, 0, 0}, r2 = 0;
    for (i = 0; i < s->ns; i++) {
        Mt += s->m[i];
        for (c = 0; c < 3; c++) com[c] += s->m[i] * s->r[3 * i + c];
    }
    for (c = 0; c < 3; c++) com[c] /= Mt;
    for (i = 0; i < s->ns; i++) {
        double d[3] = {s->r[3 * i] - com[0], s->r[3 * i + 1] - com[1], s->r[3 * i + 2] - com[2]};
        r2 += s->m[i] * dot(d, d);
    }
    r2 /= Mt;
    /* potential of the uniform field: -sum_A M_A g . r_A */
    double Uu = 0.0;
    for (A = 0; A < s->na; A++) Uu -= s->M[A] * dot(s->p.g, &s->rA[3 * A]);
    for (c = 0; c < 3; c++) { out[c] = P[c]; out[3 + c] = L[c]; out[12 + c] = com[c]; }
    out[6] = Kt; out[7] = Kr; out[8] = Es; out[9] = Ug; out[10] = maxov;
    out[11] = sqrt(5.0 / 3.0 * r2);
    out[15] = Uu;
}

/* The listed spheres are independent: with OpenMP they are shared among
 * threads; each one's sums keep their order. */
void ora_eval_subset(const ora_sim* s, const int64_t* idx, int64_t n_idx, double* F, double* tau)
{
    int64_t k;
#pragma omp parallel for schedule(dynamic, 4)
    for (k = 0; k < n_idx; k++) {
        int64_t x = idx[k], j;
        int c;
        double f[3] = {0, 0, 0}, t[3] = {0, 0, 0};
        /* contacts in canonical order: pairs (j, x) with j < x, then (x, j) */
        for (j = 0; j < s->ns; j++) {
            double d[3], hz[7] = {0, 0, 0, 0, 0, 0, 0}, hn[7], o9[9];
            if (j == x || s->agg[j] == s->agg[x]) continue;
            int64_t a = j < x ? j : x, b = j < x ? x : j;
            separation(&s->p, &s->r[3 * a], &s->r[3 * b], d);
            if (!in_contact(d, s->s[a], s->s[b])) continue;
            pair_force(s, a, b, hz, hn, o9, NULL);
            for (c = 0; c < 3; c++) {
                if (a == x) { f[c] += o9[c]; t[c] += o9[3 + c]; }
                else { f[c] -= o9[c]; t[c] += o9[6 + c]; }
            }
        }
        if (s->p.G != 0.0) {
            double acc[3] = {0, 0, 0};
            for (j = 0; j < s->ns; j++) {
                if (j == x) continue;
                gravity_pair(s->p.G, s->p.soft_frac, &s->r[3 * x], &s->r[3 * j], s->m[x], s->m[j],
                             s->s[x], s->s[j], acc);
            }
            for (c = 0; c < 3; c++) f[c] += acc[c];
        }
        {
            int w;
            for (w = 0; w < s->p.n_walls; w++) {
                double hz[7] = {0, 0, 0, 0, 0, 0, 0}, hn[7], o9[9];
                if (!(wall_distance(&s->p, w, s->t_eval, &s->r[3 * x], NULL) < s->s[x])) continue;
                pair_force(s, x, s->ns + w, hz, hn, o9, NULL);
                for (c = 0; c < 3; c++) { f[c] += o9[c]; t[c] += o9[3 + c]; }
            }
        }
        if (s->pert_on) perturber_pull(s, x, f);
        for (c = 0; c < 3; c++) { F[3 * k + c] = f[c]; tau[3 * k + c] = t[c]; }
    }
}

int64_t ora_find_contacts(const double* pos, const double* radius, const int32_t* agg, int64_t n,
                          const double* box, uint64_t* keys, int64_t cap)
{
    ora_params p;
    int64_t i, j, np = 0;
    memset(&p, 0, sizeof(p));
    if (box) { p.periodic = 1; p.box[0] = box[0]; p.box[1] = box[1]; p.box[2] = box[2]; }
    for (i = 0; i < n; i++) {
        for (j = i + 1; j < n; j++) {
            double d[3];
            if (agg[i] == agg[j]) continue;
            separation(&p, &pos[3 * i], &pos[3 * j], d);
            if (in_contact(d, radius[i], radius[j])) {
                if (np < cap) keys[np] = ((uint64_t)i << 32) | (uint64_t)j;
                np++;
            }
        }
    }
    return np;
}

/* Threads of the OpenMP target loops (gravity); 1 runs them serially.
 * Returns the count in effect (1 without OpenMP). */
int32_t ora_set_threads(int32_t n)
{
#ifdef _OPENMP
    if (n > 0) omp_set_num_threads(n);
    return (int32_t)omp_get_max_threads();
#else
    (void)n;
    return 1;
#endif
}

/* Contact part of one evaluation on given sphere states (the same-input
 * check of the contact model): n spheres at pos with velocities vel (the
 * predicted velocities of Eq. 3), radii, aggregate ids agg (0..n_agg-1),
 * aggregate masses and space-frame spins; previous contacts old_keys
 * (canonical, sorted; a wall w of sphere i is i << 32 | (n + w)) with their
 * history old_hist[7].  Walls of p are taken at t = 0.  Writes per-sphere
 * contact force F and torque tau (canonical order of sums), the new keys and
 * history (up to cap); returns the number of contacts. */
int64_t ora_contact_forces(const ora_params* p, int64_t n, const double* pos, const double* vel,
                           const double* radius, const int32_t* agg, int64_t n_agg,
                           const double* agg_mass, const double* agg_spin, int64_t n_old,
                           const uint64_t* old_keys, const double* old_hist, double* F,
                           double* tau, uint64_t* keys, double* hist, int64_t cap)
{
    int64_t i, k, np;
    ora_sim* s = ora_create(p);
    int64_t* opi = (int64_t*)malloc((n_old > 0 ? n_old : 1) * sizeof(int64_t));
    int64_t* opj = (int64_t*)malloc((n_old > 0 ? n_old : 1) * sizeof(int64_t));
    s->na = n_agg;
    s->ns = n;
    s->agg = (int64_t*)malloc(n * sizeof(int64_t));
    s->s = (double*)malloc(n * sizeof(double));
    s->r = (double*)malloc(3 * n * sizeof(double));
    s->v = (double*)malloc(3 * n * sizeof(double));
    s->F = (double*)calloc(3 * n, sizeof(double));
    s->tau = (double*)calloc(3 * n, sizeof(double));
    s->M = (double*)malloc(n_agg * sizeof(double));
    s->wA = (double*)malloc(3 * n_agg * sizeof(double));
    for (i = 0; i < n; i++) { s->agg[i] = agg[i]; s->s[i] = radius[i]; }
    memcpy(s->r, pos, 3 * n * sizeof(double));
    memcpy(s->v, vel, 3 * n * sizeof(double));
    memcpy(s->M, agg_mass, n_agg * sizeof(double));
    memcpy(s->wA, agg_spin, 3 * n_agg * sizeof(double));
    s->t_eval = 0.0;
    for (k = 0; k < n_old; k++) {
        opi[k] = (int64_t)(old_keys[k] >> 32);
        opj[k] = (int64_t)(old_keys[k] & 0xffffffffu);
    }
    contact_pass(s, opi, opj, old_hist, n_old);
    memcpy(F, s->F, 3 * n * sizeof(double));
    memcpy(tau, s->tau, 3 * n * sizeof(double));
    np = s->np;
    for (k = 0; k < np && k < cap; k++) {
        keys[k] = ((uint64_t)s->pi[k] << 32) | (uint64_t)s->pj[k];
        memcpy(&hist[7 * k], &s->hist[7 * k], 7 * sizeof(double));
    }
    free(opi);
    free(opj);
    ora_destroy(s);
    return np;
}
