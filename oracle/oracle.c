/*
 * Reference oracle for vectorized motion validation (arXiv 2309.14545).
 *
 * TEST INFRASTRUCTURE ONLY.  This file is the plain, slow, obviously-correct CPU definition of
 * what the GPU path computes.  It is used by the test suite, by the smoke check and by the
 * benchmark's CPU-baseline leg, and by nothing else.  It shares no code, header, table or
 * helper with the HIP library.
 *
 * Precision: FP64 scalar throughout.  Inputs are the canonical FP32 arrays upcast to double,
 * so both sides start from identical values.
 *
 * What it computes (each function cites the passage it follows):
 *   - forward kinematics of a revolute tree in standard DH form         (Sec. III-B)
 *   - positions of the robot's collision spheres                        (Sec. III-C, spheres
 *                                                                         only, no full pose)
 *   - signed clearance of a robot sphere to a sphere, capsule, cylinder or oriented box, and
 *     to another robot sphere (self collision)                          (Sec. III-C)
 *   - state validity: collision iff the minimum clearance is negative   (Sec. III-C)
 *   - edge discretization and edge validity as the OR over its states   (Sec. III-D)
 *   - squared-penetration cost and its gradient with respect to the joint angles (an
 *     extension used for trajectory optimisation with sphere models, Sec. III-C context)
 *
 * The method's accelerations -- the rake ordering, the per-link bounding-sphere mid-phase,
 * interleaving checks into FK and early exit (Sec. III-D) -- change the work done, never the
 * result, so none of them appears here: every state is checked against every primitive and
 * every listed self pair.
 *
 * Readings where the paper is silent (all recorded in the design notes):
 *   - joints are revolute with standard DH A = Rz(theta) Tz(d) Tx(a) Rx(alpha);
 *   - joint j hangs off link parent[j] through a fixed 3x4 mount M_j; link 0 is the fixed base
 *     at the world origin;
 *   - a state collides iff some clearance is strictly negative, or some joint value is not
 *     finite;
 *   - an edge is discretized with the per-joint (L-infinity) step: n = max(2, ceil(L/res)+1),
 *     L = max_j |qb_j - qa_j|, states q_k = qa + k/(n-1) (qb - qa), both endpoints included.
 */
#include <math.h>
#include <pthread.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#include <unistd.h>

typedef struct {
    int dof;
    const int32_t *parent_link;   /* [dof] link index the joint hangs off (0 = base)      */
    const double *mount;          /* [dof][12] row-major 3x4 fixed transform              */
    const double *dh;             /* [dof][5] a, d, cos(alpha), sin(alpha), theta offset  */
    int n_spheres;
    const int32_t *sphere_link;   /* [S] link of each sphere                               */
    const double *sphere_xyzr;    /* [S][4] centre in its link frame, radius              */
    int n_pairs;
    const int32_t *pairs;         /* [P][2] self-collision sphere pairs                    */
    const int32_t *joint_type;    /* [dof] 0 revolute, 1 prismatic; NULL = all revolute     */
} orc_robot;

static int prismatic(const orc_robot *rb, int j) { return rb->joint_type && rb->joint_type[j] == 1; }

typedef struct {
    int n_spheres;   const double *spheres;    /* [n][4]  centre, radius                    */
    int n_capsules;  const double *capsules;   /* [n][7]  p0, p1, radius                    */
    int n_cylinders; const double *cylinders;  /* [n][8]  centre, unit axis, half h, radius */
    int n_boxes;     const double *boxes;      /* [n][15] centre, R row-major, half extents */
} orc_env;

#define ORC_MAX_DOF 64

/* ------------------------------------------------------------------------------------------
 * 4x4 homogeneous transforms stored row-major as double[16].
 * ---------------------------------------------------------------------------------------- */
static void mat_identity(double m[16]) {
    memset(m, 0, 16 * sizeof(double));
    m[0] = m[5] = m[10] = m[15] = 1.0;
}

static void mat_from_3x4(const double *r, double m[16]) {
    for (int i = 0; i < 12; ++i) m[i] = r[i];
    m[12] = m[13] = m[14] = 0.0;
    m[15] = 1.0;
}

static void mat_mul(const double a[16], const double b[16], double out[16]) {
    double t[16];
    for (int i = 0; i < 4; ++i)
        for (int j = 0; j < 4; ++j) {
            double s = 0.0;
            for (int k = 0; k < 4; ++k) s += a[4 * i + k] * b[4 * k + j];
            t[4 * i + j] = s;
        }
    memcpy(out, t, sizeof t);
}

/* Standard DH link transform A = Rz(theta) Tz(d) Tx(a) Rx(alpha), written out as a matrix. */
static void dh_matrix(double a, double d, double ca, double sa, double theta, double m[16]) {
    double ct = cos(theta), st = sin(theta);
    m[0] = ct;  m[1] = -st * ca; m[2] = st * sa;   m[3] = a * ct;
    m[4] = st;  m[5] = ct * ca;  m[6] = -ct * sa;  m[7] = a * st;
    m[8] = 0.0; m[9] = sa;       m[10] = ca;       m[11] = d;
    m[12] = 0.0; m[13] = 0.0;    m[14] = 0.0;      m[15] = 1.0;
}

/*
 * Forward kinematics (Sec. III-B): pose of every link for one configuration.
 *   T_0 = I;  P_j = T_parent(j) * M_j;
 *   revolute:  T_{j+1} = P_j * Rz(q_j + theta_offset_j) Tz(d_j) Tx(a_j) Rx(alpha_j),
 *   prismatic: T_{j+1} = P_j * Rz(theta_offset_j) Tz(d_j + q_j) Tx(a_j) Rx(alpha_j)
 * (a prismatic joint slides along the z axis of P_j by q_j).
 * link_T: [(dof+1)][12] row-major 3x4 of every link (link 0 first).
 * joint_P: [dof][12] frame of each joint (its z column is the rotation axis, its last column
 * the point the axis passes through); may be NULL.
 */
void orc_fk(const orc_robot *rb, const double *q, double *link_T, double *joint_P) {
    double T[ORC_MAX_DOF + 1][16];
    mat_identity(T[0]);
    for (int j = 0; j < rb->dof; ++j) {
        double M[16], P[16], A[16];
        const double *dh = rb->dh + 5 * j;
        mat_from_3x4(rb->mount + 12 * j, M);
        mat_mul(T[rb->parent_link[j]], M, P);
        if (prismatic(rb, j))
            dh_matrix(dh[0], dh[1] + q[j], dh[2], dh[3], dh[4], A);
        else
            dh_matrix(dh[0], dh[1], dh[2], dh[3], q[j] + dh[4], A);
        mat_mul(P, A, T[j + 1]);
        if (joint_P) memcpy(joint_P + 12 * j, P, 12 * sizeof(double));
    }
    if (link_T)
        for (int k = 0; k <= rb->dof; ++k) memcpy(link_T + 12 * k, T[k], 12 * sizeof(double));
}

/* Sphere centres in the world frame (Sec. III-C): c_s = T_link(s) * (l_s, 1).  out: [S][3]. */
void orc_sphere_centres(const orc_robot *rb, const double *q, double *out) {
    double T[(ORC_MAX_DOF + 1) * 12];
    orc_fk(rb, q, T, NULL);
    for (int s = 0; s < rb->n_spheres; ++s) {
        const double *m = T + 12 * rb->sphere_link[s];
        const double *l = rb->sphere_xyzr + 4 * s;
        for (int i = 0; i < 3; ++i)
            out[3 * s + i] = m[4 * i] * l[0] + m[4 * i + 1] * l[1] + m[4 * i + 2] * l[2] +
                             m[4 * i + 3];
    }
}

/* ------------------------------------------------------------------------------------------
 * Signed distances of a point to each primitive (negative inside), Sec. III-C primitives.
 * Closest-point constructions follow Ericson, Real-Time Collision Detection, Ch. 5.
 * ---------------------------------------------------------------------------------------- */
static double dot3(const double *a, const double *b) { return a[0] * b[0] + a[1] * b[1] + a[2] * b[2]; }
static double norm3(const double *a) { return sqrt(dot3(a, a)); }

double orc_sd_sphere(const double *c, const double *prim) {
    double d[3] = {c[0] - prim[0], c[1] - prim[1], c[2] - prim[2]};
    return norm3(d) - prim[3];
}

/* Capsule: closest point on segment p0-p1 (parameter clamped to [0,1]); minus the radius. */
double orc_sd_capsule(const double *c, const double *prim) {
    const double *p0 = prim, *p1 = prim + 3;
    double u[3] = {p1[0] - p0[0], p1[1] - p0[1], p1[2] - p0[2]};
    double w[3] = {c[0] - p0[0], c[1] - p0[1], c[2] - p0[2]};
    double uu = dot3(u, u);
    double t = uu > 0.0 ? dot3(w, u) / uu : 0.0;
    if (t < 0.0) t = 0.0;
    if (t > 1.0) t = 1.0;
    double d[3] = {w[0] - t * u[0], w[1] - t * u[1], w[2] - t * u[2]};
    return norm3(d) - prim[6];
}

/* Flat-capped cylinder with centre o, unit axis w, half height H and radius R. */
double orc_sd_cylinder(const double *c, const double *prim) {
    const double *o = prim, *w = prim + 3;
    double H = prim[6], R = prim[7];
    double v[3] = {c[0] - o[0], c[1] - o[1], c[2] - o[2]};
    double h = dot3(v, w);
    double rad[3] = {v[0] - h * w[0], v[1] - h * w[1], v[2] - h * w[2]};
    double rho = norm3(rad);
    double ah = fabs(h);
    if (ah <= H && rho <= R) {
        double a = H - ah, b = R - rho;
        return -(a < b ? a : b);
    }
    double x = rho - R > 0.0 ? rho - R : 0.0;
    double y = ah - H > 0.0 ? ah - H : 0.0;
    return sqrt(x * x + y * y);
}

/* Oriented box: point in box coordinates p = R^T (c - o); q = |p| - e;
 * sd = |max(q, 0)| + min(max(q_x, q_y, q_z), 0). */
double orc_sd_box(const double *c, const double *prim) {
    const double *o = prim, *R = prim + 3, *e = prim + 12;
    double v[3] = {c[0] - o[0], c[1] - o[1], c[2] - o[2]};
    double qv[3], out2 = 0.0, mx = -INFINITY;
    for (int k = 0; k < 3; ++k) {
        double pk = R[0 + k] * v[0] + R[3 + k] * v[1] + R[6 + k] * v[2];   /* column k */
        qv[k] = fabs(pk) - e[k];
        if (qv[k] > 0.0) out2 += qv[k] * qv[k];
        if (qv[k] > mx) mx = qv[k];
    }
    return sqrt(out2) + (mx < 0.0 ? mx : 0.0);
}

/* Clearance of robot sphere (c, r) to primitive kind k: sd(c) - r. */
enum { ORC_SPHERE = 0, ORC_CAPSULE = 1, ORC_CYLINDER = 2, ORC_BOX = 3 };

double orc_clearance(int kind, const double *c, double r, const double *prim) {
    switch (kind) {
    case ORC_SPHERE: return orc_sd_sphere(c, prim) - r;
    case ORC_CAPSULE: return orc_sd_capsule(c, prim) - r;
    case ORC_CYLINDER: return orc_sd_cylinder(c, prim) - r;
    default: return orc_sd_box(c, prim) - r;
    }
}

static int prim_count(const orc_env *env, int kind) {
    switch (kind) {
    case ORC_SPHERE: return env->n_spheres;
    case ORC_CAPSULE: return env->n_capsules;
    case ORC_CYLINDER: return env->n_cylinders;
    default: return env->n_boxes;
    }
}

static const double *prim_row(const orc_env *env, int kind, int i) {
    switch (kind) {
    case ORC_SPHERE: return env->spheres + 4 * i;
    case ORC_CAPSULE: return env->capsules + 7 * i;
    case ORC_CYLINDER: return env->cylinders + 8 * i;
    default: return env->boxes + 15 * i;
    }
}

static int all_finite(const double *q, int n) {
    for (int j = 0; j < n; ++j)
        if (!isfinite(q[j])) return 0;
    return 1;
}

/*
 * Minimum clearance of one state over every (robot sphere, primitive) pair and every listed
 * self pair (Sec. III-C: environment and self collision).  +inf if there is nothing to test;
 * NaN if some joint value is not finite.
 */
double orc_state_min_clearance(const orc_robot *rb, const orc_env *env, const double *q) {
    if (!all_finite(q, rb->dof)) return NAN;
    double *c = (double *)malloc(sizeof(double) * 3 * (rb->n_spheres + 1));
    orc_sphere_centres(rb, q, c);
    double cmin = INFINITY;
    for (int s = 0; s < rb->n_spheres; ++s) {
        double r = rb->sphere_xyzr[4 * s + 3];
        for (int kind = 0; kind < 4; ++kind)
            for (int i = 0, n = prim_count(env, kind); i < n; ++i) {
                double cl = orc_clearance(kind, c + 3 * s, r, prim_row(env, kind, i));
                if (cl < cmin) cmin = cl;
            }
    }
    for (int p = 0; p < rb->n_pairs; ++p) {
        int s = rb->pairs[2 * p], t = rb->pairs[2 * p + 1];
        double d[3] = {c[3 * s] - c[3 * t], c[3 * s + 1] - c[3 * t + 1], c[3 * s + 2] - c[3 * t + 2]};
        double cl = norm3(d) - rb->sphere_xyzr[4 * s + 3] - rb->sphere_xyzr[4 * t + 3];
        if (cl < cmin) cmin = cl;
    }
    free(c);
    return cmin;
}

/* State validity (Sec. III-C): 1 = in collision (or non-finite input), 0 = free. */
int orc_state_collides(const orc_robot *rb, const orc_env *env, const double *q) {
    double cm = orc_state_min_clearance(rb, env, q);
    return isnan(cm) ? 1 : (cm < 0.0);
}

/* Number of discretized states of edge qa->qb at per-joint resolution res (Sec. III-D).
 * An edge with a non-finite endpoint is reduced to its two endpoints (it collides anyway). */
int orc_edge_n_states(const double *qa, const double *qb, int dof, double res) {
    double L = 0.0;
    for (int j = 0; j < dof; ++j) {
        double d = fabs(qb[j] - qa[j]);
        if (!isfinite(d)) return 2;
        if (d > L) L = d;
    }
    double n = ceil(L / res) + 1.0;
    if (!(n < 2147483647.0)) return 2147483647;
    return n < 2.0 ? 2 : (int)n;
}

/* k-th of n discretized states: q_k = qa + (k/(n-1)) (qb - qa). */
void orc_edge_state(const double *qa, const double *qb, int dof, int n, int k, double *q) {
    double t = (double)k / (double)(n - 1);
    for (int j = 0; j < dof; ++j) q[j] = qa[j] + t * (qb[j] - qa[j]);
}

/* ------------------------------------------------------------------------------------------
 * Squared-penetration cost and its gradient.
 *   C(q) = sum_{s,o} max(0, -clear(s,o))^2 + sum_{(s,t)} max(0, -clear(s,t))^2
 * Gradient: f_s = dC/dc_s; dC/dq_j = sum over spheres on links moved by joint j of
 * (z_j x (c_s - o_j)) . f_s, with z_j, o_j the axis and origin of joint j's frame.
 * ---------------------------------------------------------------------------------------- */

/* Gradient of the signed distance with respect to the point (unit outward direction).
 * At measure-zero kinks: zero vector on a segment axis or at a sphere centre; inside a box the
 * normal of the face of the largest q component (lowest axis on ties, sign(0) = +1); inside a
 * cylinder the cap normal when the cap is no farther than the side. */
static void grad_sd(int kind, const double *c, const double *prim, double g[3]) {
    g[0] = g[1] = g[2] = 0.0;
    if (kind == ORC_SPHERE || kind == ORC_CAPSULE) {
        double foot[3];
        if (kind == ORC_SPHERE) {
            foot[0] = prim[0]; foot[1] = prim[1]; foot[2] = prim[2];
        } else {
            const double *p0 = prim, *p1 = prim + 3;
            double u[3] = {p1[0] - p0[0], p1[1] - p0[1], p1[2] - p0[2]};
            double w[3] = {c[0] - p0[0], c[1] - p0[1], c[2] - p0[2]};
            double uu = dot3(u, u);
            double t = uu > 0.0 ? dot3(w, u) / uu : 0.0;
            if (t < 0.0) t = 0.0;
            if (t > 1.0) t = 1.0;
            for (int i = 0; i < 3; ++i) foot[i] = p0[i] + t * u[i];
        }
        double d[3] = {c[0] - foot[0], c[1] - foot[1], c[2] - foot[2]};
        double n = norm3(d);
        if (n > 0.0)
            for (int i = 0; i < 3; ++i) g[i] = d[i] / n;
        return;
    }
    if (kind == ORC_BOX) {
        const double *o = prim, *R = prim + 3, *e = prim + 12;
        double v[3] = {c[0] - o[0], c[1] - o[1], c[2] - o[2]};
        double p[3], qv[3], out2 = 0.0;
        for (int k = 0; k < 3; ++k) {
            p[k] = R[0 + k] * v[0] + R[3 + k] * v[1] + R[6 + k] * v[2];
            qv[k] = fabs(p[k]) - e[k];
            if (qv[k] > 0.0) out2 += qv[k] * qv[k];
        }
        double local[3] = {0.0, 0.0, 0.0};
        if (out2 > 0.0) {
            double n = sqrt(out2);
            for (int k = 0; k < 3; ++k)
                if (qv[k] > 0.0) local[k] = (p[k] >= 0.0 ? 1.0 : -1.0) * qv[k] / n;
        } else {
            int kmax = 0;
            for (int k = 1; k < 3; ++k)
                if (qv[k] > qv[kmax]) kmax = k;
            local[kmax] = p[kmax] >= 0.0 ? 1.0 : -1.0;
        }
        for (int i = 0; i < 3; ++i)   /* back to world: R * local */
            g[i] = R[3 * i] * local[0] + R[3 * i + 1] * local[1] + R[3 * i + 2] * local[2];
        return;
    }
    /* cylinder */
    const double *o = prim, *w = prim + 3;
    double H = prim[6], R = prim[7];
    double v[3] = {c[0] - o[0], c[1] - o[1], c[2] - o[2]};
    double h = dot3(v, w);
    double rad[3] = {v[0] - h * w[0], v[1] - h * w[1], v[2] - h * w[2]};
    double rho = norm3(rad), ah = fabs(h), sh = h >= 0.0 ? 1.0 : -1.0;
    double ru[3] = {0.0, 0.0, 0.0};
    if (rho > 0.0)
        for (int i = 0; i < 3; ++i) ru[i] = rad[i] / rho;
    if (ah <= H && rho <= R) {
        if (H - ah <= R - rho)
            for (int i = 0; i < 3; ++i) g[i] = sh * w[i];
        else
            for (int i = 0; i < 3; ++i) g[i] = ru[i];
        return;
    }
    double x = rho - R > 0.0 ? rho - R : 0.0;
    double y = ah - H > 0.0 ? ah - H : 0.0;
    double n = sqrt(x * x + y * y);
    for (int i = 0; i < 3; ++i) g[i] = (x * ru[i] + y * sh * w[i]) / n;
}

/* Cost of one state; NaN for non-finite input. */
double orc_cost(const orc_robot *rb, const orc_env *env, const double *q) {
    if (!all_finite(q, rb->dof)) return NAN;
    double *c = (double *)malloc(sizeof(double) * 3 * (rb->n_spheres + 1));
    orc_sphere_centres(rb, q, c);
    double C = 0.0;
    for (int s = 0; s < rb->n_spheres; ++s) {
        double r = rb->sphere_xyzr[4 * s + 3];
        for (int kind = 0; kind < 4; ++kind)
            for (int i = 0, n = prim_count(env, kind); i < n; ++i) {
                double p = -orc_clearance(kind, c + 3 * s, r, prim_row(env, kind, i));
                if (p > 0.0) C += p * p;
            }
    }
    for (int k = 0; k < rb->n_pairs; ++k) {
        int s = rb->pairs[2 * k], t = rb->pairs[2 * k + 1];
        double d[3] = {c[3 * s] - c[3 * t], c[3 * s + 1] - c[3 * t + 1], c[3 * s + 2] - c[3 * t + 2]};
        double p = rb->sphere_xyzr[4 * s + 3] + rb->sphere_xyzr[4 * t + 3] - norm3(d);
        if (p > 0.0) C += p * p;
    }
    free(c);
    return C;
}

/* 1 if link `lk` is moved by joint j (i.e. link j+1 is lk or one of its ancestors). */
static int moved_by(const orc_robot *rb, int lk, int j) {
    while (lk > 0) {
        if (lk == j + 1) return 1;
        lk = rb->parent_link[lk - 1];
    }
    return 0;
}

/* Analytic gradient dC/dq of one state via the explicit per-sphere Jacobian. grad: [dof]. */
void orc_cost_grad(const orc_robot *rb, const orc_env *env, const double *q, double *grad) {
    int S = rb->n_spheres, dof = rb->dof;
    if (!all_finite(q, dof)) {
        for (int j = 0; j < dof; ++j) grad[j] = NAN;
        return;
    }
    double *c = (double *)malloc(sizeof(double) * 3 * (S + 1));
    double *f = (double *)calloc(3 * (S + 1), sizeof(double));
    double P[ORC_MAX_DOF * 12];
    double T[(ORC_MAX_DOF + 1) * 12];
    orc_fk(rb, q, T, P);
    orc_sphere_centres(rb, q, c);
    for (int s = 0; s < S; ++s) {
        double r = rb->sphere_xyzr[4 * s + 3];
        for (int kind = 0; kind < 4; ++kind)
            for (int i = 0, n = prim_count(env, kind); i < n; ++i) {
                const double *prim = prim_row(env, kind, i);
                double p = -orc_clearance(kind, c + 3 * s, r, prim);
                if (p > 0.0) {
                    double g[3];
                    grad_sd(kind, c + 3 * s, prim, g);
                    for (int a = 0; a < 3; ++a) f[3 * s + a] += -2.0 * p * g[a];
                }
            }
    }
    for (int k = 0; k < rb->n_pairs; ++k) {
        int s = rb->pairs[2 * k], t = rb->pairs[2 * k + 1];
        double d[3] = {c[3 * s] - c[3 * t], c[3 * s + 1] - c[3 * t + 1], c[3 * s + 2] - c[3 * t + 2]};
        double n = norm3(d);
        double p = rb->sphere_xyzr[4 * s + 3] + rb->sphere_xyzr[4 * t + 3] - n;
        if (p > 0.0 && n > 0.0)
            for (int a = 0; a < 3; ++a) {
                f[3 * s + a] += -2.0 * p * d[a] / n;
                f[3 * t + a] += 2.0 * p * d[a] / n;
            }
    }
    for (int j = 0; j < dof; ++j) {
        const double *Pj = P + 12 * j;
        double z[3] = {Pj[2], Pj[6], Pj[10]}, o[3] = {Pj[3], Pj[7], Pj[11]};
        double acc = 0.0;
        for (int s = 0; s < S; ++s) {
            if (!moved_by(rb, rb->sphere_link[s], j)) continue;
            /* Jacobian column of the sphere centre: z x (c - o) for a revolute joint, z for a
             * prismatic one */
            double v[3] = {c[3 * s] - o[0], c[3 * s + 1] - o[1], c[3 * s + 2] - o[2]};
            double jc[3] = {z[1] * v[2] - z[2] * v[1], z[2] * v[0] - z[0] * v[2],
                            z[0] * v[1] - z[1] * v[0]};
            if (prismatic(rb, j)) {
                jc[0] = z[0];
                jc[1] = z[1];
                jc[2] = z[2];
            }
            acc += dot3(jc, f + 3 * s);
        }
        grad[j] = acc;
    }
    free(c);
    free(f);
}

/* ------------------------------------------------------------------------------------------
 * Batched drivers.  Work is split statically over threads; n_threads <= 0 uses every online
 * core.  Configurations are SoA: q[j * ldq + i] is joint j of state i.
 * ---------------------------------------------------------------------------------------- */
typedef struct {
    const orc_robot *rb;
    const orc_env *env;
    const double *q;
    int64_t n, ldq, lo, hi;
    double *out;          /* per-state scalar output (min clearance or cost)   */
    double *grad;         /* [dof][ldg] gradient output (cost-grad job)          */
    int64_t ldg;
    uint8_t *flag;
    int job;              /* 0 = min clearance, 1 = cost, 2 = gradient           */
    /* edges */
    const double *qa, *qb;
    const int32_t *n_states;
    double res;
    int8_t *cls;
    int early;
} orc_job;

static void *run_job(void *arg) {
    orc_job *jb = (orc_job *)arg;
    int dof = jb->rb->dof;
    double q[ORC_MAX_DOF], g[ORC_MAX_DOF];
    for (int64_t i = jb->lo; i < jb->hi; ++i) {
        if (jb->job <= 2) {
            for (int j = 0; j < dof; ++j) q[j] = jb->q[j * jb->ldq + i];
            if (jb->job == 0) {
                double cm = orc_state_min_clearance(jb->rb, jb->env, q);
                if (jb->out) jb->out[i] = cm;
                if (jb->flag) jb->flag[i] = isnan(cm) ? 1 : (cm < 0.0);
            } else if (jb->job == 1) {
                jb->out[i] = orc_cost(jb->rb, jb->env, q);
            } else {
                orc_cost_grad(jb->rb, jb->env, q, g);
                for (int j = 0; j < dof; ++j) jb->grad[j * jb->ldg + i] = g[j];
            }
        } else {
            /* edge job: flag = OR over states; class 1 = some state clearly colliding
             * (cmin < -1e-4), 0 = every state clearly free (cmin > 1e-4), 2 = otherwise. */
            const double *qa = jb->qa + (int64_t)dof * i, *qb = jb->qb + (int64_t)dof * i;
            int n = jb->n_states ? jb->n_states[i] : orc_edge_n_states(qa, qb, dof, jb->res);
            int hit = 0, near = 0;
            double emin = INFINITY;
            if (n < 2) n = 2;
            if (!all_finite(qa, dof) || !all_finite(qb, dof)) {
                /* a non-finite endpoint is a non-finite state of the edge: colliding */
                jb->flag[i] = 1;
                if (jb->cls) jb->cls[i] = 1;
                if (jb->out) jb->out[i] = NAN;
                continue;
            }
            for (int k = 0; k < n; ++k) {
                orc_edge_state(qa, qb, dof, n, k, q);
                double cm = orc_state_min_clearance(jb->rb, jb->env, q);
                if (isnan(cm)) { hit = 1; emin = NAN; break; }
                if (cm < emin) emin = cm;
                if (cm < 0.0) hit = 1;
                if (cm < -1e-4) { if (jb->early) break; }
                else if (cm <= 1e-4) near = 1;
            }
            jb->flag[i] = (uint8_t)hit;
            if (jb->cls) jb->cls[i] = (int8_t)(isnan(emin) || emin < -1e-4 ? 1 : (near ? 2 : 0));
            if (jb->out) jb->out[i] = emin;
        }
    }
    return NULL;
}

static int resolve_threads(int n_threads, int64_t n) {
    if (n_threads <= 0) n_threads = (int)sysconf(_SC_NPROCESSORS_ONLN);
    if (n_threads < 1) n_threads = 1;
    if (n_threads > 256) n_threads = 256;
    if ((int64_t)n_threads > n) n_threads = n > 0 ? (int)n : 1;
    return n_threads;
}

static void run_parallel(orc_job base, int64_t n, int n_threads) {
    int nt = resolve_threads(n_threads, n);
    pthread_t th[256];
    orc_job jobs[256];
    for (int t = 0; t < nt; ++t) {
        jobs[t] = base;
        jobs[t].lo = n * t / nt;
        jobs[t].hi = n * (t + 1) / nt;
        pthread_create(&th[t], NULL, run_job, &jobs[t]);
    }
    for (int t = 0; t < nt; ++t) pthread_join(th[t], NULL);
}

int orc_threads(int n_threads) { return resolve_threads(n_threads, 1 << 30); }

/* Per-state minimum clearance and collision flag for n SoA states. */
void orc_states(const orc_robot *rb, const orc_env *env, const double *q, int64_t n,
                int64_t ldq, double *cmin, uint8_t *flag, int n_threads) {
    orc_job jb;
    memset(&jb, 0, sizeof jb);
    jb.rb = rb; jb.env = env; jb.q = q; jb.n = n; jb.ldq = ldq;
    jb.out = cmin; jb.flag = flag; jb.job = 0;
    run_parallel(jb, n, n_threads);
}

/* Edge flags (OR over discretized states), classes and minimum clearance; qa/qb AoS [E][dof].
 * n_states may be NULL (then computed from res).  early != 0 stops an edge at its first clearly
 * colliding state (its minimum clearance is then that state's). */
void orc_edges(const orc_robot *rb, const orc_env *env, const double *qa, const double *qb,
               const int32_t *n_states, int64_t n_edges, double res, uint8_t *flag,
               int8_t *cls, double *emin, int early, int n_threads) {
    orc_job jb;
    memset(&jb, 0, sizeof jb);
    jb.rb = rb; jb.env = env; jb.qa = qa; jb.qb = qb; jb.n_states = n_states;
    jb.res = res; jb.flag = flag; jb.cls = cls; jb.out = emin; jb.early = early; jb.job = 3;
    run_parallel(jb, n_edges, n_threads);
}

void orc_costs(const orc_robot *rb, const orc_env *env, const double *q, int64_t n,
               int64_t ldq, double *cost, int n_threads) {
    orc_job jb;
    memset(&jb, 0, sizeof jb);
    jb.rb = rb; jb.env = env; jb.q = q; jb.n = n; jb.ldq = ldq; jb.out = cost; jb.job = 1;
    run_parallel(jb, n, n_threads);
}

void orc_cost_grads(const orc_robot *rb, const orc_env *env, const double *q, int64_t n,
                    int64_t ldq, double *grad, int64_t ldg, int n_threads) {
    orc_job jb;
    memset(&jb, 0, sizeof jb);
    jb.rb = rb; jb.env = env; jb.q = q; jb.n = n; jb.ldq = ldq; jb.grad = grad; jb.ldg = ldg;
    jb.job = 2;
    run_parallel(jb, n, n_threads);
}
