/*
 * rgg_oracle.c -- plain FP64 CPU oracle for Red-Green-Gray edge labels.
 *
 * TEST INFRASTRUCTURE.  Only the test-suite, the smoke check and the
 * benchmark's CPU-baseline leg load this library.  It shares no code, header
 * or constant table with the device library; both read the same seeded
 * arrays and nothing else.
 *
 * What it computes (paper Sec. 4.1, the Red-Green-Gray rule; Sec. 3.2, the
 * definitions of swept volumes and of outer/inner approximations; Alg. 1,
 * the per-obstacle update):
 *
 *   for every roadmap edge e and the current set O of present box obstacles
 *     C(e,o) = the outer approximation of e meets o
 *     S(e,o) = for some robot sphere, its part of the outer approximation
 *              and its part of the inner approximation both meet o
 *     outer(e) = #{o : C(e,o)},  inner(e) = #{o : S(e,o)}
 *     label(e) = RED if inner(e) > 0, else GREEN if outer(e) == 0, else GRAY
 *   plus the ascending list of GRAY edge ids;
 *   and, for edges a caller names (the unknown ones, Alg. 1 when not lazy),
 *   a full continuous collision check by dyadic refinement of the same two
 *   approximations (orc_rm_validate, below).
 *
 * Primitives (the readings of the paper used throughout this project):
 *   robot             a union of spheres (centre, radius r_i) carried by a
 *                     planar rigid body (SE2), a spatial rigid body (SE3) or
 *                     a planar serial arm (ARM);
 *   cfg(e)            n+1 configurations q(t_j), t_j = j/n, along the edge's
 *                     motion q(t) (Sec. 3.2: |e|/eps configurations);
 *   inner approx.     the robot's spheres placed at every configuration of
 *                     cfg(e): a subset of the swept volume;
 *   outer approx.     per sphere i, the capsule around the chord from its
 *                     centre at t=0 to its centre at t=1 with radius
 *                     r_i + delta_i, where delta_i bounds how far the centre
 *                     strays from the chord (second-derivative bound of
 *                     linear interpolation: |p(t) - chord(t)| <= max|p''|/8);
 *   obstacles         closed axis-aligned boxes, exact (no approximation).
 *
 * Arithmetic: IEEE binary64, round to nearest, compiled without FMA
 * contraction; every sum is taken left to right in the order written here.
 * sin, cos, acos and sqrt come from the C library, except in the full
 * validation, whose sin and cos are a fixed sequence of binary64 steps.  The incremental mode's
 * bounding-box pretest only skips pairs whose predicates are false with a
 * wide margin, so it never changes a result (tests check scratch == incremental).
 */
#include <math.h>
#include <pthread.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define ORC_SE2 0
#define ORC_SE3 1
#define ORC_ARM 2

#define GREEN 0
#define GRAY 1
#define RED 2

#define MAX_SPHERES 256
#define MAX_LINKS 32

typedef struct {
    int kind, B, L, D, dof;
    double pos[MAX_SPHERES * 3];   /* SE2 [B][2], SE3 [B][3], ARM [B] */
    int link[MAX_SPHERES];
    double rad[MAX_SPHERES];
    double len[MAX_LINKS];
    double base[2];
} orc_robot;

/* ------------------------------------------------------------------------ */
/* robot                                                                     */
/* ------------------------------------------------------------------------ */

orc_robot *orc_robot_new(int kind, int n_spheres, int n_links, const double *sphere_pos,
                         const int32_t *sphere_link, const double *sphere_radius,
                         const double *link_length, double base_x, double base_y)
{
    if (n_spheres < 1 || n_spheres > MAX_SPHERES) return NULL;
    if (kind == ORC_ARM && (n_links < 1 || n_links > MAX_LINKS)) return NULL;
    if (kind != ORC_SE2 && kind != ORC_SE3 && kind != ORC_ARM) return NULL;
    orc_robot *r = (orc_robot *)calloc(1, sizeof(orc_robot));
    r->kind = kind;
    r->B = n_spheres;
    r->L = kind == ORC_ARM ? n_links : 0;
    r->D = kind == ORC_SE3 ? 3 : 2;
    r->dof = kind == ORC_SE2 ? 3 : (kind == ORC_SE3 ? 7 : n_links);
    int per = kind == ORC_SE2 ? 2 : (kind == ORC_SE3 ? 3 : 1);
    for (int i = 0; i < n_spheres * per; ++i) r->pos[i] = sphere_pos[i];
    for (int i = 0; i < n_spheres; ++i) {
        r->rad[i] = sphere_radius[i];
        r->link[i] = kind == ORC_ARM ? sphere_link[i] : 0;
        if (kind == ORC_ARM && (r->link[i] < 0 || r->link[i] >= n_links)) { free(r); return NULL; }
    }
    for (int m = 0; m < r->L; ++m) r->len[m] = link_length[m];
    r->base[0] = base_x;
    r->base[1] = base_y;
    return r;
}

void orc_robot_free(orc_robot *r) { free(r); }
int orc_robot_dim(const orc_robot *r) { return r->D; }

/* ------------------------------------------------------------------------ */
/* edge motion q(t), t in [0,1]                                              */
/* ------------------------------------------------------------------------ */

typedef struct {
    double qa[MAX_LINKS + 7], qb[MAX_LINKS + 7];
    double dth;          /* SE2: wrapped heading change                     */
    double h, sh;        /* SE3: half rotation angle and its sine           */
} motion;

static void motion_init(const orc_robot *r, const double *qa, const double *qb, motion *m)
{
    for (int c = 0; c < r->dof; ++c) { m->qa[c] = qa[c]; m->qb[c] = qb[c]; }
    m->dth = 0.0; m->h = 0.0; m->sh = 0.0;
    if (r->kind == ORC_SE2) {
        /* heading moves the short way round: dth in (-pi, pi] */
        double d = qb[2] - qa[2];
        if (d > M_PI) d = d - 2.0 * M_PI;
        else if (d <= -M_PI) d = d + 2.0 * M_PI;
        m->dth = d;
    } else if (r->kind == ORC_SE3) {
        /* spherical linear interpolation along the shorter arc */
        double cq = qa[3] * qb[3] + qa[4] * qb[4] + qa[5] * qb[5] + qa[6] * qb[6];
        if (cq < 0.0) {
            for (int c = 3; c < 7; ++c) m->qb[c] = -qb[c];
            cq = -cq;
        }
        if (cq > 1.0) cq = 1.0;
        m->h = acos(cq);
        m->sh = sin(m->h);
    }
}

static void motion_at(const orc_robot *r, const motion *m, double t, double *q)
{
    if (r->kind == ORC_SE2) {
        q[0] = m->qa[0] + t * (m->qb[0] - m->qa[0]);
        q[1] = m->qa[1] + t * (m->qb[1] - m->qa[1]);
        q[2] = m->qa[2] + t * m->dth;
    } else if (r->kind == ORC_SE3) {
        for (int c = 0; c < 3; ++c) q[c] = m->qa[c] + t * (m->qb[c] - m->qa[c]);
        if (m->sh < 1e-12) {
            for (int c = 3; c < 7; ++c) q[c] = m->qa[c];
        } else {
            double wa = sin((1.0 - t) * m->h) / m->sh;
            double wb = sin(t * m->h) / m->sh;
            for (int c = 3; c < 7; ++c) q[c] = wa * m->qa[c] + wb * m->qb[c];
        }
    } else {
        for (int c = 0; c < r->dof; ++c) q[c] = m->qa[c] + t * (m->qb[c] - m->qa[c]);
    }
}

/* ------------------------------------------------------------------------ */
/* forward kinematics: sphere centres [B][D] at configuration q              */
/* ------------------------------------------------------------------------ */

static void fk(const orc_robot *r, const double *q, double *ctr)
{
    if (r->kind == ORC_SE2) {
        double c = cos(q[2]), s = sin(q[2]);
        for (int i = 0; i < r->B; ++i) {
            double ox = r->pos[2 * i], oy = r->pos[2 * i + 1];
            ctr[2 * i] = q[0] + (c * ox - s * oy);
            ctr[2 * i + 1] = q[1] + (s * ox + c * oy);
        }
    } else if (r->kind == ORC_SE3) {
        /* rotate the offset v by the quaternion (w, u):
         * v' = v + w*t + u x t with t = 2 (u x v) */
        double w = q[3], ux = q[4], uy = q[5], uz = q[6];
        for (int i = 0; i < r->B; ++i) {
            double vx = r->pos[3 * i], vy = r->pos[3 * i + 1], vz = r->pos[3 * i + 2];
            double tx = 2.0 * (uy * vz - uz * vy);
            double ty = 2.0 * (uz * vx - ux * vz);
            double tz = 2.0 * (ux * vy - uy * vx);
            double rx = (vx + w * tx) + (uy * tz - uz * ty);
            double ry = (vy + w * ty) + (uz * tx - ux * tz);
            double rz = (vz + w * tz) + (ux * ty - uy * tx);
            ctr[3 * i] = q[0] + rx;
            ctr[3 * i + 1] = q[1] + ry;
            ctr[3 * i + 2] = q[2] + rz;
        }
    } else {
        /* planar chain: absolute link angle Phi_m = q_0 + ... + q_m, joint
         * J_0 = base, J_{m+1} = J_m + l_m (cos Phi_m, sin Phi_m); a sphere at
         * distance s along link m sits at J_m + s (cos Phi_m, sin Phi_m). */
        double jx[MAX_LINKS + 1], jy[MAX_LINKS + 1], cph[MAX_LINKS], sph[MAX_LINKS];
        double phi = 0.0;
        jx[0] = r->base[0];
        jy[0] = r->base[1];
        for (int m = 0; m < r->L; ++m) {
            phi = m == 0 ? q[0] : phi + q[m];
            cph[m] = cos(phi);
            sph[m] = sin(phi);
            jx[m + 1] = jx[m] + r->len[m] * cph[m];
            jy[m + 1] = jy[m] + r->len[m] * sph[m];
        }
        for (int i = 0; i < r->B; ++i) {
            int m = r->link[i];
            ctr[2 * i] = jx[m] + r->pos[i] * cph[m];
            ctr[2 * i + 1] = jy[m] + r->pos[i] * sph[m];
        }
    }
}

/* number of segments n along the edge: cfg(e) has n+1 configurations */
static int64_t n_segments(const orc_robot *r, const motion *m, double resolution, int spe)
{
    if (spe > 0) return spe - 1;
    double len;
    if (r->kind == ORC_SE2) {
        double dx = m->qb[0] - m->qa[0], dy = m->qb[1] - m->qa[1];
        len = sqrt(dx * dx + dy * dy + m->dth * m->dth);
    } else if (r->kind == ORC_SE3) {
        double acc = 0.0;
        for (int c = 0; c < 3; ++c) { double d = m->qb[c] - m->qa[c]; acc = acc + d * d; }
        double phi = 2.0 * m->h;
        len = sqrt(acc + phi * phi);
    } else {
        double acc = 0.0;
        for (int c = 0; c < r->dof; ++c) { double d = m->qb[c] - m->qa[c]; acc = acc + d * d; }
        len = sqrt(acc);
    }
    double n = ceil(len / resolution);
    return n < 1.0 ? 1 : (int64_t)n;
}

/* delta_i: bound on the distance between sphere i's centre path and the
 * chord joining its end positions; max|p''| / 8 for each kind. */
static void deltas(const orc_robot *r, const motion *m, double *dl)
{
    if (r->kind == ORC_SE2) {
        for (int i = 0; i < r->B; ++i) {
            double ox = r->pos[2 * i], oy = r->pos[2 * i + 1];
            double nrm = sqrt(ox * ox + oy * oy);
            dl[i] = (nrm * m->dth) * m->dth / 8.0;
        }
    } else if (r->kind == ORC_SE3) {
        double phi = 2.0 * m->h;
        for (int i = 0; i < r->B; ++i) {
            double ox = r->pos[3 * i], oy = r->pos[3 * i + 1], oz = r->pos[3 * i + 2];
            double nrm = sqrt(ox * ox + oy * oy + oz * oz);
            dl[i] = (nrm * phi) * phi / 8.0;
        }
    } else {
        for (int i = 0; i < r->B; ++i) {
            int L = r->link[i];
            double acc = 0.0, dphi = 0.0;
            for (int k = 0; k <= L; ++k) {
                dphi = dphi + (m->qb[k] - m->qa[k]);
                /* |p''| <= sum_k |lever_k| dPhi_k^2: the lever's length */
                double arm = fabs(k < L ? r->len[k] : r->pos[i]);
                acc = acc + (arm * dphi) * dphi;
            }
            dl[i] = acc / 8.0;
        }
    }
}

/* ------------------------------------------------------------------------ */
/* second outer form: an oriented box per robot body (Sec. 4.2)              */
/* ------------------------------------------------------------------------ */
/*
 * Sec. 4.2 bounds the swept volume of each robot body along an edge by an
 * oriented box fitted to the point cloud of the body's intermediate
 * placements (an approximation of the smallest such box).  Here a body is
 * the whole robot for the rigid kinds and one link for the arm, and its cloud
 * is the centres of its spheres at every configuration of cfg(e).
 *   axes    the principal axes of the cloud: eigenvectors of its scatter
 *           matrix sum (p - mean)(p - mean)^T, found by cyclic Jacobi
 *           rotations (one rotation in 2-D, eight sweeps in 3-D); their
 *           product is a rotation, orthonormal up to rounding;
 *   extent  along axis u_k, from min(u_k . c - r_i - eta_i) to
 *           max(u_k . c + r_i + eta_i) over the cloud, eta_i = delta_i / n^2.
 * Over one step [t_j, t_j+1] of length 1/n sphere i's centre stays within
 * delta_i / n^2 of the chord between its two sampled positions (the same
 * second-derivative bound as the capsule's, on an interval 1/n long), so
 * the sphere's swept volume over that step lies in the capsule of radius
 * r_i + eta_i around the chord, whose extent along any unit vector lies
 * between the projections of the chord's ends widened by r_i + eta_i.  The
 * box, the intersection of the D slabs, therefore holds the body's whole
 * continuous swept volume.  Stored as centre c, axes u (row k = u_k) and
 * half-extents h.
 */
#define JACOBI_SWEEPS_3D 8

/* eigenvectors of the symmetric D x D matrix a (overwritten) into the
 * columns of v: cyclic Jacobi rotations over the pairs (p, q), p < q */
static void jacobi_eigen(int D, double a[3][3], double v[3][3])
{
    for (int r = 0; r < D; ++r)
        for (int c = 0; c < D; ++c) v[r][c] = r == c ? 1.0 : 0.0;
    int sweeps = D == 3 ? JACOBI_SWEEPS_3D : 1;
    for (int sw = 0; sw < sweeps; ++sw) {
        for (int p = 0; p < D - 1; ++p) {
            for (int q = p + 1; q < D; ++q) {
                double apq = a[p][q];
                if (apq == 0.0) continue;
                /* the rotation angle phi zeroes a[p][q]: t = tan(phi) is the
                 * smaller root of t^2 + 2 theta t - 1 = 0 */
                double theta = (a[q][q] - a[p][p]) / (2.0 * apq);
                double t = 1.0 / (fabs(theta) + sqrt(theta * theta + 1.0));
                if (theta < 0.0) t = -t;
                double c = 1.0 / sqrt(t * t + 1.0);
                double s = t * c;
                for (int r = 0; r < D; ++r) {
                    if (r == p || r == q) continue;
                    double arp = a[r][p], arq = a[r][q];
                    a[r][p] = c * arp - s * arq;
                    a[p][r] = a[r][p];
                    a[r][q] = s * arp + c * arq;
                    a[q][r] = a[r][q];
                }
                a[p][p] = a[p][p] - t * apq;
                a[q][q] = a[q][q] + t * apq;
                a[p][q] = 0.0;
                a[q][p] = 0.0;
                for (int r = 0; r < D; ++r) {
                    double vrp = v[r][p], vrq = v[r][q];
                    v[r][p] = c * vrp - s * vrq;
                    v[r][q] = s * vrp + c * vrq;
                }
            }
        }
    }
}

/* body of sphere i: 0 for the rigid kinds, its link for the arm */
static int body_of(const orc_robot *r, int i) { return r->kind == ORC_ARM ? r->link[i] : 0; }
static int n_bodies(const orc_robot *r) { return r->kind == ORC_ARM ? r->L : 1; }

/* Oriented box of body b for an edge with n+1 configurations of centres
 * ctr [n+1][B][D] and chord bounds dl [B].  Returns 0 (and writes nothing)
 * when the body carries no sphere. */
static int body_obb(const orc_robot *r, int b, const double *ctr, int64_t n, const double *dl, double *c,
                    double *u, double *h)
{
    int B = r->B, D = r->D;
    double mu[3] = {0.0, 0.0, 0.0};
    int64_t cnt = 0;
    for (int64_t j = 0; j <= n; ++j)
        for (int i = 0; i < B; ++i) {
            if (body_of(r, i) != b) continue;
            for (int k = 0; k < D; ++k) mu[k] = mu[k] + ctr[(j * B + i) * D + k];
            ++cnt;
        }
    if (cnt == 0) return 0;
    for (int k = 0; k < D; ++k) mu[k] = mu[k] / (double)cnt;
    double a[3][3] = {{0.0, 0.0, 0.0}, {0.0, 0.0, 0.0}, {0.0, 0.0, 0.0}};
    for (int64_t j = 0; j <= n; ++j)
        for (int i = 0; i < B; ++i) {
            if (body_of(r, i) != b) continue;
            double d[3];
            for (int k = 0; k < D; ++k) d[k] = ctr[(j * B + i) * D + k] - mu[k];
            for (int k = 0; k < D; ++k)
                for (int l = k; l < D; ++l) a[k][l] = a[k][l] + d[k] * d[l];
        }
    for (int k = 0; k < D; ++k)
        for (int l = 0; l < k; ++l) a[k][l] = a[l][k];
    double v[3][3];
    jacobi_eigen(D, a, v);
    for (int k = 0; k < D; ++k)
        for (int d = 0; d < D; ++d) u[k * D + d] = v[d][k];
    double nn = (double)n * (double)n;
    double mid[3];
    for (int k = 0; k < D; ++k) {
        double lo = INFINITY, hi = -INFINITY;
        for (int64_t j = 0; j <= n; ++j)
            for (int i = 0; i < B; ++i) {
                if (body_of(r, i) != b) continue;
                double pr = 0.0;
                for (int d = 0; d < D; ++d) pr = pr + u[k * D + d] * ctr[(j * B + i) * D + d];
                double eta = dl[i] / nn;
                double l = (pr - r->rad[i]) - eta, g = (pr + r->rad[i]) + eta;
                if (l < lo) lo = l;
                if (g > hi) hi = g;
            }
        mid[k] = 0.5 * (lo + hi);
        h[k] = 0.5 * (hi - lo);
    }
    for (int d = 0; d < D; ++d) {
        double acc = 0.0;
        for (int k = 0; k < D; ++k) acc = acc + mid[k] * u[k * D + d];
        c[d] = acc;
    }
    return 1;
}

/* 1 when the oriented box (c, u, h) and the closed box [lo, hi] share a
 * point.  Separating-axis theorem for two boxes: they are disjoint exactly
 * when their projections on one of the candidate axes are -- the box's face
 * normals e_d, the oriented box's axes u_k and, in 3-D, the nine products
 * e_d x u_k.  On an axis L the projections of the centres differ by |T . L|
 * (T = c - box centre) and the boxes reach sum_d bh_d |e_d . L| and
 * sum_k h_k |u_k . L| from them; touching counts as sharing a point. */
static int obb_box_meet(int D, const double *c, const double *u, const double *h, const double *lo,
                        const double *hi)
{
    double bh[3], t[3], au[3][3];
    for (int d = 0; d < D; ++d) {
        bh[d] = 0.5 * (hi[d] - lo[d]);
        t[d] = c[d] - 0.5 * (lo[d] + hi[d]);
    }
    for (int d = 0; d < D; ++d)
        for (int k = 0; k < D; ++k) au[d][k] = fabs(u[k * D + d]);   /* |e_d . u_k| */
    for (int d = 0; d < D; ++d) {
        double rb = 0.0;
        for (int k = 0; k < D; ++k) rb = rb + h[k] * au[d][k];
        if (fabs(t[d]) > bh[d] + rb) return 0;
    }
    for (int k = 0; k < D; ++k) {
        double ra = 0.0, tp = 0.0;
        for (int d = 0; d < D; ++d) {
            ra = ra + bh[d] * au[d][k];
            tp = tp + u[k * D + d] * t[d];
        }
        if (fabs(tp) > h[k] + ra) return 0;
    }
    if (D == 3) {
        /* L = e_d x u_k has components -u_k[d2] at d1 and u_k[d1] at d2
         * (d1, d2 the next two axes after d); u_k1 . L = +-u_k2[d] and
         * u_k2 . L = -+u_k1[d] for an orthonormal frame */
        for (int d = 0; d < 3; ++d) {
            int d1 = (d + 1) % 3, d2 = (d + 2) % 3;
            for (int k = 0; k < 3; ++k) {
                int k1 = (k + 1) % 3, k2 = (k + 2) % 3;
                double ra = bh[d1] * au[d2][k] + bh[d2] * au[d1][k];
                double rb = h[k1] * au[d][k2] + h[k2] * au[d][k1];
                double tp = t[d2] * u[k * 3 + d1] - t[d1] * u[k * 3 + d2];
                if (fabs(tp) > ra + rb) return 0;
            }
        }
    }
    return 1;
}

/* ------------------------------------------------------------------------ */
/* second inner form: shortcut splines (Sec. 4.2)                            */
/* ------------------------------------------------------------------------ */
/*
 * Sec. 4.2 joins the centres of the copies of a sphere along the edge into a
 * polyline, the sphere's spline, and shortens it with the curve
 * simplification of Agarwal et al.: vertices strictly between j and p may be
 * dropped when each lies close enough to the segment from c_j to c_p.  For
 * each sphere i, with err(a, b) = max over a < m < b of dist(c_m, [c_a, c_b])
 * (0 when b = a + 1), the simplification here is their greedy one:
 *   from vertex a (first 0), take b = a+1, a+2, a+4, ... (the last one
 *   clamped to n) while err(a, b) <= tol r_i; between the last accepted and
 *   the first rejected b, bisect for an accepted b whose successor is
 *   rejected; keep the segment (a, b) and continue from b until b = n.
 * A kept segment is the capsule around [c_a, c_b] of radius
 *   rho = r_i - err(a, b) - eta_i,   eta_i = delta_i / n^2,
 * dropped if rho < 0.  The capsule lies in the swept volume: a point x of
 * the segment lies within err(a, b) of the polyline (walking the polyline
 * from c_a to c_b passes a point y whose coordinate along the segment equals
 * x's; y is on a polyline piece whose distance from the segment's line is at
 * most its end vertices', and these are within err(a, b)); y, on the piece
 * between c_m and c_m+1, is within eta_i of the centre at the matching
 * parameter (the chord bound on an interval of length 1/n).  So x is within
 * r_i - rho of a centre of sphere i on the path, and the ball of radius rho
 * around x lies in that sphere.  The paper's splines have no thickness and
 * accept err < r_i; a thickness that the tolerance leaves makes the spline
 * a solid inner approximation of the sphere's sweep.
 */

/* squared distance from p to the segment [a, b] */
static double point_seg_d2(int D, const double *p, const double *a, const double *b)
{
    double d[3], dd = 0.0, wd = 0.0;
    for (int k = 0; k < D; ++k) {
        d[k] = b[k] - a[k];
        dd = dd + d[k] * d[k];
        wd = wd + (p[k] - a[k]) * d[k];
    }
    double t = 0.0;
    if (dd > 0.0) {
        t = wd / dd;
        if (t < 0.0) t = 0.0;
        if (t > 1.0) t = 1.0;
    }
    double acc = 0.0;
    for (int k = 0; k < D; ++k) {
        double g = (a[k] + t * d[k]) - p[k];
        acc = acc + g * g;
    }
    return acc;
}

/* err(a, b)^2 over the vertices pts + m * stride */
static double shortcut_err2(int D, const double *pts, int64_t stride, int64_t a, int64_t b)
{
    double mx = 0.0;
    for (int64_t m = a + 1; m < b; ++m) {
        double v = point_seg_d2(D, pts + m * stride, pts + a * stride, pts + b * stride);
        if (v > mx) mx = v;
    }
    return mx;
}

/* The spline of one sphere: vertices pts + j * stride, j = 0..n.  Writes
 * the kept segments (A[D], B[D], rho) to out (may be NULL) and returns
 * their count (at most n). */
static int64_t sphere_spline(int D, const double *pts, int64_t stride, int64_t n, double rad, double eta,
                             double tol, double *out)
{
    double lim = tol * rad;
    double lim2 = lim * lim;
    int64_t a = 0, K = 0;
    while (a < n) {
        int64_t lo = a + 1, hi = n + 1;   /* (a, lo) accepted; (a, hi) rejected unless hi = n + 1 */
        int64_t step = 2;
        for (;;) {
            int64_t b = a + step < n ? a + step : n;
            if (b <= lo) break;
            if (shortcut_err2(D, pts, stride, a, b) <= lim2) {
                lo = b;
                if (b == n) break;
                step = step * 2;
            } else {
                hi = b;
                break;
            }
        }
        while (hi - lo > 1 && hi <= n) {
            int64_t mid = lo + (hi - lo) / 2;
            if (shortcut_err2(D, pts, stride, a, mid) <= lim2) lo = mid;
            else hi = mid;
        }
        double rho = (rad - sqrt(shortcut_err2(D, pts, stride, a, lo))) - eta;
        if (rho >= 0.0) {
            if (out) {
                double *o = out + K * (2 * D + 1);
                for (int k = 0; k < D; ++k) {
                    o[k] = pts[a * stride + k];
                    o[D + k] = pts[lo * stride + k];
                }
                o[2 * D] = rho;
            }
            ++K;
        }
        a = lo;
    }
    return K;
}

/* ------------------------------------------------------------------------ */
/* distance predicates                                                       */
/* ------------------------------------------------------------------------ */

static double gap1(double x, double lo, double hi)
{
    double a = lo - x;
    double g = a > 0.0 ? a : 0.0;
    double b = x - hi;
    return b > g ? b : g;
}

/* squared distance from point c to the closed box [lo, hi] */
static double point_box_d2(int D, const double *c, const double *lo, const double *hi)
{
    double acc = 0.0;
    for (int k = 0; k < D; ++k) {
        double g = gap1(c[k], lo[k], hi[k]);
        acc = acc + g * g;
    }
    return acc;
}

/* F(t) = squared distance of A + t d to the box */
static double seg_F(int D, const double *A, const double *d, double t, const double *lo,
                    const double *hi)
{
    double acc = 0.0;
    for (int k = 0; k < D; ++k) {
        double p = A[k] + t * d[k];
        double g = gap1(p, lo[k], hi[k]);
        acc = acc + g * g;
    }
    return acc;
}

/* G(t) = F'(t)/2 = sum_k d_k * (excess of p_k outside [lo_k, hi_k], signed) */
static double seg_G(int D, const double *A, const double *d, double t, const double *lo,
                    const double *hi)
{
    double acc = 0.0;
    for (int k = 0; k < D; ++k) {
        double p = A[k] + t * d[k];
        double ex = p < lo[k] ? p - lo[k] : (p > hi[k] ? p - hi[k] : 0.0);
        acc = acc + d[k] * ex;
    }
    return acc;
}

/* Minimum over t in [0,1] of F(t), the squared distance from the segment
 * A->B to the box.  F is convex and piecewise quadratic; its pieces change
 * only where a coordinate crosses a face plane.  G = F'/2 is nondecreasing,
 * so the minimiser lies between the last candidate where G <= 0 and the
 * first where G >= 0 (candidates: 0, 1 and the face crossings inside
 * (0,1)).  Between those two the active faces are fixed and F is a single
 * quadratic whose stationary point is clamped into the bracket. */
static double segbox_fmin(int D, const double *A, const double *Bp, const double *lo,
                          const double *hi)
{
    double d[3];
    for (int k = 0; k < D; ++k) d[k] = Bp[k] - A[k];
    double cand[8];
    int nc = 0;
    cand[nc++] = 0.0;
    cand[nc++] = 1.0;
    for (int k = 0; k < D; ++k) {
        if (d[k] != 0.0) {
            double t1 = (lo[k] - A[k]) / d[k];
            if (t1 > 0.0 && t1 < 1.0) cand[nc++] = t1;
            double t2 = (hi[k] - A[k]) / d[k];
            if (t2 > 0.0 && t2 < 1.0) cand[nc++] = t2;
        }
    }
    double tL = 0.0, tR = 1.0;
    for (int c = 0; c < nc; ++c) {
        double g = seg_G(D, A, d, cand[c], lo, hi);
        if (g <= 0.0 && cand[c] > tL) tL = cand[c];
        if (g >= 0.0 && cand[c] < tR) tR = cand[c];
    }
    double fL = seg_F(D, A, d, tL, lo, hi);
    double fR = seg_F(D, A, d, tR, lo, hi);
    double fmin = fL < fR ? fL : fR;
    if (tL < tR) {
        double tm = 0.5 * (tL + tR);
        double num = 0.0, den = 0.0;
        for (int k = 0; k < D; ++k) {
            double p = A[k] + tm * d[k];
            if (p < lo[k]) {
                num = num + d[k] * (lo[k] - A[k]);
                den = den + d[k] * d[k];
            } else if (p > hi[k]) {
                num = num + d[k] * (hi[k] - A[k]);
                den = den + d[k] * d[k];
            }
        }
        double ts = tL;
        if (den > 0.0) {
            ts = num / den;
            if (ts < tL) ts = tL;
            if (ts > tR) ts = tR;
        }
        double fs = seg_F(D, A, d, ts, lo, hi);
        if (fs < fmin) fmin = fs;
    }
    return fmin;
}

static int box_present(int D, const double *box)
{
    for (int k = 0; k < D; ++k)
        if (box[k] > box[3 + k]) return 0;
    return 1;
}

/* ------------------------------------------------------------------------ */
/* roadmap geometry                                                          */
/* ------------------------------------------------------------------------ */

typedef struct {
    orc_robot rob;
    int64_t E;
    int64_t *soff;     /* [E+1] first sample configuration of each edge    */
    double *ctr;       /* [total configs][B][D] sphere centres            */
    double *capR;      /* [E][B] capsule radius r_i + delta_i             */
    double *aabb;      /* [E][2][3] loose bounding box for the pretest    */
    int32_t *outer, *inner;
    int64_t M;
    double *resident;  /* [M][6] obstacle slots for the incremental mode  */
    double *q;         /* [n_nodes][dof] node configurations (validation) */
    int64_t *uv;       /* [E][2] edge end nodes (validation)              */
    /* the second forms (Sec. 4.2), chosen at build */
    int obb;           /* outer: capsules and per-body oriented boxes     */
    int spl;           /* inner: shortcut splines instead of copies       */
    double tol;        /* spline tolerance, in [0, 1)                     */
    int nb;            /* bodies                                          */
    int bhas[MAX_LINKS];   /* body b carries a sphere                     */
    double *obbv;      /* [E][nb][2D + D*D] centre, axes (rows), half-extents */
    int64_t *sseg;     /* [E*B + 1] first spline segment of (edge, sphere) */
    double *seg;       /* [segments][2D + 1] spline segments (A, B, rho)  */
} orc_rm;

static int obb_len(int D) { return 2 * D + D * D; }

typedef struct {
    orc_rm *rm;
    const double *q;
    const int64_t *uv;
    double resolution;
    int spe;
    int64_t e0, e1;
    int pass;          /* 0: count samples, 1: fill geometry and count spline
                          segments, 2: fill spline segments               */
    int status;
} build_job;

static void *build_worker(void *arg)
{
    build_job *j = (build_job *)arg;
    orc_rm *rm = j->rm;
    const orc_robot *r = &rm->rob;
    int B = r->B, D = r->D;
    double qt[MAX_LINKS + 7];
    double dl[MAX_SPHERES];
    for (int64_t e = j->e0; e < j->e1; ++e) {
        motion m;
        motion_init(r, j->q + j->uv[2 * e] * r->dof, j->q + j->uv[2 * e + 1] * r->dof, &m);
        int64_t n = n_segments(r, &m, j->resolution, j->spe);
        if (j->pass == 0) {
            rm->soff[e + 1] = n + 1;
            continue;
        }
        double *c = rm->ctr + rm->soff[e] * B * D;
        if (j->pass == 2) {
            deltas(r, &m, dl);
            double nn = (double)n * (double)n;
            for (int i = 0; i < B; ++i)
                sphere_spline(D, c + i * D, (int64_t)B * D, n, r->rad[i], dl[i] / nn, rm->tol,
                              rm->seg + rm->sseg[e * B + i] * (2 * D + 1));
            continue;
        }
        for (int64_t s = 0; s <= n; ++s) {
            double t = (double)s / (double)n;
            motion_at(r, &m, t, qt);
            fk(r, qt, c + s * B * D);
        }
        deltas(r, &m, dl);
        if (rm->obb) {
            for (int b = 0; b < rm->nb; ++b) {
                double *o = rm->obbv + (e * rm->nb + b) * obb_len(D);
                if (!body_obb(r, b, c, n, dl, o, o + D, o + D + D * D))
                    for (int k = 0; k < obb_len(D); ++k) o[k] = 0.0;
            }
        }
        if (rm->spl) {
            double nn = (double)n * (double)n;
            for (int i = 0; i < B; ++i)
                rm->sseg[e * B + i + 1] =
                    sphere_spline(D, c + i * D, (int64_t)B * D, n, r->rad[i], dl[i] / nn, rm->tol, NULL);
        }
        double *first = c, *last = c + n * B * D;
        double lo[3] = {INFINITY, INFINITY, INFINITY}, hi[3] = {-INFINITY, -INFINITY, -INFINITY};
        for (int i = 0; i < B; ++i) {
            double R = r->rad[i] + dl[i];
            rm->capR[e * B + i] = R;
            for (int k = 0; k < D; ++k) {
                double a = first[i * D + k], b = last[i * D + k];
                double mn = a < b ? a : b, mx = a < b ? b : a;
                if (mn - R < lo[k]) lo[k] = mn - R;
                if (mx + R > hi[k]) hi[k] = mx + R;
            }
        }
        for (int k = 0; k < 3; ++k) {
            double plo = k < D ? lo[k] - 1e-6 * (1.0 + fabs(lo[k])) : 0.0;
            double phi = k < D ? hi[k] + 1e-6 * (1.0 + fabs(hi[k])) : 0.0;
            rm->aabb[e * 6 + k] = plo;
            rm->aabb[e * 6 + 3 + k] = phi;
        }
    }
    return NULL;
}

static int clamp_threads(int threads, int64_t work)
{
    if (threads < 1) threads = 1;
    if (threads > 256) threads = 256;
    if (work < threads) threads = work < 1 ? 1 : (int)work;
    return threads;
}

static void run_build_pass(orc_rm *rm, const double *q, const int64_t *uv, double res, int spe,
                           int pass, int threads)
{
    threads = clamp_threads(threads, rm->E);
    pthread_t tid[256];
    build_job jobs[256];
    for (int t = 0; t < threads; ++t) {
        jobs[t] = (build_job){rm, q, uv, res, spe, rm->E * t / threads, rm->E * (t + 1) / threads,
                              pass, 0};
        pthread_create(&tid[t], NULL, build_worker, &jobs[t]);
    }
    for (int t = 0; t < threads; ++t) pthread_join(tid[t], NULL);
}

void orc_rm_free(orc_rm *rm)
{
    if (!rm) return;
    free(rm->soff);
    free(rm->ctr);
    free(rm->capR);
    free(rm->aabb);
    free(rm->outer);
    free(rm->inner);
    free(rm->resident);
    free(rm->q);
    free(rm->uv);
    free(rm->obbv);
    free(rm->sseg);
    free(rm->seg);
    free(rm);
}

/* Builds the approximations of every edge.  Returns NULL on invalid input
 * (node id out of range, non-positive resolution without a sample count,
 * a sample count below 2) or when memory runs out. */
orc_rm *orc_rm_build_ex(const orc_robot *rob, int64_t n_nodes, const double *q, int64_t n_edges,
                        const int64_t *edge_uv, double resolution, int samples_per_edge, int64_t n_slots,
                        int threads, int outer_obb, int inner_splines, double spline_tol)
{
    if (!rob || n_edges < 0 || n_slots < 0) return NULL;
    if (inner_splines && !(spline_tol >= 0.0 && spline_tol < 1.0)) return NULL;
    if (samples_per_edge == 1 || samples_per_edge < 0) return NULL;
    if (samples_per_edge == 0 && !(resolution > 0.0)) return NULL;
    for (int64_t e = 0; e < 2 * n_edges; ++e)
        if (edge_uv[e] < 0 || edge_uv[e] >= n_nodes) return NULL;
    orc_rm *rm = (orc_rm *)calloc(1, sizeof(orc_rm));
    rm->rob = *rob;
    rm->E = n_edges;
    int B = rob->B, D = rob->D;
    rm->soff = (int64_t *)calloc((size_t)n_edges + 1, sizeof(int64_t));
    rm->capR = (double *)malloc(sizeof(double) * (size_t)(n_edges * B + 1));
    rm->aabb = (double *)malloc(sizeof(double) * (size_t)(n_edges * 6 + 1));
    rm->outer = (int32_t *)calloc((size_t)n_edges + 1, sizeof(int32_t));
    rm->inner = (int32_t *)calloc((size_t)n_edges + 1, sizeof(int32_t));
    rm->M = n_slots;
    rm->obb = outer_obb != 0;
    rm->spl = inner_splines != 0;
    rm->tol = spline_tol;
    rm->nb = n_bodies(rob);
    for (int b = 0; b < rm->nb; ++b) rm->bhas[b] = 0;
    for (int i = 0; i < B; ++i) rm->bhas[body_of(rob, i)] = 1;
    if (rm->obb) {
        rm->obbv = (double *)malloc(sizeof(double) * (size_t)(n_edges * rm->nb * obb_len(D) + 1));
        if (!rm->obbv) {
            orc_rm_free(rm);
            return NULL;
        }
    }
    if (rm->spl) {
        rm->sseg = (int64_t *)calloc((size_t)(n_edges * B + 1), sizeof(int64_t));
        if (!rm->sseg) {
            orc_rm_free(rm);
            return NULL;
        }
    }
    rm->resident = (double *)malloc(sizeof(double) * (size_t)(n_slots * 6 + 1));
    rm->q = (double *)malloc(sizeof(double) * (size_t)(n_nodes * rob->dof + 1));
    rm->uv = (int64_t *)malloc(sizeof(int64_t) * (size_t)(n_edges * 2 + 1));
    if (!rm->soff || !rm->capR || !rm->aabb || !rm->outer || !rm->inner || !rm->resident || !rm->q ||
        !rm->uv) {
        orc_rm_free(rm);
        return NULL;
    }
    if (n_nodes > 0) memcpy(rm->q, q, sizeof(double) * (size_t)(n_nodes * rob->dof));
    if (n_edges > 0) memcpy(rm->uv, edge_uv, sizeof(int64_t) * (size_t)(n_edges * 2));
    for (int64_t s = 0; s < n_slots; ++s) {
        for (int k = 0; k < 3; ++k) {
            rm->resident[s * 6 + k] = 1.0;
            rm->resident[s * 6 + 3 + k] = -1.0;
        }
    }
    run_build_pass(rm, q, edge_uv, resolution, samples_per_edge, 0, threads);
    rm->soff[0] = 0;
    for (int64_t e = 0; e < n_edges; ++e) rm->soff[e + 1] += rm->soff[e];
    rm->ctr = (double *)malloc(sizeof(double) * (size_t)(rm->soff[n_edges] * B * D + 1));
    if (!rm->ctr) {
        orc_rm_free(rm);
        return NULL;
    }
    run_build_pass(rm, q, edge_uv, resolution, samples_per_edge, 1, threads);
    if (rm->spl) {
        for (int64_t k = 0; k < n_edges * B; ++k) rm->sseg[k + 1] += rm->sseg[k];
        rm->seg = (double *)malloc(sizeof(double) * (size_t)(rm->sseg[n_edges * B] * (2 * D + 1) + 1));
        if (!rm->seg) {
            orc_rm_free(rm);
            return NULL;
        }
        run_build_pass(rm, q, edge_uv, resolution, samples_per_edge, 2, threads);
    }
    return rm;
}

/* the capsule and sample-copy forms of Sec. 4.2's approximations */
orc_rm *orc_rm_build(const orc_robot *rob, int64_t n_nodes, const double *q, int64_t n_edges,
                     const int64_t *edge_uv, double resolution, int samples_per_edge,
                     int64_t n_slots, int threads)
{
    return orc_rm_build_ex(rob, n_nodes, q, n_edges, edge_uv, resolution, samples_per_edge, n_slots,
                           threads, 0, 0, 0.0);
}

/* ------------------------------------------------------------------------ */
/* pair predicates                                                           */
/* ------------------------------------------------------------------------ */

/* capsule of sphere i meets the box */
static int capsule_meets(const orc_rm *rm, int64_t e, int i, const double *box)
{
    const orc_robot *r = &rm->rob;
    int B = r->B, D = r->D;
    int64_t n = rm->soff[e + 1] - rm->soff[e] - 1;
    const double *first = rm->ctr + rm->soff[e] * B * D;
    const double *last = first + n * B * D;
    double R = rm->capR[e * B + i];
    return segbox_fmin(D, first + i * D, last + i * D, box, box + 3) <= R * R;
}

/* some copy of sphere i along the edge meets the box */
static int copies_meet(const orc_rm *rm, int64_t e, int i, const double *box)
{
    const orc_robot *r = &rm->rob;
    int B = r->B, D = r->D;
    const double *c = rm->ctr + rm->soff[e] * B * D;
    int64_t cnt = rm->soff[e + 1] - rm->soff[e];
    double rr = r->rad[i];
    for (int64_t s = 0; s < cnt; ++s)
        if (point_box_d2(D, c + (s * B + i) * D, box, box + 3) <= rr * rr) return 1;
    return 0;
}

/* some kept spline segment of sphere i meets the box */
static int splines_meet(const orc_rm *rm, int64_t e, int i, const double *box)
{
    int B = rm->rob.B, D = rm->rob.D;
    for (int64_t k = rm->sseg[e * B + i]; k < rm->sseg[e * B + i + 1]; ++k) {
        const double *g = rm->seg + k * (2 * D + 1);
        if (segbox_fmin(D, g, g + D, box, box + 3) <= g[2 * D] * g[2 * D]) return 1;
    }
    return 0;
}

/* the oriented box of body b of edge e meets the box */
static int body_obb_meets(const orc_rm *rm, int64_t e, int b, const double *box)
{
    int D = rm->rob.D;
    if (!rm->bhas[b]) return 0;
    const double *o = rm->obbv + (e * rm->nb + b) * obb_len(D);
    return obb_box_meet(D, o, o + D, o + D + D * D, box, box + 3);
}

/* C and S of one (edge, box) pair, sphere by sphere:
 *   C = for some sphere i, its capsule meets the box (and, with the oriented
 *       boxes, so does the box of sphere i's body);
 *   S = for some sphere i, what C asks of sphere i holds and a copy of
 *       sphere i (a spline segment of sphere i, with the splines) meets it.
 * Every copy of sphere i, and every spline segment, lies inside capsule i
 * (the inflation delta_i bounds the centre's distance from the chord) and
 * inside the box of its body, so the conjunction never changes S in exact
 * arithmetic; it makes S imply C, and the inner parts of a sphere whose
 * outer parts miss need no test.  With the oriented boxes the outer
 * approximation is the union over spheres of capsule_i intersected with the
 * box of sphere i's body: still a superset of the swept volume. */
void orc_rm_pair(const orc_rm *rm, int64_t e, const double *box, int32_t *C, int32_t *S)
{
    const orc_robot *r = &rm->rob;
    *C = 0;
    *S = 0;
    if (!box_present(r->D, box)) return;
    for (int i = 0; i < r->B; ++i) {
        if (!capsule_meets(rm, e, i, box)) continue;
        if (rm->obb && !body_obb_meets(rm, e, body_of(r, i), box)) continue;
        *C = 1;
        if (rm->spl ? splines_meet(rm, e, i, box) : copies_meet(rm, e, i, box)) {
            *S = 1;
            return;
        }
    }
}

static int loose_overlap(const orc_rm *rm, int64_t e, const double *box)
{
    int D = rm->rob.D;
    const double *a = rm->aabb + e * 6;
    for (int k = 0; k < D; ++k)
        if (box[k] > a[3 + k] || box[3 + k] < a[k]) return 0;
    return 1;
}

/* ------------------------------------------------------------------------ */
/* classification                                                            */
/* ------------------------------------------------------------------------ */

typedef struct {
    orc_rm *rm;
    int64_t M;
    const double *boxes;   /* scratch: all slots; incremental: old        */
    const double *nboxes;  /* incremental: new                            */
    const int64_t *chg;    /* incremental: changed slot ids               */
    int64_t nchg;
    int64_t e0, e1;
    int mode;              /* 0 scratch, 1 incremental                    */
} cls_job;

static void *cls_worker(void *arg)
{
    cls_job *j = (cls_job *)arg;
    orc_rm *rm = j->rm;
    int D = rm->rob.D;
    for (int64_t e = j->e0; e < j->e1; ++e) {
        if (j->mode == 0) {
            int32_t outer = 0, inner = 0;
            for (int64_t s = 0; s < j->M; ++s) {
                const double *b = j->boxes + 6 * s;
                if (!box_present(D, b)) continue;
                int32_t C, S;
                orc_rm_pair(rm, e, b, &C, &S);
                outer += C;
                inner += S;
            }
            rm->outer[e] = outer;
            rm->inner[e] = inner;
        } else {
            for (int64_t c = 0; c < j->nchg; ++c) {
                int64_t s = j->chg[c];
                const double *ob = j->boxes + 6 * s, *nb = j->nboxes + 6 * s;
                int32_t C, S;
                if (box_present(D, ob) && loose_overlap(rm, e, ob)) {
                    orc_rm_pair(rm, e, ob, &C, &S);
                    rm->outer[e] -= C;
                    rm->inner[e] -= S;
                }
                if (box_present(D, nb) && loose_overlap(rm, e, nb)) {
                    orc_rm_pair(rm, e, nb, &C, &S);
                    rm->outer[e] += C;
                    rm->inner[e] += S;
                }
            }
        }
    }
    return NULL;
}

static void run_cls(cls_job base, int threads)
{
    threads = clamp_threads(threads, base.rm->E);
    pthread_t tid[256];
    cls_job jobs[256];
    for (int t = 0; t < threads; ++t) {
        jobs[t] = base;
        jobs[t].e0 = base.rm->E * t / threads;
        jobs[t].e1 = base.rm->E * (t + 1) / threads;
        pthread_create(&tid[t], NULL, cls_worker, &jobs[t]);
    }
    for (int t = 0; t < threads; ++t) pthread_join(tid[t], NULL);
}

/* labels from the counters; the gray list holds every GRAY id ascending.
 * Writes min(n_gray, gray_cap) ids and returns n_gray. */
static int64_t emit(const orc_rm *rm, uint8_t *labels, int64_t *gray, int64_t gray_cap)
{
    int64_t ng = 0;
    for (int64_t e = 0; e < rm->E; ++e) {
        uint8_t lab = rm->inner[e] > 0 ? RED : (rm->outer[e] == 0 ? GREEN : GRAY);
        if (labels) labels[e] = lab;
        if (lab == GRAY) {
            if (gray && ng < gray_cap) gray[ng] = e;
            ++ng;
        }
    }
    return ng;
}

static int boxes_finite(int64_t M, const double *b)
{
    for (int64_t i = 0; i < 6 * M; ++i)
        if (!isfinite(b[i])) return 0;
    return 1;
}

/* From scratch: every edge against every present box.  Replaces the
 * counters and the resident slots.  Returns n_gray, or -1 on bad input. */
int64_t orc_rm_classify(orc_rm *rm, int64_t M, const double *boxes, uint8_t *labels, int64_t *gray,
                        int64_t gray_cap, int threads)
{
    if (M != rm->M || !boxes_finite(M, boxes)) return -1;
    cls_job j = {rm, M, boxes, NULL, NULL, 0, 0, 0, 0};
    run_cls(j, threads);
    memcpy(rm->resident, boxes, sizeof(double) * 6 * (size_t)M);
    return emit(rm, labels, gray, gray_cap);
}

/* Incremental (Alg. 1 applied to every slot whose box changed): for each
 * changed slot the old box's C and S are removed from the counters and the
 * new box's added.  `old_boxes` must equal the resident slots bit for bit.
 * Returns n_gray, -1 on bad input, -3 when `old_boxes` differs from the
 * resident slots. */
int64_t orc_rm_update(orc_rm *rm, int64_t M, const double *old_boxes, const double *new_boxes,
                      uint8_t *labels, int64_t *gray, int64_t gray_cap, int threads)
{
    if (M != rm->M || !boxes_finite(M, old_boxes) || !boxes_finite(M, new_boxes)) return -1;
    if (memcmp(old_boxes, rm->resident, sizeof(double) * 6 * (size_t)M) != 0) return -3;
    int64_t *chg = (int64_t *)malloc(sizeof(int64_t) * (size_t)(M + 1));
    int64_t nchg = 0;
    for (int64_t s = 0; s < M; ++s)
        if (memcmp(old_boxes + 6 * s, new_boxes + 6 * s, sizeof(double) * 6) != 0) chg[nchg++] = s;
    cls_job j = {rm, M, old_boxes, new_boxes, chg, nchg, 0, 0, 1};
    run_cls(j, threads);
    free(chg);
    memcpy(rm->resident, new_boxes, sizeof(double) * 6 * (size_t)M);
    return emit(rm, labels, gray, gray_cap);
}

/* ------------------------------------------------------------------------ */
/* full validation of an edge (Alg. 1, the branch taken when not lazy)       */
/* ------------------------------------------------------------------------ */
/*
 * Alg. 1 gives every edge left unknown a full collision check.  Here that
 * check is continuous: it decides whether any configuration q(t), t in
 * [0,1], of the edge's motion puts a robot sphere into a present box.  It
 * refines the outer and inner approximations of Sec. 3.2 on dyadic
 * sub-intervals [j 2^-l, (j+1) 2^-l] of the edge:
 *   free(l, j): for every sphere i and every present box, the capsule from
 *               sphere i's centre at the interval's start to its centre at
 *               the interval's end, radius r_i + delta_i 4^-l, misses the
 *               box.  delta_i bounds max|p''|/8 over the whole edge, so
 *               delta_i 4^-l bounds the chord deviation over an interval
 *               of length 2^-l and the capsule holds sphere i's swept volume
 *               over that interval;
 *   hit(t):     some sphere at configuration q(t) meets a present box.
 * The search is level by level:
 *   hit(0) or hit(1)                  -> COLLIDES, witness 0 or 1
 *   free(0, 0)                        -> FREE at level 0
 *   A_0 = {0}; for l = 0, 1, ..., max_level - 1:
 *     |A_l| > max_active              -> UNRESOLVED at level l
 *     some j in A_l with hit((2j+1) 2^-(l+1))
 *                                     -> COLLIDES at level l+1, witness the
 *                                        smallest such midpoint
 *     A_{l+1} = {c in {2j, 2j+1}, j in A_l : not free(l+1, c)}
 *     A_{l+1} empty                   -> FREE at level l+1
 *   otherwise                         -> UNRESOLVED at level max_level.
 * COLLIDES is exact (a witness configuration).  FREE certifies the whole
 * motion up to the rounding of its binary64 evaluation.  UNRESOLVED edges
 * graze a box within the resolution the limits allow; a caller treats them
 * as invalid.
 *
 * The configurations are evaluated like the build's, except that sin and
 * cos come from vsincos below: a fixed sequence of binary64 +, -, * and
 * rint, which any IEEE evaluator (this oracle, a GPU) reproduces bit for
 * bit.  The build's samples keep the C library's sin and cos.
 */

#define V_FREE 0
#define V_COLLIDES 2
#define V_UNRESOLVED 3

/* sin and cos by Cody and Waite's reduction x = k (pi/2) + r, pi/2 split
 * into a 24-bit head (exact products with k) and its binary64 remainder,
 * then the Taylor series of sin r to r^19 and of cos r to r^20 in Horner
 * form (|r| <= pi/4 up to rounding; the first omitted terms are below
 * 1e-19).  The quadrant k mod 4 maps (sin r, cos r) to (sin x, cos x). */
static void vsincos(double x, double *sn, double *cs)
{
    const double pi = 3.14159265358979323846;
    const double half_pi = pi / 2.0;
    const double head = (double)(float)half_pi;
    const double tail = half_pi - head;
    double k = rint(x * (2.0 / pi));
    double r = (x - k * head) - k * tail;
    double z = r * r;
    double ps = -1.0 / 121645100408832000.0;     /* -1/19! */
    ps = ps * z + 1.0 / 355687428096000.0;       /* 1/17!  */
    ps = ps * z - 1.0 / 1307674368000.0;         /* -1/15! */
    ps = ps * z + 1.0 / 6227020800.0;            /* 1/13!  */
    ps = ps * z - 1.0 / 39916800.0;              /* -1/11! */
    ps = ps * z + 1.0 / 362880.0;                /* 1/9!   */
    ps = ps * z - 1.0 / 5040.0;                  /* -1/7!  */
    ps = ps * z + 1.0 / 120.0;                   /* 1/5!   */
    ps = ps * z - 1.0 / 6.0;                     /* -1/3!  */
    double s = r + (r * z) * ps;
    double pc = 1.0 / 2432902008176640000.0;     /* 1/20!  */
    pc = pc * z - 1.0 / 6402373705728000.0;      /* -1/18! */
    pc = pc * z + 1.0 / 20922789888000.0;        /* 1/16!  */
    pc = pc * z - 1.0 / 87178291200.0;           /* -1/14! */
    pc = pc * z + 1.0 / 479001600.0;             /* 1/12!  */
    pc = pc * z - 1.0 / 3628800.0;               /* -1/10! */
    pc = pc * z + 1.0 / 40320.0;                 /* 1/8!   */
    pc = pc * z - 1.0 / 720.0;                   /* -1/6!  */
    pc = pc * z + 1.0 / 24.0;                    /* 1/4!   */
    pc = pc * z - 1.0 / 2.0;                     /* -1/2!  */
    double c = 1.0 + z * pc;
    int64_t quadrant = (int64_t)k & 3;
    if (quadrant == 0) { *sn = s; *cs = c; }
    else if (quadrant == 1) { *sn = c; *cs = -s; }
    else if (quadrant == 2) { *sn = -s; *cs = -c; }
    else { *sn = -c; *cs = s; }
}

/* q(t) as motion_at, with vsincos for the slerp weights */
static void motion_at_v(const orc_robot *r, const motion *m, double t, double *q)
{
    if (r->kind == ORC_SE3 && !(m->sh < 1e-12)) {
        for (int c = 0; c < 3; ++c) q[c] = m->qa[c] + t * (m->qb[c] - m->qa[c]);
        double sa, ca, sb, cb;
        vsincos((1.0 - t) * m->h, &sa, &ca);
        vsincos(t * m->h, &sb, &cb);
        double wa = sa / m->sh;
        double wb = sb / m->sh;
        for (int c = 3; c < 7; ++c) q[c] = wa * m->qa[c] + wb * m->qb[c];
        return;
    }
    motion_at(r, m, t, q);   /* no trigonometry on the other paths */
}

/* sphere centres at q, as fk, with vsincos */
static void fk_v(const orc_robot *r, const double *q, double *ctr)
{
    if (r->kind == ORC_SE2) {
        double s, c;
        vsincos(q[2], &s, &c);
        for (int i = 0; i < r->B; ++i) {
            double ox = r->pos[2 * i], oy = r->pos[2 * i + 1];
            ctr[2 * i] = q[0] + (c * ox - s * oy);
            ctr[2 * i + 1] = q[1] + (s * ox + c * oy);
        }
    } else if (r->kind == ORC_SE3) {
        fk(r, q, ctr);           /* quaternion rotation: no trigonometry */
    } else {
        double jx[MAX_LINKS + 1], jy[MAX_LINKS + 1], cph[MAX_LINKS], sph[MAX_LINKS];
        double phi = 0.0;
        jx[0] = r->base[0];
        jy[0] = r->base[1];
        for (int m = 0; m < r->L; ++m) {
            phi = m == 0 ? q[0] : phi + q[m];
            vsincos(phi, &sph[m], &cph[m]);
            jx[m + 1] = jx[m] + r->len[m] * cph[m];
            jy[m + 1] = jy[m] + r->len[m] * sph[m];
        }
        for (int i = 0; i < r->B; ++i) {
            int m = r->link[i];
            ctr[2 * i] = jx[m] + r->pos[i] * cph[m];
            ctr[2 * i + 1] = jy[m] + r->pos[i] * sph[m];
        }
    }
}

typedef struct {
    const orc_rm *rm;
    motion m;
    double dl[MAX_SPHERES];
} vedge;

static void centres_v(const vedge *v, double t, double *ctr)
{
    double q[MAX_LINKS + 7];
    motion_at_v(&v->rm->rob, &v->m, t, q);
    fk_v(&v->rm->rob, q, ctr);
}

/* hit(t): some sphere at q(t) meets a present box */
static int hit_v(const vedge *v, double t)
{
    const orc_robot *r = &v->rm->rob;
    double ctr[MAX_SPHERES * 3];
    centres_v(v, t, ctr);
    for (int64_t s = 0; s < v->rm->M; ++s) {
        const double *b = v->rm->resident + 6 * s;
        if (!box_present(r->D, b)) continue;
        for (int i = 0; i < r->B; ++i)
            if (point_box_d2(r->D, ctr + i * r->D, b, b + 3) <= r->rad[i] * r->rad[i]) return 1;
    }
    return 0;
}

/* free(l, j) */
static int free_v(const vedge *v, int l, int64_t j)
{
    const orc_robot *r = &v->rm->rob;
    double w = ldexp(1.0, -l);
    double ca[MAX_SPHERES * 3], cb[MAX_SPHERES * 3];
    centres_v(v, ldexp((double)j, -l), ca);
    centres_v(v, ldexp((double)(j + 1), -l), cb);
    for (int64_t s = 0; s < v->rm->M; ++s) {
        const double *b = v->rm->resident + 6 * s;
        if (!box_present(r->D, b)) continue;
        for (int i = 0; i < r->B; ++i) {
            double R = r->rad[i] + v->dl[i] * (w * w);
            if (segbox_fmin(r->D, ca + i * r->D, cb + i * r->D, b, b + 3) <= R * R) return 0;
        }
    }
    return 1;
}

static int validate_edge(const orc_rm *rm, int64_t e, int max_level, int max_active, int32_t *level,
                         double *witness, int64_t *act, int64_t *nxt)
{
    vedge v;
    v.rm = rm;
    const orc_robot *r = &rm->rob;
    motion_init(r, rm->q + rm->uv[2 * e] * r->dof, rm->q + rm->uv[2 * e + 1] * r->dof, &v.m);
    deltas(r, &v.m, v.dl);
    *witness = NAN;
    *level = 0;
    if (hit_v(&v, 0.0)) { *witness = 0.0; return V_COLLIDES; }
    if (hit_v(&v, 1.0)) { *witness = 1.0; return V_COLLIDES; }
    if (free_v(&v, 0, 0)) return V_FREE;
    int64_t na = 1;
    act[0] = 0;
    for (int l = 0; l < max_level; ++l) {
        *level = l;
        if (na > max_active) return V_UNRESOLVED;
        for (int64_t a = 0; a < na; ++a) {
            double t = ldexp((double)(2 * act[a] + 1), -(l + 1));
            if (hit_v(&v, t)) {
                *level = l + 1;
                *witness = t;
                return V_COLLIDES;
            }
        }
        int64_t nn = 0;
        for (int64_t a = 0; a < na; ++a)
            for (int64_t c = 2 * act[a]; c <= 2 * act[a] + 1; ++c)
                if (!free_v(&v, l + 1, c)) nxt[nn++] = c;
        *level = l + 1;
        if (nn == 0) return V_FREE;
        for (int64_t a = 0; a < nn; ++a) act[a] = nxt[a];
        na = nn;
    }
    *level = max_level;
    return V_UNRESOLVED;
}

typedef struct {
    const orc_rm *rm;
    const int64_t *ids;
    int64_t i0, i1;
    int max_level, max_active;
    uint8_t *verdict;
    int32_t *level;
    double *witness;
} val_job;

static void *val_worker(void *arg)
{
    val_job *j = (val_job *)arg;
    int64_t *act = (int64_t *)malloc(sizeof(int64_t) * (size_t)(2 * j->max_active + 2));
    int64_t *nxt = (int64_t *)malloc(sizeof(int64_t) * (size_t)(2 * j->max_active + 2));
    for (int64_t i = j->i0; i < j->i1; ++i)
        j->verdict[i] = (uint8_t)validate_edge(j->rm, j->ids[i], j->max_level, j->max_active, &j->level[i],
                                               &j->witness[i], act, nxt);
    free(act);
    free(nxt);
    return NULL;
}

/* Full validation of edges ids[0..n) against the resident obstacle slots.
 * verdict[i] is 0 (FREE), 2 (COLLIDES) or 3 (UNRESOLVED); level[i] the
 * level where the search stopped; witness[i] the colliding parameter t
 * (NaN unless COLLIDES).  Returns 0, or -1 on bad input. */
int orc_rm_validate(const orc_rm *rm, const int64_t *ids, int64_t n, int max_level, int max_active,
                    uint8_t *verdict, int32_t *level, double *witness, int threads)
{
    if (n < 0 || max_level < 0 || max_level > 30 || max_active < 1 || max_active > 1024) return -1;
    for (int64_t i = 0; i < n; ++i)
        if (ids[i] < 0 || ids[i] >= rm->E) return -1;
    if (n == 0) return 0;
    if (threads < 1) threads = 1;
    if (threads > 256) threads = 256;
    if (n < threads) threads = (int)n;
    pthread_t tid[256];
    val_job jobs[256];
    for (int t = 0; t < threads; ++t) {
        jobs[t] = (val_job){rm, ids, n * t / threads, n * (t + 1) / threads, max_level, max_active,
                            verdict, level, witness};
        pthread_create(&tid[t], NULL, val_worker, &jobs[t]);
    }
    for (int t = 0; t < threads; ++t) pthread_join(tid[t], NULL);
    return 0;
}

void orc_vsincos(double x, double *s, double *c) { vsincos(x, s, c); }

/* centres at parameter t of the motion qa -> qb, as the validation evaluates them */
void orc_centres_v(const orc_robot *r, const double *qa, const double *qb, double t, double *ctr)
{
    motion m;
    motion_init(r, qa, qb, &m);
    double q[MAX_LINKS + 7];
    motion_at_v(r, &m, t, q);
    fk_v(r, q, ctr);
}

/* ------------------------------------------------------------------------ */
/* accessors used by the pin tests                                           */
/* ------------------------------------------------------------------------ */

int64_t orc_rm_n_edges(const orc_rm *rm) { return rm->E; }
int64_t orc_rm_n_configs(const orc_rm *rm, int64_t e) { return rm->soff[e + 1] - rm->soff[e]; }

/* sphere centres of edge e, [n_configs][B][D] */
void orc_rm_centres(const orc_rm *rm, int64_t e, double *out)
{
    int64_t cnt = (rm->soff[e + 1] - rm->soff[e]) * rm->rob.B * rm->rob.D;
    memcpy(out, rm->ctr + rm->soff[e] * rm->rob.B * rm->rob.D, sizeof(double) * (size_t)cnt);
}

void orc_rm_capsule_radius(const orc_rm *rm, int64_t e, double *out)
{
    memcpy(out, rm->capR + e * rm->rob.B, sizeof(double) * (size_t)rm->rob.B);
}

/* oriented box of body b of edge e: centre [D], axes [D][D], half-extents
 * [D]; returns 0 without writing when the roadmap has no boxes or the body
 * carries no sphere */
int orc_rm_obb(const orc_rm *rm, int64_t e, int b, double *c, double *u, double *h)
{
    int D = rm->rob.D;
    if (!rm->obb || b < 0 || b >= rm->nb || !rm->bhas[b]) return 0;
    const double *o = rm->obbv + (e * rm->nb + b) * obb_len(D);
    memcpy(c, o, sizeof(double) * D);
    memcpy(u, o + D, sizeof(double) * D * D);
    memcpy(h, o + D + D * D, sizeof(double) * D);
    return 1;
}

/* spline segments of sphere i of edge e, [K][2D + 1] (A, B, rho) into out
 * (may be NULL); returns K, or -1 when the roadmap has no splines */
int64_t orc_rm_spline(const orc_rm *rm, int64_t e, int i, double *out)
{
    int B = rm->rob.B, D = rm->rob.D;
    if (!rm->spl) return -1;
    int64_t k0 = rm->sseg[e * B + i], k1 = rm->sseg[e * B + i + 1];
    if (out) memcpy(out, rm->seg + k0 * (2 * D + 1), sizeof(double) * (size_t)((k1 - k0) * (2 * D + 1)));
    return k1 - k0;
}

/* the building blocks, for the tests */
void orc_jacobi_eigen(int D, const double *a, double *v)
{
    double A[3][3], V[3][3];
    for (int r = 0; r < D; ++r)
        for (int c = 0; c < D; ++c) A[r][c] = a[r * D + c];
    jacobi_eigen(D, A, V);
    for (int r = 0; r < D; ++r)
        for (int c = 0; c < D; ++c) v[r * D + c] = V[r][c];
}

int orc_obb_box_meet(int D, const double *c, const double *u, const double *h, const double *box)
{
    return obb_box_meet(D, c, u, h, box, box + 3);
}

int64_t orc_sphere_spline(int D, const double *pts, int64_t n, double rad, double eta, double tol, double *out)
{
    return sphere_spline(D, pts, D, n, rad, eta, tol, out);
}

void orc_rm_counters(const orc_rm *rm, int32_t *outer, int32_t *inner)
{
    memcpy(outer, rm->outer, sizeof(int32_t) * (size_t)rm->E);
    memcpy(inner, rm->inner, sizeof(int32_t) * (size_t)rm->E);
}

void orc_interp(const orc_robot *r, const double *qa, const double *qb, double t, double *q)
{
    motion m;
    motion_init(r, qa, qb, &m);
    motion_at(r, &m, t, q);
}

void orc_fk(const orc_robot *r, const double *q, double *ctr) { fk(r, q, ctr); }

void orc_deltas(const orc_robot *r, const double *qa, const double *qb, double *dl)
{
    motion m;
    motion_init(r, qa, qb, &m);
    deltas(r, &m, dl);
}

int64_t orc_n_segments(const orc_robot *r, const double *qa, const double *qb, double resolution,
                       int spe)
{
    motion m;
    motion_init(r, qa, qb, &m);
    return n_segments(r, &m, resolution, spe);
}

double orc_point_box_d2(int D, const double *c, const double *box)
{
    return point_box_d2(D, c, box, box + 3);
}

double orc_segbox_fmin(int D, const double *A, const double *Bp, const double *box)
{
    return segbox_fmin(D, A, Bp, box, box + 3);
}
