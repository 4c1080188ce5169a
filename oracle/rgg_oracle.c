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
} orc_rm;

typedef struct {
    orc_rm *rm;
    const double *q;
    const int64_t *uv;
    double resolution;
    int spe;
    int64_t e0, e1;
    int pass;          /* 0: count samples, 1: fill geometry             */
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
        for (int64_t s = 0; s <= n; ++s) {
            double t = (double)s / (double)n;
            motion_at(r, &m, t, qt);
            fk(r, qt, c + s * B * D);
        }
        deltas(r, &m, dl);
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
    free(rm);
}

/* Builds the approximations of every edge.  Returns NULL on invalid input
 * (node id out of range, non-positive resolution without a sample count,
 * a sample count below 2) or when memory runs out. */
orc_rm *orc_rm_build(const orc_robot *rob, int64_t n_nodes, const double *q, int64_t n_edges,
                     const int64_t *edge_uv, double resolution, int samples_per_edge,
                     int64_t n_slots, int threads)
{
    if (!rob || n_edges < 0 || n_slots < 0) return NULL;
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
    return rm;
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

/* C and S of one (edge, box) pair, sphere by sphere:
 *   C = some capsule meets the box;
 *   S = for some sphere i, its capsule meets the box and a copy of sphere i
 *       meets it.
 * Every copy of sphere i lies inside capsule i (the inflation delta_i bounds
 * the centre's distance from the chord), so the conjunction never changes S
 * in exact arithmetic; it makes S imply C, and the copies of a sphere whose
 * capsule misses need no test. */
void orc_rm_pair(const orc_rm *rm, int64_t e, const double *box, int32_t *C, int32_t *S)
{
    const orc_robot *r = &rm->rob;
    *C = 0;
    *S = 0;
    if (!box_present(r->D, box)) return;
    for (int i = 0; i < r->B; ++i) {
        if (!capsule_meets(rm, e, i, box)) continue;
        *C = 1;
        if (copies_meet(rm, e, i, box)) {
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
