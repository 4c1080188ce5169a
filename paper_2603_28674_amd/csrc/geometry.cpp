// Host build stage of librgg: approximations of every roadmap edge.
//
// Paper Sec. 3.2 defines cfg(e) (|e|/eps configurations along an edge), the
// forward kinematics FK and outer/inner approximations (superset/subset of the
// swept volume).  This file computes, in binary64 with the C library's sin,
// cos, acos and sqrt and without FMA contraction (compile flags), for each
// edge:
//   - the sphere centres at every configuration of cfg(e) (inner
//     approximation: the robot itself at those configurations);
//   - for every sphere, a capsule around the chord of its centre path with
//     radius r_i + delta_i (outer approximation), where delta_i = max|p''|/8
//     bounds the distance between a C^2 path and the chord of its ends;
//   - a padded, outward-rounded binary32 box around all capsules, used by the
//     grid and by the pair pretest.
// The expression order is part of the definition of the labels: every
// binary64 quantity here is written in one fixed order, so the device's
// binary64 re-tests see the same numbers as any other evaluator of the same
// definition.
#include <math.h>
#include <string.h>

#include <algorithm>
#include <new>
#include <thread>

#include "rgg_internal.h"

namespace rgg {

namespace {

constexpr double kPi = 3.14159265358979323846;

int dof_of(const rgg_robot *r)
{
    return r->kind == RGG_SE2 ? 3 : (r->kind == RGG_SE3 ? 7 : r->n_links);
}

int dim_of(const rgg_robot *r) { return r->kind == RGG_SE3 ? 3 : 2; }

// Parameters of the straight-line motion between two configurations.
struct Motion {
    double a[kMaxLinks + 7];
    double b[kMaxLinks + 7];   // SE3: quaternion sign chosen for the short arc
    double turn = 0.0;         // SE2: heading change in (-pi, pi]
    double half = 0.0;         // SE3: half the rotation angle
    double sin_half = 0.0;
};

void make_motion(const rgg_robot *r, const double *qa, const double *qb, Motion *m)
{
    int n = dof_of(r);
    memcpy(m->a, qa, sizeof(double) * n);
    memcpy(m->b, qb, sizeof(double) * n);
    if (r->kind == RGG_SE2) {
        double turn = qb[2] - qa[2];
        if (turn > kPi)
            turn = turn - 2.0 * kPi;
        else if (turn <= -kPi)
            turn = turn + 2.0 * kPi;
        m->turn = turn;
    } else if (r->kind == RGG_SE3) {
        double dot = qa[3] * qb[3] + qa[4] * qb[4] + qa[5] * qb[5] + qa[6] * qb[6];
        if (dot < 0.0) {
            dot = -dot;
            m->b[3] = -qb[3];
            m->b[4] = -qb[4];
            m->b[5] = -qb[5];
            m->b[6] = -qb[6];
        }
        dot = std::min(dot, 1.0);
        m->half = acos(dot);
        m->sin_half = sin(m->half);
    }
}

// Configuration at parameter t in [0, 1].
void config_at(const rgg_robot *r, const Motion &m, double t, double *q)
{
    switch (r->kind) {
    case RGG_SE2:
        q[0] = m.a[0] + t * (m.b[0] - m.a[0]);
        q[1] = m.a[1] + t * (m.b[1] - m.a[1]);
        q[2] = m.a[2] + t * m.turn;
        break;
    case RGG_SE3: {
        q[0] = m.a[0] + t * (m.b[0] - m.a[0]);
        q[1] = m.a[1] + t * (m.b[1] - m.a[1]);
        q[2] = m.a[2] + t * (m.b[2] - m.a[2]);
        if (m.sin_half < 1e-12) {
            q[3] = m.a[3];
            q[4] = m.a[4];
            q[5] = m.a[5];
            q[6] = m.a[6];
        } else {
            // spherical linear interpolation, not renormalised
            double wa = sin((1.0 - t) * m.half) / m.sin_half;
            double wb = sin(t * m.half) / m.sin_half;
            for (int c = 3; c < 7; ++c) q[c] = wa * m.a[c] + wb * m.b[c];
        }
        break;
    }
    default:
        for (int c = 0; c < r->n_links; ++c) q[c] = m.a[c] + t * (m.b[c] - m.a[c]);
    }
}

// Writes the sphere centres of configuration j (of J) into a [B][J][S] block:
// coordinate d of sphere i lands at blk[(i*J + j)*S + d].
void place_spheres(const rgg_robot *r, const double *q, double *blk, int64_t S, int64_t J, int64_t j)
{
    const int B = r->n_spheres;
    if (r->kind == RGG_SE2) {
        double c = cos(q[2]);
        double s = sin(q[2]);
        for (int i = 0; i < B; ++i) {
            double ox = r->sphere_pos[2 * i], oy = r->sphere_pos[2 * i + 1];
            blk[(i * J + j) * S] = q[0] + (c * ox - s * oy);
            blk[(i * J + j) * S + 1] = q[1] + (s * ox + c * oy);
        }
    } else if (r->kind == RGG_SE3) {
        // v' = v + w*t + u x t, t = 2 (u x v), for the quaternion (w, u)
        const double w = q[3], ux = q[4], uy = q[5], uz = q[6];
        for (int i = 0; i < B; ++i) {
            const double *v = r->sphere_pos + 3 * i;
            double tx = 2.0 * (uy * v[2] - uz * v[1]);
            double ty = 2.0 * (uz * v[0] - ux * v[2]);
            double tz = 2.0 * (ux * v[1] - uy * v[0]);
            blk[(i * J + j) * S] = q[0] + ((v[0] + w * tx) + (uy * tz - uz * ty));
            blk[(i * J + j) * S + 1] = q[1] + ((v[1] + w * ty) + (uz * tx - ux * tz));
            blk[(i * J + j) * S + 2] = q[2] + ((v[2] + w * tz) + (ux * ty - uy * tx));
        }
    } else {
        // planar chain: link angle Phi_m accumulates q_0..q_m; joint
        // J_{m+1} = J_m + l_m (cos Phi_m, sin Phi_m)
        double jx[kMaxLinks + 1], jy[kMaxLinks + 1], cs[kMaxLinks], sn[kMaxLinks];
        double phi = q[0];
        jx[0] = r->base[0];
        jy[0] = r->base[1];
        for (int k = 0; k < r->n_links; ++k) {
            if (k > 0) phi = phi + q[k];
            cs[k] = cos(phi);
            sn[k] = sin(phi);
            jx[k + 1] = jx[k] + r->link_length[k] * cs[k];
            jy[k + 1] = jy[k] + r->link_length[k] * sn[k];
        }
        for (int i = 0; i < B; ++i) {
            int k = r->sphere_link[i];
            blk[(i * J + j) * S] = jx[k] + r->sphere_pos[i] * cs[k];
            blk[(i * J + j) * S + 1] = jy[k] + r->sphere_pos[i] * sn[k];
        }
    }
}

// Number of segments: cfg(e) holds segments + 1 configurations.
int64_t segments_of(const rgg_robot *r, const rgg_build_opts *o, const Motion &m)
{
    if (o->samples_per_edge > 1) return o->samples_per_edge - 1;
    double len;
    if (r->kind == RGG_SE2) {
        double dx = m.b[0] - m.a[0], dy = m.b[1] - m.a[1];
        len = sqrt(dx * dx + dy * dy + m.turn * m.turn);
    } else if (r->kind == RGG_SE3) {
        double s = 0.0;
        for (int c = 0; c < 3; ++c) {
            double d = m.b[c] - m.a[c];
            s = s + d * d;
        }
        double ang = 2.0 * m.half;
        len = sqrt(s + ang * ang);
    } else {
        double s = 0.0;
        for (int c = 0; c < r->n_links; ++c) {
            double d = m.b[c] - m.a[c];
            s = s + d * d;
        }
        len = sqrt(s);
    }
    double n = ceil(len / o->resolution);
    return n < 1.0 ? 1 : (int64_t)n;
}

// Chord-deviation bound of each sphere centre: max|p''| / 8.
//   SE2: |o| turn^2 / 8   (centre moves on a circle at the turning rate)
//   SE3: |o| phi^2 / 8    (slerp turns about a fixed axis at rate phi = 2*half)
//   arm: (sum_{k<L} |l_k| dPhi_k^2 + |s| dPhi_L^2) / 8, dPhi_k = sum_{j<=k} (qb_j - qa_j);
//        a lever enters by its length, so a sphere behind its joint (s < 0) is
//        bounded as one in front of it
void inflation(const rgg_robot *r, const Motion &m, double *out)
{
    const int B = r->n_spheres;
    if (r->kind == RGG_SE2) {
        for (int i = 0; i < B; ++i) {
            double ox = r->sphere_pos[2 * i], oy = r->sphere_pos[2 * i + 1];
            double len = sqrt(ox * ox + oy * oy);
            out[i] = (len * m.turn) * m.turn / 8.0;
        }
    } else if (r->kind == RGG_SE3) {
        double ang = 2.0 * m.half;
        for (int i = 0; i < B; ++i) {
            const double *v = r->sphere_pos + 3 * i;
            double len = sqrt(v[0] * v[0] + v[1] * v[1] + v[2] * v[2]);
            out[i] = (len * ang) * ang / 8.0;
        }
    } else {
        for (int i = 0; i < B; ++i) {
            const int link = r->sphere_link[i];
            double sum = 0.0, dphi = 0.0;
            for (int k = 0; k <= link; ++k) {
                dphi = dphi + (m.b[k] - m.a[k]);
                double lever = fabs(k < link ? r->link_length[k] : r->sphere_pos[i]);
                sum = sum + (lever * dphi) * dphi;
            }
            out[i] = sum / 8.0;
        }
    }
}

// ---------------------------------------------------------------------------
// Second outer form (Sec. 4.2): an oriented box around each body's sweep.
// A body is the robot (SE2, SE3) or one link (arm).  The box's axes are the
// principal axes of the body's sphere centres over cfg(e), its extent along
// axis u the range of u.c -+ (r_i + delta_i / n^2) over those centres: over
// one step of length 1/n a centre stays within delta_i / n^2 of the chord of
// its sampled ends, so the box holds the continuous sweep.  The binary64
// steps (sums over configurations, then spheres; Jacobi rotations; the
// extents) are one fixed order, so the boxes are a function of the inputs.
// ---------------------------------------------------------------------------

int body_index(const rgg_robot *r, int i) { return r->kind == RGG_PLANAR_ARM ? r->sphere_link[i] : 0; }
int body_count(const rgg_robot *r) { return r->kind == RGG_PLANAR_ARM ? r->n_links : 1; }

// Columns of ev: eigenvectors of the symmetric D x D matrix m (overwritten),
// by cyclic Jacobi rotations (pairs (p, q), p < q; one sweep in 2-D, where
// one rotation diagonalises, eight in 3-D).
void principal_axes(int D, double m[3][3], double ev[3][3])
{
    for (int r = 0; r < D; ++r)
        for (int c = 0; c < D; ++c) ev[r][c] = r == c ? 1.0 : 0.0;
    const int sweeps = D == 3 ? 8 : 1;
    for (int sw = 0; sw < sweeps; ++sw)
        for (int p = 0; p + 1 < D; ++p)
            for (int q = p + 1; q < D; ++q) {
                const double off = m[p][q];
                if (off == 0.0) continue;
                // tan of the angle that zeroes m[p][q]: the root of
                // t^2 + 2 theta t - 1 of smaller magnitude
                const double theta = (m[q][q] - m[p][p]) / (2.0 * off);
                double t = 1.0 / (fabs(theta) + sqrt(theta * theta + 1.0));
                if (theta < 0.0) t = -t;
                const double c = 1.0 / sqrt(t * t + 1.0);
                const double sn = t * c;
                for (int r = 0; r < D; ++r) {
                    if (r == p || r == q) continue;
                    const double mp = m[r][p], mq = m[r][q];
                    m[r][p] = c * mp - sn * mq;
                    m[p][r] = m[r][p];
                    m[r][q] = sn * mp + c * mq;
                    m[q][r] = m[r][q];
                }
                m[p][p] = m[p][p] - t * off;
                m[q][q] = m[q][q] + t * off;
                m[p][q] = 0.0;
                m[q][p] = 0.0;
                for (int r = 0; r < D; ++r) {
                    const double ep = ev[r][p], eq = ev[r][q];
                    ev[r][p] = c * ep - sn * eq;
                    ev[r][q] = sn * ep + c * eq;
                }
            }
}

// Box of body b: centres blk[(i*J + j)*S + d] (j = 0..nseg), bounds infl[B].
// Writes centre[D], axes[D][D] (row k = axis k), half[D] to o; false (and
// nothing written) when the body carries no sphere.
bool body_box(const rgg_robot *r, int D, int b, const double *blk, int S, int64_t J, const double *infl,
              double *o)
{
    const int B = r->n_spheres;
    const int64_t nseg = J - 1;
    double mean[3] = {0.0, 0.0, 0.0};
    int64_t npts = 0;
    for (int64_t j = 0; j < J; ++j)
        for (int i = 0; i < B; ++i) {
            if (body_index(r, i) != b) continue;
            for (int d = 0; d < D; ++d) mean[d] = mean[d] + blk[(i * J + j) * S + d];
            ++npts;
        }
    if (npts == 0) return false;
    for (int d = 0; d < D; ++d) mean[d] = mean[d] / (double)npts;
    double sc[3][3] = {{0.0, 0.0, 0.0}, {0.0, 0.0, 0.0}, {0.0, 0.0, 0.0}};
    for (int64_t j = 0; j < J; ++j)
        for (int i = 0; i < B; ++i) {
            if (body_index(r, i) != b) continue;
            double dv[3];
            for (int d = 0; d < D; ++d) dv[d] = blk[(i * J + j) * S + d] - mean[d];
            for (int k = 0; k < D; ++k)
                for (int l = k; l < D; ++l) sc[k][l] = sc[k][l] + dv[k] * dv[l];
        }
    for (int k = 1; k < D; ++k)
        for (int l = 0; l < k; ++l) sc[k][l] = sc[l][k];
    double ev[3][3];
    principal_axes(D, sc, ev);
    double *ctr = o, *ax = o + D, *half = o + D + D * D;
    for (int k = 0; k < D; ++k)
        for (int d = 0; d < D; ++d) ax[k * D + d] = ev[d][k];
    const double n2 = (double)nseg * (double)nseg;
    double mid[3];
    for (int k = 0; k < D; ++k) {
        double lo = INFINITY, hi = -INFINITY;
        for (int64_t j = 0; j < J; ++j)
            for (int i = 0; i < B; ++i) {
                if (body_index(r, i) != b) continue;
                double pr = 0.0;
                for (int d = 0; d < D; ++d) pr = pr + ax[k * D + d] * blk[(i * J + j) * S + d];
                const double eta = infl[i] / n2;
                const double a = (pr - r->sphere_radius[i]) - eta, z = (pr + r->sphere_radius[i]) + eta;
                if (a < lo) lo = a;
                if (z > hi) hi = z;
            }
        mid[k] = 0.5 * (lo + hi);
        half[k] = 0.5 * (hi - lo);
    }
    for (int d = 0; d < D; ++d) {
        double acc = 0.0;
        for (int k = 0; k < D; ++k) acc = acc + mid[k] * ax[k * D + d];
        ctr[d] = acc;
    }
    return true;
}

// ---------------------------------------------------------------------------
// Second inner form (Sec. 4.2): each sphere's spline through its centres,
// simplified by Agarwal et al.'s greedy shortcuts.  From vertex a the
// candidates b = a+2, a+4, a+8, ... (the last clamped to n) are accepted
// while err(a, b), the largest distance of the skipped centres from the
// segment [c_a, c_b], is at most tol * r; a bisection between the last
// accepted and the first rejected candidate then finds an accepted b whose
// successor is rejected.  The segment (a, b) becomes a capsule of radius
// r - err(a, b) - delta / n^2, kept when that is not negative: each of its
// points is within err(a, b) of the polyline and so within err(a, b) +
// delta / n^2 of the sphere's centre path, which keeps the capsule inside
// the swept sphere.
// ---------------------------------------------------------------------------

// squared distance from p to the segment [a, b]
double seg_point_d2(int D, const double *p, const double *a, const double *b)
{
    double d[3], dd = 0.0, wd = 0.0;
    for (int k = 0; k < D; ++k) {
        d[k] = b[k] - a[k];
        dd = dd + d[k] * d[k];
        wd = wd + (p[k] - a[k]) * d[k];
    }
    double t = 0.0;
    if (dd > 0.0) t = std::min(std::max(wd / dd, 0.0), 1.0);
    double acc = 0.0;
    for (int k = 0; k < D; ++k) {
        const double g = (a[k] + t * d[k]) - p[k];
        acc = acc + g * g;
    }
    return acc;
}

// err(a, b)^2 of the centres c + j * S
double skip_err2(int D, const double *c, int S, int64_t a, int64_t b)
{
    double worst = 0.0;
    for (int64_t m = a + 1; m < b; ++m) worst = std::max(worst, seg_point_d2(D, c + m * S, c + a * S, c + b * S));
    return worst;
}

// Segments of the spline through c + j * S, j = 0..n, into out ([K][2D+1]:
// A, B, rho; may be null); returns K.
int64_t spline_segments(int D, const double *c, int S, int64_t n, double rad, double eta, double tol, double *out)
{
    const double lim = tol * rad;
    const double lim2 = lim * lim;
    int64_t a = 0, K = 0;
    while (a < n) {
        int64_t good = a + 1, bad = n + 1;   // (a, good) accepted, (a, bad) rejected or past the end
        for (int64_t span = 2;; span *= 2) {
            const int64_t b = std::min(a + span, n);
            if (b <= good) break;
            if (skip_err2(D, c, S, a, b) > lim2) {
                bad = b;
                break;
            }
            good = b;
            if (b == n) break;
        }
        while (bad - good > 1 && bad <= n) {
            const int64_t mid = good + (bad - good) / 2;
            if (skip_err2(D, c, S, a, mid) <= lim2)
                good = mid;
            else
                bad = mid;
        }
        const double rho = (rad - sqrt(skip_err2(D, c, S, a, good))) - eta;
        if (rho >= 0.0) {
            if (out) {
                double *o = out + K * (2 * D + 1);
                for (int k = 0; k < D; ++k) {
                    o[k] = c[a * S + k];
                    o[D + k] = c[good * S + k];
                }
                o[2 * D] = rho;
            }
            ++K;
        }
        a = good;
    }
    return K;
}

double pad_of(double x) { return ldexp(std::max(1.0, fabs(x)), -20); }

bool finite_all(const double *p, int64_t n)
{
    for (int64_t i = 0; i < n; ++i)
        if (!std::isfinite(p[i])) return false;
    return true;
}

}  // namespace

float f32_down(double x)
{
    float f = (float)x;
    if ((double)f > x) f = nextafterf(f, -INFINITY);
    return f;
}

float f32_up(double x)
{
    float f = (float)x;
    if ((double)f < x) f = nextafterf(f, INFINITY);
    return f;
}

rgg_status validate_build_inputs(const rgg_roadmap_desc *rd, const rgg_robot *r,
                                 const rgg_build_opts *o, std::string *err)
{
    auto bad = [&](const char *msg) {
        *err = msg;
        return RGG_E_INVALID_ARG;
    };
    if (!rd || !r || !o) return bad("null roadmap, robot or options");
    if (r->kind != RGG_SE2 && r->kind != RGG_SE3 && r->kind != RGG_PLANAR_ARM)
        return bad("unknown robot kind");
    if (r->n_spheres < 1 || r->n_spheres > kMaxSpheres) return bad("n_spheres must be 1..64");
    if (!r->sphere_pos || !r->sphere_radius) return bad("null sphere arrays");
    const int B = r->n_spheres;
    if (r->kind == RGG_PLANAR_ARM) {
        if (r->n_links < 1 || r->n_links > kMaxLinks) return bad("n_links must be 1..32");
        if (!r->sphere_link || !r->link_length) return bad("null arm arrays");
        for (int i = 0; i < B; ++i)
            if (r->sphere_link[i] < 0 || r->sphere_link[i] >= r->n_links)
                return bad("sphere_link out of range");
        if (!finite_all(r->link_length, r->n_links) || !finite_all(r->base, 2))
            return bad("non-finite arm geometry");
    }
    int per = r->kind == RGG_SE2 ? 2 : (r->kind == RGG_SE3 ? 3 : 1);
    if (!finite_all(r->sphere_pos, (int64_t)B * per)) return bad("non-finite sphere offsets");
    for (int i = 0; i < B; ++i)
        if (!(r->sphere_radius[i] > 0.0) || !std::isfinite(r->sphere_radius[i]))
            return bad("sphere radii must be finite and positive");
    if (rd->n_nodes < 0 || rd->n_edges < 0) return bad("negative node or edge count");
    if (rd->n_edges > (int64_t)INT32_MAX - 1) return bad("too many edges");
    if (rd->n_nodes > 0 && !rd->q) return bad("null node array");
    if (rd->n_edges > 0 && !rd->edge_uv) return bad("null edge array");
    const int dof = dof_of(r);
    if (!finite_all(rd->q, rd->n_nodes * dof)) return bad("non-finite node configuration");
    if (r->kind == RGG_SE3) {
        for (int64_t v = 0; v < rd->n_nodes; ++v) {
            const double *q = rd->q + v * dof;
            double n2 = q[3] * q[3] + q[4] * q[4] + q[5] * q[5] + q[6] * q[6];
            if (fabs(n2 - 1.0) > 1e-9) return bad("SE3 node quaternion is not unit length");
        }
    }
    for (int64_t e = 0; e < 2 * rd->n_edges; ++e)
        if (rd->edge_uv[e] < 0 || rd->edge_uv[e] >= rd->n_nodes) return bad("edge node id out of range");
    if (o->samples_per_edge == 1 || o->samples_per_edge < 0)
        return bad("samples_per_edge must be 0 or >= 2");
    if (o->samples_per_edge == 0 && !(o->resolution > 0.0 && std::isfinite(o->resolution)))
        return bad("resolution must be positive when samples_per_edge is 0");
    if (o->precision != RGG_PREC_FP64 && o->precision != RGG_PREC_FP32_RECHECK)
        return bad("unknown precision");
    if (!(o->band_rel >= 0.0) && !(o->band_rel <= 0.0)) return bad("band_rel is NaN");
    if (o->n_obstacle_slots < 0 || o->n_obstacle_slots > 4096) return bad("n_obstacle_slots must be 0..4096");
    if (o->retest_capacity < 0 || o->retest_capacity > (1 << 20)) return bad("retest_capacity must be 0..2^20");
    if (o->item_edges < 0 || o->item_edges > 512) return bad("item_edges must be 0..512");
    if (std::isnan(o->cell_size)) return bad("cell_size is NaN");
    if (o->mem_budget < 0) return bad("mem_budget must be 0 (the free device memory) or positive");
    if (o->pair_list_capacity < 0 || o->pair_list_capacity > (1 << 20))
        return bad("pair_list_capacity must be 0..2^20");
    if (o->inline_rounds < RGG_INLINE_NONE || o->inline_rounds > (1 << 20))
        return bad("inline_rounds must be RGG_INLINE_NONE, RGG_INLINE_ALL or a round count up to 2^20");
    if (o->outer_obb != 0 && o->outer_obb != 1) return bad("outer_obb must be 0 or 1");
    if (o->inner_splines != 0 && o->inner_splines != 1) return bad("inner_splines must be 0 or 1");
    if (o->inner_splines && !(o->spline_tol >= 0.0 && o->spline_tol < 1.0))
        return bad("spline_tol must be in [0, 1) (0 selects 0.05)");
    return RGG_OK;
}

rgg_status build_geometry(const rgg_roadmap_desc *rd, const rgg_robot *r, const rgg_build_opts *o,
                          int64_t e0, int64_t e1, int threads, HostGeometry *g, std::string *err)
{
    const int B = r->n_spheres, D = dim_of(r), dof = dof_of(r);
    const int64_t E = e1 - e0;
    g->kind = r->kind;
    g->D = D;
    g->B = B;
    g->E = E;
    g->radius.assign(r->sphere_radius, r->sphere_radius + B);
    g->soff.assign(E + 1, 0);
    g->dof = dof;
    g->L = r->kind == RGG_PLANAR_ARM ? r->n_links : 0;
    const int per = r->kind == RGG_SE2 ? 2 : (r->kind == RGG_SE3 ? 3 : 1);
    g->rob_pos.assign(r->sphere_pos, r->sphere_pos + B * per);
    g->rob_link.assign((size_t)B, 0);
    if (r->kind == RGG_PLANAR_ARM) {
        g->rob_link.assign(r->sphere_link, r->sphere_link + B);
        g->rob_len.assign(r->link_length, r->link_length + r->n_links);
        g->rob_base[0] = r->base[0];
        g->rob_base[1] = r->base[1];
    }
    const int vstride = 2 * dof + 3;
    const double tol = o->spline_tol > 0.0 ? o->spline_tol : kDefaultSplineTol;
    if (threads < 1) threads = 1;
    threads = (int)std::min<int64_t>(threads, std::max<int64_t>(E, 1));

    auto run = [&](auto &&fn) {
        std::vector<std::thread> pool;
        for (int t = 0; t < threads; ++t)
            pool.emplace_back([&, t] { fn(E * t / threads, E * (t + 1) / threads); });
        for (auto &th : pool) th.join();
    };
    // pass 1: configuration counts
    run([&](int64_t a, int64_t b) {
        for (int64_t k = a; k < b; ++k) {
            const int64_t e = e0 + k;
            Motion m;
            make_motion(r, rd->q + rd->edge_uv[2 * e] * dof, rd->q + rd->edge_uv[2 * e + 1] * dof, &m);
            g->soff[k + 1] = std::min(segments_of(r, o, m) + 1, kMaxEdgeConfigs + 1) * B;
        }
    });
    for (int64_t k = 0; k < E; ++k)
        if (g->soff[k + 1] > kMaxEdgeConfigs * B) {
            *err = "an edge needs more than 2^24 configurations (resolution too fine)";
            return RGG_E_INVALID_ARG;
        }
    for (int64_t k = 0; k < E; ++k) g->soff[k + 1] += g->soff[k];
    const int64_t total = g->soff[E];
    const int S = copy_stride(D);
    if (total > ((int64_t)1 << 40) / S) {
        *err = "too many sphere samples (resolution too fine)";
        return RGG_E_OUT_OF_MEMORY;
    }
    try {
        g->samp.assign((size_t)(total * S), 0.0);
        g->cap.assign((size_t)(E * (2 * D + 1) * B), 0.0);
        g->aabb.assign((size_t)(E * kAabbStride), 0.0f);
        g->motion.assign((size_t)(E * vstride), 0.0);
        g->delta.assign((size_t)(E * B), 0.0);
        g->n_bodies = body_count(r);
        g->body.assign((size_t)B, 0);
        g->body_has.assign((size_t)g->n_bodies, 0);
        for (int i = 0; i < B; ++i) {
            g->body[i] = body_index(r, i);
            g->body_has[g->body[i]] = 1;
        }
        if (o->outer_obb) g->obb.assign((size_t)(E * g->n_bodies * obb_stride(D)), 0.0);
        if (o->inner_splines) g->sseg.assign((size_t)(E * B + 1), 0);
    } catch (const std::bad_alloc &) {
        *err = "host memory for the build";
        return RGG_E_OUT_OF_MEMORY;
    }
    // pass 2: centres, capsules, boxes
    run([&](int64_t a, int64_t b) {
        double q[kMaxLinks + 7];
        double infl[kMaxSpheres];
        for (int64_t k = a; k < b; ++k) {
            const int64_t e = e0 + k;
            Motion m;
            make_motion(r, rd->q + rd->edge_uv[2 * e] * dof, rd->q + rd->edge_uv[2 * e + 1] * dof, &m);
            const int64_t P = g->soff[k + 1] - g->soff[k];
            const int64_t J = P / B, nseg = J - 1;
            double *blk = g->samp.data() + S * g->soff[k];
            for (int64_t j = 0; j <= nseg; ++j) {
                config_at(r, m, (double)j / (double)nseg, q);
                place_spheres(r, q, blk, S, J, j);
            }
            inflation(r, m, infl);
            double *mv = g->motion.data() + k * vstride;
            for (int c = 0; c < dof; ++c) {
                mv[c] = m.a[c];
                mv[dof + c] = m.b[c];
            }
            mv[2 * dof] = m.turn;
            mv[2 * dof + 1] = m.half;
            mv[2 * dof + 2] = m.sin_half;
            for (int i = 0; i < B; ++i) g->delta[k * B + i] = infl[i];
            if (o->outer_obb)
                for (int b = 0; b < g->n_bodies; ++b)
                    body_box(r, D, b, blk, S, J, infl, g->obb.data() + (k * g->n_bodies + b) * obb_stride(D));
            if (o->inner_splines) {
                const double n2 = (double)nseg * (double)nseg;
                for (int i = 0; i < B; ++i)
                    g->sseg[k * B + i + 1] = spline_segments(D, blk + i * J * S, S, nseg, r->sphere_radius[i],
                                                             infl[i] / n2, tol, nullptr);
            }
            double *cp = g->cap.data() + k * (2 * D + 1) * B;
            double lo[3] = {INFINITY, INFINITY, INFINITY}, hi[3] = {-INFINITY, -INFINITY, -INFINITY};
            for (int i = 0; i < B; ++i) {
                const double R = r->sphere_radius[i] + infl[i];
                cp[2 * D * B + i] = R;
                for (int d = 0; d < D; ++d) {
                    const double s = blk[(i * J) * S + d], t = blk[(i * J + nseg) * S + d];
                    cp[d * B + i] = s;
                    cp[(D + d) * B + i] = t;
                    lo[d] = std::min(lo[d], std::min(s, t) - R);
                    hi[d] = std::max(hi[d], std::max(s, t) + R);
                }
            }
            float *bx = g->aabb.data() + k * kAabbStride;
            float smax = 0.0f;
            for (int d = 0; d < 3; ++d) {
                float l = 0.0f, h = 0.0f;
                if (d < D) {
                    l = f32_down(lo[d] - pad_of(lo[d]));
                    h = f32_up(hi[d] + pad_of(hi[d]));
                    smax = std::max(smax, std::max(fabsf(l), fabsf(h)));
                }
                bx[d] = l;
                bx[4 + d] = h;
            }
            bx[3] = smax;
            bx[7] = 0.0f;
        }
    });
    if (o->inner_splines) {
        // pass 3: the spline segments, at the offsets their counts give
        for (int64_t k = 0; k < E * B; ++k) g->sseg[k + 1] += g->sseg[k];
        try {
            g->seg.assign((size_t)(g->sseg[E * B] * (2 * D + 1)), 0.0);
        } catch (const std::bad_alloc &) {
            *err = "host memory for the splines";
            return RGG_E_OUT_OF_MEMORY;
        }
        run([&](int64_t a, int64_t b) {
            for (int64_t k = a; k < b; ++k) {
                const int64_t P = g->soff[k + 1] - g->soff[k];
                const int64_t J = P / B, nseg = J - 1;
                const double *blk = g->samp.data() + S * g->soff[k];
                const double n2 = (double)nseg * (double)nseg;
                for (int i = 0; i < B; ++i)
                    spline_segments(D, blk + i * J * S, S, nseg, r->sphere_radius[i], g->delta[k * B + i] / n2, tol,
                                    g->seg.data() + g->sseg[k * B + i] * (2 * D + 1));
            }
        });
    }
    return RGG_OK;
}

int32_t cell_coord(double x, double org, double inv, int32_t n)
{
    double c = floor((x - org) * inv);
    if (c < 0.0) return -1;
    if (c >= (double)n) return n;
    return (int32_t)c;
}

namespace {

rgg_status build_grid_body(const HostGeometry &g, double cell_size, int32_t chunk, HostGrid *out,
                           std::string *err)
{
    const int D = g.D;
    const int64_t E = g.E;
    double lo[3] = {0, 0, 0}, hi[3] = {0, 0, 0}, ext_sum = 0.0;
    for (int d = 0; d < D; ++d) {
        lo[d] = INFINITY;
        hi[d] = -INFINITY;
    }
    for (int64_t e = 0; e < E; ++e) {
        const float *b = g.aabb.data() + e * kAabbStride;
        double ext = 0.0;
        for (int d = 0; d < D; ++d) {
            lo[d] = std::min(lo[d], (double)b[d]);
            hi[d] = std::max(hi[d], (double)b[4 + d]);
            ext = std::max(ext, (double)b[4 + d] - (double)b[d]);
        }
        ext_sum += ext;
    }
    if (E == 0)
        for (int d = 0; d < D; ++d) lo[d] = hi[d] = 0.0;
    double h = cell_size;
    if (h == 0.0) h = E ? 2.0 * ext_sum / (double)E : 1.0;    // heuristic: twice the mean edge extent
    bool single = !(h > 0.0) || !std::isfinite(h);
    // keep the grid within 2^22 cells
    if (!single) {
        for (int it = 0; it < 64; ++it) {
            double cells = 1.0;
            for (int d = 0; d < D; ++d) cells *= std::max(1.0, ceil((hi[d] - lo[d]) / h));
            if (cells <= (double)(1 << 22)) break;
            h *= 1.25;
        }
    }
    for (int d = 0; d < 3; ++d) {
        out->org[d] = d < D ? lo[d] : 0.0;
        out->dim[d] = 1;
        if (!single && d < D) out->dim[d] = (int32_t)std::max(1.0, ceil((hi[d] - lo[d]) / h));
    }
    out->inv = single ? 0.0 : 1.0 / h;
    out->cell = single ? INFINITY : h;
    // block-local slab masks: local_slabs(D) slabs per axis over the bounds
    for (int d = 0; d < 3; ++d) {
        out->sl_org[d] = d < D ? (float)lo[d] : 0.0f;
        const double ext = d < D ? hi[d] - lo[d] : 0.0;
        out->sl_inv[d] = ext > 0.0 && std::isfinite(ext) ? (float)(local_slabs(D) / ext) : 0.0f;
    }
    const int64_t ncell = (int64_t)out->dim[0] * out->dim[1] * out->dim[2];
    std::vector<int64_t> count(ncell + 1, 0);
    auto range = [&](const float *b, int d, int32_t *c0, int32_t *c1) {
        if (d >= D) {
            *c0 = *c1 = 0;
            return;
        }
        int32_t n = out->dim[d];
        *c0 = std::min(std::max(cell_coord((double)b[d], out->org[d], out->inv, n), 0), n - 1);
        *c1 = std::min(std::max(cell_coord((double)b[4 + d], out->org[d], out->inv, n), 0), n - 1);
    };
    for (int pass = 0; pass < 2; ++pass) {
        std::vector<int64_t> cursor;
        if (pass == 1) {
            for (int64_t c = 0; c < ncell; ++c) count[c + 1] += count[c];
            if (count[ncell] > (int64_t)INT32_MAX) {
                *err = "grid too fine: more than 2^31 registrations";
                return RGG_E_OUT_OF_MEMORY;
            }
            out->edges.assign(count[ncell], 0);
            cursor.assign(count.begin(), count.end() - 1);
        }
        for (int64_t e = 0; e < E; ++e) {
            const float *b = g.aabb.data() + e * kAabbStride;
            int32_t r0[3], r1[3];
            for (int d = 0; d < 3; ++d) range(b, d, &r0[d], &r1[d]);
            for (int32_t z = r0[2]; z <= r1[2]; ++z)
                for (int32_t y = r0[1]; y <= r1[1]; ++y)
                    for (int32_t x = r0[0]; x <= r1[0]; ++x) {
                        int64_t c = ((int64_t)z * out->dim[1] + y) * out->dim[0] + x;
                        if (pass == 0)
                            count[c + 1]++;
                        else
                            out->edges[cursor[c]++] = (int32_t)e;
                    }
        }
    }
    out->start.assign(ncell + 1, 0);
    int64_t items = 0;
    for (int64_t c = 0; c <= ncell; ++c) out->start[c] = (int32_t)count[c];
    for (int64_t c = 0; c < ncell; ++c) {
        int64_t n = count[c + 1] - count[c];
        items += std::max<int64_t>(1, (n + chunk - 1) / chunk);
    }
    out->items_cap = items;
    return RGG_OK;
}

}  // namespace

rgg_status build_grid(const HostGeometry &g, double cell_size, int32_t chunk, HostGrid *out,
                      std::string *err)
{
    try {
        return build_grid_body(g, cell_size, chunk, out, err);
    } catch (const std::bad_alloc &) {
        *err = "host memory for the grid";
        return RGG_E_OUT_OF_MEMORY;
    }
}

}  // namespace rgg
