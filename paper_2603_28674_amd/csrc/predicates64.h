// The binary64 predicates behind every exact decision of librgg: the update
// kernels' binary64 re-tests and deferred items, the oriented-box test (always
// decided in binary64), and the full validation.  Each is one fixed expression order; device code is compiled
// without FMA contraction, so any IEEE binary64 evaluator of the same
// expressions reaches the same values.
#pragma once

#include <hip/hip_runtime.h>

namespace rgg {

__device__ inline double gap64(double x, double lo, double hi)
{
    double a = lo - x;
    double g = a > 0.0 ? a : 0.0;
    double b = x - hi;
    return b > g ? b : g;
}

template <int D>
__device__ inline double point_box64(const double *c, const double *lo, const double *hi)
{
    double acc = 0.0;
#pragma unroll
    for (int k = 0; k < D; ++k) {
        double g = gap64(c[k], lo[k], hi[k]);
        acc = acc + g * g;
    }
    return acc;
}

template <int D>
__device__ inline double seg_F64(const double *A, const double *d, double t, const double *lo,
                                 const double *hi)
{
    double acc = 0.0;
#pragma unroll
    for (int k = 0; k < D; ++k) {
        double p = A[k] + t * d[k];
        double g = gap64(p, lo[k], hi[k]);
        acc = acc + g * g;
    }
    return acc;
}

template <int D>
__device__ inline double seg_G64(const double *A, const double *d, double t, const double *lo,
                                 const double *hi)
{
    double acc = 0.0;
#pragma unroll
    for (int k = 0; k < D; ++k) {
        double p = A[k] + t * d[k];
        double ex = p < lo[k] ? p - lo[k] : (p > hi[k] ? p - hi[k] : 0.0);
        acc = acc + d[k] * ex;
    }
    return acc;
}

// Minimum over t in [0,1] of the squared distance from A + t (B - A) to the
// box.  The function is convex and piecewise quadratic with breaks where a
// coordinate crosses a face plane; its half-derivative G is nondecreasing.
// The minimiser lies between the largest candidate with G <= 0 and the
// smallest with G >= 0 (candidates: 0, 1, face crossings strictly inside);
// there the faces in play are fixed and the single quadratic's stationary
// point is clamped into that bracket.
// When `targ` is given it receives the parameter of the value returned (which
// does not change the value).
template <int D>
__device__ inline double segbox64(const double *A, const double *Bp, const double *lo, const double *hi,
                                  double *targ = nullptr)
{
    double d[D];
#pragma unroll
    for (int k = 0; k < D; ++k) d[k] = Bp[k] - A[k];
    double tL = 0.0, tR = 1.0;
    auto take = [&](double t) {
        double g = seg_G64<D>(A, d, t, lo, hi);
        if (g <= 0.0 && t > tL) tL = t;
        if (g >= 0.0 && t < tR) tR = t;
    };
    take(0.0);
    take(1.0);
#pragma unroll
    for (int k = 0; k < D; ++k) {
        if (d[k] != 0.0) {
            double t1 = (lo[k] - A[k]) / d[k];
            if (t1 > 0.0 && t1 < 1.0) take(t1);
            double t2 = (hi[k] - A[k]) / d[k];
            if (t2 > 0.0 && t2 < 1.0) take(t2);
        }
    }
    double fL = seg_F64<D>(A, d, tL, lo, hi);
    double fR = seg_F64<D>(A, d, tR, lo, hi);
    double fmin = fL < fR ? fL : fR;
    double tmin = fL < fR ? tL : tR;
    if (tL < tR) {
        double tm = 0.5 * (tL + tR);
        double num = 0.0, den = 0.0;
#pragma unroll
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
        double fs = seg_F64<D>(A, d, ts, lo, hi);
        if (fs < fmin) {
            fmin = fs;
            tmin = ts;
        }
    }
    if (targ) *targ = tmin;
    return fmin;
}

// Oriented box o = (centre[D], axes[D][D] as rows, half-extents[D]) against
// the closed box [lo, hi]: true when they share a point.  Separating-axis
// theorem for two boxes: the candidate axes are the box's face normals e_d,
// the oriented box's axes u_k and, in 3-D, the products e_d x u_k; on an axis
// the centres' projections differ by |T . axis| (T = centre - box centre) and
// the boxes reach the sums of their half-extents times |face normal . axis|.
template <int D>
__device__ inline bool obb_box_meet64(const double *o, const double *lo, const double *hi)
{
    const double *c = o, *u = o + D, *h = o + D + D * D;
    double bh[D], t[D], au[D][D];
#pragma unroll
    for (int d = 0; d < D; ++d) {
        bh[d] = 0.5 * (hi[d] - lo[d]);
        t[d] = c[d] - 0.5 * (lo[d] + hi[d]);
    }
#pragma unroll
    for (int d = 0; d < D; ++d)
#pragma unroll
        for (int k = 0; k < D; ++k) au[d][k] = fabs(u[k * D + d]);
    bool sep = false;
#pragma unroll
    for (int d = 0; d < D; ++d) {
        double rb = 0.0;
#pragma unroll
        for (int k = 0; k < D; ++k) rb = rb + h[k] * au[d][k];
        sep = sep || fabs(t[d]) > bh[d] + rb;
    }
#pragma unroll
    for (int k = 0; k < D; ++k) {
        double ra = 0.0, tp = 0.0;
#pragma unroll
        for (int d = 0; d < D; ++d) {
            ra = ra + bh[d] * au[d][k];
            tp = tp + u[k * D + d] * t[d];
        }
        sep = sep || fabs(tp) > h[k] + ra;
    }
    if constexpr (D == 3) {
        // e_d x u_k: components -u_k[d2] at d1 and u_k[d1] at d2
#pragma unroll
        for (int d = 0; d < 3; ++d) {
            const int d1 = (d + 1) % 3, d2 = (d + 2) % 3;
#pragma unroll
            for (int k = 0; k < 3; ++k) {
                const int k1 = (k + 1) % 3, k2 = (k + 2) % 3;
                const double ra = bh[d1] * au[d2][k] + bh[d2] * au[d1][k];
                const double rb = h[k1] * au[d][k2] + h[k2] * au[d][k1];
                const double tp = t[d2] * u[k * 3 + d1] - t[d1] * u[k * 3 + d2];
                sep = sep || fabs(tp) > ra + rb;
            }
        }
    }
    return !sep;
}

}  // namespace rgg
