// Full validation of listed edges (Alg. 1, the branch taken when not lazy:
// every edge left unknown gets a full collision check).
//
// The check is continuous: does any configuration q(t), t in [0, 1], of the
// edge's motion put a robot sphere into a present box?  It refines the two
// approximations of Sec. 3.2 on dyadic sub-intervals [j 2^-l, (j+1) 2^-l]:
//   free(l, j)  every sphere's capsule from its centre at the interval's start
//               to its centre at the end, radius r_i + delta_i 4^-l, misses
//               every present box (delta_i 4^-l bounds the chord deviation
//               over an interval of length 2^-l, since delta_i bounds
//               max|p''|/8 over the edge);
//   hit(t)      some sphere at q(t) meets a present box.
// Level by level: hit(0) or hit(1) -> COLLIDES (witness 0, then 1); free(0, 0)
// -> FREE at level 0; then with A_0 = {0} and l = 0, 1, ...: more than
// max_active unknown intervals -> UNRESOLVED at l; a midpoint of A_l hits ->
// COLLIDES at l+1, witness the smallest such midpoint; A_{l+1} = the children
// that are not free; none -> FREE at l+1; after max_level levels ->
// UNRESOLVED.
//
// The configurations use the build's binary64 motion parameters and a sin/cos
// made of a fixed sequence of binary64 +, -, * and rint (Cody and Waite's
// reduction by pi/2, Taylor series to degree 19/20), compiled without
// contraction, so any IEEE evaluator of the same steps reaches the same
// verdicts.  The distance predicates are the binary64 definitions of the
// update kernels (predicates64.h).
//
// One wavefront (a 64-thread block) validates one listed edge at a time (grid-stride
// over the list).  Its present boxes near the edge are staged in LDS: a box
// can matter only if it meets the box around the edge's chords widened by
// r_i + 2 delta_i (each sub-chord stays within delta_i of the edge's chord,
// each sub-capsule adds at most r_i + delta_i), plus a rounding margin.  More
// than kValBoxes such boxes are handled in pages.
#include <hip/hip_runtime.h>
#include <math.h>

#include "predicates64.h"
#include "rgg_device.h"

namespace rgg {

namespace {

constexpr int kVT = 64;            // threads per block
constexpr int kVGrid = 16384;      // blocks at most (the hardware balances them)
constexpr int kNoHit = 0x7fffffff;

constexpr uint8_t kFree = RGG_VERDICT_FREE;
constexpr uint8_t kCollides = RGG_VERDICT_COLLIDES;
constexpr uint8_t kUnresolved = RGG_VERDICT_UNRESOLVED;

// ---- configurations --------------------------------------------------------

// sin and cos: x = k (pi/2) + r with pi/2 split into a 24-bit head (exact
// products with k) and its binary64 remainder; Taylor series of sin r to r^19
// and cos r to r^20 in Horner form; the quadrant k mod 4 maps the pair.
__device__ inline void vsincos(double x, double *sn, double *cs)
{
    const double pi = 3.14159265358979323846;
    const double half_pi = pi / 2.0;
    const double head = (double)(float)half_pi;
    const double tail = half_pi - head;
    const double k = rint(x * (2.0 / pi));
    const double r = (x - k * head) - k * tail;
    const double z = r * r;
    double ps = -1.0 / 121645100408832000.0;
    ps = ps * z + 1.0 / 355687428096000.0;
    ps = ps * z - 1.0 / 1307674368000.0;
    ps = ps * z + 1.0 / 6227020800.0;
    ps = ps * z - 1.0 / 39916800.0;
    ps = ps * z + 1.0 / 362880.0;
    ps = ps * z - 1.0 / 5040.0;
    ps = ps * z + 1.0 / 120.0;
    ps = ps * z - 1.0 / 6.0;
    const double s = r + (r * z) * ps;
    double pc = 1.0 / 2432902008176640000.0;
    pc = pc * z - 1.0 / 6402373705728000.0;
    pc = pc * z + 1.0 / 20922789888000.0;
    pc = pc * z - 1.0 / 87178291200.0;
    pc = pc * z + 1.0 / 479001600.0;
    pc = pc * z - 1.0 / 3628800.0;
    pc = pc * z + 1.0 / 40320.0;
    pc = pc * z - 1.0 / 720.0;
    pc = pc * z + 1.0 / 24.0;
    pc = pc * z - 1.0 / 2.0;
    const double c = 1.0 + z * pc;
    const int64_t quadrant = (int64_t)k & 3;
    if (quadrant == 0) {
        *sn = s;
        *cs = c;
    } else if (quadrant == 1) {
        *sn = c;
        *cs = -s;
    } else if (quadrant == 2) {
        *sn = -s;
        *cs = -c;
    } else {
        *sn = -c;
        *cs = s;
    }
}

// centre of sphere i at parameter t of the motion `mot` (a, b, turn, half,
// sin_half), in the build's expression order
template <int D>
__device__ inline void centre_at(const VRobot &rb, const double *mot, double t, int i, double *c)
{
    const int dof = rb.dof;
    const double *a = mot, *b = mot + dof;
    if (rb.kind == RGG_SE2) {
        const double q0 = a[0] + t * (b[0] - a[0]);
        const double q1 = a[1] + t * (b[1] - a[1]);
        const double q2 = a[2] + t * mot[2 * dof];
        double s, co;
        vsincos(q2, &s, &co);
        const double ox = rb.pos[2 * i], oy = rb.pos[2 * i + 1];
        c[0] = q0 + (co * ox - s * oy);
        c[1] = q1 + (s * ox + co * oy);
    } else if (rb.kind == RGG_SE3) {
        const double q0 = a[0] + t * (b[0] - a[0]);
        const double q1 = a[1] + t * (b[1] - a[1]);
        const double q2 = a[2] + t * (b[2] - a[2]);
        const double half = mot[2 * dof + 1], sh = mot[2 * dof + 2];
        double w, ux, uy, uz;
        if (sh < 1e-12) {
            w = a[3];
            ux = a[4];
            uy = a[5];
            uz = a[6];
        } else {
            double sa, ca, sb, cb;
            vsincos((1.0 - t) * half, &sa, &ca);
            vsincos(t * half, &sb, &cb);
            const double wa = sa / sh;
            const double wb = sb / sh;
            w = wa * a[3] + wb * b[3];
            ux = wa * a[4] + wb * b[4];
            uy = wa * a[5] + wb * b[5];
            uz = wa * a[6] + wb * b[6];
        }
        const double vx = rb.pos[3 * i], vy = rb.pos[3 * i + 1], vz = rb.pos[3 * i + 2];
        const double tx = 2.0 * (uy * vz - uz * vy);
        const double ty = 2.0 * (uz * vx - ux * vz);
        const double tz = 2.0 * (ux * vy - uy * vx);
        const double rx = (vx + w * tx) + (uy * tz - uz * ty);
        const double ry = (vy + w * ty) + (uz * tx - ux * tz);
        const double rz = (vz + w * tz) + (ux * ty - uy * tx);
        c[0] = q0 + rx;
        c[1] = q1 + ry;
        if (D == 3) c[D - 1] = q2 + rz;
    } else {
        // planar chain up to the sphere's link
        const int link = rb.link[i];
        double jx = rb.base[0], jy = rb.base[1], phi = 0.0, sph = 0.0, cph = 1.0;
        for (int m = 0; m <= link; ++m) {
            const double qm = a[m] + t * (b[m] - a[m]);
            phi = m == 0 ? qm : phi + qm;
            vsincos(phi, &sph, &cph);
            if (m < link) {
                jx = jx + rb.len[m] * cph;
                jy = jy + rb.len[m] * sph;
            }
        }
        c[0] = jx + rb.pos[i] * cph;
        c[1] = jy + rb.pos[i] * sph;
    }
}

// ---- the kernel ------------------------------------------------------------

struct ValShared {
    VRobot rob;
    double mot[2 * 32 + 3];
    double del[64];
    double ebox[6];                 // lo[3], hi[3] of the candidate region
    double box[kValBoxes][6];       // staged candidate boxes: lo[3], hi[3]
    int32_t act[kValMaxActive];
    int32_t nxt[2 * kValMaxActive];
    uint8_t flag[2 * kValMaxActive];
    int32_t wave_cnt[kVT / 64];
    int32_t n_cand, n_page, hit, n_next, nonfree;
};

// Threads per (point or interval, sphere) item: the block's threads are
// spread over the items and then over the staged boxes, so few items with
// many boxes still use the whole block (each group recomputes the centres).
__device__ inline int groups(int items, int nb)
{
    int g = items > 0 ? kVT / items : 1;
    if (g > nb) g = nb;
    return g < 1 ? 1 : g;
}

__device__ inline bool present_near(const rgg_box &b, const double *ebox, int D)
{
    bool ok = true;
    for (int k = 0; k < D; ++k) {
        ok = ok && b.lo[k] <= b.hi[k];
        ok = ok && b.lo[k] <= ebox[3 + k] && b.hi[k] >= ebox[k];
    }
    return ok;
}

// Stages candidate boxes [page * kValBoxes, ...) into sh.box (in slot order)
// and leaves their number in sh.n_page and the total in sh.n_cand.
template <int D>
__device__ __forceinline__ void gather_page(ValShared &sh, const ValDev &v, int page)
{
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int64_t lo_rank = (int64_t)page * kValBoxes;
    int32_t base = 0;
    for (int64_t s0 = 0; s0 < v.M; s0 += kVT) {
        const int64_t s = s0 + tid;
        bool cand = false;
        if (s < v.M) cand = present_near(v.resident[s], sh.ebox, D);
        const unsigned long long bal = __ballot(cand);
        if (lane == 0) sh.wave_cnt[wave] = __popcll(bal);
        __syncthreads();
        int32_t before = base;
        for (int w = 0; w < wave; ++w) before += sh.wave_cnt[w];
        int32_t total = 0;
        for (int w = 0; w < kVT / 64; ++w) total += sh.wave_cnt[w];
        const int32_t rank = before + __popcll(bal & ((1ull << lane) - 1ull));
        if (cand && rank >= lo_rank && rank < lo_rank + kValBoxes) {
            const rgg_box &b = v.resident[s];
            double *dst = sh.box[rank - lo_rank];
            for (int k = 0; k < 3; ++k) {
                dst[k] = b.lo[k];
                dst[3 + k] = b.hi[k];
            }
        }
        base += total;
        __syncthreads();
    }
    if (tid == 0) {
        sh.n_cand = base;
        const int64_t left = (int64_t)base - lo_rank;
        sh.n_page = (int32_t)(left < 0 ? 0 : (left > kValBoxes ? kValBoxes : left));
    }
    __syncthreads();
}

// Runs `test(n_boxes)` over every page of candidate boxes (the staged page
// when there is only one).
template <int D, typename F>
__device__ __forceinline__ void over_pages(ValShared &sh, const ValDev &v, int n_pages, F &&test)
{
    if (n_pages <= 1) {
        test(sh.n_page);
        __syncthreads();
        return;
    }
    for (int p = 0; p < n_pages; ++p) {
        gather_page<D>(sh, v, p);
        test(sh.n_page);
        __syncthreads();
    }
}

template <int D>
__device__ __forceinline__ void validate_one(ValShared &sh, const ValDev &v, int64_t e, int max_level, int max_active,
                             uint8_t *verdict, int32_t *level, double *witness, uint8_t *labels)
{
    const int tid = threadIdx.x;
    const int B = v.B;
    for (int k = tid; k < v.vstride; k += kVT) sh.mot[k] = v.motion[e * v.vstride + k];
    for (int k = tid; k < B; k += kVT) sh.del[k] = v.delta[e * B + k];
    __syncthreads();
    if (tid < D) {
        // the candidate region: chords widened by r_i + 2 delta_i, plus margin
        const double *cp = v.cap64 + e * (2 * D + 1) * B;
        double lo = INFINITY, hi = -INFINITY;
        for (int i = 0; i < B; ++i) {
            const double A = cp[tid * B + i], Bv = cp[(D + tid) * B + i];
            const double w = cp[2 * D * B + i] + sh.del[i];
            const double mn = A < Bv ? A : Bv, mx = A < Bv ? Bv : A;
            if (mn - w < lo) lo = mn - w;
            if (mx + w > hi) hi = mx + w;
        }
        sh.ebox[tid] = lo - 1e-6 * (1.0 + fabs(lo));
        sh.ebox[3 + tid] = hi + 1e-6 * (1.0 + fabs(hi));
    }
    __syncthreads();
    gather_page<D>(sh, v, 0);
    const int n_pages = (int)((sh.n_cand + kValBoxes - 1) / kValBoxes);

    uint8_t out = kUnresolved;
    int32_t out_level = 0;
    double out_t = NAN;

    // One phase of the search: hit(t) at the points ldexp(key(k), -ex),
    // k < n_pts (sh.hit = the smallest key that hits, kNoHit if none), and
    // free(lc, child(k)) for k < n_children (sh.flag[k] = 1 when not free).
    // The children's tests only matter when no point hits; computing both in
    // one pass saves a barrier-separated phase per level.
    auto step = [&](int n_pts, int ex, auto &&key, int lc, int n_children, auto &&child) {
        if (tid == 0) sh.hit = kNoHit;
        for (int k = tid; k < n_children; k += kVT) sh.flag[k] = 0;
        __syncthreads();
        const double wl = ldexp(1.0, -lc);
        const int hit_items = n_pts * B, all_items = (n_pts + n_children) * B;
        over_pages<D>(sh, v, n_pages, [&](int nb) {
            const int G = groups(all_items, nb);
            for (int w = tid; w < all_items * G; w += kVT) {
                const int item = w / G, grp = w - item * G;
                if (item < hit_items) {
                    const int k = item / B, i = item - k * B;
                    const int32_t kk = key(k);
                    if (kk >= sh.hit) continue;
                    double c[D];
                    centre_at<D>(sh.rob, sh.mot, ldexp((double)kk, -ex), i, c);
                    const double r2 = sh.rob.rad[i] * sh.rob.rad[i];
                    for (int b = grp; b < nb; b += G) {
                        if (point_box64<D>(c, sh.box[b], sh.box[b] + 3) <= r2) {
                            atomicMin(&sh.hit, kk);
                            break;
                        }
                    }
                } else {
                    const int it = item - hit_items;
                    const int k = it / B, i = it - k * B;
                    if (sh.flag[k] || sh.hit != kNoHit) continue;
                    const int32_t j = child(k);
                    double ca[D], cb[D];
                    centre_at<D>(sh.rob, sh.mot, ldexp((double)j, -lc), i, ca);
                    centre_at<D>(sh.rob, sh.mot, ldexp((double)(j + 1), -lc), i, cb);
                    const double R = sh.rob.rad[i] + sh.del[i] * (wl * wl);
                    // the capsule's bounding box, widened far beyond rounding:
                    // a box outside it is farther than R from the segment
                    double clo[D], chi[D];
#pragma unroll
                    for (int d = 0; d < D; ++d) {
                        const double mn = ca[d] < cb[d] ? ca[d] : cb[d], mx = ca[d] < cb[d] ? cb[d] : ca[d];
                        clo[d] = mn - (R * 1.000001 + 1e-9 * (1.0 + fabs(mn)));
                        chi[d] = mx + (R * 1.000001 + 1e-9 * (1.0 + fabs(mx)));
                    }
                    for (int b = grp; b < nb; b += G) {
                        bool apart = false;
#pragma unroll
                        for (int d = 0; d < D; ++d)
                            apart = apart || sh.box[b][d] > chi[d] || sh.box[b][3 + d] < clo[d];
                        if (apart) continue;
                        if (segbox64<D>(ca, cb, sh.box[b], sh.box[b] + 3) <= R * R) {
                            sh.flag[k] = 1;
                            break;
                        }
                    }
                }
            }
        });
        return sh.hit;
    };

    do {
        // t = 0, then t = 1 (key = t), and the whole edge's capsules
        const int h0 = step(2, 0, [](int k) { return (int32_t)k; }, 0, 1, [](int) { return 0; });
        if (h0 != kNoHit) {
            out = kCollides;
            out_t = (double)h0;
            break;
        }
        if (!sh.flag[0]) {
            out = kFree;
            break;
        }
        int na = 1;
        if (tid == 0) sh.act[0] = 0;
        __syncthreads();
        bool done = false;
        for (int l = 0; l < max_level && !done; ++l) {
            out_level = l;
            if (na > max_active) {
                out = kUnresolved;
                done = true;
                break;
            }
            const int h = step(na, l + 1, [&](int k) { return 2 * sh.act[k] + 1; }, l + 1, 2 * na,
                               [&](int k) { return 2 * sh.act[k >> 1] + (k & 1); });
            if (h != kNoHit) {
                out = kCollides;
                out_level = l + 1;
                out_t = ldexp((double)h, -(l + 1));
                done = true;
                break;
            }
            if (tid == 0) sh.n_next = 0;
            __syncthreads();
            for (int k = tid; k < 2 * na; k += kVT)
                if (sh.flag[k]) sh.nxt[atomicAdd(&sh.n_next, 1)] = 2 * sh.act[k >> 1] + (k & 1);
            __syncthreads();
            const int nn = sh.n_next;
            out_level = l + 1;
            if (nn == 0) {
                out = kFree;
                done = true;
                break;
            }
            // more than max_active stops the search at the next level (or
            // after the last one) before act is read again
            if (nn <= max_active)
                for (int k = tid; k < nn; k += kVT) sh.act[k] = sh.nxt[k];
            __syncthreads();
            na = nn;
        }
        if (!done) {
            out = kUnresolved;
            out_level = max_level;
        }
    } while (false);
    __syncthreads();
    if (tid == 0) {
        if (verdict) verdict[0] = out;
        if (level) level[0] = out_level;
        if (witness) witness[0] = out_t;
        if (labels) labels[e] = out == kFree ? (uint8_t)RGG_GREEN : (uint8_t)RGG_RED;
    }
    __syncthreads();
}

// One wavefront per edge with 14 KB of LDS: about eleven edges are in
// flight per CU.  The search is a chain of dependent phases per edge, so
// edges in flight matter more than threads per edge.
template <int D>
__global__ __launch_bounds__(kVT) __attribute__((amdgpu_waves_per_eu(4))) void k_validate(
    ValDev v, const int64_t *ids, int64_t n, const rgg_update_result *count, int max_level, int max_active,
    uint8_t *verdict, int32_t *level, double *witness, uint8_t *labels)
{
    __shared__ ValShared sh;
    const int tid = threadIdx.x;
    int64_t nn = n;
    if (count) {
        const int64_t g = count->status == RGG_OK ? count->n_gray : 0;
        nn = g < n ? g : n;
    }
    // blocks beyond the list (the grid is sized for its capacity when the
    // count comes from the device) leave at once
    if ((int64_t)blockIdx.x >= nn) return;
    {
        const int32_t *src = reinterpret_cast<const int32_t *>(v.rob);
        int32_t *dst = reinterpret_cast<int32_t *>(&sh.rob);
        for (int k = tid; k < (int)(sizeof(VRobot) / 4); k += kVT) dst[k] = src[k];
    }
    __syncthreads();
    for (int64_t i = blockIdx.x; i < nn; i += gridDim.x) {
        const int64_t e = ids[i];
        if (e < 0 || e >= v.E) {
            if (tid == 0) {
                if (verdict) verdict[i] = RGG_VERDICT_BAD_ID;
                if (level) level[i] = 0;
                if (witness) witness[i] = NAN;
            }
            continue;
        }
        validate_one<D>(sh, v, e, max_level, max_active, verdict ? verdict + i : nullptr, level ? level + i : nullptr,
                        witness ? witness + i : nullptr, labels);
    }
}

}  // namespace

hipError_t launch_validate(const ValDev &v, const int64_t *ids, int64_t n, const rgg_update_result *count,
                           int32_t max_level, int32_t max_active, uint8_t *verdict, int32_t *level,
                           double *witness, uint8_t *labels, hipStream_t s)
{
    if (n <= 0) return hipSuccess;
    const int grid = (int)(n < kVGrid ? n : kVGrid);
    if (v.D == 3)
        k_validate<3><<<grid, kVT, 0, s>>>(v, ids, n, count, max_level, max_active, verdict, level, witness, labels);
    else
        k_validate<2><<<grid, kVT, 0, s>>>(v, ids, n, count, max_level, max_active, verdict, level, witness, labels);
    return hipGetLastError();
}

}  // namespace rgg
