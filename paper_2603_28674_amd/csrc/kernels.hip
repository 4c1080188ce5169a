// Update pipeline of librgg for gfx950 (wave64).
//
// One update = these kernels on one stream (or one graph):
//   k_diff      validate the old/new boxes against the resident slots, list
//               the changed (box, sign) entries in slot order, commit the
//               slots (Alg. 1: a moved obstacle's old and new poses);
//   k_cells     activate every grid cell a changed box overlaps and emit one
//               work item per (cell, chunk of 256 of its edges)  (Sec. 3.3);
//   k_item      one block per work item: pairs of the item's edges with the
//               changed boxes of the cell, outer test (per-sphere capsule vs
//               box), inner test (copies of the spheres whose capsule met),
//               counter update (Sec. 3.1 rule; Alg. 1's intersection lists
//               kept as counts).  In the FP32 mode a pair whose margin falls
//               inside the rounding band is left to
//   k_recheck_pairs   which decides it in binary64; an item whose block ran
//               out of re-test room is run again whole by the binary64 k_item;
//   k_count + k_write   labels from the counters and the ordered gray list.
//
// Binary64 code is compiled without FMA contraction and its sums run left to
// right from 0.0, so a re-test reproduces the definition's values exactly.
// No hot path uses a single global counter: on MI355X device-scope atomics on
// one address serialise across the eight XCDs, so work lists are positional
// and statistics are per-block partial sums.
#include <hip/hip_runtime.h>

#include <type_traits>

#include "rgg_device.h"

namespace rgg {

namespace {

constexpr int kDiffBlock = 1024;
constexpr int kBlock = 256;
constexpr int kWaves = kBlock / 64;
constexpr int kCellsGrid = 128;
constexpr int kGrid = kStatBlocks; // blocks of k_item and k_recheck_pairs

enum : int { kMiss = 0, kHit = 1, kUnsure = 2, kOpen = 3 };

__device__ inline int lane_id() { return __lane_id(); }
__device__ inline uint64_t lanes_below() { return (1ull << lane_id()) - 1ull; }

__device__ inline void wave_sync()
{
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

__device__ inline int wave_prefix(int v, int *total)
{
    // inclusive scan over the wavefront, returned exclusive
    const int lane = lane_id();
    int x = v;
    for (int o = 1; o < 64; o <<= 1) {
        int y = __shfl_up(x, o);
        if (lane >= o) x += y;
    }
    *total = __shfl(x, 63);
    return x - v;
}

__device__ inline float next_down(float f)
{
    uint32_t b = __float_as_uint(f);
    if (f > 0.0f) return __uint_as_float(b - 1u);
    if (f < 0.0f) return __uint_as_float(b + 1u);
    return -__uint_as_float(1u);
}

__device__ inline float round_down(double x)
{
    float f = (float)x;
    return (double)f > x ? next_down(f) : f;
}

__device__ inline float round_up(double x)
{
    float f = (float)x;
    return (double)f < x ? -next_down(-f) : f;
}

__device__ inline int32_t cell_of(double x, double org, double inv, int32_t n)
{
    double c = floor((x - org) * inv);
    if (c < 0.0) return -1;
    if (c >= (double)n) return n;
    return (int32_t)c;
}

__device__ inline bool overlap3(const float *lo, const float *hi, const float4 &bl, const float4 &bh)
{
    return lo[0] <= bh.x && hi[0] >= bl.x && lo[1] <= bh.y && hi[1] >= bl.y && lo[2] <= bh.z &&
           hi[2] >= bl.z;
}

// ------------------------------------------------------------------------
// binary64 predicates: the definition, evaluated in a fixed order
// ------------------------------------------------------------------------

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
template <int D>
__device__ inline double segbox64(const double *A, const double *Bp, const double *lo, const double *hi)
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
        if (fs < fmin) fmin = fs;
    }
    return fmin;
}

// ------------------------------------------------------------------------
// binary32 filter: the same quantities, any rounding; only a margin outside
// the band +-band_rel*s^2 is trusted (s bounds every coordinate of the pair)
// ------------------------------------------------------------------------

template <int D>
__device__ inline float point_box32(const float *c, const float *lo, const float *hi)
{
    float acc = 0.0f;
#pragma unroll
    for (int k = 0; k < D; ++k) {
        float g = fmaxf(fmaxf(lo[k] - c[k], 0.0f), c[k] - hi[k]);
        acc = __builtin_fmaf(g, g, acc);
    }
    return acc;
}

template <int D>
__device__ inline float seg_F32(const float *A, const float *d, float t, const float *lo, const float *hi)
{
    float acc = 0.0f;
#pragma unroll
    for (int k = 0; k < D; ++k) {
        float p = __builtin_fmaf(t, d[k], A[k]);
        float g = fmaxf(fmaxf(lo[k] - p, 0.0f), p - hi[k]);
        acc = __builtin_fmaf(g, g, acc);
    }
    return acc;
}

template <int D>
__device__ inline float segbox32(const float *A, const float *Bp, const float *lo, const float *hi)
{
    float d[D], inv[D];
#pragma unroll
    for (int k = 0; k < D; ++k) {
        d[k] = Bp[k] - A[k];
        inv[k] = d[k] != 0.0f ? __builtin_amdgcn_rcpf(d[k]) : 0.0f;
    }
    float tL = 0.0f, tR = 1.0f;
    auto take = [&](float t) {
        float g = 0.0f;
#pragma unroll
        for (int k = 0; k < D; ++k) {
            float p = __builtin_fmaf(t, d[k], A[k]);
            float ex = fminf(p - lo[k], 0.0f) + fmaxf(p - hi[k], 0.0f);
            g = __builtin_fmaf(d[k], ex, g);
        }
        tL = (g <= 0.0f && t > tL) ? t : tL;
        tR = (g >= 0.0f && t < tR) ? t : tR;
    };
    take(0.0f);
    take(1.0f);
#pragma unroll
    for (int k = 0; k < D; ++k) {
        // a crossing outside (0,1) (or of an axis the segment does not
        // move along) is replaced by t = 0, which repeats the first candidate
        float t1 = (lo[k] - A[k]) * inv[k];
        float t2 = (hi[k] - A[k]) * inv[k];
        take(t1 > 0.0f && t1 < 1.0f ? t1 : 0.0f);
        take(t2 > 0.0f && t2 < 1.0f ? t2 : 0.0f);
    }
    float fmin = fminf(seg_F32<D>(A, d, tL, lo, hi), seg_F32<D>(A, d, tR, lo, hi));
    float tm = 0.5f * (tL + tR);
    float num = 0.0f, den = 0.0f;
#pragma unroll
    for (int k = 0; k < D; ++k) {
        float p = __builtin_fmaf(tm, d[k], A[k]);
        float b = p < lo[k] ? lo[k] : (p > hi[k] ? hi[k] : A[k]);
        float w = (p < lo[k] || p > hi[k]) ? d[k] : 0.0f;
        num = __builtin_fmaf(w, b - A[k], num);
        den = __builtin_fmaf(w, w, den);
    }
    float ts = den > 0.0f ? fminf(fmaxf(num * __builtin_amdgcn_rcpf(den), tL), tR) : tL;
    return fminf(fmin, seg_F32<D>(A, d, ts, lo, hi));
}

__device__ inline int classify_margin(float m, float band)
{
    return m < -band ? kHit : (m > band ? kMiss : kUnsure);
}

// ------------------------------------------------------------------------
// k_diff: validation, changed entries, commit
// ------------------------------------------------------------------------

__device__ inline bool box_ok(const rgg_box &b)
{
    for (int k = 0; k < 3; ++k)
        if (!(fabs(b.lo[k]) <= 1e30) || !(fabs(b.hi[k]) <= 1e30)) return false;
    return true;
}

__device__ inline bool same_box(const rgg_box &a, const rgg_box &b)
{
    bool s = true;
    for (int k = 0; k < 3; ++k)
        s = s && __double_as_longlong(a.lo[k]) == __double_as_longlong(b.lo[k]) &&
            __double_as_longlong(a.hi[k]) == __double_as_longlong(b.hi[k]);
    return s;
}

__device__ inline bool present(const rgg_box &b, int D)
{
    for (int k = 0; k < D; ++k)
        if (b.lo[k] > b.hi[k]) return false;
    return true;
}

__device__ void write_entry(const RmDev &rm, int pos, const rgg_box &b, int sign)
{
    ChgEntry en;
    float s = 0.0f;
    bool empty = false;
    for (int k = 0; k < 3; ++k) {
        if (k < rm.D) {
            en.lo[k] = b.lo[k];
            en.hi[k] = b.hi[k];
            en.lo32[k] = round_down(b.lo[k]);
            en.hi32[k] = round_up(b.hi[k]);
            s = fmaxf(s, fmaxf(fabsf(en.lo32[k]), fabsf(en.hi32[k])));
            int32_t a = cell_of((double)en.lo32[k], rm.gorg[k], rm.ginv, rm.gdim[k]);
            int32_t z = cell_of((double)en.hi32[k], rm.gorg[k], rm.ginv, rm.gdim[k]);
            if (z < 0 || a > rm.gdim[k] - 1) empty = true;
            en.c0[k] = a < 0 ? 0 : a;
            en.c1[k] = z > rm.gdim[k] - 1 ? rm.gdim[k] - 1 : z;
        } else {
            en.lo[k] = en.hi[k] = 0.0;
            en.lo32[k] = en.hi32[k] = 0.0f;
            en.c0[k] = en.c1[k] = 0;
        }
    }
    if (empty) {
        en.c0[0] = 1;
        en.c1[0] = 0;
    }
    en.sbox = s;
    en.sign = sign;
    rm.chg[pos] = en;
}

__global__ void __launch_bounds__(kDiffBlock) k_diff(RmDev rm, const rgg_box *__restrict__ old_b,
                                                     const rgg_box *__restrict__ new_b)
{
    __shared__ int s_tot[kDiffBlock / 64];
    __shared__ int s_bad, s_mism, s_base;
    const int tid = threadIdx.x, lane = lane_id(), wave = tid >> 6;
    if (tid == 0) {
        s_bad = 0;
        s_mism = 0;
        s_base = 0;
        rm.ctl->n_items = 0;
    }
    __syncthreads();
    for (int64_t base = 0; base < rm.M; base += kDiffBlock) {
        const int64_t k = base + tid;
        int cnt = 0;
        bool po = false, pn = false;
        rgg_box o, n;
        if (k < rm.M) {
            o = old_b[k];
            n = new_b[k];
            if (!box_ok(o) || !box_ok(n)) atomicOr(&s_bad, 1);
            if (!same_box(o, rm.resident[k])) atomicOr(&s_mism, 1);
            if (!same_box(o, n)) {
                po = present(o, rm.D);
                pn = present(n, rm.D);
                cnt = (int)po + (int)pn;
            }
        }
        const uint64_t b1 = __ballot(cnt >= 1), b2 = __ballot(cnt >= 2);
        const int pre = __popcll(b1 & lanes_below()) + __popcll(b2 & lanes_below());
        if (lane == 0) s_tot[wave] = __popcll(b1) + __popcll(b2);
        __syncthreads();
        int off = s_base, tot = 0;
        for (int w = 0; w < kDiffBlock / 64; ++w) {
            if (w < wave) off += s_tot[w];
            tot += s_tot[w];
        }
        int pos = off + pre;
        if (po) write_entry(rm, pos++, o, -1);
        if (pn) write_entry(rm, pos, n, +1);
        __syncthreads();
        if (tid == 0) s_base += tot;
        __syncthreads();
    }
    const int status = s_bad ? RGG_E_INVALID_ARG : (s_mism ? RGG_E_STATE_MISMATCH : RGG_OK);
    if (tid == 0) {
        rm.ctl->status = status;
        rm.ctl->n_chg = status ? 0 : s_base;
    }
    if (status == RGG_OK) {
        for (int64_t k = tid; k < rm.M; k += kDiffBlock) {
            rgg_box n = new_b[k];
            if (!same_box(n, rm.resident[k])) rm.resident[k] = n;
        }
    }
}

// ------------------------------------------------------------------------
// k_cells: touched cells -> work items (cell, chunk)
// ------------------------------------------------------------------------

__global__ void __launch_bounds__(kBlock) k_cells(RmDev rm)
{
    const Ctl *ctl = rm.ctl;
    if (ctl->status != RGG_OK) return;
    const int n_chg = ctl->n_chg;
    const int lane = lane_id();
    const int nw = gridDim.x * kWaves;
    for (int q = blockIdx.x * kWaves + (threadIdx.x >> 6); q < n_chg; q += nw) {
        const ChgEntry &en = rm.chg[q];
        const int32_t nx = en.c1[0] - en.c0[0] + 1, ny = en.c1[1] - en.c0[1] + 1,
                      nz = en.c1[2] - en.c0[2] + 1;
        if (nx <= 0 || ny <= 0 || nz <= 0) continue;
        const int64_t total = (int64_t)nx * ny * nz;
        for (int64_t base = 0; base < total; base += 64) {
            const int64_t k = base + lane;
            int64_t c = 0;
            int nch = 0;
            if (k < total) {
                const int32_t x = en.c0[0] + (int32_t)(k % nx);
                const int32_t y = en.c0[1] + (int32_t)((k / nx) % ny);
                const int32_t z = en.c0[2] + (int32_t)(k / ((int64_t)nx * ny));
                c = ((int64_t)z * rm.gdim[1] + y) * rm.gdim[0] + x;
                const uint32_t bit = 1u << (c & 31);
                if (!(atomicOr(&rm.cell_bits[c >> 5], bit) & bit)) {
                    const int32_t n = rm.cell_start[c + 1] - rm.cell_start[c];
                    nch = n > 0 ? (n + rm.chunk - 1) / rm.chunk : 1;
                }
            }
            int tot;
            const int pre = wave_prefix(nch, &tot);
            if (tot == 0) continue;
            int pos0 = 0;
            if (lane == 0) pos0 = atomicAdd(&rm.ctl->n_items, tot);
            pos0 = __shfl(pos0, 0);
            // every winner's items are written by the whole wavefront
            uint64_t wm = __ballot(nch > 0);
            while (wm) {
                const int src = __ffsll((unsigned long long)wm) - 1;
                wm &= wm - 1;
                const int64_t cw = __shfl((long long)c, src);
                const int nw_ = __shfl(nch, src);
                const int pw = pos0 + __shfl(pre, src);
                for (int h = lane; h < nw_; h += 64)
                    if (pw + h < rm.items_cap) rm.items[pw + h] = make_int2((int32_t)cw, h);
            }
        }
    }
}

// ------------------------------------------------------------------------
// block-level helpers
// ------------------------------------------------------------------------

// exclusive prefix of v over the block; *total receives the block sum.
// Contains barriers: every thread must call it.
__device__ inline int block_scan(int v, int *total, int *wsum)
{
    const int lane = lane_id(), wv = threadIdx.x >> 6;
    int wt;
    const int pre = wave_prefix(v, &wt);
    __syncthreads();
    if (lane == 0) wsum[wv] = wt;
    __syncthreads();
    int off = 0, tot = 0;
    for (int w = 0; w < kWaves; ++w) {
        off += w < wv ? wsum[w] : 0;
        tot += wsum[w];
    }
    *total = tot;
    return off + pre;
}

// Adds the counter deltas of one edge as fire-and-forget atomics (no value is
// returned, so they cost no round trip; integer adds commute, so the result
// does not depend on their order).
__device__ inline void add_counts(const RmDev &rm, int64_t e, int dC, int dS)
{
    int *c = reinterpret_cast<int *>(rm.cnt + e);
    if (dC) __hip_atomic_fetch_add(c, dC, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    if (dS) __hip_atomic_fetch_add(c + 1, dS, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

__device__ inline int32_t clamp_cell(double x, double org, double inv, int32_t n)
{
    int32_t c = cell_of(x, org, inv, n);
    return c < 0 ? 0 : (c > n - 1 ? n - 1 : c);
}

// ------------------------------------------------------------------------
// k_item: one block per grid work item (cell c, chunk of 256 of its edges).
//
//   1. every thread owns one edge of the item; the changed entries covering
//      the cell are staged in LDS (tiles of 256); a thread lists the entries
//      whose box meets its edge's box.  With several cells a pair is taken
//      only by the cell holding the lower corner of the two boxes'
//      intersection, so each (edge, entry) pair is tested exactly once.
//   2. outer test, lanes = (pair, sphere): capsule of sphere i against the
//      entry's box (FP32: separation and end-sphere tests first, the exact
//      segment-box minimum where they do not decide).
//   3. inner test, lanes = (pair, sphere whose capsule met, configuration):
//      that sphere's copies against the box.
//   4. per pair C and S; the edge's counter deltas are summed in LDS and
//      added once per edge.  In FP32 a pair whose decision fell inside the
//      rounding band goes to the block's re-test region; if that region is
//      full the whole item is deferred to the binary64 item kernel.
// ------------------------------------------------------------------------

constexpr int kSubTile = 256;   // changed entries staged per tile
constexpr int kPairCap = 512;   // pairs per round (two per thread)
constexpr int kRowCap = 1024;   // (pair, sphere) rows per copy round

template <typename T>
struct ItemLds {
    T lo[3][kSubTile], hi[3][kSubTile];
    float sb[kSubTile];
    int sign[kSubTile], gidx[kSubTile];
    int64_t es0[kBlock];                 // first sample of each edge of the item
    int edge[kBlock], ej[kBlock];        // edge id, configurations per sphere
    float es[kBlock];                    // edge s (largest |coordinate| of its box)
    int dC[kBlock], dS[kBlock];
    uint16_t pe[kPairCap];               // edge slot << 8 | staged entry
    unsigned long long hm[kPairCap], um[kPairCap];
    uint32_t roff[kPairCap], sf[kPairCap];
    uint32_t row[kRowCap];               // pair << 6 | sphere
    uint32_t rcopy[kRowCap + 1];
    int wsum[kWaves];
    int rc_n, rc_start, defer, df_n;
    unsigned long long acc[kStats];
};

template <int D, typename T>
__device__ inline bool pair_owned(const RmDev &rm, const float4 &bl, const T *lo32, int64_t c)
{
    // lower corner of the intersection of the edge box and the entry box
    int64_t cell = 0, mul = 1;
    for (int k = 0; k < D; ++k) {
        const float ek = k == 0 ? bl.x : (k == 1 ? bl.y : bl.z);
        const float x = fmaxf(ek, (float)lo32[k]);
        cell += (int64_t)clamp_cell((double)x, rm.gorg[k], rm.ginv, rm.gdim[k]) * mul;
        mul *= rm.gdim[k];
    }
    return cell == c;
}

template <int D, typename T>
__global__ void __launch_bounds__(kBlock) k_item(RmDev rm, int deferred)
{
    constexpr bool kF32 = std::is_same<T, float>::value;
    __shared__ ItemLds<T> L;
    __shared__ T s_rad2[64];
    const Ctl *ctl = rm.ctl;
    const int tid = threadIdx.x, lane = lane_id(), wv = tid >> 6;
    const int B = rm.B;
    const int Gw = 64 / B, slot = lane / B, ci = lane - slot * B;
    const uint64_t gmask = B == 64 ? ~0ull : ((1ull << B) - 1ull);
    if (tid < kStats) L.acc[tid] = 0;
    if (tid < B) s_rad2[tid] = kF32 ? (T)rm.rad2_32[tid] : (T)(rm.rad64[tid] * rm.rad64[tid]);
    if (tid == 0) {
        L.rc_n = 0;
        L.df_n = 0;
    }
    __syncthreads();
    unsigned long long n_pairs = 0, n_outer = 0, bytes = 0, visited = 0, cand = 0;
    const int status = ctl->status;
    const int n_chg = ctl->n_chg;
    const int n_items = min(ctl->n_items, (int32_t)rm.items_cap);
    const bool single = rm.ncells == 1;
    const float4 *aabb = reinterpret_cast<const float4 *>(rm.aabb);
    const T *capb = kF32 ? (const T *)rm.cap32 : (const T *)rm.cap64;
    const T *samp = kF32 ? (const T *)rm.samp32 : (const T *)rm.samp64;
    const float band_rel = rm.band_rel;
    const int n_list = status != RGG_OK ? 0 : (deferred ? rm.df_cnt[blockIdx.x] : n_items);
    const int first = deferred ? 0 : (int)blockIdx.x, stride = deferred ? 1 : (int)gridDim.x;
    for (int li = first; li < n_list; li += stride) {
        const int it = deferred ? rm.df[(int64_t)blockIdx.x * rm.df_cap + li] : li;
        const int2 item = rm.items[it];
        const int64_t c = item.x;
        const int32_t cx = (int32_t)(c % rm.gdim[0]);
        const int32_t cy = (int32_t)((c / rm.gdim[0]) % rm.gdim[1]);
        const int32_t cz = (int32_t)(c / ((int64_t)rm.gdim[0] * rm.gdim[1]));
        const int64_t beg = (int64_t)rm.cell_start[c] + (int64_t)item.y * rm.chunk;
        const int64_t end = min((int64_t)rm.cell_start[c + 1], beg + rm.chunk);
        const bool have = beg + tid < end;
        int e = 0;
        float4 bl = make_float4(0, 0, 0, 0), bh = bl;
        int64_t s0 = 0;
        int J = 0;
        if (have) {
            e = rm.cell_edges[beg + tid];
            bl = aabb[2 * (int64_t)e];
            bh = aabb[2 * (int64_t)e + 1];
            s0 = rm.p_fixed ? (int64_t)e * rm.p_fixed : rm.soff[e];
            J = (int)((rm.p_fixed ? rm.p_fixed : rm.soff[e + 1] - s0) / B);
            ++visited;
            bytes += 32;
        }
        __syncthreads();
        L.edge[tid] = e;
        L.es[tid] = bl.w;
        L.es0[tid] = s0;
        L.ej[tid] = J;
        L.dC[tid] = 0;
        L.dS[tid] = 0;
        if (tid == 0) {
            L.rc_start = L.rc_n;
            L.defer = 0;
            // the main pass visits every item once: clear the cell's mark with
            // its first chunk, so the next update starts from zero marks
            if (!deferred && item.y == 0) atomicAnd(&rm.cell_bits[c >> 5], ~(1u << (c & 31)));
        }
        int my_pairs = 0;
        for (int j0 = 0; j0 < n_chg; j0 += kSubTile) {
            // stage the entries covering this cell
            const int j = j0 + tid;
            bool in = false;
            if (j < n_chg) {
                const ChgEntry &en = rm.chg[j];
                in = single || (cx >= en.c0[0] && cx <= en.c1[0] && cy >= en.c0[1] && cy <= en.c1[1] &&
                                cz >= en.c0[2] && cz <= en.c1[2]);
            }
            int nt;
            const int pos = block_scan(in ? 1 : 0, &nt, L.wsum);
            if (in) {
                const ChgEntry &en = rm.chg[j];
                for (int k = 0; k < 3; ++k) {
                    L.lo[k][pos] = kF32 ? (T)en.lo32[k] : (T)en.lo[k];
                    L.hi[k][pos] = kF32 ? (T)en.hi32[k] : (T)en.hi[k];
                }
                L.sb[pos] = en.sbox;
                L.sign[pos] = en.sign;
                L.gidx[pos] = j;
            }
            __syncthreads();
            if (nt == 0) continue;
            // pairs of this thread's edge with the staged entries
            auto meets = [&](int s) {
                float lo[3], hi[3];
                if constexpr (kF32) {
                    for (int k = 0; k < 3; ++k) {
                        lo[k] = L.lo[k][s];
                        hi[k] = L.hi[k][s];
                    }
                } else {
                    const ChgEntry &en = rm.chg[L.gidx[s]];
                    for (int k = 0; k < 3; ++k) {
                        lo[k] = en.lo32[k];
                        hi[k] = en.hi32[k];
                    }
                }
                if (!overlap3(lo, hi, bl, bh)) return false;
                return single || pair_owned<D, float>(rm, bl, lo, c);
            };
            // the staged entries this thread's edge meets, as a 256-bit mask
            uint64_t om[kSubTile / 64] = {0, 0, 0, 0};
            int cnt = 0;
            if (have)
                for (int s = 0; s < nt; ++s)
                    if (meets(s)) {
                        om[s >> 6] |= 1ull << (s & 63);
                        ++cnt;
                    }
            my_pairs += cnt;
            int tp;
            const int pre = block_scan(cnt, &tp, L.wsum);
            for (int r0 = 0; r0 < tp; r0 += kPairCap) {
                const int np = min(kPairCap, tp - r0);
                if (cnt > 0 && pre < r0 + np && pre + cnt > r0) {
                    int k = pre;
#pragma unroll
                    for (int w = 0; w < kSubTile / 64; ++w) {
                        uint64_t m = om[w];
                        while (m && k < r0 + np) {
                            const int s = (w << 6) + __ffsll((unsigned long long)m) - 1;
                            m &= m - 1;
                            if (k >= r0) L.pe[k - r0] = (uint16_t)((tid << 8) | s);
                            ++k;
                        }
                    }
                }
                __syncthreads();
                if (tid == 0) n_pairs += np;
                // ---- outer test: lanes = (pair, sphere); each lane takes two
                // pairs per step and issues both capsules' loads first
                constexpr int kCapU = 2;
                for (int p0 = 0; p0 < np; p0 += kWaves * Gw * kCapU) {
                    T A[kCapU][D], Bq[kCapU][D], R2[kCapU];
                    int pu[kCapU];
#pragma unroll
                    for (int u = 0; u < kCapU; ++u) {
                        pu[u] = p0 + (u * kWaves + wv) * Gw + slot;
                        R2[u] = T(0);
                        if (slot < Gw && pu[u] < np) {
                            const int te = L.pe[pu[u]] >> 8;
                            const T *cp = capb + (int64_t)L.edge[te] * (2 * D + 1) * B;
#pragma unroll
                            for (int k = 0; k < D; ++k) {
                                A[u][k] = cp[k * B + ci];
                                Bq[u][k] = cp[(D + k) * B + ci];
                            }
                            R2[u] = cp[2 * D * B + ci];
                        }
                    }
#pragma unroll
                    for (int u = 0; u < kCapU; ++u) {
                        const int p = pu[u];
                        int cls = kMiss;
                        T lo[D], hi[D];
                        float band = 0.0f;
                        const T R = R2[u];
                        const T RR = R * R;
                        if (slot < Gw && p < np) {
                            const int pv = L.pe[p], te = pv >> 8, s = pv & 255;
#pragma unroll
                            for (int k = 0; k < D; ++k) {
                                lo[k] = L.lo[k][s];
                                hi[k] = L.hi[k][s];
                            }
                            if constexpr (kF32) {
                                const float sc = fmaxf(L.es[te], L.sb[s]);
                                band = band_rel * sc * sc;
                                float sep = 0.0f;
#pragma unroll
                                for (int k = 0; k < D; ++k)
                                    sep = fmaxf(sep, fmaxf(lo[k] - fmaxf(A[u][k], Bq[u][k]), fminf(A[u][k], Bq[u][k]) - hi[k]));
                                const float m_end = fminf(point_box32<D>(A[u], lo, hi), point_box32<D>(Bq[u], lo, hi)) - RR;
                                cls = (sep > 0.0f && sep * sep - RR > band) ? kMiss : (m_end < -band ? kHit : kOpen);
                            } else {
                                cls = segbox64<D>(A[u], Bq[u], lo, hi) <= RR ? kHit : kMiss;
                            }
                        }
                        if constexpr (kF32) {
                            if (__ballot(cls == kOpen)) {
                                if (cls == kOpen) cls = classify_margin(segbox32<D>(A[u], Bq[u], lo, hi) - RR, band);
                            }
                        }
                        const uint64_t hmw = __ballot(cls == kHit), umw = __ballot(cls == kUnsure);
                        if (slot < Gw && ci == 0 && p < np) {
                            L.hm[p] = (hmw >> (slot * B)) & gmask;
                            L.um[p] = (umw >> (slot * B)) & gmask;
                        }
                    }
                }
                __syncthreads();
                // ---- rows: one per (pair, sphere whose capsule met)
                const int pa = tid, pb = tid + kBlock;
                const int ra = pa < np ? __popcll(L.hm[pa]) : 0;
                const int rb = pb < np ? __popcll(L.hm[pb]) : 0;
                int nrows;
                const int rpre = block_scan(ra + rb, &nrows, L.wsum);
                if (pa < np) {
                    L.roff[pa] = rpre;
                    L.sf[pa] = 0;
                }
                if (pb < np) {
                    L.roff[pb] = rpre + ra;
                    L.sf[pb] = 0;
                }
                __syncthreads();
                for (int q0 = 0; q0 < nrows; q0 += kRowCap) {
                    const int nr = min(kRowCap, nrows - q0);
                    for (int h = 0; h < 2; ++h) {
                        const int p = tid + h * kBlock;
                        if (p >= np) continue;
                        uint64_t m = L.hm[p];
                        int r = L.roff[p];
                        while (m && r < q0 + nr) {
                            const int i = __ffsll((unsigned long long)m) - 1;
                            m &= m - 1;
                            if (r >= q0) L.row[r - q0] = ((uint32_t)p << 6) | (uint32_t)i;
                            ++r;
                        }
                    }
                    __syncthreads();
                    // copies of each row: fixed count, or a scan over the rows
                    const int jfix = rm.p_fixed ? rm.p_fixed / B : 0;
                    int ncopies = nr * jfix;
                    if (!jfix) {
                        int cj[4], sum = 0;
                        for (int h = 0; h < 4; ++h) {
                            const int r = tid * 4 + h;
                            cj[h] = r < nr ? L.ej[L.pe[L.row[r] >> 6] >> 8] : 0;
                            sum += cj[h];
                        }
                        const int cpre = block_scan(sum, &ncopies, L.wsum);
                        int acc = cpre;
                        for (int h = 0; h < 4; ++h) {
                            const int r = tid * 4 + h;
                            if (r < nr) L.rcopy[r] = acc;
                            acc += cj[h];
                        }
                        if (tid == 0) L.rcopy[nr] = ncopies;
                        __syncthreads();
                    }
                    // each thread gathers kCopyU copies (all their loads in
                    // flight together), then tests them
                    constexpr int kCopyU = 4;
                    for (int c0 = 0; c0 < ncopies; c0 += kBlock * kCopyU) {
                        T q[kCopyU][D];
                        int cu_p[kCopyU], cu_i[kCopyU];
#pragma unroll
                        for (int u = 0; u < kCopyU; ++u) {
                            const int cidx = c0 + u * kBlock + tid;
                            cu_p[u] = -1;
                            cu_i[u] = 0;
                            if (cidx < ncopies) {
                                int r, jj;
                                if (jfix) {
                                    r = cidx / jfix;
                                    jj = cidx - r * jfix;
                                } else {
                                    int lo_ = 0, hi_ = nr - 1;   // last row with rcopy[r] <= cidx
                                    while (lo_ < hi_) {
                                        const int mid = (lo_ + hi_ + 1) >> 1;
                                        if (L.rcopy[mid] <= (uint32_t)cidx) lo_ = mid;
                                        else hi_ = mid - 1;
                                    }
                                    r = lo_;
                                    jj = cidx - (int)L.rcopy[r];
                                }
                                const uint32_t rv = L.row[r];
                                const int p = (int)(rv >> 6);
                                const int i = (int)(rv & 63u);
                                const int te = L.pe[p] >> 8;
                                const int Je = L.ej[te];
                                const int64_t P = (int64_t)Je * B;
                                const T *sb = samp + D * L.es0[te] + (int64_t)i * Je + jj;
#pragma unroll
                                for (int k = 0; k < D; ++k) q[u][k] = sb[k * P];
                                cu_p[u] = p;
                                cu_i[u] = i;
                            }
                        }
#pragma unroll
                        for (int u = 0; u < kCopyU; ++u) {
                            const int p = cu_p[u];
                            if (p < 0) continue;
                            const int pv = L.pe[p], te = pv >> 8, s = pv & 255;
                            T lo[D], hi[D];
#pragma unroll
                            for (int k = 0; k < D; ++k) {
                                lo[k] = L.lo[k][s];
                                hi[k] = L.hi[k][s];
                            }
                            bytes += D * sizeof(T);
                            int cls;
                            if constexpr (kF32) {
                                const float sc = fmaxf(L.es[te], L.sb[s]);
                                cls = classify_margin(point_box32<D>(q[u], lo, hi) - s_rad2[cu_i[u]], band_rel * sc * sc);
                            } else {
                                cls = point_box64<D>(q[u], lo, hi) <= s_rad2[cu_i[u]] ? kHit : kMiss;
                            }
                            if (cls == kHit) atomicOr(&L.sf[p], 1u);
                            else if (cls == kUnsure) atomicOr(&L.sf[p], 2u);
                        }
                    }
                    __syncthreads();
                }
                // ---- decisions
                int unsure_n = 0;
                int2 rec0 = make_int2(0, 0), rec1 = make_int2(0, 0);   // registers, not a local array
                for (int h = 0; h < 2; ++h) {
                    const int p = tid + h * kBlock;
                    if (p >= np) continue;
                    const uint64_t hmp = L.hm[p], ump = kF32 ? L.um[p] : 0ull;
                    if (!hmp && !ump) continue;
                    const uint32_t f = L.sf[p];
                    const int pv = L.pe[p], te = pv >> 8, s = pv & 255;
                    const bool unsure = kF32 && (!hmp || (!(f & 1u) && ((f & 2u) || ump)));
                    if (unsure) {
                        const int2 r = make_int2(L.edge[te], L.gidx[s]);
                        if (unsure_n == 0) rec0 = r;
                        else rec1 = r;
                        ++unsure_n;
                    } else {
                        const int sign = L.sign[s];
                        atomicAdd(&L.dC[te], sign);
                        if (f & 1u) atomicAdd(&L.dS[te], sign);
                        ++n_outer;
                    }
                }
                if constexpr (kF32) {
                    int tot_u;
                    const int upre = block_scan(unsure_n, &tot_u, L.wsum);
                    if (tot_u > 0) {
                        const int base = L.rc_n;
                        const bool fits = !L.defer && base + tot_u <= rm.rc_cap;
                        if (fits) {
                            int2 *dst = rm.rc + (int64_t)blockIdx.x * rm.rc_cap + base + upre;
                            if (unsure_n > 0) dst[0] = rec0;
                            if (unsure_n > 1) dst[1] = rec1;
                        }
                        __syncthreads();
                        if (tid == 0) {
                            if (fits) L.rc_n = base + tot_u;
                            else L.defer = 1;
                        }
                    }
                }
                __syncthreads();
            }
        }
        if (have && my_pairs > 0) {
            ++cand;
            bytes += (2 * D + 1) * B * sizeof(T) + 16;
        }
        __syncthreads();
        if (!L.defer) {
            if (have) add_counts(rm, e, L.dC[tid], L.dS[tid]);
        } else if (tid == 0) {
            L.rc_n = L.rc_start;
            rm.df[(int64_t)blockIdx.x * rm.df_cap + L.df_n] = it;
            L.df_n += 1;
        }
    }
    __syncthreads();
    atomicAdd(&L.acc[0], n_pairs);
    atomicAdd(&L.acc[1], n_outer);
    atomicAdd(&L.acc[3], bytes);
    atomicAdd(&L.acc[4], visited);
    atomicAdd(&L.acc[5], cand);
    __syncthreads();
    if (tid == 0) {
        unsigned long long *bs = rm.blk_stats + blockIdx.x * kStats;
        if (!deferred) {
            bs[0] = L.acc[0];
            bs[1] = L.acc[1];
            bs[2] = 0;
            bs[3] = L.acc[3];
            bs[4] = L.acc[4];
            bs[5] = L.acc[5];
            if (kF32) {
                rm.rc_cnt[blockIdx.x] = L.rc_n;
                rm.df_cnt[blockIdx.x] = L.df_n;
            }
        } else {
            bs[1] += L.acc[1];
            bs[2] += L.acc[0];
            bs[3] += L.acc[3];
        }
    }
}

// ------------------------------------------------------------------------
// k_recheck_pairs: binary64 decision of every pair an FP32 block left unsure
// (the definition: C = some capsule meets, S = some sphere's capsule and one
// of its copies meet), one wavefront per pair
// ------------------------------------------------------------------------

struct CopyMap {
    int J, jw, spc, sub, jj;
};

__device__ inline CopyMap copy_map(int J)
{
    CopyMap c;
    c.J = J;
    c.jw = J < 64 ? J : 64;
    c.spc = 64 / c.jw;
    c.sub = lane_id() / c.jw;
    c.jj = lane_id() - c.sub * c.jw;
    return c;
}

template <int D>
__device__ bool copies_meet64(const RmDev &rm, const double *sb, int64_t P, const CopyMap &cm, uint64_t m,
                              const double *lo, const double *hi, const double *rad, int *lst,
                              unsigned long long *bytes)
{
    const int lane = lane_id();
    if (lane < rm.B && ((m >> lane) & 1ull)) lst[__popcll(m & lanes_below())] = lane;
    wave_sync();
    const int nsph = __popcll(m);
    for (int sp0 = 0; sp0 < nsph; sp0 += cm.spc) {
        for (int j0 = 0; j0 < cm.J; j0 += cm.jw) {
            const int js = j0 + cm.jj;
            const bool valid = cm.sub < cm.spc && sp0 + cm.sub < nsph && js < cm.J;
            bool hit = false;
            if (valid) {
                const int i = lst[sp0 + cm.sub];
                double p[D];
#pragma unroll
                for (int k = 0; k < D; ++k) p[k] = sb[k * P + (int64_t)i * cm.J + js];
                const double r = rad[i];
                hit = point_box64<D>(p, lo, hi) <= r * r;
            }
            *bytes += (unsigned long long)(__popcll(__ballot(valid)) * D * 8);
            if (__ballot(hit)) {
                wave_sync();
                return true;
            }
        }
    }
    wave_sync();
    return false;
}

template <int D>
__global__ void __launch_bounds__(kBlock) k_recheck_pairs(RmDev rm)
{
    __shared__ int s_lst[kWaves][64];
    __shared__ double s_rad[64];
    __shared__ unsigned long long s_acc[3];
    const Ctl *ctl = rm.ctl;
    const int lane = lane_id(), wv = threadIdx.x >> 6;
    if (threadIdx.x < rm.B) s_rad[threadIdx.x] = rm.rad64[threadIdx.x];
    if (threadIdx.x < 3) s_acc[threadIdx.x] = 0;
    __syncthreads();
    unsigned long long n_re = 0, n_outer = 0, bytes = 0;
    const int n = ctl->status == RGG_OK ? rm.rc_cnt[blockIdx.x] : 0;
    const int B = rm.B;
    for (int k = wv; k < n; k += kWaves) {
        const int2 pr = rm.rc[(int64_t)blockIdx.x * rm.rc_cap + k];
        const int64_t e = pr.x;
        const ChgEntry &en = rm.chg[pr.y];
        double lo[D], hi[D];
#pragma unroll
        for (int d = 0; d < D; ++d) {
            lo[d] = en.lo[d];
            hi[d] = en.hi[d];
        }
        bool hit = false;
        if (lane < B) {
            const double *cp = rm.cap64 + e * (2 * D + 1) * B;
            double A[D], Bp[D];
#pragma unroll
            for (int d = 0; d < D; ++d) {
                A[d] = cp[d * B + lane];
                Bp[d] = cp[(D + d) * B + lane];
            }
            const double R = cp[2 * D * B + lane];
            hit = segbox64<D>(A, Bp, lo, hi) <= R * R;
        }
        const uint64_t hm = __ballot(hit);
        bytes += (2 * D + 1) * B * 8;
        ++n_re;
        if (!hm) continue;
        const int64_t s0 = rm.p_fixed ? e * rm.p_fixed : rm.soff[e];
        const int64_t P = rm.p_fixed ? rm.p_fixed : rm.soff[e + 1] - s0;
        const CopyMap cm = copy_map((int)(P / B));
        const bool S = copies_meet64<D>(rm, rm.samp64 + D * s0, P, cm, hm, lo, hi, s_rad, s_lst[wv], &bytes);
        ++n_outer;
        if (lane == 0) add_counts(rm, e, en.sign, S ? en.sign : 0);
    }
    if (lane == 0) {
        atomicAdd(&s_acc[0], n_re);
        atomicAdd(&s_acc[1], n_outer);
        atomicAdd(&s_acc[2], bytes);
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        unsigned long long *bs = rm.blk_stats + blockIdx.x * kStats;
        bs[1] += s_acc[1];
        bs[2] += s_acc[0];
        bs[3] += s_acc[2];
    }
}
// ------------------------------------------------------------------------
// labels and the ordered gray list
// ------------------------------------------------------------------------

__device__ inline uint8_t label_of(int2 c)
{
    return c.y > 0 ? (uint8_t)RGG_RED : (c.x == 0 ? (uint8_t)RGG_GREEN : (uint8_t)RGG_GRAY);
}

__device__ inline int block_sum(int v, int *s_w)
{
    for (int o = 32; o > 0; o >>= 1) v += __shfl_down(v, o);
    const int lane = lane_id(), wv = threadIdx.x >> 6;
    __syncthreads();
    if (lane == 0) s_w[wv] = v;
    __syncthreads();
    int t = 0;
    for (int w = 0; w < kWaves; ++w) t += s_w[w];
    return t;
}

__global__ void __launch_bounds__(kBlock) k_count(RmDev rm, uint8_t *labels,
                                                  rgg_update_result *res, int force)
{
    __shared__ int s_w[kWaves];
    const int status = force ? RGG_OK : rm.ctl->status;
    const int64_t t0 = (int64_t)blockIdx.x * kLabelTile;
    int ng = 0;
    for (int it = 0; it < kLabelTile / kBlock; ++it) {
        const int64_t e = t0 + it * kBlock + threadIdx.x;
        if (e < rm.E) {
            const uint8_t lab = label_of(rm.cnt[e]);
            if (status == RGG_OK && labels) labels[e] = lab;
            ng += lab == RGG_GRAY;
        }
    }
    const int64_t nwords = (rm.E + 31) / 32;
    if (threadIdx.x < kLabelTile / 32) {
        const int64_t w = t0 / 32 + threadIdx.x;
        if (w < nwords) rm.edge_bits[w] = 0u;
    }
    const int tot = block_sum(ng, s_w);
    if (threadIdx.x == 0) {
        rm.tile_cnt[blockIdx.x] = tot;
        if (blockIdx.x == 0 && res && !force) {
            res->status = status;
            res->n_changed = rm.ctl->n_chg;
        }
    }
}

__global__ void __launch_bounds__(kBlock) k_write(RmDev rm, int64_t *gray, int64_t cap,
                                                  rgg_update_result *res, int force)
{
    __shared__ int s_w[kWaves];
    __shared__ int s_wt[kWaves];
    __shared__ unsigned long long s_st[kStats];
    const int status = force ? RGG_OK : rm.ctl->status;
    const int tid = threadIdx.x, lane = lane_id(), wv = tid >> 6;
    int pre = 0;
    for (int j = tid; j < (int)blockIdx.x; j += kBlock) pre += rm.tile_cnt[j];
    int64_t off = block_sum(pre, s_w);
    const int64_t t0 = (int64_t)blockIdx.x * kLabelTile;
    for (int it = 0; it < kLabelTile / kBlock; ++it) {
        const int64_t e = t0 + it * kBlock + tid;
        const bool g = e < rm.E && label_of(rm.cnt[e]) == RGG_GRAY;
        const uint64_t m = __ballot(g);
        __syncthreads();
        if (lane == 0) s_wt[wv] = __popcll(m);
        __syncthreads();
        int64_t woff = off;
        int tot = 0;
        for (int w = 0; w < kWaves; ++w) {
            if (w < wv) woff += s_wt[w];
            tot += s_wt[w];
        }
        const int64_t pos = woff + __popcll(m & lanes_below());
        if (g && status == RGG_OK && gray && pos < cap) gray[pos] = e;
        off += tot;
    }
    if (blockIdx.x != gridDim.x - 1 || !res) return;
    if (force) {
        if (tid == 0) res->n_gray = off;
        return;
    }
    // the last block also folds the per-block statistics
    if (tid < kStats) s_st[tid] = 0;
    __syncthreads();
    unsigned long long acc[kStats] = {0, 0, 0, 0, 0, 0};
    for (int b = tid; b < kStatBlocks; b += kBlock)
        for (int k = 0; k < kStats; ++k) acc[k] += rm.blk_stats[b * kStats + k];
    for (int k = 0; k < kStats; ++k) atomicAdd(&s_st[k], acc[k]);
    __syncthreads();
    if (tid == 0) {
        res->n_gray = status == RGG_OK ? off : 0;
        res->n_pairs = (int64_t)s_st[0];
        res->n_outer_hits = (int64_t)s_st[1];
        res->n_rechecked = (int64_t)s_st[2];
        res->test_bytes = (int64_t)s_st[3];
        res->n_cells_visited = (int64_t)s_st[4];
        res->n_candidate_edges = (int64_t)s_st[5];
    }
}

}  // namespace

namespace {

void *item_fn(const RmDev &rm, bool f64)
{
    if (rm.D == 3) return f64 ? (void *)k_item<3, double> : (void *)k_item<3, float>;
    return f64 ? (void *)k_item<2, double> : (void *)k_item<2, float>;
}

void *recheck_fn(const RmDev &rm)
{
    return rm.D == 3 ? (void *)k_recheck_pairs<3> : (void *)k_recheck_pairs<2>;
}

struct Node {
    void *fn;
    dim3 grid, block;
    int kind;   // 0 diff, 1 rm only, 2 item (deferred flag), 3 count, 4 write
    int flag;
};

// the kernels of one update, in order; stage boundaries for the events after
// the indices listed in `marks`
int plan(const RmDev &rm, Node out[8])
{
    int n = 0;
    out[n++] = {(void *)k_diff, dim3(1), dim3(kDiffBlock), 0, 0};
    out[n++] = {(void *)k_cells, dim3(kCellsGrid), dim3(kBlock), 1, 0};
    out[n++] = {item_fn(rm, !rm.mixed), dim3(kGrid), dim3(kBlock), 2, 0};
    if (rm.mixed) {
        out[n++] = {recheck_fn(rm), dim3(kGrid), dim3(kBlock), 1, 0};
        out[n++] = {item_fn(rm, true), dim3(kGrid), dim3(kBlock), 2, 1};
    }
    out[n++] = {(void *)k_count, dim3(rm.ntiles), dim3(kBlock), 3, 0};
    out[n++] = {(void *)k_write, dim3(rm.ntiles), dim3(kBlock), 4, 0};
    return n;
}

}  // namespace

hipError_t launch_update(const RmDev &rm, const UpdateArgs &a, hipStream_t s, hipEvent_t *ev)
{
    if (rm.chunk != kBlock) return hipErrorInvalidValue;   // one edge of an item per thread
    Node nodes[8];
    const int n = plan(rm, nodes);
    hipError_t err;
    RmDev r = rm;
    const rgg_box *ob = a.old_b, *nb = a.new_b;
    uint8_t *lab = a.labels;
    int64_t *gray = a.gray;
    int64_t cap = a.gray_cap;
    rgg_update_result *res = a.res;
    int zero = 0, one = 1;
    if (ev && (err = hipEventRecord(ev[0], s)) != hipSuccess) return err;
    for (int k = 0; k < n; ++k) {
        void *args_diff[] = {&r, (void *)&ob, (void *)&nb};
        void *args_one[] = {&r};
        void *args_item[] = {&r, nodes[k].flag ? (void *)&one : (void *)&zero};
        void *args_count[] = {&r, &lab, &res, &zero};
        void *args_write[] = {&r, &gray, &cap, &res, &zero};
        void **args = nodes[k].kind == 0 ? args_diff
                    : nodes[k].kind == 1 ? args_one
                    : nodes[k].kind == 2 ? args_item
                    : nodes[k].kind == 3 ? args_count
                                         : args_write;
        if ((err = hipLaunchKernel(nodes[k].fn, nodes[k].grid, nodes[k].block, args, 0, s)) != hipSuccess) return err;
        if (ev) {
            // ev[1] after diff, ev[2] after cells, ev[3] == ev[2] (the grid scan is
            // part of the item kernel), ev[4] after the item kernel, ev[5] after
            // the binary64 re-test, ev[6] after the labels
            int mark = -1;
            if (k == 0) mark = 1;
            if (k == 1) mark = 2;
            if (k == 2) mark = 4;
            if (nodes[k].kind == 2 && nodes[k].flag) mark = 5;
            if (!rm.mixed && k == 2) mark = 4;
            if (mark == 2) {
                if ((err = hipEventRecord(ev[2], s)) != hipSuccess) return err;
                mark = 3;
            }
            if (mark == 4 && !rm.mixed) {
                if ((err = hipEventRecord(ev[4], s)) != hipSuccess) return err;
                mark = 5;
            }
            if (mark >= 0 && (err = hipEventRecord(ev[mark], s)) != hipSuccess) return err;
        }
    }
    if (ev && (err = hipEventRecord(ev[6], s)) != hipSuccess) return err;
    return hipSuccess;
}

hipError_t launch_labels(const RmDev &rm, const UpdateArgs &a, hipStream_t s)
{
    k_count<<<rm.ntiles, kBlock, 0, s>>>(rm, a.labels, a.res, 1);
    hipError_t err = hipGetLastError();
    if (err != hipSuccess) return err;
    k_write<<<rm.ntiles, kBlock, 0, s>>>(rm, a.gray, a.gray_cap, a.res, 1);
    return hipGetLastError();
}

hipError_t add_update_nodes(hipGraph_t g, const RmDev &rm, const UpdateArgs &a, hipGraphNode_t dep,
                            hipGraphNode_t *last)
{
    if (rm.chunk != kBlock) return hipErrorInvalidValue;
    Node nodes[8];
    const int n = plan(rm, nodes);
    // argument storage: hipGraphAddKernelNode copies the values
    RmDev r = rm;
    const rgg_box *ob = a.old_b, *nb = a.new_b;
    uint8_t *lab = a.labels;
    int64_t *gray = a.gray;
    int64_t cap = a.gray_cap;
    rgg_update_result *res = a.res;
    int zero = 0, one = 1;
    hipGraphNode_t prev = dep;
    for (int k = 0; k < n; ++k) {
        void *args_diff[] = {&r, (void *)&ob, (void *)&nb};
        void *args_one[] = {&r};
        void *args_item[] = {&r, nodes[k].flag ? (void *)&one : (void *)&zero};
        void *args_count[] = {&r, &lab, &res, &zero};
        void *args_write[] = {&r, &gray, &cap, &res, &zero};
        void **args = nodes[k].kind == 0 ? args_diff
                    : nodes[k].kind == 1 ? args_one
                    : nodes[k].kind == 2 ? args_item
                    : nodes[k].kind == 3 ? args_count
                                         : args_write;
        hipKernelNodeParams p = {};
        p.func = nodes[k].fn;
        p.gridDim = nodes[k].grid;
        p.blockDim = nodes[k].block;
        p.sharedMemBytes = 0;
        p.kernelParams = args;
        p.extra = nullptr;
        hipGraphNode_t node;
        hipError_t err = hipGraphAddKernelNode(&node, g, prev ? &prev : nullptr, prev ? 1 : 0, &p);
        if (err != hipSuccess) return err;
        prev = node;
    }
    *last = prev;
    return hipSuccess;
}

}  // namespace rgg
