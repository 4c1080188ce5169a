// Update pipeline of librgg for gfx950 (wave64).
//
// One update = up to seven kernels on one stream:
//   k_diff      validate the old/new boxes against the resident slots, list
//               the changed (box, sign) entries in slot order, commit the
//               slots (Alg. 1: a moved obstacle's old and new poses);
//   k_cells     activate every grid cell a changed box overlaps and emit one
//               work item per (cell, chunk of its edge list)  (Sec. 3.3 grid);
//   k_grid      per item, keep the edges whose box meets a changed box of that
//               cell; candidates are written in place, no global counter;
//   k_classify  one wavefront per candidate edge: outer test (per-sphere
//               capsule vs box), inner test (sphere samples vs box, stopping at
//               the first hit), counter update (Sec. 3.1 rule; Alg. 1's
//               intersection lists kept as counts).  In the FP32 mode a pair
//               whose margin falls inside the rounding band is left to
//   k_recheck   which re-decides it in binary64;
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
constexpr int kTile = 256;         // changed entries staged in LDS per pass
constexpr int kSubCap = 1024;      // entries of one cell staged by k_grid
constexpr int kCellsGrid = 128;
constexpr int kGrid = kStatBlocks; // blocks of k_grid, k_classify, k_recheck

enum : int { kMiss = 0, kHit = 1, kUnsure = 2, kOpen = 3 };
enum : uint8_t { kCHit = 1, kCUnsure = 2, kSHit = 4, kSUnsure = 8 };

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
// k_grid: scan the edges of each item, keep those meeting a changed box
// ------------------------------------------------------------------------

__global__ void __launch_bounds__(kBlock) k_grid(RmDev rm)
{
    __shared__ float s_lo[3][kSubCap], s_hi[3][kSubCap];
    __shared__ int s_n, s_w[kWaves];
    const Ctl *ctl = rm.ctl;
    unsigned long long visited = 0;
    if (ctl->status == RGG_OK) {
        const int n_items = min(ctl->n_items, (int32_t)rm.items_cap);
        const int n_chg = ctl->n_chg;
        const int tid = threadIdx.x, lane = lane_id(), wv = tid >> 6;
        const bool single = rm.ncells == 1;
        const float4 *aabb = reinterpret_cast<const float4 *>(rm.aabb);
        for (int it = blockIdx.x; it < n_items; it += gridDim.x) {
            const int2 item = rm.items[it];
            const int64_t c = item.x;
            const int32_t cx = (int32_t)(c % rm.gdim[0]);
            const int32_t cy = (int32_t)((c / rm.gdim[0]) % rm.gdim[1]);
            const int32_t cz = (int32_t)(c / ((int64_t)rm.gdim[0] * rm.gdim[1]));
            __syncthreads();
            if (tid == 0) {
                s_n = 0;
                if (item.y == 0) atomicAnd(&rm.cell_bits[c >> 5], ~(1u << (c & 31)));
            }
            __syncthreads();
            // the changed entries whose cell range contains this cell
            for (int j0 = 0; j0 < n_chg; j0 += kBlock) {
                const int j = j0 + tid;
                bool in = false;
                if (j < n_chg) {
                    const ChgEntry &en = rm.chg[j];
                    in = single || (cx >= en.c0[0] && cx <= en.c1[0] && cy >= en.c0[1] &&
                                    cy <= en.c1[1] && cz >= en.c0[2] && cz <= en.c1[2]);
                }
                const uint64_t m = __ballot(in);
                if (lane == 0) s_w[wv] = __popcll(m);
                __syncthreads();
                int off = s_n, tot = 0;
                for (int w = 0; w < kWaves; ++w) {
                    off += w < wv ? s_w[w] : 0;
                    tot += s_w[w];
                }
                const int s = off + __popcll(m & lanes_below());
                if (in && s < kSubCap) {
                    const ChgEntry &en = rm.chg[j];
                    for (int k = 0; k < 3; ++k) {
                        s_lo[k][s] = en.lo32[k];
                        s_hi[k][s] = en.hi32[k];
                    }
                }
                __syncthreads();
                if (tid == 0) s_n += tot;
                __syncthreads();
            }
            const int ns = s_n;
            const int64_t beg = (int64_t)rm.cell_start[c] + (int64_t)item.y * rm.chunk;
            const int64_t end = min((int64_t)rm.cell_start[c + 1], beg + rm.chunk);
            // one edge per thread (chunk == block size)
            const int64_t j = beg + tid;
            bool keep = false;
            int32_t e = 0;
            if (j < end) {
                e = rm.cell_edges[j];
                const float4 bl = aabb[2 * (int64_t)e], bh = aabb[2 * (int64_t)e + 1];
                bool hit = false;
                if (ns <= kSubCap) {
                    for (int s = 0; s < ns && !hit; ++s) {
                        const float lo[3] = {s_lo[0][s], s_lo[1][s], s_lo[2][s]};
                        const float hi[3] = {s_hi[0][s], s_hi[1][s], s_hi[2][s]};
                        hit = overlap3(lo, hi, bl, bh);
                    }
                } else {
                    for (int s = 0; s < n_chg && !hit; ++s) {
                        const ChgEntry &en = rm.chg[s];
                        hit = (single || (cx >= en.c0[0] && cx <= en.c1[0] && cy >= en.c0[1] &&
                                          cy <= en.c1[1] && cz >= en.c0[2] && cz <= en.c1[2])) &&
                              overlap3(en.lo32, en.hi32, bl, bh);
                    }
                }
                if (hit) {
                    if (single) {
                        keep = true;
                    } else {   // an edge registered in several active cells is kept once
                        const uint32_t bit = 1u << (e & 31);
                        keep = !(atomicOr(&rm.edge_bits[e >> 5], bit) & bit);
                    }
                }
            }
            const uint64_t m = __ballot(keep);
            if (lane == 0) s_w[wv] = __popcll(m);
            __syncthreads();
            int off = 0, tot = 0;
            for (int w = 0; w < kWaves; ++w) {
                off += w < wv ? s_w[w] : 0;
                tot += s_w[w];
            }
            if (keep) rm.work[beg + off + __popcll(m & lanes_below())] = e;
            if (tid == 0) {
                rm.item_cnt[it] = tot;
                visited += (unsigned long long)max((int64_t)0, end - beg);
            }
        }
    }
    if (threadIdx.x == 0) rm.blk_stats[blockIdx.x * kStats + 4] = visited;
}

// ------------------------------------------------------------------------
// candidates of one block: items it = blockIdx.x, + gridDim.x, ...; within
// an item the wavefronts take candidates wv, wv + kWaves, ...
// ------------------------------------------------------------------------

struct Cursor {
    int it, k, cnt;
    int64_t beg;
};

__device__ inline bool cursor_next(const RmDev &rm, int n_items, Cursor &cu, int wv, int64_t *slot)
{
    for (;;) {
        if (cu.it >= n_items) return false;
        if (cu.k < 0) {
            const int2 item = rm.items[cu.it];
            cu.cnt = rm.item_cnt[cu.it];
            cu.beg = (int64_t)rm.cell_start[item.x] + (int64_t)item.y * rm.chunk;
            cu.k = wv;
        }
        if (cu.k < cu.cnt) {
            *slot = cu.beg + cu.k;
            cu.k += kWaves;
            return true;
        }
        cu.it += gridDim.x;
        cu.k = -1;
    }
}

// Adds the counter deltas of one edge.  Each edge is owned by one wavefront
// within a kernel, so the adds need no returned value: they are issued as
// fire-and-forget atomics and cost no round trip.
__device__ inline void add_counts(const RmDev &rm, int64_t e, int dC, int dS)
{
    int *c = reinterpret_cast<int *>(rm.cnt + e);
    if (dC) __hip_atomic_fetch_add(c, dC, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    if (dS) __hip_atomic_fetch_add(c + 1, dS, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// ------------------------------------------------------------------------
// per-wavefront LDS scratch of the classify kernels
// ------------------------------------------------------------------------

struct WaveScratch {
    int act[kTile];   // staged-entry index of each pair of the current edge
    int lst[64];      // sphere indices whose copies are tested
};

// Lane mapping of the copies of up to 64/jw spheres onto one wavefront:
// lane -> (sub = lane / jw, jj = lane % jw), jw = min(J, 64) configurations.
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

// writes the indices of the set bits of m (wave-uniform, bits < B) to lst
__device__ inline int list_spheres(uint64_t m, int B, int *lst)
{
    const int lane = lane_id();
    if (lane < B && ((m >> lane) & 1ull)) lst[__popcll(m & lanes_below())] = lane;
    wave_sync();
    return __popcll(m);
}

// ------------------------------------------------------------------------
// binary64 classification of one edge against entries [t0, t0+nt): the
// definition, sphere by sphere (C: some capsule meets the box; S: for some
// sphere, its capsule and one of its copies meet the box).  Used by the FP64
// mode and by the re-test of the FP32 mode; every lane returns the same
// counter deltas.
// ------------------------------------------------------------------------

template <int D>
__device__ bool copies_meet64(const RmDev &rm, const double *sb, int64_t P, const CopyMap &cm,
                              uint64_t m, const double *lo, const double *hi, const double *rad,
                              int *lst, unsigned long long *bytes)
{
    const int nsph = list_spheres(m, rm.B, lst);
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
            if (__ballot(hit)) return true;
        }
    }
    return false;
}

template <int D>
__device__ int2 edge_exact(const RmDev &rm, int64_t e, const ChgEntry *__restrict__ chg, int t0, int nt,
                           WaveScratch &ws, const double *rad, unsigned long long *n_pairs,
                           unsigned long long *n_outer, unsigned long long *bytes)
{
    const int lane = lane_id(), B = rm.B;
    const int G = 64 / B, slot = lane / B, ci = lane - slot * B;
    const uint64_t gmask = B == 64 ? ~0ull : ((1ull << B) - 1ull);
    const float4 *aabb = reinterpret_cast<const float4 *>(rm.aabb);
    const float4 bl = aabb[2 * e], bh = aabb[2 * e + 1];
    int n_act = 0;
    for (int b0 = 0; b0 < nt; b0 += 64) {
        const int j = b0 + lane;
        const bool ov = j < nt && overlap3(chg[t0 + j].lo32, chg[t0 + j].hi32, bl, bh);
        const uint64_t m = __ballot(ov);
        if (ov) ws.act[n_act + __popcll(m & lanes_below())] = t0 + j;
        n_act += __popcll(m);
    }
    *bytes += 32;
    wave_sync();
    if (n_act == 0) return make_int2(0, 0);
    *n_pairs += n_act;
    const double *cp = rm.cap64 + e * (2 * D + 1) * B;
    double A[D], Bp[D];
#pragma unroll
    for (int k = 0; k < D; ++k) {
        A[k] = cp[k * B + ci];
        Bp[k] = cp[(D + k) * B + ci];
    }
    const double R = cp[2 * D * B + ci];
    *bytes += (unsigned long long)((2 * D + 1) * B * 8);
    const int64_t s0 = rm.p_fixed ? e * rm.p_fixed : rm.soff[e];
    const int64_t P = rm.p_fixed ? rm.p_fixed : rm.soff[e + 1] - s0;
    const double *sb = rm.samp64 + D * s0;
    const CopyMap cm = copy_map((int)(P / B));
    int dC = 0, dS = 0;
    for (int a0 = 0; a0 < n_act; a0 += G) {
        const int a = a0 + slot;
        bool hit = false;
        if (slot < G && a < n_act) {
            const ChgEntry &en = chg[ws.act[a]];
            double lo[D], hi[D];
#pragma unroll
            for (int k = 0; k < D; ++k) {
                lo[k] = en.lo[k];
                hi[k] = en.hi[k];
            }
            hit = segbox64<D>(A, Bp, lo, hi) <= R * R;
        }
        const uint64_t hm = __ballot(hit);
        for (int s = 0; s < G && a0 + s < n_act; ++s) {
            const uint64_t m = (hm >> (s * B)) & gmask;
            if (!m) continue;
            const ChgEntry &en = chg[ws.act[a0 + s]];
            double lo[D], hi[D];
#pragma unroll
            for (int k = 0; k < D; ++k) {
                lo[k] = en.lo[k];
                hi[k] = en.hi[k];
            }
            ++*n_outer;
            dC += en.sign;
            if (copies_meet64<D>(rm, sb, P, cm, m, lo, hi, rad, ws.lst, bytes)) dS += en.sign;
        }
    }
    wave_sync();
    return make_int2(dC, dS);
}

// ------------------------------------------------------------------------
// k_classify, FP64 mode
// ------------------------------------------------------------------------

__device__ inline void store_partials(const RmDev &rm, unsigned long long n_pairs,
                                      unsigned long long n_outer, unsigned long long bytes)
{
    __shared__ unsigned long long s_acc[3];
    if (threadIdx.x < 3) s_acc[threadIdx.x] = 0;
    __syncthreads();
    if (lane_id() == 0) {
        atomicAdd(&s_acc[0], n_pairs);
        atomicAdd(&s_acc[1], n_outer);
        atomicAdd(&s_acc[2], bytes);
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        unsigned long long *bs = rm.blk_stats + blockIdx.x * kStats;
        bs[0] = s_acc[0];
        bs[1] = s_acc[1];
        bs[2] = 0;
        bs[3] = s_acc[2];
    }
}

template <int D>
__global__ void __launch_bounds__(kBlock) k_classify64(RmDev rm)
{
    __shared__ WaveScratch s_ws[kWaves];
    __shared__ double s_rad[64];
    const Ctl *ctl = rm.ctl;
    if (threadIdx.x < rm.B) s_rad[threadIdx.x] = rm.rad64[threadIdx.x];
    __syncthreads();
    unsigned long long n_pairs = 0, n_outer = 0, bytes = 0;
    if (ctl->status == RGG_OK) {
        const int n_chg = ctl->n_chg;
        const int n_items = min(ctl->n_items, (int32_t)rm.items_cap);
        const int wv = threadIdx.x >> 6;
        Cursor cu = {(int)blockIdx.x, -1, 0, 0};
        int64_t slot;
        while (cursor_next(rm, n_items, cu, wv, &slot)) {
            const int64_t e = rm.work[slot];
            int2 d = make_int2(0, 0);
            for (int t0 = 0; t0 < n_chg; t0 += kTile) {
                int2 x = edge_exact<D>(rm, e, rm.chg, t0, min(kTile, n_chg - t0), s_ws[wv], s_rad,
                                       &n_pairs, &n_outer, &bytes);
                d.x += x.x;
                d.y += x.y;
            }
            if (lane_id() == 0) add_counts(rm, e, d.x, d.y);
            bytes += 16;
        }
    }
    store_partials(rm, n_pairs, n_outer, bytes);
}

// ------------------------------------------------------------------------
// k_classify, FP32 mode: one wavefront per candidate edge.  A decision is
// kept only when its binary32 margin lies outside the rounding band; a tile
// of pairs with any undecided pair is left whole to k_recheck.
// ------------------------------------------------------------------------

// copies of the spheres in m against one box: kHit (some copy certainly
// meets it), kMiss (every copy certainly misses) or kUnsure
template <int D>
__device__ int copies_meet32(const float *sb, int64_t P, const CopyMap &cm, uint64_t m, int B,
                             const float *lo, const float *hi, float band, const float *rad2,
                             int *lst, unsigned long long *bytes)
{
    const int nsph = list_spheres(m, B, lst);
    bool unsure = false;
    for (int sp0 = 0; sp0 < nsph; sp0 += cm.spc) {
        for (int j0 = 0; j0 < cm.J; j0 += cm.jw) {
            const int js = j0 + cm.jj;
            const bool valid = cm.sub < cm.spc && sp0 + cm.sub < nsph && js < cm.J;
            int cls = kMiss;
            if (valid) {
                const int i = lst[sp0 + cm.sub];
                float p[D];
#pragma unroll
                for (int k = 0; k < D; ++k) p[k] = sb[k * P + i * cm.J + js];
                cls = classify_margin(point_box32<D>(p, lo, hi) - rad2[i], band);
            }
            *bytes += (unsigned long long)(__popcll(__ballot(valid)) * D * 4);
            if (__ballot(cls == kHit)) return kHit;
            unsure |= __ballot(cls == kUnsure) != 0;
        }
    }
    return unsure ? kUnsure : kMiss;
}

template <int D>
__global__ void __launch_bounds__(kBlock) k_classify32(RmDev rm)
{
    __shared__ float s_lo[3][kTile], s_hi[3][kTile];
    __shared__ float s_sb[kTile];
    __shared__ int s_sign[kTile];
    __shared__ WaveScratch s_ws[kWaves];
    __shared__ float s_rad2[64];
    const Ctl *ctl = rm.ctl;
    const int tid = threadIdx.x, lane = lane_id(), wv = tid >> 6;
    if (tid < rm.B) s_rad2[tid] = rm.rad2_32[tid];
    unsigned long long n_pairs = 0, n_outer = 0, bytes = 0;
    if (ctl->status == RGG_OK) {
        const int n_chg = ctl->n_chg;
        const int n_items = min(ctl->n_items, (int32_t)rm.items_cap);
        const int B = rm.B;
        const int G = 64 / B, slot = lane / B, ci = lane - slot * B;
        const uint64_t gmask = B == 64 ? ~0ull : ((1ull << B) - 1ull);
        const float4 *aabb = reinterpret_cast<const float4 *>(rm.aabb);
        const float band_rel = rm.band_rel;
        WaveScratch &ws = s_ws[wv];
        for (int t0 = 0, tile = 0; t0 < n_chg; t0 += kTile, ++tile) {
            const int nt = min(kTile, n_chg - t0);
            __syncthreads();
            for (int j = tid; j < nt; j += kBlock) {
                const ChgEntry &en = rm.chg[t0 + j];
                for (int k = 0; k < 3; ++k) {
                    s_lo[k][j] = en.lo32[k];
                    s_hi[k][j] = en.hi32[k];
                }
                s_sb[j] = en.sbox;
                s_sign[j] = en.sign;
            }
            __syncthreads();
            Cursor cu = {(int)blockIdx.x, -1, 0, 0};
            int64_t wslot;
            while (cursor_next(rm, n_items, cu, wv, &wslot)) {
                const int64_t e = rm.work[wslot];
                const float4 bl = aabb[2 * e], bh = aabb[2 * e + 1];
                const float *cp = rm.cap32 + e * (2 * D + 1) * B;
                float A[D], Bq[D];
#pragma unroll
                for (int k = 0; k < D; ++k) {
                    A[k] = cp[k * B + ci];
                    Bq[k] = cp[(D + k) * B + ci];
                }
                const float R = cp[2 * D * B + ci];
                const int64_t s0 = rm.p_fixed ? e * rm.p_fixed : rm.soff[e];
                const int64_t P = rm.p_fixed ? rm.p_fixed : rm.soff[e + 1] - s0;
                // pretest against the staged entries
                int n_act = 0;
                for (int b0 = 0; b0 < nt; b0 += 64) {
                    const int j = b0 + lane;
                    bool ov = false;
                    if (j < nt) {
                        const float lo[3] = {s_lo[0][j], s_lo[1][j], s_lo[2][j]};
                        const float hi[3] = {s_hi[0][j], s_hi[1][j], s_hi[2][j]};
                        ov = overlap3(lo, hi, bl, bh);
                    }
                    const uint64_t m = __ballot(ov);
                    if (ov) ws.act[n_act + __popcll(m & lanes_below())] = j;
                    n_act += __popcll(m);
                }
                bytes += 32;
                uint32_t unsure_tiles = 0;
                if (n_act > 0) {
                    wave_sync();
                    n_pairs += n_act;
                    bytes += (unsigned long long)((2 * D + 1) * B * 4);
                    const float *sb = rm.samp32 + D * s0;
                    const CopyMap cm = copy_map((int)(P / B));
                    const float R2 = R * R;
                    bool any_unsure = false;
                    int dC = 0, dS = 0;
                    for (int a0 = 0; a0 < n_act; a0 += G) {
                        // capsule tests: separation -> miss, an end sphere
                        // meeting the box -> hit, else the full minimum
                        const int a = a0 + slot;
                        int cls = kMiss;
                        float lo[D], hi[D], band = 0.0f;
                        if (slot < G && a < n_act) {
                            const int j = ws.act[a];
#pragma unroll
                            for (int k = 0; k < D; ++k) {
                                lo[k] = s_lo[k][j];
                                hi[k] = s_hi[k][j];
                            }
                            const float s = fmaxf(bl.w, s_sb[j]);
                            band = band_rel * s * s;
                            float sep = 0.0f;
#pragma unroll
                            for (int k = 0; k < D; ++k)
                                sep = fmaxf(sep, fmaxf(lo[k] - fmaxf(A[k], Bq[k]), fminf(A[k], Bq[k]) - hi[k]));
                            const float m_end = fminf(point_box32<D>(A, lo, hi), point_box32<D>(Bq, lo, hi)) - R2;
                            cls = (sep > 0.0f && sep * sep - R2 > band) ? kMiss : (m_end < -band ? kHit : kOpen);
                        }
                        if (__ballot(cls == kOpen)) {
                            if (cls == kOpen) cls = classify_margin(segbox32<D>(A, Bq, lo, hi) - R2, band);
                        }
                        const uint64_t hm = __ballot(cls == kHit), um = __ballot(cls == kUnsure);
                        // per pair: copies of the spheres whose capsule met
                        for (int s = 0; s < G && a0 + s < n_act; ++s) {
                            const uint64_t h = (hm >> (s * B)) & gmask, u = (um >> (s * B)) & gmask;
                            if (!h) {
                                any_unsure |= u != 0;   // C rests on undecided capsules
                                continue;
                            }
                            const int j = ws.act[a0 + s];
                            float plo[D], phi[D];
#pragma unroll
                            for (int k = 0; k < D; ++k) {
                                plo[k] = s_lo[k][j];
                                phi[k] = s_hi[k][j];
                            }
                            const float sc = fmaxf(bl.w, s_sb[j]);
                            const int r = copies_meet32<D>(sb, P, cm, h, B, plo, phi, band_rel * sc * sc,
                                                           s_rad2, ws.lst, &bytes);
                            const int sign = s_sign[j];
                            ++n_outer;
                            if (r == kHit) {
                                dC += sign;
                                dS += sign;
                            } else if (r == kUnsure || u) {
                                any_unsure = true;
                            } else {
                                dC += sign;
                            }
                        }
                    }
                    if (any_unsure) {
                        unsure_tiles = 1u << tile;
                    } else if (lane == 0) {
                        add_counts(rm, e, dC, dS);
                    }
                    bytes += 16;
                    wave_sync();
                }
                if (lane == 0) rm.unsure[wslot] = tile == 0 ? unsure_tiles : (rm.unsure[wslot] | unsure_tiles);
            }
        }
    }
    store_partials(rm, n_pairs, n_outer, bytes);
}

// ------------------------------------------------------------------------
// k_recheck: binary64 re-test of the tiles the FP32 filter left unsure.
// Wavefronts scan the unsure marks of whole items, 64 candidates at a time.
// ------------------------------------------------------------------------

template <int D>
__global__ void __launch_bounds__(kBlock) k_recheck(RmDev rm)
{
    __shared__ WaveScratch s_ws[kWaves];
    __shared__ double s_rad[64];
    const Ctl *ctl = rm.ctl;
    if (threadIdx.x < rm.B) s_rad[threadIdx.x] = rm.rad64[threadIdx.x];
    __syncthreads();
    if (ctl->status != RGG_OK) return;
    const int n_chg = ctl->n_chg;
    const int n_items = min(ctl->n_items, (int32_t)rm.items_cap);
    const int lane = lane_id(), wv = threadIdx.x >> 6;
    unsigned long long n_pairs = 0, n_outer = 0, bytes = 0;
    for (int it = blockIdx.x * kWaves + wv; it < n_items; it += gridDim.x * kWaves) {
        const int2 item = rm.items[it];
        const int cnt = rm.item_cnt[it];
        const int64_t beg = (int64_t)rm.cell_start[item.x] + (int64_t)item.y * rm.chunk;
        for (int k0 = 0; k0 < cnt; k0 += 64) {
            const uint32_t mk = k0 + lane < cnt ? rm.unsure[beg + k0 + lane] : 0u;
            uint64_t fl = __ballot(mk != 0u);
            while (fl) {
                const int src = __ffsll((unsigned long long)fl) - 1;
                fl &= fl - 1;
                uint32_t mask = (uint32_t)__shfl((int)mk, src);
                const int64_t e = rm.work[beg + k0 + src];
                int2 d = make_int2(0, 0);
                while (mask) {
                    const int tile = __ffs(mask) - 1;
                    mask &= mask - 1;
                    const int t0 = tile * kTile;
                    int2 x = edge_exact<D>(rm, e, rm.chg, t0, min(kTile, n_chg - t0), s_ws[wv], s_rad,
                                           &n_pairs, &n_outer, &bytes);
                    d.x += x.x;
                    d.y += x.y;
                }
                if (lane == 0) add_counts(rm, e, d.x, d.y);
            }
        }
    }
    __shared__ unsigned long long s_acc[2];
    if (threadIdx.x < 2) s_acc[threadIdx.x] = 0;
    __syncthreads();
    if (lane == 0) {
        atomicAdd(&s_acc[0], n_pairs);   // pairs re-decided in binary64
        atomicAdd(&s_acc[1], bytes);
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        unsigned long long *bs = rm.blk_stats + blockIdx.x * kStats;
        bs[2] = s_acc[0];
        bs[3] += s_acc[1];
    }
}

// ------------------------------------------------------------------------
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
    unsigned long long acc[kStats] = {0, 0, 0, 0, 0};
    for (int b = tid; b < kStatBlocks; b += kBlock)
        for (int k = 0; k < kStats; ++k) acc[k] += rm.blk_stats[b * kStats + k];
    for (int k = 0; k < kStats; ++k) atomicAdd(&s_st[k], acc[k]);
    __syncthreads();
    if (tid == 0) {
        int64_t cand = 0;
        res->n_gray = status == RGG_OK ? off : 0;
        res->n_pairs = (int64_t)s_st[0];
        res->n_outer_hits = (int64_t)s_st[1];
        res->n_rechecked = (int64_t)s_st[2];
        res->test_bytes = (int64_t)s_st[3];
        res->n_cells_visited = (int64_t)s_st[4];
        (void)cand;
    }
}

// candidate count: sum of per-item counts, folded by one block
__global__ void __launch_bounds__(kBlock) k_candidates(RmDev rm, rgg_update_result *res)
{
    __shared__ int s_w[kWaves];
    const Ctl *ctl = rm.ctl;
    const int n_items = ctl->status == RGG_OK ? min(ctl->n_items, (int32_t)rm.items_cap) : 0;
    int acc = 0;
    for (int i = threadIdx.x; i < n_items; i += kBlock) acc += rm.item_cnt[i];
    const int tot = block_sum(acc, s_w);
    if (threadIdx.x == 0 && res) res->n_candidate_edges = tot;
}

}  // namespace

hipError_t launch_update(const RmDev &rm, const UpdateArgs &a, hipStream_t s, hipEvent_t *ev)
{
    hipError_t err;
#define RGG_TRY(x)                                 \
    do {                                           \
        if ((err = (x)) != hipSuccess) return err; \
    } while (0)
    if (rm.chunk != kBlock) return hipErrorInvalidValue;   // k_grid: one edge per thread
    if (ev) RGG_TRY(hipEventRecord(ev[0], s));
    k_diff<<<1, kDiffBlock, 0, s>>>(rm, a.old_b, a.new_b);
    RGG_TRY(hipGetLastError());
    if (ev) RGG_TRY(hipEventRecord(ev[1], s));
    k_cells<<<kCellsGrid, kBlock, 0, s>>>(rm);
    RGG_TRY(hipGetLastError());
    if (ev) RGG_TRY(hipEventRecord(ev[2], s));
    k_grid<<<kGrid, kBlock, 0, s>>>(rm);
    RGG_TRY(hipGetLastError());
    if (ev) RGG_TRY(hipEventRecord(ev[3], s));
    if (rm.mixed) {
        if (rm.D == 3) k_classify32<3><<<kGrid, kBlock, 0, s>>>(rm);
        else k_classify32<2><<<kGrid, kBlock, 0, s>>>(rm);
    } else {
        if (rm.D == 3) k_classify64<3><<<kGrid, kBlock, 0, s>>>(rm);
        else k_classify64<2><<<kGrid, kBlock, 0, s>>>(rm);
    }
    RGG_TRY(hipGetLastError());
    if (ev) RGG_TRY(hipEventRecord(ev[4], s));
    if (rm.mixed) {
        if (rm.D == 3) k_recheck<3><<<kGrid, kBlock, 0, s>>>(rm);
        else k_recheck<2><<<kGrid, kBlock, 0, s>>>(rm);
        RGG_TRY(hipGetLastError());
    }
    if (ev) RGG_TRY(hipEventRecord(ev[5], s));
    k_count<<<rm.ntiles, kBlock, 0, s>>>(rm, a.labels, a.res, 0);
    RGG_TRY(hipGetLastError());
    k_write<<<rm.ntiles, kBlock, 0, s>>>(rm, a.gray, a.gray_cap, a.res, 0);
    RGG_TRY(hipGetLastError());
    k_candidates<<<1, kBlock, 0, s>>>(rm, a.res);
    RGG_TRY(hipGetLastError());
    if (ev) RGG_TRY(hipEventRecord(ev[6], s));
    return hipSuccess;
#undef RGG_TRY
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
    // argument storage: hipGraphAddKernelNode copies the values
    RmDev r = rm;
    const rgg_box *ob = a.old_b, *nb = a.new_b;
    uint8_t *lab = a.labels;
    int64_t *gray = a.gray;
    int64_t cap = a.gray_cap;
    rgg_update_result *res = a.res;
    int zero = 0;
    void *args_diff[] = {&r, (void *)&ob, (void *)&nb};
    void *args_one[] = {&r};
    void *args_count[] = {&r, &lab, &res, &zero};
    void *args_write[] = {&r, &gray, &cap, &res, &zero};
    void *args_cand[] = {&r, &res};
    struct Node {
        void *fn;
        dim3 grid;
        void **args;
    };
    void *cls = rm.mixed ? (rm.D == 3 ? (void *)k_classify32<3> : (void *)k_classify32<2>)
                         : (rm.D == 3 ? (void *)k_classify64<3> : (void *)k_classify64<2>);
    Node nodes[8];
    int n = 0;
    nodes[n++] = {(void *)k_diff, dim3(1), args_diff};
    nodes[n++] = {(void *)k_cells, dim3(kCellsGrid), args_one};
    nodes[n++] = {(void *)k_grid, dim3(kGrid), args_one};
    nodes[n++] = {cls, dim3(kGrid), args_one};
    if (rm.mixed) nodes[n++] = {rm.D == 3 ? (void *)k_recheck<3> : (void *)k_recheck<2>, dim3(kGrid), args_one};
    nodes[n++] = {(void *)k_count, dim3(rm.ntiles), args_count};
    nodes[n++] = {(void *)k_write, dim3(rm.ntiles), args_write};
    nodes[n++] = {(void *)k_candidates, dim3(1), args_cand};
    hipGraphNode_t prev = dep;
    for (int k = 0; k < n; ++k) {
        hipKernelNodeParams p = {};
        p.func = nodes[k].fn;
        p.gridDim = nodes[k].grid;
        p.blockDim = dim3(k == 0 ? kDiffBlock : kBlock);
        p.sharedMemBytes = 0;
        p.kernelParams = nodes[k].args;
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
