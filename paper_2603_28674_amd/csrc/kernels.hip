// Update pipeline of librgg for gfx950 (wave64).
//
// One update = five kernels on one stream:
//   k_diff     validate old/new boxes against the resident slots, list the
//              changed (box, sign) entries in slot order, commit the slots
//              (Alg. 1: the moved obstacle's old and new poses);
//   k_cells    activate the grid cells each changed box overlaps and emit one
//              work item per (cell, chunk of its edge list)  (Sec. 3.3 grid);
//   k_grid     scan the edges of the active cells, keep those whose box meets
//              a changed box of that cell, and queue each such edge once;
//   k_classify one wavefront per queued edge: outer test (per-sphere capsule
//              vs box), inner test (sphere samples vs box, stop at the first
//              hit), FP64 re-test of pairs inside the rounding band, counter
//              update (Sec. 3.1 rule, Alg. 1 intersection lists as counts);
//   k_count + k_write   labels from the counters and the ordered gray list.
//
// All binary64 code below is compiled without FMA contraction; its sums run
// left to right from 0.0 so that a re-test reproduces the definition's
// values exactly.
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
constexpr int kGridGrid = 2048;
constexpr int kClassifyGrid = 2048;

enum : int { kMiss = 0, kHit = 1, kUnsure = 2 };
enum : uint8_t { kCHit = 1, kCUnsure = 2, kSHit = 4, kSUnsure = 8 };

__device__ inline int lane_id() { return __lane_id(); }
__device__ inline uint64_t lanes_below() { return (1ull << lane_id()) - 1ull; }

__device__ inline void wave_sync()
{
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
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

// ------------------------------------------------------------------------
// distance predicates (templated on the floating type and the dimension)
// ------------------------------------------------------------------------

template <typename T>
__device__ inline T gap1(T x, T lo, T hi)
{
    T a = lo - x;
    T g = a > T(0) ? a : T(0);
    T b = x - hi;
    return b > g ? b : g;
}

// squared distance from point c to the box
template <typename T, int D>
__device__ inline T point_box_d2(const T *c, const T *lo, const T *hi)
{
    T acc = T(0);
#pragma unroll
    for (int k = 0; k < D; ++k) {
        T g = gap1(c[k], lo[k], hi[k]);
        acc = acc + g * g;
    }
    return acc;
}

template <typename T, int D>
__device__ inline T seg_F(const T *A, const T *d, T t, const T *lo, const T *hi)
{
    T acc = T(0);
#pragma unroll
    for (int k = 0; k < D; ++k) {
        T p = A[k] + t * d[k];
        T g = gap1(p, lo[k], hi[k]);
        acc = acc + g * g;
    }
    return acc;
}

template <typename T, int D>
__device__ inline T seg_G(const T *A, const T *d, T t, const T *lo, const T *hi)
{
    T acc = T(0);
#pragma unroll
    for (int k = 0; k < D; ++k) {
        T p = A[k] + t * d[k];
        T ex = p < lo[k] ? p - lo[k] : (p > hi[k] ? p - hi[k] : T(0));
        acc = acc + d[k] * ex;
    }
    return acc;
}

// Minimum over t in [0,1] of the squared distance from A + t (B - A) to the
// box.  The function is convex and piecewise quadratic with breaks where a
// coordinate crosses a face plane; its half-derivative G is nondecreasing.
// Bracket the minimiser between the largest candidate with G <= 0 and the
// smallest with G >= 0 (candidates: 0, 1, face crossings strictly inside),
// then minimise the single quadratic of that bracket.
template <typename T, int D>
__device__ inline T segbox_fmin(const T *A, const T *Bp, const T *lo, const T *hi)
{
    T d[D];
#pragma unroll
    for (int k = 0; k < D; ++k) d[k] = Bp[k] - A[k];
    T tL = T(0), tR = T(1);
    auto take = [&](T t) {
        T g = seg_G<T, D>(A, d, t, lo, hi);
        if (g <= T(0) && t > tL) tL = t;
        if (g >= T(0) && t < tR) tR = t;
    };
    take(T(0));
    take(T(1));
#pragma unroll
    for (int k = 0; k < D; ++k) {
        if (d[k] != T(0)) {
            T t1 = (lo[k] - A[k]) / d[k];
            if (t1 > T(0) && t1 < T(1)) take(t1);
            T t2 = (hi[k] - A[k]) / d[k];
            if (t2 > T(0) && t2 < T(1)) take(t2);
        }
    }
    T fL = seg_F<T, D>(A, d, tL, lo, hi);
    T fR = seg_F<T, D>(A, d, tR, lo, hi);
    T fmin = fL < fR ? fL : fR;
    if (tL < tR) {
        T tm = T(0.5) * (tL + tR);
        T num = T(0), den = T(0);
#pragma unroll
        for (int k = 0; k < D; ++k) {
            T p = A[k] + tm * d[k];
            if (p < lo[k]) {
                num = num + d[k] * (lo[k] - A[k]);
                den = den + d[k] * d[k];
            } else if (p > hi[k]) {
                num = num + d[k] * (hi[k] - A[k]);
                den = den + d[k] * d[k];
            }
        }
        T ts = tL;
        if (den > T(0)) {
            ts = num / den;
            if (ts < tL) ts = tL;
            if (ts > tR) ts = tR;
        }
        T fs = seg_F<T, D>(A, d, ts, lo, hi);
        if (fs < fmin) fmin = fs;
    }
    return fmin;
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
        Ctl *c = rm.ctl;
        c->n_items = 0;
        c->n_work = 0;
        c->n_pairs = 0;
        c->n_outer = 0;
        c->n_recheck = 0;
        c->n_visited = 0;
        c->test_bytes = 0;
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
// k_cells: touched cells -> work items
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
        for (int64_t k = lane; k < total; k += 64) {
            const int32_t x = en.c0[0] + (int32_t)(k % nx);
            const int32_t y = en.c0[1] + (int32_t)((k / nx) % ny);
            const int32_t z = en.c0[2] + (int32_t)(k / ((int64_t)nx * ny));
            const int64_t c = ((int64_t)z * rm.gdim[1] + y) * rm.gdim[0] + x;
            const uint32_t bit = 1u << (c & 31);
            const uint32_t old = atomicOr(&rm.cell_bits[c >> 5], bit);
            if (!(old & bit)) {
                const int32_t n = rm.cell_start[c + 1] - rm.cell_start[c];
                const int32_t nch = n > 0 ? (n + rm.chunk - 1) / rm.chunk : 1;
                const int32_t pos = atomicAdd(&rm.ctl->n_items, nch);
                for (int32_t h = 0; h < nch; ++h)
                    if (pos + h < rm.items_cap) rm.items[pos + h] = make_int2((int32_t)c, h);
            }
        }
    }
}

// ------------------------------------------------------------------------
// k_grid: scan active cells, queue candidate edges once
// ------------------------------------------------------------------------

__device__ inline bool overlap3(const float *lo, const float *hi, const float4 &bl, const float4 &bh)
{
    return lo[0] <= bh.x && hi[0] >= bl.x && lo[1] <= bh.y && hi[1] >= bl.y && lo[2] <= bh.z &&
           hi[2] >= bl.z;
}

__global__ void __launch_bounds__(kBlock) k_grid(RmDev rm)
{
    __shared__ float s_lo[kSubCap * 3], s_hi[kSubCap * 3];
    __shared__ int s_n;
    const Ctl *ctl = rm.ctl;
    if (ctl->status != RGG_OK) return;
    const int n_items = min(ctl->n_items, (int32_t)rm.items_cap);
    const int n_chg = ctl->n_chg;
    const int tid = threadIdx.x, lane = lane_id();
    const float4 *aabb = reinterpret_cast<const float4 *>(rm.aabb);
    unsigned long long visited = 0;
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
        for (int j = tid; j < n_chg; j += kBlock) {
            const ChgEntry &en = rm.chg[j];
            if (cx >= en.c0[0] && cx <= en.c1[0] && cy >= en.c0[1] && cy <= en.c1[1] &&
                cz >= en.c0[2] && cz <= en.c1[2]) {
                const int s = atomicAdd(&s_n, 1);
                if (s < kSubCap)
                    for (int k = 0; k < 3; ++k) {
                        s_lo[k * kSubCap + s] = en.lo32[k];
                        s_hi[k * kSubCap + s] = en.hi32[k];
                    }
            }
        }
        __syncthreads();
        const int ns = s_n;
        const int64_t beg = (int64_t)rm.cell_start[c] + (int64_t)item.y * rm.chunk;
        const int64_t end = min((int64_t)rm.cell_start[c + 1], beg + rm.chunk);
        if (tid == 0) visited += (unsigned long long)max((int64_t)0, end - beg);
        for (int64_t j = beg + tid; j < end; j += kBlock) {
            const int32_t e = rm.cell_edges[j];
            const float4 bl = aabb[2 * (int64_t)e], bh = aabb[2 * (int64_t)e + 1];
            bool hit = false;
            if (ns <= kSubCap) {
                for (int s = 0; s < ns && !hit; ++s) {
                    const float lo[3] = {s_lo[s], s_lo[kSubCap + s], s_lo[2 * kSubCap + s]};
                    const float hi[3] = {s_hi[s], s_hi[kSubCap + s], s_hi[2 * kSubCap + s]};
                    hit = overlap3(lo, hi, bl, bh);
                }
            } else {
                for (int s = 0; s < n_chg && !hit; ++s) {
                    const ChgEntry &en = rm.chg[s];
                    hit = cx >= en.c0[0] && cx <= en.c1[0] && cy >= en.c0[1] && cy <= en.c1[1] &&
                          cz >= en.c0[2] && cz <= en.c1[2] && overlap3(en.lo32, en.hi32, bl, bh);
                }
            }
            bool first = false;
            if (hit) {
                const uint32_t bit = 1u << (e & 31);
                first = !(atomicOr(&rm.edge_bits[e >> 5], bit) & bit);
            }
            const uint64_t m = __ballot(first);
            if (m) {
                const int leader = __ffsll((unsigned long long)m) - 1;
                int base = 0;
                if (lane == leader) base = atomicAdd(&rm.ctl->n_work, __popcll(m));
                base = __shfl(base, leader);
                if (first) rm.work[base + __popcll(m & lanes_below())] = e;
            }
        }
    }
    if (tid == 0 && visited) atomicAdd(&rm.ctl->n_visited, visited);
}

// ------------------------------------------------------------------------
// k_classify: one wavefront per candidate edge
// ------------------------------------------------------------------------

template <int D>
struct Lds {
    float lo32[3][kTile], hi32[3][kTile];
    float sbox[kTile];
    int sign[kTile];
    double lo64[3][kTile], hi64[3][kTile];
    int act[kWaves][kTile];
    uint8_t st[kWaves][kTile];
};

// exact (binary64) outer test of one pair; every lane returns the same value
template <int D>
__device__ bool outer64(const RmDev &rm, int64_t e, const double *lo, const double *hi)
{
    const int B = rm.B, lane = lane_id();
    bool hit = false;
    if (lane < B) {
        const double *cp = rm.cap64 + e * (2 * D + 1) * B;
        double A[D], Bp[D];
#pragma unroll
        for (int k = 0; k < D; ++k) {
            A[k] = cp[k * B + lane];
            Bp[k] = cp[(D + k) * B + lane];
        }
        const double R = cp[2 * D * B + lane];
        hit = segbox_fmin<double, D>(A, Bp, lo, hi) <= R * R;
    }
    return __ballot(hit) != 0;
}

// exact (binary64) inner test of one pair
template <int D>
__device__ bool inner64(const RmDev &rm, int64_t e, const double *lo, const double *hi,
                        unsigned long long *bytes)
{
    const int B = rm.B, lane = lane_id();
    const int64_t s0 = rm.soff[e], P = rm.soff[e + 1] - s0;
    const double *base = rm.samp64 + D * s0;
    const int step = 64 % B, lane_b = lane % B;
    int cmod = 0;   // c mod B
    for (int64_t c = 0; c < P; c += 64) {
        const int64_t n = c + lane;
        bool hit = false;
        int ir = cmod + lane_b;
        ir = ir >= B ? ir - B : ir;
        cmod += step;
        cmod = cmod >= B ? cmod - B : cmod;
        if (n < P) {
            double p[D];
#pragma unroll
            for (int k = 0; k < D; ++k) p[k] = base[k * P + n];
            const double r = rm.rad64[ir];
            hit = point_box_d2<double, D>(p, lo, hi) <= r * r;
        }
        *bytes += (unsigned long long)(min((int64_t)64, P - c) * D * 8);
        if (__ballot(hit)) return true;
    }
    return false;
}

template <int D, bool kMixed>
__global__ void __launch_bounds__(kBlock) k_classify(RmDev rm)
{
    using T = typename std::conditional<kMixed, float, double>::type;
    __shared__ Lds<D> L;
    const Ctl *ctl = rm.ctl;
    if (ctl->status != RGG_OK) return;
    const int n_chg = ctl->n_chg, n_work = ctl->n_work;
    if (n_chg == 0 || n_work == 0) return;
    const int tid = threadIdx.x, lane = lane_id(), wv = tid >> 6;
    const int B = rm.B;
    const int G = 64 / B;                 // pairs per capsule pass
    const int slot = lane / B, ci = lane % B;
    const uint64_t gmask = B == 64 ? ~0ull : ((1ull << B) - 1ull);
    const float4 *aabb = reinterpret_cast<const float4 *>(rm.aabb);
    const T *cap = kMixed ? (const T *)rm.cap32 : (const T *)rm.cap64;
    const T *samp = kMixed ? (const T *)rm.samp32 : (const T *)rm.samp64;
    int *act = L.act[wv];
    uint8_t *st = L.st[wv];
    unsigned long long n_pairs = 0, n_outer = 0, n_re = 0, bytes = 0;

    for (int t0 = 0; t0 < n_chg; t0 += kTile) {
        const int nt = min(kTile, n_chg - t0);
        __syncthreads();
        for (int j = tid; j < nt; j += kBlock) {
            const ChgEntry &en = rm.chg[t0 + j];
            for (int k = 0; k < 3; ++k) {
                L.lo32[k][j] = en.lo32[k];
                L.hi32[k][j] = en.hi32[k];
                L.lo64[k][j] = en.lo[k];
                L.hi64[k][j] = en.hi[k];
            }
            L.sbox[j] = en.sbox;
            L.sign[j] = en.sign;
        }
        __syncthreads();
        for (int w = blockIdx.x * kWaves + wv; w < n_work; w += gridDim.x * kWaves) {
            const int64_t e = rm.work[w];
            const float4 bl = aabb[2 * e], bh = aabb[2 * e + 1];
            // box pretest against the staged entries
            int n_act = 0;
            for (int b0 = 0; b0 < nt; b0 += 64) {
                const int j = b0 + lane;
                bool ov = false;
                if (j < nt) {
                    const float lo[3] = {L.lo32[0][j], L.lo32[1][j], L.lo32[2][j]};
                    const float hi[3] = {L.hi32[0][j], L.hi32[1][j], L.hi32[2][j]};
                    ov = overlap3(lo, hi, bl, bh);
                }
                const uint64_t m = __ballot(ov);
                if (ov) act[n_act + __popcll(m & lanes_below())] = j;
                n_act += __popcll(m);
            }
            bytes += 32;
            if (n_act == 0) continue;
            wave_sync();
            n_pairs += n_act;
            // outer test: lane (slot, ci) tests capsule ci against pair slot
            const T *cp = cap + e * (2 * D + 1) * B;
            T A[D], Bp[D];
#pragma unroll
            for (int k = 0; k < D; ++k) {
                A[k] = cp[k * B + ci];
                Bp[k] = cp[(D + k) * B + ci];
            }
            const T R = cp[2 * D * B + ci];
            bytes += (unsigned long long)((2 * D + 1) * B * sizeof(T));
            int pend = 0;
            for (int a0 = 0; a0 < n_act; a0 += G) {
                const int a = a0 + slot;
                int cls = kMiss;
                if (slot < G && a < n_act) {
                    const int j = act[a];
                    T lo[D], hi[D];
#pragma unroll
                    for (int k = 0; k < D; ++k) {
                        lo[k] = kMixed ? (T)L.lo32[k][j] : (T)L.lo64[k][j];
                        hi[k] = kMixed ? (T)L.hi32[k][j] : (T)L.hi64[k][j];
                    }
                    const T m = segbox_fmin<T, D>(A, Bp, lo, hi) - R * R;
                    if (kMixed) {
                        const float s = fmaxf(bl.w, L.sbox[j]);
                        const float band = rm.band_rel * s * s;
                        cls = m < -band ? kHit : (m > band ? kMiss : kUnsure);
                    } else {
                        cls = m <= T(0) ? kHit : kMiss;
                    }
                }
                const uint64_t hm = __ballot(cls == kHit), um = __ballot(cls == kUnsure);
                if (lane < G && a0 + lane < n_act) {
                    const uint64_t g = gmask << (lane * B);
                    st[a0 + lane] = (hm & g) ? kCHit : ((um & g) ? kCUnsure : 0);
                }
                // count how many pairs need the inner test
                for (int s = 0; s < G && a0 + s < n_act; ++s)
                    pend += ((hm >> (s * B)) & gmask) ? 1 : 0;
            }
            wave_sync();
            // inner test over chunks of 64 sphere samples, all pending pairs per chunk
            const int64_t s0 = rm.soff[e], P = rm.soff[e + 1] - s0;
            const T *sb = samp + D * s0;
            const int step = 64 % B;
            int cmod = 0;   // c mod B
            for (int64_t c = 0; c < P && pend > 0; c += 64) {
                const int64_t n = c + lane;
                const bool valid = n < P;
                int ir = cmod + ci;
                ir = ir >= B ? ir - B : ir;
                cmod += step;
                cmod = cmod >= B ? cmod - B : cmod;
                T p[D];
                T r2 = T(0);
                if (valid) {
#pragma unroll
                    for (int k = 0; k < D; ++k) p[k] = sb[k * P + n];
                    r2 = kMixed ? (T)rm.rad2_32[ir] : (T)(rm.rad64[ir] * rm.rad64[ir]);
                }
                bytes += (unsigned long long)(min((int64_t)64, P - c) * D * sizeof(T));
                for (int a = 0; a < n_act; ++a) {
                    uint8_t s = st[a];
                    if (!(s & kCHit) || (s & kSHit)) continue;
                    const int j = act[a];
                    int cls = kMiss;
                    if (valid) {
                        T lo[D], hi[D];
#pragma unroll
                        for (int k = 0; k < D; ++k) {
                            lo[k] = kMixed ? (T)L.lo32[k][j] : (T)L.lo64[k][j];
                            hi[k] = kMixed ? (T)L.hi32[k][j] : (T)L.hi64[k][j];
                        }
                        const T m = point_box_d2<T, D>(p, lo, hi) - r2;
                        if (kMixed) {
                            const float sc = fmaxf(bl.w, L.sbox[j]);
                            const float band = rm.band_rel * sc * sc;
                            cls = m < -band ? kHit : (m > band ? kMiss : kUnsure);
                        } else {
                            cls = m <= T(0) ? kHit : kMiss;
                        }
                    }
                    const uint64_t hm = __ballot(cls == kHit), um = __ballot(cls == kUnsure);
                    if (hm) {
                        s |= kSHit;
                        --pend;
                    } else if (um) {
                        s |= kSUnsure;
                    }
                    st[a] = s;
                    wave_sync();
                }
            }
            // resolve every pair; unsure ones are re-decided in binary64
            int dC = 0, dS = 0;
            for (int a = 0; a < n_act; ++a) {
                const uint8_t s = st[a];
                const int j = act[a];
                int C = 0, S = 0;
                if (s & kCUnsure) {
                    double lo3[3] = {L.lo64[0][j], L.lo64[1][j], L.lo64[2][j]};
                    double hi3[3] = {L.hi64[0][j], L.hi64[1][j], L.hi64[2][j]};
                    C = outer64<D>(rm, e, lo3, hi3) ? 1 : 0;
                    S = C && inner64<D>(rm, e, lo3, hi3, &bytes) ? 1 : 0;
                    bytes += (unsigned long long)((2 * D + 1) * B * 8);
                    ++n_re;
                } else if (s & kCHit) {
                    C = 1;
                    if (s & kSHit) {
                        S = 1;
                    } else if (s & kSUnsure) {
                        double lo3[3] = {L.lo64[0][j], L.lo64[1][j], L.lo64[2][j]};
                        double hi3[3] = {L.hi64[0][j], L.hi64[1][j], L.hi64[2][j]};
                        S = inner64<D>(rm, e, lo3, hi3, &bytes) ? 1 : 0;
                        ++n_re;
                    }
                }
                n_outer += C;
                dC += L.sign[j] * C;
                dS += L.sign[j] * S;
            }
            if (lane == 0 && (dC != 0 || dS != 0)) {
                int2 v = rm.cnt[e];
                v.x += dC;
                v.y += dS;
                rm.cnt[e] = v;
            }
            bytes += 16;
            wave_sync();
        }
    }
    if (lane == 0) {
        Ctl *c = rm.ctl;
        if (n_pairs) atomicAdd(&c->n_pairs, n_pairs);
        if (n_outer) atomicAdd(&c->n_outer, n_outer);
        if (n_re) atomicAdd(&c->n_recheck, n_re);
        if (bytes) atomicAdd(&c->test_bytes, bytes);
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
    if (tid == 0 && res && blockIdx.x == gridDim.x - 1) {
        if (force) {
            res->n_gray = off;
        } else {
            const Ctl *c = rm.ctl;
            res->n_gray = status == RGG_OK ? off : 0;
            res->n_candidate_edges = c->n_work;
            res->n_pairs = (int64_t)c->n_pairs;
            res->n_outer_hits = (int64_t)c->n_outer;
            res->n_rechecked = (int64_t)c->n_recheck;
            res->n_cells_visited = (int64_t)c->n_visited;
            res->test_bytes = (int64_t)c->test_bytes;
        }
    }
}

void *classify_fn(const RmDev &rm)
{
    if (rm.D == 3) return rm.mixed ? (void *)k_classify<3, true> : (void *)k_classify<3, false>;
    return rm.mixed ? (void *)k_classify<2, true> : (void *)k_classify<2, false>;
}

struct Launch {
    void *fn;
    dim3 grid, block;
};

// the five launches of one update, in order
void plan(const RmDev &rm, Launch out[6])
{
    out[0] = {(void *)k_diff, dim3(1), dim3(kDiffBlock)};
    out[1] = {(void *)k_cells, dim3(kCellsGrid), dim3(kBlock)};
    out[2] = {(void *)k_grid, dim3(kGridGrid), dim3(kBlock)};
    out[3] = {classify_fn(rm), dim3(kClassifyGrid), dim3(kBlock)};
    out[4] = {(void *)k_count, dim3(rm.ntiles), dim3(kBlock)};
    out[5] = {(void *)k_write, dim3(rm.ntiles), dim3(kBlock)};
}

}  // namespace

hipError_t launch_update(const RmDev &rm, const UpdateArgs &a, hipStream_t s, hipEvent_t *ev)
{
    hipError_t err;
#define RGG_TRY(x)                               \
    do {                                         \
        if ((err = (x)) != hipSuccess) return err; \
    } while (0)
    if (ev) RGG_TRY(hipEventRecord(ev[0], s));
    k_diff<<<1, kDiffBlock, 0, s>>>(rm, a.old_b, a.new_b);
    RGG_TRY(hipGetLastError());
    if (ev) RGG_TRY(hipEventRecord(ev[1], s));
    k_cells<<<kCellsGrid, kBlock, 0, s>>>(rm);
    RGG_TRY(hipGetLastError());
    if (ev) RGG_TRY(hipEventRecord(ev[2], s));
    k_grid<<<kGridGrid, kBlock, 0, s>>>(rm);
    RGG_TRY(hipGetLastError());
    if (ev) RGG_TRY(hipEventRecord(ev[3], s));
    if (rm.D == 3) {
        if (rm.mixed) k_classify<3, true><<<kClassifyGrid, kBlock, 0, s>>>(rm);
        else k_classify<3, false><<<kClassifyGrid, kBlock, 0, s>>>(rm);
    } else {
        if (rm.mixed) k_classify<2, true><<<kClassifyGrid, kBlock, 0, s>>>(rm);
        else k_classify<2, false><<<kClassifyGrid, kBlock, 0, s>>>(rm);
    }
    RGG_TRY(hipGetLastError());
    if (ev) RGG_TRY(hipEventRecord(ev[4], s));
    k_count<<<rm.ntiles, kBlock, 0, s>>>(rm, a.labels, a.res, 0);
    RGG_TRY(hipGetLastError());
    k_write<<<rm.ntiles, kBlock, 0, s>>>(rm, a.gray, a.gray_cap, a.res, 0);
    RGG_TRY(hipGetLastError());
    if (ev) RGG_TRY(hipEventRecord(ev[5], s));
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
    Launch L[6];
    plan(rm, L);
    // argument storage: copied by hipGraphAddKernelNode
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
    void **args[6] = {args_diff, args_one, args_one, args_one, args_count, args_write};
    hipGraphNode_t prev = dep;
    for (int k = 0; k < 6; ++k) {
        hipKernelNodeParams p = {};
        p.func = L[k].fn;
        p.gridDim = L[k].grid;
        p.blockDim = L[k].block;
        p.sharedMemBytes = 0;
        p.kernelParams = args[k];
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
