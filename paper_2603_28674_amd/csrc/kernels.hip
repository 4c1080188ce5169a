// Update pipeline of librgg for gfx950 (wave64).
//
// One update = these kernels on one stream (or one graph):
//   k_diff      validate the old/new boxes against the resident slots, list
//               the changed (box, sign) entries in slot order, commit the
//               slots (Alg. 1: a moved obstacle's old and new poses); with
//               one grid cell it also hands out the fixed work items, with
//               several it activates every grid cell a changed box overlaps
//               and emits one work item per (cell, chunk of its edges)
//               (Sec. 4.3);
//   k_item32/64 one block per work item: pairs of the item's edges with the
//               changed boxes of the cell, outer test (per-sphere capsule vs
//               box), inner test (copies of the spheres whose capsule met),
//               counter update (Sec. 4.1 rule; Alg. 1's intersection lists
//               kept as counts).  Optionally (inline_rounds) the FP32 item
//               kernel tests only an item's first pair rounds and lists the
//               rest for
//   k_pairs     which cuts the listed pairs into equal shares, one per
//               block, and runs the same tests on them.  In the FP32 mode a
//               pair whose margin falls inside the rounding band is left to
//   k_fp64      which decides it in binary64, one wavefront per pair; an
//               item whose block ran out of re-test room is then run again
//               whole in binary64 by the same kernel (skipped otherwise);
//   k_labels    labels from the counters and the ordered gray list, in one
//               pass (k_count + k_write, the two-pass form, serve the label
//               queries and the batch).
// The *_batch kernels run the same stages for many roadmaps in one launch
// each, reading every roadmap's arguments from a request table.
//
// Binary64 code is compiled without FMA contraction and its sums run left to
// right from 0.0, so a re-test reproduces the definition's values exactly.
// Hot loops keep off single global counters: on MI355X device-scope atomics
// on one address serialise across the eight XCDs, so work lists are
// positional and statistics go to 256 rows shared through atomics.  The few
// single-address counters are k_labels' tickets (one per 4096-edge tile),
// the batched item kernel's claims (one per item past two per block) and
// the rare appends to a roadmap's list of items left whole.
#include <hip/hip_runtime.h>

#include <type_traits>

#include "predicates64.h"
#include "rgg_device.h"

namespace rgg {

namespace {

constexpr int kDiffBlock = 1024;
constexpr int kBlock = 256;
constexpr int kWaves = kBlock / 64;
constexpr int kGrid = kStatBlocks; // blocks of the item kernels
constexpr int kFp64Grid = 256;     // blocks of the binary64 pass of the FP32 mode
constexpr int kBatchItemGrid = 1024;  // blocks of a batched item kernel: the blocks of the
                                      // FP32 kernel resident at once (4 per CU, 256 CUs)
constexpr int kBatchStatic = 2;       // items a batched item block takes before it claims
constexpr int kFp64BatchGrid = 32; // blocks per roadmap of the batched binary64 pass
static_assert(kStatBlocks % kFp64Grid == 0 && kStatBlocks / kFp64BatchGrid <= 64, "re-test regions per block");
static_assert(kBatchItemGrid <= kStatBlocks, "a batched item block's row and region exist");
static_assert(kFp64Grid <= kStatRows && kFp64BatchGrid <= kStatRows, "a binary64 block owns a statistics row");
static_assert(kStatBlocks % 256 == 0, "statistics rows are folded 256 at a time");

enum : int { kMiss = 0, kHit = 1, kUnsure = 2, kOpen = 3 };

__device__ inline int lane_id() { return __lane_id(); }
__device__ inline uint64_t lanes_below() { return (1ull << lane_id()) - 1ull; }

__device__ inline void wave_sync()
{
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

__device__ inline unsigned long long wave_sum_u64(unsigned long long v)
{
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o);
    return v;
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
    // c is integral, so comparing its int32 value with n decides c >= n
    // exactly (and keeps n out of binary64 registers)
    double c = floor((x - org) * inv);
    if (c < 0.0) return -1;
    if (!(c < 2147483647.0)) return n;
    const int32_t ci = (int32_t)c;
    return ci >= n ? n : ci;
}

__device__ inline bool overlap3(const float *lo, const float *hi, const float4 &bl, const float4 &bh)
{
    return lo[0] <= bh.x && hi[0] >= bl.x && lo[1] <= bh.y && hi[1] >= bl.y && lo[2] <= bh.z &&
           hi[2] >= bl.z;
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

// `targ` receives the parameter of the value returned.  Scheduling barriers
// between the candidates keep one candidate's temporaries live at a time, so
// this binary32 filter stays small in registers.
template <int D>
__device__ inline float segbox32(const float *A, const float *Bp, const float *lo, const float *hi, float &targ)
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
        __builtin_amdgcn_sched_barrier(0);
    };
    take(0.0f);
    take(1.0f);
#pragma unroll
    for (int k = 0; k < D; ++k) {
        // a crossing outside (0,1) (or of an axis the segment does not
        // move along) is replaced by t = 0, which repeats the first candidate
        float t1 = (lo[k] - A[k]) * inv[k];
        take(t1 > 0.0f && t1 < 1.0f ? t1 : 0.0f);
        float t2 = (hi[k] - A[k]) * inv[k];
        take(t2 > 0.0f && t2 < 1.0f ? t2 : 0.0f);
    }
    const float fL = seg_F32<D>(A, d, tL, lo, hi), fR = seg_F32<D>(A, d, tR, lo, hi);
    const float fmin = fminf(fL, fR);
    const float tmin = fL <= fR ? tL : tR;
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
    const float fs = seg_F32<D>(A, d, ts, lo, hi);
    targ = fs < fmin ? ts : tmin;
    return fminf(fmin, fs);
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

template <int D>
__device__ inline bool present(const rgg_box &b)
{
    bool p = true;
#pragma unroll
    for (int k = 0; k < 3; ++k) p = p && (k >= D || b.lo[k] <= b.hi[k]);
    return p;
}

// returns whether the box covers at least one grid cell (D is the
// roadmap's dimension, so the loop below is straight-line code)
template <int D>
__device__ bool write_entry(const RmDev &rm, int pos, const rgg_box &b, int sign)
{
    ChgEntry en;
    float s = 0.0f;
    bool empty = false;
#pragma unroll
    for (int k = 0; k < 3; ++k) {
        if (k < D) {
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
    return !empty;
}

// Block-wide exclusive prefix over the kNW wavefronts of a block (64-bit
// values): returns this thread's prefix, *total the block's sum.
template <int kNW>
__device__ inline long long block_prefix64(long long v, long long *total, long long *wsum)
{
    const int lane = lane_id(), wv = (int)(threadIdx.x >> 6);
    long long x = v;
    for (int o = 1; o < 64; o <<= 1) {
        const long long y = __shfl_up(x, o);
        if (lane >= o) x += y;
    }
    __syncthreads();
    if (lane == 63) wsum[wv] = x;
    __syncthreads();
    long long off = 0, tot = 0;
    for (int w = 0; w < kNW; ++w) {
        off += w < wv ? wsum[w] : 0;
        tot += wsum[w];
    }
    *total = tot;
    return off + x - v;
}

// Grid roadmaps: the cells the n_chg changed entries cover are marked and
// each newly marked cell emits one work item per chunk of its edges (an
// empty cell one item, whose first chunk clears the mark).  One block of
// kDiffBlock threads, right after the entries are written: the (entry,
// cell) pairs are dealt over the threads (a prefix over the entries' cell
// counts), so every mark of a pass is in flight at once, and the items go
// to positions from a block scan (one block per roadmap: no global counter).
__device__ __forceinline__ void activate_cells(const RmDev &rm, int n_chg)
{
    constexpr int kNW = kDiffBlock / 64;
    __shared__ long long s_cpre[kDiffBlock];
    __shared__ int s_rng[kDiffBlock][5];   // first cell (x, y, z), cells along x and y
    __shared__ long long s_w64[kNW];
    __shared__ int s_w32[kNW];
    __shared__ int s_items;
    const int tid = threadIdx.x, lane = lane_id(), wv = tid >> 6;
    if (tid == 0) s_items = 0;
    for (int q0 = 0; q0 < n_chg; q0 += kDiffBlock) {
        const int q = q0 + tid;
        long long cnt = 0;
        if (q < n_chg) {
            const ChgEntry &en = rm.chg[q];
            const int32_t nx = en.c1[0] - en.c0[0] + 1, ny = en.c1[1] - en.c0[1] + 1, nz = en.c1[2] - en.c0[2] + 1;
            if (nx > 0 && ny > 0 && nz > 0) cnt = (long long)nx * ny * nz;
            s_rng[tid][0] = en.c0[0];
            s_rng[tid][1] = en.c0[1];
            s_rng[tid][2] = en.c0[2];
            s_rng[tid][3] = nx;
            s_rng[tid][4] = ny;
        }
        long long tot;
        const long long pre = block_prefix64<kNW>(cnt, &tot, s_w64);
        s_cpre[tid] = pre;
        __syncthreads();
        const int ne = min(kDiffBlock, n_chg - q0);
        for (long long t0 = 0; t0 < tot; t0 += kDiffBlock) {
            const long long t = t0 + tid;
            int nch = 0;
            long long c = 0;
            if (t < tot) {
                // the entry holding pair t: the last j with s_cpre[j] <= t
                int lo = 0, hi = ne - 1;
                while (lo < hi) {
                    const int mid = (lo + hi + 1) >> 1;
                    if (s_cpre[mid] <= t) lo = mid;
                    else hi = mid - 1;
                }
                const long long k = t - s_cpre[lo];
                const int nx = s_rng[lo][3], ny = s_rng[lo][4];
                const int32_t x = s_rng[lo][0] + (int32_t)(k % nx);
                const int32_t y = s_rng[lo][1] + (int32_t)((k / nx) % ny);
                const int32_t z = s_rng[lo][2] + (int32_t)(k / ((long long)nx * ny));
                c = ((long long)z * rm.gdim[1] + y) * rm.gdim[0] + x;
                const uint32_t bit = 1u << (c & 31);
                const int32_t s0 = rm.cell_start[c], s1 = rm.cell_start[c + 1];
                if (!(atomicOr(&rm.cell_bits[c >> 5], bit) & bit)) {
                    const int32_t n = s1 - s0;
                    nch = n > 0 ? (n + rm.chunk - 1) / rm.chunk : 1;
                }
            }
            // positions of this pass's items
            int x = nch;
            for (int o = 1; o < 64; o <<= 1) {
                const int y = __shfl_up(x, o);
                if (lane >= o) x += y;
            }
            __syncthreads();
            if (lane == 63) s_w32[wv] = x;
            __syncthreads();
            int off = s_items, ntot = 0;
            for (int w = 0; w < kNW; ++w) {
                off += w < wv ? s_w32[w] : 0;
                ntot += s_w32[w];
            }
            const int pos = off + x - nch;
            for (int h = 0; h < nch; ++h)
                if ((int64_t)pos + h < rm.items_cap) rm.items[pos + h] = make_int2((int32_t)c, h);
            __syncthreads();
            if (tid == 0) s_items += ntot;
            __syncthreads();
        }
    }
    if (tid == 0) rm.ctl->n_items = s_items;
}

// One block: validates the update, writes the changed entries and commits
// the new boxes.  The block's first half takes the entry of a slot's old
// box, the second half that of its new box, so each thread writes at most
// one entry (the entry is a chain of binary64 roundings and cell indices,
// which one wavefront runs at its latency); a chunk of the update covers
// kDiffBlock / 2 slots, its old boxes' entries first.
template <int D>
__device__ __forceinline__ void diff_body(const RmDev &rm, const rgg_box *__restrict__ old_b,
                                          const rgg_box *__restrict__ new_b)
{
    constexpr int kHalf = kDiffBlock / 2;
    __shared__ int s_tot[kDiffBlock / 64];
    __shared__ int s_bad, s_mism, s_base, s_any;
    const int tid = threadIdx.x, lane = lane_id(), wave = tid >> 6;
    const int side = tid / kHalf;        // 0: the old box's entry, 1: the new box's
    const int j = tid - side * kHalf;    // slot within the chunk
    if (tid == 0) {
        s_bad = 0;
        s_mism = 0;
        s_base = 0;
        s_any = 0;
        rm.ctl->n_items = 0;
        rm.ctl->n_df = 0;
        rm.ctl->claim = 0;
        rm.ctl->label_ticket = 0;
    }
    for (int t = tid; t < rm.ntiles; t += kDiffBlock) rm.tile_state[t] = 0ull;
    __syncthreads();
    bool dirty0 = false;   // the first chunk's slot changes (kept for the commit)
    rgg_box n0;
    for (int64_t base = 0; base < rm.M; base += kHalf) {
        const int64_t k = base + j;
        bool emit = false;
        rgg_box b;
        if (k < rm.M) {
            const rgg_box o = old_b[k], n = new_b[k], r = rm.resident[k];
            if (side == 0) {
                if (!box_ok(o) || !box_ok(n)) atomicOr(&s_bad, 1);
                if (!same_box(o, r)) atomicOr(&s_mism, 1);
            } else if (base == 0) {
                dirty0 = !same_box(n, r);
                n0 = n;
            }
            b = side ? n : o;
            emit = !same_box(o, n) && present<D>(b);
        }
        const uint64_t bm = __ballot(emit);
        if (lane == 0) s_tot[wave] = __popcll(bm);
        __syncthreads();
        int pos = s_base, tot = 0;
        for (int w = 0; w < kDiffBlock / 64; ++w) {
            if (w < wave) pos += s_tot[w];
            tot += s_tot[w];
        }
        pos += __popcll(bm & lanes_below());
        if (emit && write_entry<D>(rm, pos, b, side ? +1 : -1)) s_any = 1;
        __syncthreads();
        if (tid == 0) s_base += tot;
        __syncthreads();
    }
    const int status = s_bad ? RGG_E_INVALID_ARG : (s_mism ? RGG_E_STATE_MISMATCH : RGG_OK);
    if (tid == 0) {
        rm.ctl->status = status;
        rm.ctl->n_chg = status ? 0 : s_base;
        // one grid cell: its items (0, h) are fixed at build; they are all
        // work as soon as one changed box lies inside the grid
        if (rm.ncells == 1) rm.ctl->n_items = (status == RGG_OK && s_any) ? (int32_t)rm.items_cap : 0;
    }
    if (status == RGG_OK) {
        if (dirty0) rm.resident[j] = n0;
        for (int64_t k = kHalf + tid; k < rm.M; k += kDiffBlock) {
            rgg_box n = new_b[k];
            if (!same_box(n, rm.resident[k])) rm.resident[k] = n;
        }
        // the entries written above are read back by this block's threads
        if (rm.ncells > 1) {
            __syncthreads();
            activate_cells(rm, s_base);
        }
    }
}

template <int D>
__global__ void __launch_bounds__(kDiffBlock) k_diff(RmDev rm, const rgg_box *__restrict__ old_b,
                                                     const rgg_box *__restrict__ new_b)
{
    diff_body<D>(rm, old_b, new_b);
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
// sphere samples: per edge a [B][J][S] block at S * soff[e], S values per copy
// (xyz + pad in 3-D, xy in 2-D), so one copy is one aligned vector load
// ------------------------------------------------------------------------

template <int D>
__host__ __device__ constexpr int copy_stride()
{
    return D == 3 ? kCopyStride3 : kCopyStride2;
}

// copy `idx` (= soff[e] + sphere * J + configuration) of the sample array
template <int D, typename T>
__device__ inline void load_copy(const T *samp, int64_t idx, T (&q)[D])
{
    const T *p = samp + copy_stride<D>() * idx;
    if constexpr (std::is_same<T, float>::value && D == 3) {
        const float4 v = *reinterpret_cast<const float4 *>(p);
        q[0] = v.x;
        q[1] = v.y;
        q[2] = v.z;
    } else if constexpr (std::is_same<T, float>::value && D == 2) {
        const float2 v = *reinterpret_cast<const float2 *>(p);
        q[0] = v.x;
        q[1] = v.y;
    } else {
#pragma unroll
        for (int k = 0; k < D; ++k) q[k] = p[k];
    }
}

// ------------------------------------------------------------------------
// binary64 re-test of one (edge, box) pair by one wavefront: the definition
// (C = some capsule meets, S = some sphere's capsule and one of its copies
// meet), used for the pairs whose binary32 decision fell inside the band
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
                for (int k = 0; k < D; ++k) p[k] = sb[((int64_t)i * cm.J + js) * copy_stride<D>() + k];
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

// some kept spline segment of a sphere in m meets the box (binary64, one
// wavefront: the spheres in turn, their segments across the lanes)
template <int D>
__device__ bool splines_meet64(const RmDev &rm, int64_t e, uint64_t m, const double *lo, const double *hi,
                               unsigned long long *bytes)
{
    constexpr int W = 2 * D + 1;
    const int lane = lane_id();
    while (m) {
        const int i = __ffsll((unsigned long long)m) - 1;
        m &= m - 1;
        const int64_t k = e * rm.B + i;
        const int32_t k0 = rm.sseg[k], k1 = rm.sseg[k + 1];
        for (int32_t j0 = k0; j0 < k1; j0 += 64) {
            const int32_t j = j0 + lane;
            bool hit = false;
            if (j < k1) {
                const double *g = rm.seg64 + (int64_t)j * W;
                double A[D], Bq[D];
#pragma unroll
                for (int d = 0; d < D; ++d) {
                    A[d] = g[d];
                    Bq[d] = g[D + d];
                }
                hit = segbox64<D>(A, Bq, lo, hi) <= g[2 * D] * g[2 * D];
            }
            *bytes += (unsigned long long)(min(64, k1 - j0) * W * 8);
            if (__ballot(hit)) return true;
        }
    }
    return false;
}

// Binary64 decision of one (edge e, changed entry ci) pair by one wavefront:
// C and S by their definition (capsules, the oriented boxes, then copies or
// spline segments), added to the edge's counters.  lst: 64 ints of LDS for
// the wavefront; rad: the binary64 radii in LDS.
template <int D, int MODE>
__device__ inline void retest_one(const RmDev &rm, int64_t e, int ci, int *lst, const double *rad, uint32_t &n_outer,
                                  unsigned long long &bytes)
{
    const int lane = lane_id();
    const int B = rm.B;
    const ChgEntry &en = rm.chg[ci];
    double lo[D], hi[D];
#pragma unroll
    for (int d = 0; d < D; ++d) {
        lo[d] = en.lo[d];
        hi[d] = en.hi[d];
    }
    // the edge's sample range is loaded with its capsules: it is needed as
    // soon as one capsule meets, and would otherwise add a round trip
    int64_t s0 = 0, P = 0;
    if constexpr ((MODE & kModeSplines) == 0) {
        s0 = rm.p_fixed ? e * rm.p_fixed : rm.soff[e];
        P = rm.p_fixed ? rm.p_fixed : rm.soff[e + 1] - s0;
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
    uint64_t hm = __ballot(hit);
    bytes += (2 * D + 1) * B * 8;
    if constexpr ((MODE & kModeObb) != 0) {
        // spheres whose body's oriented box misses are dropped
        bool keep = false;
        uint64_t sp = 0;
        if (hm && lane < rm.nbody) {
            sp = rm.body_sph[lane];
            if (sp & hm) {
                keep = obb_box_meet64<D>(rm.obb64 + (e * rm.nbody + lane) * obb_words(D), lo, hi);
                bytes += obb_words(D) * 8;
            }
        }
        uint64_t allowed = keep ? sp : 0ull;
        for (int o = 32; o > 0; o >>= 1) allowed |= __shfl_xor(allowed, o);
        hm &= allowed;
    }
    if (!hm) return;
    bool S;
    if constexpr ((MODE & kModeSplines) != 0) {
        S = splines_meet64<D>(rm, e, hm, lo, hi, &bytes);
    } else {
        const CopyMap cm = copy_map((int)(P / B));
        S = copies_meet64<D>(rm, rm.samp64 + copy_stride<D>() * s0, P, cm, hm, lo, hi, rad, lst, &bytes);
    }
    ++n_outer;
    if (lane == 0) add_counts(rm, e, en.sign, S ? en.sign : 0);
}

// ------------------------------------------------------------------------
// k_item: one block per work item (grid cell c, a chunk of at most 256 of
// its edges; the chunk size is the roadmap's work-item size).
//
//   1. every thread owns one edge of the item.  The changed entries covering
//      the cell are staged in LDS (tiles of kSubTile) and registered in a
//      block-local pruning grid (an entry over more than kWideCells of its
//      cells is a candidate of every edge); a thread ORs the masks of the
//      pruning cells its edge's box covers and marks the candidates whose
//      box meets its edge's box, 32 per LDS word.  With several grid cells a
//      pair is taken only by the cell holding the lower corner of the two
//      boxes' intersection, so each (edge, entry) pair is tested once.
//   2. outer test, lanes = (pair, sphere): separation and end-sphere tests
//      first; the tests they leave open are queued in LDS and run densely
//      with the exact segment-box minimum.  Each pair keeps the sphere whose
//      capsule met deepest and the configuration nearest the capsule axis'
//      closest point to the box.
//   3. probe: that one copy is tested first.  S is an existence test, so a
//      copy found to meet settles the pair and its other copies are not
//      tested; the result is the same, only the order of the tests changes.
//   4. inner test of the pairs the probe left open, rows = (pair, sphere
//      whose capsule met), lanes = configurations: every copy of those
//      spheres.
//   5. per pair C and S; the edge's counter deltas are summed in LDS and
//      added once per edge.  In FP32 a pair whose decision fell inside the
//      rounding band goes to the block's re-test region, decided in binary64
//      by k_fp64 (one wavefront per pair); when the region is full the
//      whole item is left to k_fp64's second part, which runs it in binary64.
// ------------------------------------------------------------------------

constexpr int kSubTile = 128;             // changed entries staged per tile
constexpr int kSlots = 2;                 // edge slots per thread
constexpr int kItemCap = kSlots * kBlock; // edges per work item at most
constexpr int kWords = kSubTile / 32;     // overlap words per edge
constexpr int kPairCap = kBlock;          // pairs per round (one per thread)
static_assert(rt_cap_of(1) == kPairCap, "a share's re-test region holds a round");
constexpr int kRowCap = 256;              // (pair, sphere) rows per copy round
constexpr int kOpenCap = 1024;            // capsule tests queued for the exact part
static_assert(kWords == 4, "a slab mask holds one uint4 of entry bits");
static_assert(kSubTile <= 65536 && kItemCap <= 65536, "a pair is (edge slot << 16) | entry in 32 bits");
static_assert(kLocalCells * 4 == kWords * kItemCap, "the overlap words reuse the slab masks' storage");
static_assert(2 * 3 * slabs_of(3) <= kLocalCells && 2 * 2 * slabs_of(2) <= kLocalCells && slabs_of(2) <= 128 &&
                  slabs_of(3) <= 128,
              "the slab masks fit their storage and one wavefront's scan (two slabs a lane)");
static_assert(kOpenCap >= 3 * kRowCap + 1, "the rows fit the capsule queue's storage");
static_assert(kOpenCap * 4 >= kPairCap * 8 + kBlock * 4 + 64 * 8, "the overflow re-test fits the queue's storage");

__device__ inline int pe_slot(uint32_t v) { return (int)(v >> 16); }
__device__ inline int pe_entry(uint32_t v) { return (int)(v & 0xFFFFu); }

template <typename T>
struct ExactBoxes {
    T lo[3][kSubTile], hi[3][kSubTile];
};
struct NoBoxes {};
struct Radii32 {
    float r32[64];                        // sphere radii, binary32 (for the band)
};
struct NoRadii {};

template <typename T>
struct ItemLds {
    float4 blo[kSubTile], bhi[kSubTile];  // binary32 boxes: (lo, sbox), (hi, 0)
    int sign[kSubTile], gidx[kSubTile];
    // binary64 boxes for the binary64 kernel (the binary32 ones serve FP32)
    typename std::conditional<std::is_same<T, double>::value, ExactBoxes<double>, NoBoxes>::type x;
    typename std::conditional<std::is_same<T, float>::value, Radii32, NoRadii>::type r;
    union {
        // slab masks: sm[(2 d + 0) n + s] the staged entries whose slab range
        // on axis d starts at or before slab s, sm[(2 d + 1) n + s] those
        // whose range ends at or after it (n = slabs_of(D))
        uint4 sm[kLocalCells];
        uint32_t om[kWords][kItemCap];    // then the staged entries each edge's box meets
    } g;
    uint32_t cfg0[kItemCap];              // first configuration of each edge (sample / B)
    int edge[kItemCap], ej[kItemCap];     // edge id, configurations per sphere
    float es[kItemCap];                   // edge s (largest |coordinate| of its box)
    int dC[kItemCap], dS[kItemCap];
    uint32_t pe[kPairCap];                // edge slot << 16 | staged entry
    unsigned long long hm[kPairCap], um[kPairCap];
    uint32_t key[kPairCap];               // probe_key of the deepest capsule hit
    // the capsule-test queue is dead once the exact part has run; the rows
    // and their copy offsets live after it, in the same storage, and after
    // the decisions it is the scratch of a binary64 overflow re-test
    union alignas(8) {
        uint32_t open[kOpenCap];          // queued (pair << 6 | sphere) capsule tests
        struct {
            uint32_t row[kRowCap];        // pair << 6 | sphere
            uint32_t rcopy[kRowCap + 1];
            uint32_t rbase[kRowCap];      // splines: the row's first segment
        } rw;
    } u;
    int nopen;
    uint32_t sf[kPairCap];
    int wsum[kWaves];
    int rc_n, rc_start, defer;
    int pl_n, pl_start;                   // pairs this block listed (pair listing)
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

// Rounding band of a binary32 margin (squared-distance units): tau (s + R)
// (R + L) + tau^2 s^2, where s bounds every coordinate of the pair, R is the
// radius tested and L the L1 length of the capsule axis (0 for a sphere).
// The margin's rounding error is below 28 u s (R + L) + 7 u R^2 + O(u^2 s^2)
// (u = 2^-24), so tau = 1e-5 (about 168 u) leaves a factor of six.  The
// derivation assumes s <= 2^20 R; beyond that every decision is re-tested.
__device__ inline float band_of(float tau, float s, float R, float L)
{
    if (!(s <= 1048576.0f * R)) return INFINITY;
    return tau * (s + R) * (R + L) + (s > 0.0f ? tau * tau * s * s : 0.0f);
}

// Slab of coordinate x on axis d of the block-local slab masks, clamped to
// [0, n).  The subtraction, the product and floor are monotone, so the slab
// ranges of two boxes that share a point overlap on every axis.
__device__ inline int slab_of(const RmDev &rm, int d, float x, int n)
{
    const float f = floorf((x - rm.sl_org[d]) * rm.sl_inv[d]);
    return (int)fminf(fmaxf(f, 0.0f), (float)(n - 1));
}

// order-preserving map of a binary32 value to an unsigned key
__device__ inline uint32_t ordered_key(float f)
{
    const uint32_t u = __float_as_uint(f);
    return (u & 0x80000000u) ? ~u : (u | 0x80000000u);
}

// Probe key of a capsule hit: the margin's order (16 high bits), the
// parameter of the closest point (10 bits) and the sphere (6 bits); the
// minimum over a pair's hits names its deepest one.
__device__ inline uint32_t probe_key(float mg, float t, int sphere)
{
    const uint32_t tq = (uint32_t)fminf(fmaxf(t, 0.0f) * 1023.0f + 0.5f, 1023.0f);
    return (ordered_key(mg) & 0xFFFF0000u) | (tq << 6) | (uint32_t)sphere;
}

// A step in [1, n) coprime with n, near n / 2 (1 for n <= 2): k * step % n
// then visits 0 .. n-1 in a spread order.
__device__ inline int coprime_step(int n)
{
    if (n <= 2) return 1;
    for (int s = n / 2 + 1; s < n; ++s) {
        int a = s, b = n;
        while (b) {
            const int t = a % b;
            a = b;
            b = t;
        }
        if (a == 1) return s;
    }
    return 1;
}

// One round of at most kPairCap pairs listed in L.pe (edge slot << 16 |
// entry): the outer test (capsules, then the oriented boxes), the probe, the
// inner test (copies or spline segments) and the decisions.  Item blocks
// (kShare false) sum each edge's counter deltas in L.dC / L.dS and leave
// their item whole to the binary64 pass when the re-test region is full;
// pair-share blocks (kShare true: slot and entry are the pair itself) add
// the deltas to the counters at once and re-test an overflow themselves.
template <int D, typename T, int MODE, bool kShare, typename Lds>
__device__ __forceinline__ void test_round(const RmDev &rm, Lds &L, const T *s_rad2, const int *s_lane, int np,
                                           uint32_t &n_pairs, uint32_t &n_outer, unsigned long long &bytes)
{
    constexpr bool kF32 = std::is_same<T, float>::value;
    constexpr bool kObb = (MODE & kModeObb) != 0;
    constexpr bool kSpl = (MODE & kModeSplines) != 0;
    constexpr int kSegW = 2 * D + 1;   // values per spline segment
    const int tid = threadIdx.x, lane = lane_id(), wv = tid >> 6;
    const int B = rm.B;
    const int Gw = 64 / B;
    const T *capb = kF32 ? (const T *)rm.cap32 : (const T *)rm.cap64;
    const T *samp = kF32 ? (const T *)rm.samp32 : (const T *)rm.samp64;
    const float band_rel = rm.band_rel;
    const int jfix = rm.p_fixed ? rm.p_fixed / B : 0;
    // coordinates of entry s in the kernel's precision
    auto box_lo = [&](int k, int s) -> T {
        if constexpr (kF32) return k == 0 ? L.blo[s].x : (k == 1 ? L.blo[s].y : L.blo[s].z);
        else return L.x.lo[k][s];
    };
    auto box_hi = [&](int k, int s) -> T {
        if constexpr (kF32) return k == 0 ? L.bhi[s].x : (k == 1 ? L.bhi[s].y : L.bhi[s].z);
        else return L.x.hi[k][s];
    };
    // per-pair results start empty (kPairCap == kBlock: pair tid)
    if (tid < np) {
        L.hm[tid] = 0ull;
        L.um[tid] = 0ull;
        L.key[tid] = ~0u;
    }
    if (tid == 0) L.nopen = 0;
    __syncthreads();
    n_pairs += np;
    // a (pair, sphere) result: capsule hit bits, the deepest hit as
    // the probe key, undecided bits
    auto record = [&](int p, int i, int cls, float mg, float tpar) {
        if (cls == kHit) {
            atomicOr(&L.hm[p], 1ull << i);
            atomicMin(&L.key[p], probe_key(mg, tpar, i));
        } else if (cls == kUnsure) {
            atomicOr(&L.um[p], 1ull << i);
        }
    };
    // ---- outer test, quick part: lanes = (pair, sphere); each lane
    // takes two pairs per step and issues both capsules' loads first.
    // FP32 lanes the quick tests leave open are queued for the exact
    // part, so the segment-box minimum runs on dense wavefronts.
    constexpr int kCapU = 2;
    const int slot = s_lane[lane] >> 8, ci = s_lane[lane] & 255;
    for (int p0 = 0; p0 < np; p0 += kWaves * Gw * kCapU) {
        T A[kCapU][D], Bq[kCapU][D], R2[kCapU];
        int pu[kCapU];
#pragma unroll
        for (int u = 0; u < kCapU; ++u) {
            pu[u] = p0 + (u * kWaves + wv) * Gw + slot;
            R2[u] = T(0);
            if (slot < Gw && pu[u] < np) {
                const int te = pe_slot(L.pe[pu[u]]);
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
            const bool act = slot < Gw && p < np;
            int cls = kMiss;
            T lo[D], hi[D];
            float band = 0.0f, mg = 0.0f, tpar = 0.0f;
            const T R = R2[u];
            const T RR = R * R;
            if (act) {
                const int s = pe_entry(L.pe[p]);
#pragma unroll
                for (int k = 0; k < D; ++k) {
                    lo[k] = box_lo(k, s);
                    hi[k] = box_hi(k, s);
                }
                if constexpr (kF32) {
                    const float sc = fmaxf(L.es[pe_slot(L.pe[p])], L.blo[s].w);
                    float len = 0.0f;
#pragma unroll
                    for (int k = 0; k < D; ++k) len += fabsf(Bq[u][k] - A[u][k]);
                    band = band_of(band_rel, sc, R, len);
                    float sep = 0.0f;
#pragma unroll
                    for (int k = 0; k < D; ++k)
                        sep = fmaxf(sep, fmaxf(lo[k] - fmaxf(A[u][k], Bq[u][k]), fminf(A[u][k], Bq[u][k]) - hi[k]));
                    const float dA = point_box32<D>(A[u], lo, hi), dB = point_box32<D>(Bq[u], lo, hi);
                    mg = fminf(dA, dB) - RR;
                    tpar = dA <= dB ? 0.0f : 1.0f;
                    cls = (sep > 0.0f && sep * sep - RR > band) ? kMiss : (mg < -band ? kHit : kOpen);
                } else {
                    double ts;
                    const double v = segbox64<D>(A[u], Bq[u], lo, hi, &ts);
                    cls = v <= RR ? kHit : kMiss;
                    mg = (float)(v - RR);
                    tpar = (float)ts;
                }
            }
            if constexpr (kF32) {
                const bool op = cls == kOpen;
                const uint64_t ob = __ballot(op);
                if (ob) {
                    int base = 0;
                    if (lane == 0) base = atomicAdd(&L.nopen, __popcll(ob));
                    base = __shfl(base, 0);
                    if (op) {
                        const int q = base + __popcll(ob & lanes_below());
                        if (q < kOpenCap) {
                            L.u.open[q] = ((uint32_t)p << 6) | (uint32_t)ci;
                            cls = kMiss;     // decided by the exact part
                        } else {
                            cls = kUnsure;   // queue full: the binary64 re-test decides
                        }
                    }
                }
            }
            if (act) record(p, ci, cls, mg, tpar);
        }
    }
    __syncthreads();
    if constexpr (kF32) {
        // ---- outer test, exact part: the queued tasks, one per lane
        const int nq = min(L.nopen, kOpenCap);
        for (int q = tid; q < nq; q += kBlock) {
            const uint32_t tk = L.u.open[q];
            const int p = (int)(tk >> 6), i = (int)(tk & 63u);
            const uint32_t pv = L.pe[p], te = pe_slot(pv), s = pe_entry(pv);
            const float *cp = (const float *)capb + (int64_t)L.edge[te] * (2 * D + 1) * B;
            float A[D], Bq[D], lo[D], hi[D];
#pragma unroll
            for (int k = 0; k < D; ++k) {
                A[k] = cp[k * B + i];
                Bq[k] = cp[(D + k) * B + i];
                lo[k] = box_lo(k, s);
                hi[k] = box_hi(k, s);
            }
            const float R = cp[2 * D * B + i];
            const float sc = fmaxf(L.es[te], L.blo[s].w);
            float len = 0.0f;
#pragma unroll
            for (int k = 0; k < D; ++k) len += fabsf(Bq[k] - A[k]);
            float ts;
            const float mg = segbox32<D>(A, Bq, lo, hi, ts) - R * R;
            record(p, i, classify_margin(mg, band_of(band_rel, sc, R, len)), mg, ts);
        }
        __syncthreads();
    }
    if constexpr (kObb) {
        // ---- oriented boxes: the outer part of sphere i is its
        // capsule intersected with its body's box, so a sphere
        // whose body's box misses is dropped (decided in binary64)
        if (tid < np) {
            const uint64_t cnd = L.hm[tid] | (kF32 ? L.um[tid] : 0ull);
            if (cnd) {
                const uint32_t pv = L.pe[tid], te = pe_slot(pv), s = pe_entry(pv);
                double lo[D], hi[D];
                if constexpr (kF32) {
                    const ChgEntry &en = rm.chg[L.gidx[s]];
#pragma unroll
                    for (int k = 0; k < D; ++k) {
                        lo[k] = en.lo[k];
                        hi[k] = en.hi[k];
                    }
                } else {
#pragma unroll
                    for (int k = 0; k < D; ++k) {
                        lo[k] = L.x.lo[k][s];
                        hi[k] = L.x.hi[k][s];
                    }
                }
                const double *ob = rm.obb64 + (int64_t)L.edge[te] * rm.nbody * obb_words(D);
                uint64_t keep = 0;
                for (int bd = 0; bd < rm.nbody; ++bd) {
                    const uint64_t sp = rm.body_sph[bd];
                    if (!(sp & cnd)) continue;
                    bytes += obb_words(D) * 8;
                    if (obb_box_meet64<D>(ob + bd * obb_words(D), lo, hi)) keep |= sp;
                }
                L.hm[tid] &= keep;
                if constexpr (kF32) L.um[tid] &= keep;
            }
        }
        __syncthreads();
    }
    // ---- probe: one copy per pair whose capsule met (the copy
    // form only; a sphere the boxes dropped is not probed)
    const int p = tid;   // kPairCap == kBlock: this thread's pair
    uint32_t f = 0;
    uint64_t hmp = 0;
    if (p < np) {
        hmp = L.hm[p];
        if (hmp && !kSpl && (!kObb || ((hmp >> (L.key[p] & 63u)) & 1ull))) {
            const uint32_t key = L.key[p];
            const int i = (int)(key & 63u);
            const uint32_t pv = L.pe[p], te = pe_slot(pv), s = pe_entry(pv);
            const int Je = L.ej[te];
            // the configuration nearest the deepest capsule's closest point
            const int jj = min(Je - 1, (int)((float)((key >> 6) & 1023u) * (1.0f / 1023.0f) * (float)(Je - 1) + 0.5f));
            T q[D], lo[D], hi[D];
            load_copy<D>(samp, (int64_t)L.cfg0[te] * B + (int64_t)i * Je + jj, q);
#pragma unroll
            for (int k = 0; k < D; ++k) {
                lo[k] = box_lo(k, s);
                hi[k] = box_hi(k, s);
            }
            bytes += D * sizeof(T);
            if constexpr (kF32) {
                const float sc = fmaxf(L.es[te], L.blo[s].w);
                const int cls = classify_margin(point_box32<D>(q, lo, hi) - s_rad2[i],
                                                band_of(band_rel, sc, L.r.r32[i], 0.0f));
                f = cls == kHit ? 1u : (cls == kUnsure ? 2u : 0u);
            } else {
                f = point_box64<D>(q, lo, hi) <= s_rad2[i] ? 1u : 0u;
            }
        }
        L.sf[p] = f;
    }
    // ---- rows: one per (open pair, sphere whose capsule met)
    const int ra = (p < np && !(f & 1u)) ? __popcll(hmp) : 0;
    int nrows;
    const int rpre = block_scan(ra, &nrows, L.wsum);
    __syncthreads();
    for (int q0 = 0; q0 < nrows; q0 += kRowCap) {
        const int nr = min(kRowCap, nrows - q0);
        if (ra > 0 && rpre < q0 + nr && rpre + ra > q0) {
            uint64_t m = hmp;
            int r = rpre;
            while (m && r < q0 + nr) {
                const int i = __ffsll((unsigned long long)m) - 1;
                m &= m - 1;
                if (r >= q0) L.u.rw.row[r - q0] = ((uint32_t)p << 6) | (uint32_t)i;
                ++r;
            }
        }
        __syncthreads();
        // the row's copies (spline segments): fixed count, or a scan
        // over the rows
        int ncopies = kSpl ? 0 : nr * jfix;
        if (kSpl || !jfix) {
            int cj[2], sum = 0;
            for (int h = 0; h < 2; ++h) {
                const int r = tid * 2 + h;
                cj[h] = 0;
                if (r < nr) {
                    const uint32_t rv = L.u.rw.row[r];
                    const int te = pe_slot(L.pe[rv >> 6]);
                    if constexpr (kSpl) {
                        const int64_t k = (int64_t)L.edge[te] * B + (int64_t)(rv & 63u);
                        const int32_t k0 = rm.sseg[k];
                        cj[h] = rm.sseg[k + 1] - k0;
                        L.u.rw.rbase[r] = (uint32_t)k0;
                    } else {
                        cj[h] = L.ej[te];
                    }
                }
                sum += cj[h];
            }
            const int cpre = block_scan(sum, &ncopies, L.wsum);
            int acc = cpre;
            for (int h = 0; h < 2; ++h) {
                const int r = tid * 2 + h;
                if (r < nr) L.u.rw.rcopy[r] = acc;
                acc += cj[h];
            }
            if (tid == 0) L.u.rw.rcopy[nr] = ncopies;
            __syncthreads();
        }
        // each thread gathers kCopyU copies (all their loads in
        // flight together), then tests them.  When the copies take several
        // passes (every sphere has jfix copies), the passes go through the
        // copy indices in groups of kCopyU, a group of one row per thread,
        // the groups in a strided order; a row whose pair has already met
        // the box is skipped: that pair's S is decided.
        constexpr int kCopyU = 4;
        const T *segb = kF32 ? (const T *)rm.seg32 : (const T *)rm.seg64;
        const bool grouped = !kSpl && jfix && ncopies > kBlock * kCopyU;
        const int ngr = grouped ? (jfix + kCopyU - 1) / kCopyU : 1;
        const int gstep = grouped ? coprime_step(ngr) : 1;
        const int nloop = grouped ? nr * ngr * kCopyU : ncopies;
        for (int c0 = 0; c0 < nloop; c0 += kBlock * kCopyU) {
            T q[kCopyU][kSpl ? kSegW : D];
            int cu_p[kCopyU], cu_i[kCopyU];
            int g_r = -1, g_j0 = 0;   // grouped: this thread's row and first copy index
            if (grouped) {
                const int f = c0 / kCopyU + tid;
                if (f < nr * ngr) {
                    const int g = f / nr;
                    g_r = f - g * nr;
                    g_j0 = ((g * gstep) % ngr) * kCopyU;
                    // other waves may be setting the bit now: reading it
                    // late only costs a skipped skip
                    if (c0 > 0 && (__hip_atomic_load(&L.sf[L.u.rw.row[g_r] >> 6], __ATOMIC_RELAXED,
                                                     __HIP_MEMORY_SCOPE_WORKGROUP) & 1u))
                        g_r = -1;
                }
            }
#pragma unroll
            for (int u = 0; u < kCopyU; ++u) {
                const int cidx = c0 + u * kBlock + tid;
                cu_p[u] = -1;
                cu_i[u] = 0;
                if (grouped ? (g_r >= 0 && g_j0 + u < jfix) : cidx < ncopies) {
                    int r, jj;
                    if (grouped) {
                        r = g_r;
                        jj = g_j0 + u;
                    } else if (!kSpl && jfix) {
                        r = cidx / jfix;
                        jj = cidx - r * jfix;
                    } else {
                        int lo_ = 0, hi_ = nr - 1;   // last row with rcopy[r] <= cidx
                        while (lo_ < hi_) {
                            const int mid = (lo_ + hi_ + 1) >> 1;
                            if (L.u.rw.rcopy[mid] <= (uint32_t)cidx) lo_ = mid;
                            else hi_ = mid - 1;
                        }
                        r = lo_;
                        jj = cidx - (int)L.u.rw.rcopy[r];
                    }
                    const uint32_t rv = L.u.rw.row[r];
                    const int pp = (int)(rv >> 6);
                    const int i = (int)(rv & 63u);
                    const int te = pe_slot(L.pe[pp]);
                    if constexpr (kSpl) {
                        const T *sg = segb + ((int64_t)L.u.rw.rbase[r] + jj) * kSegW;
#pragma unroll
                        for (int k = 0; k < kSegW; ++k) q[u][k] = sg[k];
                    } else {
                        const int Je = L.ej[te];
                        load_copy<D>(samp, (int64_t)L.cfg0[te] * B + (int64_t)i * Je + jj, q[u]);
                    }
                    cu_p[u] = pp;
                    cu_i[u] = i;
                }
            }
#pragma unroll
            for (int u = 0; u < kCopyU; ++u) {
                const int pp = cu_p[u];
                if (pp < 0) continue;
                const uint32_t pv = L.pe[pp], te = pe_slot(pv), s = pe_entry(pv);
                T lo[D], hi[D];
#pragma unroll
                for (int k = 0; k < D; ++k) {
                    lo[k] = box_lo(k, s);
                    hi[k] = box_hi(k, s);
                }
                int cls;
                if constexpr (kSpl) {
                    // a spline segment: the capsule (A, B, rho)
                    T A[D], Bq[D];
#pragma unroll
                    for (int k = 0; k < D; ++k) {
                        A[k] = q[u][k];
                        Bq[k] = q[u][D + k];
                    }
                    const T rho = q[u][2 * D];
                    bytes += kSegW * sizeof(T);
                    if constexpr (kF32) {
                        const float sc = fmaxf(L.es[te], L.blo[s].w);
                        float len = 0.0f;
#pragma unroll
                        for (int k = 0; k < D; ++k) len += fabsf(Bq[k] - A[k]);
                        float ts;
                        const float mg = segbox32<D>(A, Bq, lo, hi, ts) - rho * rho;
                        cls = classify_margin(mg, band_of(band_rel, sc, rho, len));
                    } else {
                        cls = segbox64<D>(A, Bq, lo, hi) <= rho * rho ? kHit : kMiss;
                    }
                } else {
                    bytes += D * sizeof(T);
                    if constexpr (kF32) {
                        const float sc = fmaxf(L.es[te], L.blo[s].w);
                        cls = classify_margin(point_box32<D>(q[u], lo, hi) - s_rad2[cu_i[u]],
                                              band_of(band_rel, sc, L.r.r32[cu_i[u]], 0.0f));
                    } else {
                        cls = point_box64<D>(q[u], lo, hi) <= s_rad2[cu_i[u]] ? kHit : kMiss;
                    }
                }
                if (cls == kHit) atomicOr(&L.sf[pp], 1u);
                else if (cls == kUnsure) atomicOr(&L.sf[pp], 2u);
            }
        }
        __syncthreads();
    }
    // ---- decisions
    bool unsure = false;
    int2 rec = make_int2(0, 0);
    if (p < np) {
        const uint64_t ump = kF32 ? L.um[p] : 0ull;
        if (hmp || ump) {
            const uint32_t fp = L.sf[p];
            const uint32_t pv = L.pe[p], te = pe_slot(pv), s = pe_entry(pv);
            unsure = kF32 && (!hmp || (!(fp & 1u) && ((fp & 2u) || ump)));
            if (unsure) {
                rec = make_int2(L.edge[te], L.gidx[s]);
            } else {
                const int sign = L.sign[s];
                if constexpr (kShare) {
                    add_counts(rm, L.edge[te], sign, (fp & 1u) ? sign : 0);
                } else {
                    atomicAdd(&L.dC[te], sign);
                    if (fp & 1u) atomicAdd(&L.dS[te], sign);
                }
                ++n_outer;
            }
        }
    }
    if constexpr (kF32) {
        // undecided pairs go to the block's re-test region for the binary64
        // pass.  An item block whose region is full leaves its item whole to
        // that pass; a pair share never fills its own region (it holds at
        // most rt_cap_of(pl_cap) pairs)
        int tot_u;
        const int upre = block_scan(unsure ? 1 : 0, &tot_u, L.wsum);
        if (tot_u > 0) {
            const int base = L.rc_n;
            if constexpr (kShare) {
                if (unsure) rm.rt[(int64_t)blockIdx.x * rt_cap_of(rm.pl_cap) + base + upre] = rec;
                __syncthreads();
                if (tid == 0) L.rc_n = base + tot_u;
            } else {
                const bool fits = !L.defer && base + tot_u <= rm.rc_cap;
                if (fits && unsure) rm.rc[(int64_t)blockIdx.x * rm.rc_cap + base + upre] = rec;
                __syncthreads();
                if (tid == 0) {
                    if (fits) L.rc_n = base + tot_u;
                    else L.defer = 1;
                }
            }
        }
    }
    __syncthreads();
}

// deferred == 0: the main pass: items li0, li0 + lstride, ... (statistics
// row and re-test region blockIdx.x).
// deferred == 1: the binary64 pass over the items the FP32 blocks left whole
// (their list rm.df, ctl->n_df long): entries li0, li0 + lstride, ...
// (statistics row li0).
//
// kList: the pair listing of the FP32 mode.  Each round of pairs goes to this
// block's region of the pair list (rm.pl, for the pair-share kernel) while
// the region has room; a round that does not fit is tested here, as the
// fused kernel does.
// kCont: this block may have visited the roadmap before in this launch (the
// batched kernel's claimed items): its re-test region continues from the
// count it wrote then, and its statistics are added to its row, which
// start from zero (both are cleared after they are read).
template <int D, typename T, int MODE, bool kList = false, bool kCont = false>
__device__ __forceinline__ void item_body(const RmDev &rm, int deferred, int li0, int lstride)
{
    constexpr bool kF32 = std::is_same<T, float>::value;
    static_assert(!kList || kF32, "the pair listing serves the FP32 mode");
    __shared__ ItemLds<T> L;
    __shared__ T s_rad2[64];
    const Ctl *ctl = rm.ctl;
    const int tid = threadIdx.x, lane = lane_id(), wv = tid >> 6;
    const int B = rm.B;
    // lane -> (pair slot, sphere) of the capsule phase, read from LDS where
    // needed rather than held in registers through the whole kernel
    __shared__ int s_lane[64];
    if (tid < 64) s_lane[tid] = ((tid / B) << 8) | (tid - (tid / B) * B);
    if (tid < kStats) L.acc[tid] = 0;
    if (tid < B) s_rad2[tid] = kF32 ? (T)rm.rad2_32[tid] : (T)(rm.rad64[tid] * rm.rad64[tid]);
    if constexpr (kF32) {
        if (tid < B) L.r.r32[tid] = (float)rm.rad64[tid];
    }
    if (tid == 0) {
        L.rc_n = (kCont && kF32 && !deferred) ? rm.rc_cnt[blockIdx.x] : 0;
        L.pl_n = 0;
    }
    const int status = ctl->status;
    const int n_df = (deferred && status == RGG_OK) ? ctl->n_df : 0;
    __syncthreads();
    // wavefront-uniform counts (kept in scalar registers) and per-lane ones
    uint32_t n_pairs = 0, visited = 0, cand = 0, n_outer = 0;
    unsigned long long bytes = 0;
    const int n_chg = ctl->n_chg;
    const int n_items = min(ctl->n_items, (int32_t)rm.items_cap);
    const bool single = rm.ncells == 1;
    const float4 *aabb = reinterpret_cast<const float4 *>(rm.aabb);
    const int jfix = rm.p_fixed ? rm.p_fixed / B : 0;
    constexpr int kSl = slabs_of(D);   // slabs per axis of the slab masks
    // next work item of this block; false when there is none
    int li = li0;
    auto next_item = [&](int &it) -> bool {
        if (!deferred) {
            if (status != RGG_OK || li >= n_items) return false;
            it = li;
        } else {
            if (li >= n_df) return false;
            it = rm.df[li];
        }
        li += lstride;
        return true;
    };
    int it;
    while (next_item(it)) {
        // with one cell the items are (0, h) and the cell's list is every
        // edge in order: the item's edges are beg .. end - 1 themselves
        const int2 item = single ? make_int2(0, it) : rm.items[it];
        const int64_t c = item.x;
        const int32_t cx = (int32_t)(c % rm.gdim[0]);
        const int32_t cy = (int32_t)((c / rm.gdim[0]) % rm.gdim[1]);
        const int32_t cz = (int32_t)(c / ((int64_t)rm.gdim[0] * rm.gdim[1]));
        int64_t beg, end;
        if (single) {
            beg = (int64_t)item.y * rm.chunk;
            end = min(rm.E, beg + rm.chunk);
        } else {
            beg = (int64_t)rm.cell_start[c] + (int64_t)item.y * rm.chunk;
            end = min((int64_t)rm.cell_start[c + 1], beg + rm.chunk);
        }
        const int n_e = (int)(end - beg);   // edge slots in use: tid, tid + kBlock
        int e[kSlots], J[kSlots];
        float es[kSlots];
        uint32_t j0[kSlots];
#pragma unroll
        for (int h = 0; h < kSlots; ++h) {
            const int sl = tid + h * kBlock;
            e[h] = 0;
            J[h] = 0;
            es[h] = 0.0f;
            j0[h] = 0;
            if (sl < n_e) {
                if (!single) {
                    // the cell list's slot: one contiguous load, no gather
                    const int4 cs = rm.cell_slot[beg + sl];
                    e[h] = cs.x;
                    es[h] = __int_as_float(cs.y);
                    j0[h] = (uint32_t)cs.z;
                    J[h] = cs.w;
                } else {
                    e[h] = (int)(beg + sl);
                    es[h] = aabb[2 * (int64_t)e[h]].w;
                    if (jfix) {
                        J[h] = jfix;
                        j0[h] = (uint32_t)((int64_t)e[h] * jfix);
                    } else {
                        const int64_t s0 = rm.soff[e[h]];
                        j0[h] = (uint32_t)(s0 / B);
                        J[h] = (int)((rm.soff[e[h] + 1] - s0) / B);
                    }
                }
                bytes += 32;
            }
        }
        // with one cell every entry covers it: the first tile's entries are
        // requested together with the edges (binary32 boxes, size, sign)
        const bool pf = kF32 && single;
        float4 pf_a = make_float4(0.0f, 0.0f, 0.0f, 0.0f), pf_b = pf_a;
        if (pf && tid < kSubTile && tid < n_chg) {
            const float4 *q = reinterpret_cast<const float4 *>(&rm.chg[tid]);
            pf_a = q[0];   // lo32[0..2], hi32[0]
            pf_b = q[1];   // hi32[1..2], sbox, sign
        }
        __syncthreads();   // the previous item is done with the LDS arrays
#pragma unroll
        for (int h = 0; h < kSlots; ++h) {
            const int sl = tid + h * kBlock;
            L.edge[sl] = e[h];
            L.es[sl] = es[h];
            L.cfg0[sl] = j0[h];
            L.ej[sl] = J[h];
            L.dC[sl] = 0;
            L.dS[sl] = 0;
        }
        if (wv == 0) visited += (uint32_t)n_e;
        if (tid == 0) {
            L.rc_start = L.rc_n;
            L.pl_start = L.pl_n;
            L.defer = 0;
            // the main pass visits every item once: clear the cell's mark with
            // its first chunk, so the next update starts from zero marks
            if (!deferred && !single && item.y == 0) atomicAnd(&rm.cell_bits[c >> 5], ~(1u << (c & 31)));
        }
        uint32_t had = 0;   // bit h: edge slot h has pairs
        bool fused = !kList;   // some round of this item was tested here
        int n_round = 0;       // this item's pair rounds so far
        for (int j0 = 0; j0 < n_chg; j0 += kSubTile) {
            // the slab masks start empty (the previous tile or item is done
            // with their storage); the staging scan's barriers order this
            // before they are filled
            for (int q = tid; q < 2 * D * kSl; q += kBlock) L.g.sm[q] = make_uint4(0u, 0u, 0u, 0u);
            // stage the entries covering this cell
            const int j = j0 + tid;
            const bool first = pf && j0 == 0;
            bool in = false;
            if (tid < kSubTile && j < n_chg) {
                if (first) {
                    in = true;
                } else {
                    const ChgEntry &en = rm.chg[j];
                    in = single || (cx >= en.c0[0] && cx <= en.c1[0] && cy >= en.c0[1] && cy <= en.c1[1] &&
                                    cz >= en.c0[2] && cz <= en.c1[2]);
                }
            }
            int nt;
            const int pos = block_scan(in ? 1 : 0, &nt, L.wsum);
            if (in) {
                if (first) {
                    L.blo[pos] = make_float4(pf_a.x, pf_a.y, pf_a.z, pf_b.z);
                    L.bhi[pos] = make_float4(pf_a.w, pf_b.x, pf_b.y, 0.0f);
                    L.sign[pos] = __float_as_int(pf_b.w);
                } else {
                    const ChgEntry &en = rm.chg[j];
                    L.blo[pos] = make_float4(en.lo32[0], en.lo32[1], en.lo32[2], en.sbox);
                    L.bhi[pos] = make_float4(en.hi32[0], en.hi32[1], en.hi32[2], 0.0f);
                    if constexpr (!kF32) {
                        for (int k = 0; k < 3; ++k) {
                            L.x.lo[k][pos] = en.lo[k];
                            L.x.hi[k][pos] = en.hi[k];
                        }
                    }
                    L.sign[pos] = en.sign;
                }
                L.gidx[pos] = j;
            }
            if (nt == 0) continue;   // uniform: nt is the block total
            const int nw = (nt + 31) >> 5;
            __syncthreads();
            // block-local slab masks: each staged entry marks the slab its
            // range starts in and the slab it ends in, on every axis ...
            if (tid < nt) {
                const float4 l = L.blo[tid], h = L.bhi[tid];
                const float lo3[3] = {l.x, l.y, l.z}, hi3[3] = {h.x, h.y, h.z};
                const uint32_t bit = 1u << (tid & 31);
                const int wd = tid >> 5;
                uint32_t *mw = reinterpret_cast<uint32_t *>(L.g.sm);
#pragma unroll
                for (int d = 0; d < D; ++d) {
                    atomicOr(&mw[((2 * d) * kSl + slab_of(rm, d, lo3[d], kSl)) * 4 + wd], bit);
                    atomicOr(&mw[((2 * d + 1) * kSl + slab_of(rm, d, hi3[d], kSl)) * 4 + wd], bit);
                }
            }
            __syncthreads();
            // ... then each axis's start marks become "starts at or before s"
            // (an OR over slabs 0..s) and its end marks "ends at or after s"
            // (an OR over s..n-1): one wavefront per (axis, mark), each lane
            // two slabs, the lanes joined by a wavefront scan
            for (int a = wv; a < 2 * D; a += kWaves) {
                const bool up = (a & 1) == 0;   // start marks: forward
                uint4 *arr = L.g.sm + a * kSl;
                const int s0 = 2 * lane, s1 = 2 * lane + 1;
                auto at = [&](int s) -> uint4 & { return arr[up ? s : kSl - 1 - s]; };
                uint4 v0 = s0 < kSl ? at(s0) : make_uint4(0u, 0u, 0u, 0u);
                uint4 v1 = s1 < kSl ? at(s1) : make_uint4(0u, 0u, 0u, 0u);
                v1 = make_uint4(v1.x | v0.x, v1.y | v0.y, v1.z | v0.z, v1.w | v0.w);
                uint4 ex = v1;   // inclusive OR over lanes 0..lane, then shifted
#pragma unroll
                for (int o = 1; o < 64; o <<= 1) {
                    const uint32_t x = __shfl_up(ex.x, o), y = __shfl_up(ex.y, o), z = __shfl_up(ex.z, o),
                                   w = __shfl_up(ex.w, o);
                    if (lane >= o) ex = make_uint4(ex.x | x, ex.y | y, ex.z | z, ex.w | w);
                }
                uint4 pre = make_uint4(__shfl_up(ex.x, 1), __shfl_up(ex.y, 1), __shfl_up(ex.z, 1),
                                       __shfl_up(ex.w, 1));
                if (lane == 0) pre = make_uint4(0u, 0u, 0u, 0u);
                if (s0 < kSl) at(s0) = make_uint4(pre.x | v0.x, pre.y | v0.y, pre.z | v0.z, pre.w | v0.w);
                if (s1 < kSl) at(s1) = make_uint4(pre.x | v1.x, pre.y | v1.y, pre.z | v1.z, pre.w | v1.w);
            }
            __syncthreads();
            // the staged entries each of this thread's edges meets, 32 per
            // word: the candidates whose slab range meets the edge's on
            // every axis (all reads of the slab masks first: their storage
            // then takes the words), then the exact test against the edge's
            // box
            float4 bl[kSlots], bh[kSlots];
            uint32_t cw[kSlots][kWords];
            // both slots' boxes are requested before either is used
#pragma unroll
            for (int h = 0; h < kSlots; ++h) {
                const int sl = tid + h * kBlock;
                bl[h] = make_float4(0, 0, 0, 0);
                bh[h] = bl[h];
                if (sl < n_e) {
                    bl[h] = aabb[2 * (int64_t)L.edge[sl]];
                    bh[h] = aabb[2 * (int64_t)L.edge[sl] + 1];
                }
            }
#pragma unroll
            for (int h = 0; h < kSlots; ++h) {
                const int sl = tid + h * kBlock;
#pragma unroll
                for (int w = 0; w < kWords; ++w) cw[h][w] = 0u;
                if (sl < n_e) {
                    const float lo3[3] = {bl[h].x, bl[h].y, bl[h].z}, hi3[3] = {bh[h].x, bh[h].y, bh[h].z};
                    uint4 m = make_uint4(~0u, ~0u, ~0u, ~0u);
#pragma unroll
                    for (int d = 0; d < D; ++d) {
                        // entries starting at or before the edge's last slab
                        // and ending at or after its first
                        const uint4 st = L.g.sm[(2 * d) * kSl + slab_of(rm, d, hi3[d], kSl)];
                        const uint4 en = L.g.sm[(2 * d + 1) * kSl + slab_of(rm, d, lo3[d], kSl)];
                        m = make_uint4(m.x & st.x & en.x, m.y & st.y & en.y, m.z & st.z & en.z, m.w & st.w & en.w);
                    }
                    cw[h][0] = m.x;
                    cw[h][1] = m.y;
                    cw[h][2] = m.z;
                    cw[h][3] = m.w;
                }
            }
            __syncthreads();
            int cnt = 0;
#pragma unroll
            for (int h = 0; h < kSlots; ++h) {
                const int sl = tid + h * kBlock;
                if (sl >= n_e) continue;
                int ch = 0;
#pragma unroll
                for (int w = 0; w < kWords; ++w) {
                    if (w < nw) {
                        const int left = nt - 32 * w;   // staged entries from this word on
                        uint32_t m = cw[h][w] & (left >= 32 ? ~0u : ((1u << left) - 1u)), bits = 0;
                        while (m) {
                            const int b = __ffs(m) - 1;
                            m &= m - 1;
                            const float4 l = L.blo[w * 32 + b], hb = L.bhi[w * 32 + b];
                            bool hit = (l.x <= bh[h].x) & (hb.x >= bl[h].x) & (l.y <= bh[h].y) & (hb.y >= bl[h].y) &
                                       (l.z <= bh[h].z) & (hb.z >= bl[h].z);
                            if (hit && !single) {
                                const float lo3[3] = {l.x, l.y, l.z};
                                hit = pair_owned<D, float>(rm, bl[h], lo3, c);
                            }
                            bits |= (uint32_t)hit << b;
                        }
                        L.g.om[w][sl] = bits;
                        ch += __popc(bits);
                    }
                }
                cnt += ch;
                if (ch) had |= 1u << h;
            }
            int tp;
            const int pre = block_scan(cnt, &tp, L.wsum);
            for (int r0 = 0; r0 < tp; r0 += kPairCap) {
                const int np = min(kPairCap, tp - r0);
                if (cnt > 0 && pre < r0 + np && pre + cnt > r0) {
                    int k = pre;
                    for (int h = 0; h < kSlots && k < r0 + np; ++h) {
                        const int sl = tid + h * kBlock;
                        if (sl >= n_e) break;
                        for (int w = 0; w < nw && k < r0 + np; ++w) {
                            uint32_t m = L.g.om[w][sl];
                            while (m && k < r0 + np) {
                                const int s = (w << 5) + __ffs(m) - 1;
                                m &= m - 1;
                                if (k >= r0) L.pe[k - r0] = ((uint32_t)sl << 16) | (uint32_t)s;
                                ++k;
                            }
                        }
                    }
                }
                if constexpr (kList) {
                    // after the item's first inline_rounds rounds, a round
                    // goes to the pair list when the region has room
                    if (n_round++ >= rm.inline_rounds) {
                        __syncthreads();   // the round's pairs are in L.pe
                        const int base = L.pl_n;
                        if (base + np <= rm.pl_cap) {
                            if (tid < np) {
                                const uint32_t v = L.pe[tid];
                                rm.pl[(int64_t)blockIdx.x * rm.pl_cap + base + tid] =
                                    make_int2(L.edge[pe_slot(v)], L.gidx[pe_entry(v)]);
                            }
                            bytes += tid < np ? 8 : 0;
                            __syncthreads();
                            if (tid == 0) L.pl_n = base + np;
                            __syncthreads();
                            continue;
                        }
                    }
                    fused = true;
                }
                test_round<D, T, MODE, false>(rm, L, s_rad2, s_lane, np, n_pairs, n_outer, bytes);
            }
        }
        cand += (uint32_t)(__popcll(__ballot(had & 1u)) + __popcll(__ballot(had & 2u)));
        if (fused) bytes += (unsigned long long)__popc(had) * ((2 * D + 1) * B * sizeof(T) + 16);
        __syncthreads();
        if (!L.defer) {
#pragma unroll
            for (int h = 0; h < kSlots; ++h) {
                const int sl = tid + h * kBlock;
                if (sl < n_e) add_counts(rm, L.edge[sl], L.dC[sl], L.dS[sl]);
            }
        } else if (tid == 0) {
            // the whole item goes to the binary64 pass: its queued re-tests
            // and listed pairs are withdrawn (the withdrawn pairs are
            // counted here, as the rounds this block tested are)
            L.acc[0] += (unsigned long long)(L.pl_n - L.pl_start);
            L.rc_n = L.rc_start;
            L.pl_n = L.pl_start;
            // each item is left whole at most once per update, so the
            // list (items_cap long) has room
            rm.df[atomicAdd(&rm.ctl->n_df, 1)] = it;
        }
    }
    __syncthreads();
    // the binary64 pass counts its pairs as re-tested
    // per-lane counts are summed over the wavefront first: LDS atomics on
    // one address from every lane are slow
    const unsigned long long w_outer = wave_sum_u64(n_outer), w_bytes = wave_sum_u64(bytes);
    if (tid == 0 && n_pairs) atomicAdd(&L.acc[deferred ? 2 : 0], (unsigned long long)n_pairs);
    const int byte_row = deferred ? kStatFp64Bytes : (kList ? kStatItemBytes : kStatPairBytes);
    if (lane == 0) {
        if (w_outer) atomicAdd(&L.acc[1], w_outer);
        if (w_bytes) atomicAdd(&L.acc[byte_row], w_bytes);
        if (visited) atomicAdd(&L.acc[4], (unsigned long long)visited);
        if (cand) atomicAdd(&L.acc[5], (unsigned long long)cand);
    }
    __syncthreads();
    // statistic k at bs[k * kStatBlocks]: item blocks add to row blockIdx &
    // (kStatRows - 1), shared with other blocks (atomics); the binary64 pass's
    // block li0 owns row li0
    unsigned long long *bs = rm.blk_stats + (deferred ? li0 : (int)(blockIdx.x & (kStatRows - 1)));
    if (!deferred) {
        if (tid < kStats && L.acc[tid]) atomicAdd(&bs[tid * kStatBlocks], L.acc[tid]);
        if (kF32 && tid == 0) {
            rm.rc_cnt[blockIdx.x] = L.rc_n;
            if (kList) rm.pl_cnt[blockIdx.x] = L.pl_n;
        }
    } else if (tid == 0 && (L.acc[1] | L.acc[2] | L.acc[kStatFp64Bytes])) {
        bs[1 * kStatBlocks] += L.acc[1];
        bs[2 * kStatBlocks] += L.acc[2];
        bs[kStatFp64Bytes * kStatBlocks] += L.acc[kStatFp64Bytes];
    }
}

// The binary32 kernel is held to 128 VGPRs (four waves per SIMD, four
// blocks per CU); the binary64 one keeps the compiler's choice.
template <int D, int MODE>
__global__ void __launch_bounds__(kBlock, 4) k_item32(RmDev rm)
{
    item_body<D, float, MODE, true>(rm, 0, (int)blockIdx.x, (int)gridDim.x);
}

template <int D, int MODE>
__global__ void __launch_bounds__(kBlock) k_item64(RmDev rm)
{
    item_body<D, double, MODE>(rm, 0, (int)blockIdx.x, (int)gridDim.x);
}

// Binary64 re-test of the pairs queued by the FP32 blocks whose regions this
// block takes, one wavefront per pair: the item blocks' re-test regions b,
// b + G, ... (at most 64 of them), then the pair shares' regions of the same
// blocks; statistics row b.
template <int D, int MODE>
__device__ __forceinline__ void retest_pairs(const RmDev &rm, int b, int G)
{
    const int kReg = kStatBlocks / G;
    __shared__ int s_lst[kWaves][64];
    __shared__ double s_rad[64];
    __shared__ int s_off[65];
    __shared__ unsigned long long s_acc[3];
    const int tid = threadIdx.x, lane = lane_id(), wv = tid >> 6;
    const bool ok = rm.ctl->status == RGG_OK;
    if (tid < rm.B) s_rad[tid] = rm.rad64[tid];
    if (tid < 3) s_acc[tid] = 0;
    unsigned long long n_re = 0, bytes = 0;
    uint32_t n_outer = 0;
    // regions [kReg] at reg[(b + k G) * cap], counts cnt[b + k G]
    auto run = [&](int32_t *cnt, const int2 *reg_base, int32_t cap) {
        __syncthreads();   // s_off is free
        // pair counts of this block's regions, as an exclusive prefix
        if (tid < 64) {
            int n = 0;
            if (tid < kReg) {
                int *rc = cnt + b + tid * G;
                const int v = *rc;   // loaded whatever the status, so both loads are in flight at once
                n = ok ? v : 0;
                *rc = 0;   // cleared for the next update
            }
            int tot;
            const int pre = wave_prefix(n, &tot);
            if (tid < kReg) s_off[tid] = pre;
            if (tid == 0) s_off[kReg] = tot;
        }
        __syncthreads();
        const int total = s_off[kReg];
        int reg = 0;
        for (int q = wv; q < total; q += kWaves) {
            while (s_off[reg + 1] <= q) ++reg;
            const int k = q - s_off[reg];
            const int2 pr = reg_base[(int64_t)(b + reg * G) * cap + k];
            retest_one<D, MODE>(rm, pr.x, pr.y, s_lst[wv], s_rad, n_outer, bytes);
            ++n_re;
        }
    };
    run(rm.rc_cnt, rm.rc, rm.rc_cap);
    if (rm.rt) run(rm.rt_cnt, rm.rt, rt_cap_of(rm.pl_cap));
    if (lane == 0 && n_re) {
        atomicAdd(&s_acc[0], n_re);
        atomicAdd(&s_acc[1], (unsigned long long)n_outer);
        atomicAdd(&s_acc[2], bytes);
    }
    __syncthreads();
    if (tid == 0 && s_acc[0]) {
        unsigned long long *bs = rm.blk_stats + b;
        bs[1 * kStatBlocks] += s_acc[1];
        bs[2 * kStatBlocks] += s_acc[0];
        bs[kStatFp64Bytes * kStatBlocks] += s_acc[2];
    }
}

// Binary64 re-test of the queued pairs of one roadmap, spread over the whole
// grid: every block sums the pair counts of all re-test regions (the item
// blocks' regions r, then the pair shares' as regions kStatBlocks + r) into
// one prefix in LDS, and wavefront w of W takes pairs w, w + W, ... of the
// regions' concatenation.  The pairs of a heavy region are thus spread over
// many wavefronts instead of one block's four.  The counts are not cleared
// here (another block may still be reading them): every block of the item
// kernel and of the pair-share kernel writes its own region's count at its
// end, and the label kernel's statistics block clears them for the batched
// pass, whose blocks write only the regions of roadmaps they visit.
template <int D, int MODE>
__device__ __forceinline__ void retest_spread(const RmDev &rm)
{
    constexpr int kReg = 2 * kStatBlocks;   // item regions, then share regions
    constexpr int kPer = kReg / kBlock;     // consecutive regions per thread
    __shared__ int s_pre[kReg];
    __shared__ int s_lst[kWaves][64];
    __shared__ double s_rad[64];
    __shared__ int s_w[kWaves];
    __shared__ unsigned long long s_acc[3];
    const int tid = threadIdx.x, lane = lane_id(), wv = tid >> 6;
    const int32_t *rt_cnt = rm.rt ? rm.rt_cnt : nullptr;
    if (tid < rm.B) s_rad[tid] = rm.rad64[tid];
    if (tid < 3) s_acc[tid] = 0;
    // coalesced loads of the counts, issued with the status load rather
    // than after it, then each thread sums its own kPer
    int n[kPer];
#pragma unroll
    for (int h = 0; h < kPer; ++h) {
        const int r = h * kBlock + tid;
        n[h] = r < kStatBlocks ? rm.rc_cnt[r] : (rt_cnt ? rt_cnt[r - kStatBlocks] : 0);
    }
    const bool ok = rm.ctl->status == RGG_OK;
#pragma unroll
    for (int h = 0; h < kPer; ++h) s_pre[h * kBlock + tid] = ok ? n[h] : 0;
    __syncthreads();
    int v[kPer], sum = 0;
#pragma unroll
    for (int j = 0; j < kPer; ++j) {
        v[j] = s_pre[tid * kPer + j];
        sum += v[j];
    }
    int total;
    int pre = block_scan(sum, &total, s_w);   // its barriers order the reads above before the writes below
#pragma unroll
    for (int j = 0; j < kPer; ++j) {
        s_pre[tid * kPer + j] = pre;
        pre += v[j];
    }
    __syncthreads();
    unsigned long long n_re = 0, bytes = 0;
    uint32_t n_outer = 0;
    const int W = (int)gridDim.x * kWaves;
    const int32_t rt_cap = rt_cap_of(rm.pl_cap);
    for (int q = (int)blockIdx.x * kWaves + wv; q < total; q += W) {
        // the region holding pair q: the last r with s_pre[r] <= q
        int lo = 0, hi = kReg - 1;
        while (lo < hi) {
            const int mid = (lo + hi + 1) >> 1;
            if (s_pre[mid] <= q) lo = mid;
            else hi = mid - 1;
        }
        const int k = q - s_pre[lo];
        const int2 pr = lo < kStatBlocks ? rm.rc[(int64_t)lo * rm.rc_cap + k]
                                         : rm.rt[(int64_t)(lo - kStatBlocks) * rt_cap + k];
        retest_one<D, MODE>(rm, pr.x, pr.y, s_lst[wv], s_rad, n_outer, bytes);
        ++n_re;
    }
    if (lane == 0 && n_re) {
        atomicAdd(&s_acc[0], n_re);
        atomicAdd(&s_acc[1], (unsigned long long)n_outer);
        atomicAdd(&s_acc[2], bytes);
    }
    __syncthreads();
    if (tid == 0 && s_acc[0]) {
        unsigned long long *bs = rm.blk_stats + blockIdx.x;
        bs[1 * kStatBlocks] += s_acc[1];
        bs[2 * kStatBlocks] += s_acc[0];
        bs[kStatFp64Bytes * kStatBlocks] += s_acc[2];
    }
}

// The binary64 pass of the FP32 mode of one roadmap: the queued pairs
// (spread over the grid), then the items left whole because their blocks'
// re-test regions were full (rare: skipped unless one was deferred in this
// update; entries b, b + G, ... of the roadmap's list).  One kernel for both, so the common case
// costs one launch; it runs one block per CU, so the binary64 item path's
// registers cost no occupancy.
template <int D, int MODE>
__global__ void __launch_bounds__(kBlock) k_fp64(RmDev rm)
{
    const int n_df = rm.ctl->n_df;
    retest_spread<D, MODE>(rm);
    if (!n_df) return;
    item_body<D, double, MODE>(rm, 1, (int)blockIdx.x, (int)gridDim.x);
}

// ------------------------------------------------------------------------
// k_pairs: the balanced pair testing of the FP32 mode (launched only when
// the item kernel lists pairs).  The listing leaves each block's pairs in
// its region of rm.pl; this kernel cuts the concatenation of the regions
// into equal shares, as many as the device holds at once while a share fits
// one round, so every block tests the same number of pairs whatever the
// items' sizes were.  A share runs in rounds of kPairCap pairs through the
// same phases as an item block's round (each pair is its own edge slot and
// entry); counter deltas go to the counters at once.
// ------------------------------------------------------------------------

struct ShareLds {
    float4 blo[kPairCap], bhi[kPairCap];  // the pairs' entries: (lo, sbox), (hi, 0)
    int sign[kPairCap], gidx[kPairCap];
    NoBoxes x;
    Radii32 r;
    uint32_t cfg0[kPairCap];              // first configuration of each pair's edge
    int edge[kPairCap], ej[kPairCap];     // edge id, configurations per sphere
    float es[kPairCap];                   // edge s (largest |coordinate| of its box)
    uint32_t pe[kPairCap];                // pair << 16 | pair
    unsigned long long hm[kPairCap], um[kPairCap];
    uint32_t key[kPairCap];
    union alignas(8) {
        uint32_t open[kOpenCap];
        struct {
            uint32_t row[kRowCap];
            uint32_t rcopy[kRowCap + 1];
            uint32_t rbase[kRowCap];
        } rw;
    } u;
    int nopen;
    uint32_t sf[kPairCap];
    int wsum[kWaves];
    int rc_n;
    int pref[kStatBlocks + 1];            // listed pairs before each region
    unsigned long long acc[kStats];
};

template <int D, int MODE>
__device__ __forceinline__ void share_body(const RmDev &rm)
{
    __shared__ ShareLds L;
    __shared__ float s_rad2[64];
    __shared__ int s_lane[64];
    const int tid = threadIdx.x, lane = lane_id();
    const int B = rm.B;
    if (tid < 64) s_lane[tid] = ((tid / B) << 8) | (tid - (tid / B) * B);
    if (tid < kStats) L.acc[tid] = 0;
    if (tid < B) {
        s_rad2[tid] = rm.rad2_32[tid];
        L.r.r32[tid] = (float)rm.rad64[tid];
    }
    if (tid == 0) L.rc_n = 0;   // pairs queued in this share's re-test region
    // prefix of the regions' pair counts: kPer consecutive regions per thread
    constexpr int kPer = kStatBlocks / kBlock;
    static_assert(kStatBlocks % kBlock == 0, "regions are scanned kPer per thread");
    int c[kPer], sum = 0;
#pragma unroll
    for (int k = 0; k < kPer; ++k) {
        c[k] = rm.pl_cnt[tid * kPer + k];
        sum += c[k];
    }
    int total;
    int pre = block_scan(sum, &total, L.wsum);
#pragma unroll
    for (int k = 0; k < kPer; ++k) {
        L.pref[tid * kPer + k] = pre;
        pre += c[k];
    }
    if (tid == 0) L.pref[kStatBlocks] = total;
    __syncthreads();
    // the shares: as many as fit on the device at once while each is at most
    // one round, more (up to the grid) when the pairs need more rounds; a
    // share then holds at most max(kPairCap, pl_cap) pairs
    const int G = min((int)gridDim.x, max(rm.test_slots, (total + kPairCap - 1) / kPairCap));
    const int b = (int)blockIdx.x;
    const int64_t lo = b < G ? (int64_t)total * b / G : 0;
    const int64_t hi = b < G ? (int64_t)total * (b + 1) / G : 0;
    const float4 *aabb = reinterpret_cast<const float4 *>(rm.aabb);
    const int jfix = rm.p_fixed ? rm.p_fixed / B : 0;
    uint32_t n_pairs = 0, n_outer = 0;
    unsigned long long bytes = 0;
    for (int64_t r0 = lo; r0 < hi; r0 += kPairCap) {
        const int np = (int)min((int64_t)kPairCap, hi - r0);
        if (tid < np) {
            // the pair's region: the last one whose first pair is at most g
            const int g = (int)(r0 + tid);
            int a = 0, z = kStatBlocks - 1;
            while (a < z) {
                const int m = (a + z + 1) >> 1;
                if (L.pref[m] <= g) a = m;
                else z = m - 1;
            }
            const int2 pr = rm.pl[(int64_t)a * rm.pl_cap + (g - L.pref[a])];
            const int e = pr.x, j = pr.y;
            const float4 *q = reinterpret_cast<const float4 *>(&rm.chg[j]);
            const float4 qa = q[0], qb = q[1];   // lo32[0..2], hi32[0]; hi32[1..2], sbox, sign
            L.blo[tid] = make_float4(qa.x, qa.y, qa.z, qb.z);
            L.bhi[tid] = make_float4(qa.w, qb.x, qb.y, 0.0f);
            L.sign[tid] = __float_as_int(qb.w);
            L.gidx[tid] = j;
            L.edge[tid] = e;
            L.es[tid] = aabb[2 * (int64_t)e].w;
            if (jfix) {
                L.ej[tid] = jfix;
                L.cfg0[tid] = (uint32_t)((int64_t)e * jfix);
            } else {
                const int64_t s0 = rm.soff[e];
                L.cfg0[tid] = (uint32_t)(s0 / B);
                L.ej[tid] = (int)((rm.soff[e + 1] - s0) / B);
            }
            L.pe[tid] = ((uint32_t)tid << 16) | (uint32_t)tid;
            // the pair record and entry, the edge's box word; its capsules
            // once per run of pairs of one edge
            bytes += 8 + 32 + 4;
        }
        __syncthreads();
        if (tid < np && (tid == 0 || L.edge[tid] != L.edge[tid - 1]))
            bytes += (unsigned long long)((2 * D + 1) * B * sizeof(float) + (jfix ? 0 : 16));
        test_round<D, float, MODE, true>(rm, L, s_rad2, s_lane, np, n_pairs, n_outer, bytes);
    }
    __syncthreads();
    const unsigned long long w_outer = wave_sum_u64(n_outer), w_bytes = wave_sum_u64(bytes);
    if (tid == 0 && n_pairs) atomicAdd(&L.acc[0], (unsigned long long)n_pairs);
    if (lane == 0) {
        if (w_outer) atomicAdd(&L.acc[1], w_outer);
        if (w_bytes) atomicAdd(&L.acc[kStatPairBytes], w_bytes);
    }
    __syncthreads();
    // the statistics rows are shared by blocks (atomics)
    unsigned long long *bs = rm.blk_stats + (blockIdx.x & (kStatRows - 1));
    if (tid == 0) {
        if (L.acc[0]) atomicAdd(&bs[0], L.acc[0]);
        if (L.acc[1]) atomicAdd(&bs[1 * kStatBlocks], L.acc[1]);
        if (L.acc[2]) atomicAdd(&bs[2 * kStatBlocks], L.acc[2]);
        if (L.acc[kStatPairBytes]) atomicAdd(&bs[kStatPairBytes * kStatBlocks], L.acc[kStatPairBytes]);
        rm.rt_cnt[blockIdx.x] = L.rc_n;
    }
}

template <int D, int MODE>
__global__ void __launch_bounds__(kBlock, 4) k_pairs(RmDev rm)
{
    share_body<D, MODE>(rm);
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

// Each thread of a label block owns kLabelRun consecutive edges of the tile.
constexpr int kLabelRun = kLabelTile / kBlock;
static_assert(kLabelRun == 16, "a run is stored as one 16-byte label word");

__device__ inline void load_run(const RmDev &rm, int64_t e0, int2 (&c)[kLabelRun])
{
    if (e0 + kLabelRun <= rm.E) {
        const int4 *src = reinterpret_cast<const int4 *>(rm.cnt + e0);   // 16-byte aligned: e0 % 16 == 0
#pragma unroll
        for (int h = 0; h < kLabelRun / 2; ++h) {
            const int4 v = src[h];
            c[2 * h] = make_int2(v.x, v.y);
            c[2 * h + 1] = make_int2(v.z, v.w);
        }
    } else {
#pragma unroll
        for (int h = 0; h < kLabelRun; ++h) c[h] = e0 + h < rm.E ? rm.cnt[e0 + h] : make_int2(0, 0);
    }
}

// k_count: gray edges per tile
__device__ __forceinline__ void count_body(const RmDev &rm, int tile)
{
    __shared__ int s_w[kWaves];
    const int tid = threadIdx.x;
    const int64_t e0 = (int64_t)tile * kLabelTile + (int64_t)tid * kLabelRun;
    int2 c[kLabelRun];
    load_run(rm, e0, c);
    int ng = 0;
#pragma unroll
    for (int h = 0; h < kLabelRun; ++h) ng += (e0 + h < rm.E && label_of(c[h]) == RGG_GRAY) ? 1 : 0;
    const int tot = block_sum(ng, s_w);
    if (tid == 0) rm.tile_cnt[tile] = tot;
}

// Folds the statistics rows of the update into *res (when res is not null)
// and clears them for the next update (the item kernels add to them).
__device__ __forceinline__ void fold_stats(const RmDev &rm, rgg_update_result *res)
{
    __shared__ unsigned long long s_part[kWaves][kStats];
    const int tid = threadIdx.x;
    static_assert(kStatRows == kBlock, "one statistics row a thread");
    unsigned long long v[kStats];
#pragma unroll
    for (int k = 0; k < kStats; ++k) v[k] = rm.blk_stats[k * kStatBlocks + tid];
#pragma unroll
    for (int k = 0; k < kStats; ++k) rm.blk_stats[k * kStatBlocks + tid] = 0ull;
    const int lane = lane_id(), wv = tid >> 6;
#pragma unroll
    for (int k = 0; k < kStats; ++k) {
        const unsigned long long w = wave_sum_u64(v[k]);
        if (lane == 0) s_part[wv][k] = w;
    }
    __syncthreads();
    if (tid == 0 && res) {
        int64_t a[kStats];
        for (int k = 0; k < kStats; ++k) {
            unsigned long long t = 0;
            for (int w = 0; w < kWaves; ++w) t += s_part[w][k];
            a[k] = (int64_t)t;
        }
        res->n_pairs = a[0];
        res->n_outer_hits = a[1];
        res->n_rechecked = a[2];
        res->test_bytes = a[kStatPairBytes] + a[kStatItemBytes] + a[kStatFp64Bytes];
        res->n_cells_visited = a[4];
        res->n_candidate_edges = a[5];
        res->item_bytes = a[kStatItemBytes];
        res->fp64_bytes = a[kStatFp64Bytes];
    }
}

// Labels of this thread's run of edges e0 .. e0 + kLabelRun - 1; returns
// how many are GRAY.
__device__ __forceinline__ int run_labels(const RmDev &rm, int64_t e0, uint8_t (&lab)[kLabelRun])
{
    int2 c[kLabelRun];
    load_run(rm, e0, c);
    int ng = 0;
#pragma unroll
    for (int h = 0; h < kLabelRun; ++h) {
        lab[h] = label_of(c[h]);
        ng += (e0 + h < rm.E && lab[h] == RGG_GRAY) ? 1 : 0;
    }
    return ng;
}

// Stores a run's labels (when labels is not null).
__device__ __forceinline__ void store_run(const RmDev &rm, uint8_t *labels, int64_t e0, const uint8_t (&lab)[kLabelRun])
{
    if (!labels) return;
    if (e0 + kLabelRun <= rm.E && ((uintptr_t)(labels + e0) & 15u) == 0) {
        uint32_t wds[kLabelRun / 4];
#pragma unroll
        for (int q = 0; q < kLabelRun / 4; ++q)
            wds[q] = (uint32_t)lab[4 * q] | ((uint32_t)lab[4 * q + 1] << 8) | ((uint32_t)lab[4 * q + 2] << 16) |
                     ((uint32_t)lab[4 * q + 3] << 24);
        *reinterpret_cast<uint4 *>(labels + e0) = make_uint4(wds[0], wds[1], wds[2], wds[3]);
    } else {
#pragma unroll
        for (int h = 0; h < kLabelRun; ++h)
            if (e0 + h < rm.E) labels[e0 + h] = lab[h];
    }
}

// Stores a tile's GRAY ids in ascending order from gray-list position
// `before` on (when gray is not null; ids past cap are dropped).  Each
// thread puts its run's ids in LDS at the tile-local positions pre, pre + 1,
// ..., then consecutive threads write consecutive positions, so the 8-byte
// stores coalesce instead of each thread's landing a few positions apart.
// Every thread of the block calls it (one barrier).
__device__ __forceinline__ void store_gray(const RmDev &rm, int64_t *gray, int64_t cap, int64_t e0,
                                           const uint8_t (&lab)[kLabelRun], int64_t before, int pre, int tot)
{
    __shared__ uint16_t s_gid[kLabelTile];   // tile-local edge index of each GRAY id
    static_assert(kLabelTile <= 65536, "a tile-local index fits 16 bits");
    if (!gray) return;
    const int64_t t0 = e0 - (int64_t)threadIdx.x * kLabelRun;   // the tile's first edge
    int p = pre;
#pragma unroll
    for (int h = 0; h < kLabelRun; ++h)
        if (e0 + h < rm.E && lab[h] == RGG_GRAY) s_gid[p++] = (uint16_t)(threadIdx.x * kLabelRun + h);
    __syncthreads();
    for (int i = threadIdx.x; i < tot; i += kBlock) {
        const int64_t pos = before + i;
        if (pos < cap) gray[pos] = t0 + s_gid[i];
    }
}

// k_write: labels and the ordered gray list, one tile per block (its first
// position is the sum of the earlier tiles' counts from k_count; the last
// tile reports n_gray, tile 0 the status); block `ntiles` instead folds the
// per-block statistics of the update.
__device__ __forceinline__ void write_body(const RmDev &rm, uint8_t *labels, int64_t *gray, int64_t cap,
                                          rgg_update_result *res, int force, int tile)
{
    __shared__ int s_w[kWaves];
    const int tid = threadIdx.x;
    if (tile == rm.ntiles) {
        if (!force) fold_stats(rm, res);
        return;
    }
    const int status = force ? RGG_OK : rm.ctl->status;
    if (tid == 0 && tile == 0 && res && !force) {
        res->status = status;
        res->n_changed = rm.ctl->n_chg;
        if (status != RGG_OK) res->n_gray = 0;
    }
    if (status != RGG_OK) return;
    const int64_t e0 = (int64_t)tile * kLabelTile + (int64_t)tid * kLabelRun;
    uint8_t lab[kLabelRun];
    const int ng = run_labels(rm, e0, lab);
    // gray edges before this tile
    int before = 0;
    for (int t = tid; t < tile; t += kBlock) before += rm.tile_cnt[t];
    before = block_sum(before, s_w);
    int tot;
    const int pre = block_scan(ng, &tot, s_w);
    if (tid == 0 && tile == rm.ntiles - 1 && res) res->n_gray = (int64_t)before + tot;
    if (tot == 0 && labels == nullptr) return;
    store_run(rm, labels, e0, lab);
    store_gray(rm, gray, cap, e0, lab, before, pre, tot);
}

// k_labels: k_count and k_write in one pass.  Blocks take their tiles in
// dispatch order (a ticket), publish their gray count, and add up the
// earlier tiles' counts by looking back over their published words,
// sixty-four at a time, stopping at the nearest tile that already published
// its inclusive prefix (the decoupled look-back scan of Merrill and Garland,
// "Single-pass Parallel Prefix Scan with Decoupled Look-back", 2016).  A
// block only waits on tiles whose blocks took earlier tickets and are
// therefore running, so every wait ends; the waits are bounded all the same
// and report RGG_E_DEVICE if a bound is ever reached.  The block with the
// last ticket folds the statistics.  k_diff clears the words and the ticket
// before each update.
constexpr unsigned long long kTileAgg = 1ull << 62, kTilePre = 2ull << 62, kTileVal = (1ull << 62) - 1;
constexpr int kLookBackSpins = 1 << 20;

__device__ __forceinline__ void labels_body(const RmDev &rm, uint8_t *labels, int64_t *gray, int64_t cap,
                                           rgg_update_result *res)
{
    __shared__ int s_w[kWaves];
    __shared__ int s_tile, s_fail;
    __shared__ long long s_before;
    const int tid = threadIdx.x, lane = lane_id(), wv = tid >> 6;
    if (tid == 0) s_tile = __hip_atomic_fetch_add(&rm.ctl->label_ticket, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    __syncthreads();
    const int tile = s_tile;
    if (tile >= rm.ntiles) {
        // every block has its ticket: the counter starts from zero next time
        if (tid == 0) __hip_atomic_store(&rm.ctl->label_ticket, 0, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        // the binary64 pass read the re-test counts without clearing them;
        // a batched pass needs them zero, as its item blocks write only the
        // regions of the roadmaps they visit
        if (rm.mixed) {
            for (int r = tid; r < kStatBlocks; r += kBlock) {
                rm.rc_cnt[r] = 0;
                if (rm.rt) rm.rt_cnt[r] = 0;
            }
        }
        fold_stats(rm, res);
        return;
    }
    const int status = rm.ctl->status;
    if (tid == 0 && tile == 0 && res) {
        res->status = status;
        res->n_changed = rm.ctl->n_chg;
        if (status != RGG_OK) res->n_gray = 0;
    }
    if (status != RGG_OK) return;   // every block returns here: no one waits
    const int64_t e0 = (int64_t)tile * kLabelTile + (int64_t)tid * kLabelRun;
    uint8_t lab[kLabelRun];
    const int ng = run_labels(rm, e0, lab);
    int tot;
    const int pre = block_scan(ng, &tot, s_w);
    unsigned long long *st = rm.tile_state;
    if (tid == 0)
        __hip_atomic_store(&st[tile], (tile == 0 ? kTilePre : kTileAgg) | (unsigned long long)tot, __ATOMIC_RELEASE,
                           __HIP_MEMORY_SCOPE_AGENT);
    if (wv == 0) {
        unsigned long long before = 0;
        bool fail = false;
        for (int t = tile - 1; t >= 0; t -= 64) {
            const int q = t - lane;              // lane l looks at tile t - l
            unsigned long long v = kTilePre;     // before tile 0: an inclusive prefix of 0
            bool ready = q < 0;
            for (int spin = 0;; ++spin) {
                if (!ready) {
                    v = __hip_atomic_load(&st[q], __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_AGENT);
                    ready = (v >> 62) != 0;
                }
                if (__ballot(!ready) == 0) break;
                if (spin >= kLookBackSpins) {
                    fail = true;
                    break;
                }
                __builtin_amdgcn_s_sleep(1);
            }
            if (fail) break;
            const uint64_t pm = __ballot((v >> 62) == 2);
            const int stop = pm ? __ffsll((unsigned long long)pm) - 1 : 63;
            before += wave_sum_u64(lane <= stop ? (v & kTileVal) : 0ull);
            if (pm) break;
        }
        if (lane == 0) {
            s_before = (long long)before;
            s_fail = fail ? 1 : 0;
        }
    }
    __syncthreads();
    const long long before = s_before;
    if (tid == 0) {
        __hip_atomic_store(&st[tile], kTilePre | (unsigned long long)(before + tot), __ATOMIC_RELEASE,
                           __HIP_MEMORY_SCOPE_AGENT);
        if (res && s_fail) res->status = RGG_E_DEVICE;
        if (res && tile == rm.ntiles - 1) res->n_gray = before + tot;
    }
    store_run(rm, labels, e0, lab);
    store_gray(rm, gray, cap, e0, lab, before, pre, tot);
}

__global__ void __launch_bounds__(kBlock) k_labels(RmDev rm, uint8_t *labels, int64_t *gray, int64_t cap,
                                                   rgg_update_result *res, int)
{
    labels_body(rm, labels, gray, cap, res);
}

__global__ void __launch_bounds__(kBlock) k_count(RmDev rm)
{
    count_body(rm, (int)blockIdx.x);
}

__global__ void __launch_bounds__(kBlock) k_write(RmDev rm, uint8_t *labels, int64_t *gray, int64_t cap,
                                                  rgg_update_result *res, int force)
{
    write_body(rm, labels, gray, cap, res, force, (int)blockIdx.x);
}

// ------------------------------------------------------------------------
// batched updates of distinct roadmaps: one launch per stage for all of
// them; each kernel finds its request in the device table
// ------------------------------------------------------------------------

// Copies a table row (or its device view) into LDS, all threads, barriers
// around.  One round of vector loads replaces the chain of scalar loads the
// compiler would otherwise issue field by field as the kernel needs them
// (each waiting on the one before, since the view holds the pointers).
template <typename R>
__device__ inline void load_row(R *dst, const R &src)
{
    static_assert(sizeof(R) % 4 == 0, "a row is copied as 32-bit words");
    __syncthreads();
    const uint32_t *a = reinterpret_cast<const uint32_t *>(&src);
    uint32_t *b = reinterpret_cast<uint32_t *>(dst);
    for (int k = threadIdx.x; k < (int)(sizeof(R) / 4); k += blockDim.x) b[k] = a[k];
    __syncthreads();
}
__device__ inline void load_rm(RmDev *dst, const RmDev &src) { load_row(dst, src); }

// One block per roadmap.  With h_tab (this launch's pinned host rows) the
// block reads its row from host memory and writes it to the device table,
// where the later stages read it.
__global__ void __launch_bounds__(kDiffBlock) k_diff_batch(BatchReq *tab, const BatchReq *h_tab)
{
    __shared__ BatchReq q;
    if (h_tab) {
        load_row(&q, h_tab[blockIdx.x]);
        const uint32_t *a = reinterpret_cast<const uint32_t *>(&q);
        uint32_t *b = reinterpret_cast<uint32_t *>(&tab[blockIdx.x]);
        for (int k = threadIdx.x; k < (int)(sizeof(BatchReq) / 4); k += blockDim.x) b[k] = a[k];
    } else {
        load_row(&q, tab[blockIdx.x]);
    }
    if (q.rm.D == 3) diff_body<3>(q.rm, q.a.old_b, q.a.new_b);
    else diff_body<2>(q.rm, q.a.old_b, q.a.new_b);
}

// The items of all requests of one group form one range: request r owns
// [P_r, P_r + n_items_r).  Block b of G takes items b, b + G, ..., up to
// kBatchStatic of them, then claims the rest one at a time from a counter
// (items kBatchStatic * G on), so blocks whose items were light take more
// and the launch ends near the mean block time rather than the heaviest
// block's.  A block may then visit a roadmap more than once: its re-test
// region and statistics row continue across the visits (kCont).  The next
// claim is issued before the current item runs, so its latency is hidden.
template <int D, typename T>
__device__ __forceinline__ void item_batch_body(const BatchReq *tab, const int32_t *grp, int n)
{
    __shared__ RmDev s_rm;
    __shared__ int s_pref[kMaxBatch + 1];
    __shared__ int s_w[kWaves];
    __shared__ int s_next;
    const int tid = threadIdx.x;
    int v = 0;
    if (tid < n) {
        const RmDev &rm = tab[grp[tid]].rm;
        v = rm.ctl->status == RGG_OK ? min(rm.ctl->n_items, (int32_t)rm.items_cap) : 0;
    }
    int tot;
    const int pre = block_scan(v, &tot, s_w);
    if (tid < n) s_pref[tid] = pre;
    if (tid == 0) s_pref[n] = tot;
    __syncthreads();
    const int G = (int)gridDim.x;
    int32_t *const claim = &tab[grp[0]].rm.ctl->claim;   // reset by the diff of this update
    int cur = -1;                                        // the request whose view s_rm holds
    int g = (int)blockIdx.x;
    for (int k = 0; g < tot; ++k) {
        // the request owning item g: the last r with s_pref[r] <= g (uniform)
        int lo = 0, hi = n - 1;
        while (lo < hi) {
            const int mid = (lo + hi + 1) >> 1;
            if (s_pref[mid] <= g) lo = mid;
            else hi = mid - 1;
        }
        const bool claims = k + 1 >= kBatchStatic;
        int nxt = 0;
        if (claims && tid == 0) nxt = kBatchStatic * G + atomicAdd(claim, 1);
        if (lo != cur) {
            load_rm(&s_rm, tab[grp[lo]].rm);
            cur = lo;
        }
        item_body<D, T, 0, false, true>(s_rm, 0, g - s_pref[lo], 1 << 30);
        if (claims && tid == 0) s_next = nxt;
        __syncthreads();
        g = claims ? s_next : g + G;
    }
}

template <int D>
__global__ void __launch_bounds__(kBlock, 4) k_item32_batch(const BatchReq *tab, const int32_t *grp, int n)
{
    item_batch_body<D, float>(tab, grp, n);
}

template <int D>
__global__ void __launch_bounds__(kBlock) k_item64_batch(const BatchReq *tab, const int32_t *grp, int n)
{
    item_batch_body<D, double>(tab, grp, n);
}

// kFp64BatchGrid blocks per request of the group: its queued pairs, then
// (if any) its items left whole
template <int D>
__global__ void __launch_bounds__(kBlock) k_fp64_batch(const BatchReq *tab, const int32_t *grp)
{
    __shared__ RmDev s_rm;
    const int r = (int)blockIdx.x / kFp64BatchGrid, b = (int)blockIdx.x % kFp64BatchGrid;
    load_rm(&s_rm, tab[grp[r]].rm);
    const int n_df = s_rm.ctl->n_df;
    retest_pairs<D, 0>(s_rm, b, kFp64BatchGrid);
    if (!n_df) return;
    item_body<D, double, 0>(s_rm, 1, b, kFp64BatchGrid);
}

// request owning a tile: the last r with first[r] <= tile (n <= kMaxBatch)
__device__ inline int owner_of(const BatchReq *tab, int n, int tile, bool write_tiles)
{
    __shared__ int s_r;
    if (threadIdx.x < 64) {
        int best = -1;
        for (int r = threadIdx.x; r < n; r += 64) {
            const int f = write_tiles ? tab[r].wtile0 : tab[r].tile0;
            if (f <= tile) best = max(best, r);
        }
        for (int o = 32; o > 0; o >>= 1) best = max(best, __shfl_xor(best, o));
        if (threadIdx.x == 0) s_r = best;
    }
    __syncthreads();
    return s_r;
}

// The batch's two label passes.  The first writes the labels as it counts
// a tile's GRAY edges (when the update succeeded and the caller asked for
// labels), so the second reads one byte per edge instead of the 8-byte
// counters to place the GRAY ids.
__global__ void __launch_bounds__(kBlock) k_count_batch(const BatchReq *tab, int n)
{
    __shared__ int s_w[kWaves];
    __shared__ BatchReq q;
    const int r = owner_of(tab, n, (int)blockIdx.x, false);
    load_row(&q, tab[r]);
    const RmDev &rm = q.rm;
    const int tile = (int)blockIdx.x - q.tile0;
    const int tid = threadIdx.x;
    const int64_t e0 = (int64_t)tile * kLabelTile + (int64_t)tid * kLabelRun;
    const int status = rm.ctl->status;   // issued before the counters' loads are waited on
    uint8_t lab[kLabelRun];
    const int ng = run_labels(rm, e0, lab);
    if (status == RGG_OK) store_run(rm, q.a.labels, e0, lab);
    const int tot = block_sum(ng, s_w);
    if (tid == 0) rm.tile_cnt[tile] = tot;
}

// A run's labels as k_count_batch wrote them.
__device__ __forceinline__ int load_labels(const RmDev &rm, const uint8_t *labels, int64_t e0,
                                           uint8_t (&lab)[kLabelRun])
{
    if (e0 + kLabelRun <= rm.E && ((uintptr_t)(labels + e0) & 15u) == 0) {
        const uint4 v = *reinterpret_cast<const uint4 *>(labels + e0);
        const uint32_t w[4] = {v.x, v.y, v.z, v.w};
#pragma unroll
        for (int h = 0; h < kLabelRun; ++h) lab[h] = (uint8_t)(w[h >> 2] >> (8 * (h & 3)));
    } else {
#pragma unroll
        for (int h = 0; h < kLabelRun; ++h) lab[h] = e0 + h < rm.E ? labels[e0 + h] : (uint8_t)RGG_GREEN;
    }
    int ng = 0;
#pragma unroll
    for (int h = 0; h < kLabelRun; ++h) ng += (e0 + h < rm.E && lab[h] == RGG_GRAY) ? 1 : 0;
    return ng;
}

__global__ void __launch_bounds__(kBlock) k_write_batch(const BatchReq *tab, int n)
{
    __shared__ BatchReq q;
    const int r = owner_of(tab, n, (int)blockIdx.x, true);
    load_row(&q, tab[r]);
    const int tile = (int)blockIdx.x - q.wtile0;
    if (!q.a.labels || tile == q.rm.ntiles) {
        write_body(q.rm, q.a.labels, q.a.gray, q.a.gray_cap, q.a.res, 0, tile);
        return;
    }
    // the labels are written: the GRAY ids from them
    __shared__ int s_w[kWaves];
    const RmDev &rm = q.rm;
    const int tid = threadIdx.x;
    // the labels and the earlier tiles' counts are loaded with the status,
    // not after it (unused when the update failed)
    const int status = rm.ctl->status;
    int before = 0;
    for (int t = tid; t < tile; t += kBlock) before += rm.tile_cnt[t];
    const int64_t e0 = (int64_t)tile * kLabelTile + (int64_t)tid * kLabelRun;
    uint8_t lab[kLabelRun];
    const int ng = load_labels(rm, q.a.labels, e0, lab);
    if (tid == 0 && tile == 0 && q.a.res) {
        q.a.res->status = status;
        q.a.res->n_changed = rm.ctl->n_chg;
        if (status != RGG_OK) q.a.res->n_gray = 0;
    }
    if (status != RGG_OK) return;
    before = block_sum(before, s_w);
    int tot;
    const int pre = block_scan(ng, &tot, s_w);
    if (tid == 0 && tile == rm.ntiles - 1 && q.a.res) q.a.res->n_gray = (int64_t)before + tot;
    if (tot == 0) return;
    store_gray(rm, q.a.gray, q.a.gray_cap, e0, lab, before, pre, tot);
}

}  // namespace

namespace {

// The kernel of role k for the roadmap's dimension and form: 0 the pair
// listing, 1 the pair testing, 2 the binary64 pass (FP32 mode), 3 the
// binary64 item kernel (FP64 mode).
template <int D, int MODE>
void *fn_of(int k)
{
    switch (k) {
    case 0: return (void *)k_item32<D, MODE>;
    case 1: return (void *)k_pairs<D, MODE>;
    case 2: return (void *)k_fp64<D, MODE>;
    default: return (void *)k_item64<D, MODE>;
    }
}

template <int D>
void *fn_dim(int mode, int k)
{
    switch (mode) {
    case kModeObb: return fn_of<D, kModeObb>(k);
    case kModeSplines: return fn_of<D, kModeSplines>(k);
    case kModeObb | kModeSplines: return fn_of<D, kModeObb | kModeSplines>(k);
    default: return fn_of<D, 0>(k);
    }
}

void *fn(const RmDev &rm, int k) { return rm.D == 3 ? fn_dim<3>(rm.mode, k) : fn_dim<2>(rm.mode, k); }


struct Node {
    void *fn;
    dim3 grid;
    int kind;      // argument list: 0 diff, 1 (rm) only, 4 write
    int ev0, ev1;  // stage events ev[ev0..ev1] are recorded after the node
};

// The kernels of one update, in order.  Stage events: ev[0] before, ev[1]
// after the diff, ev[2] after the cell activation, ev[3] after the pair
// listing, ev[4] after the pair testing, ev[5] after the binary64 pass,
// ev[6] after the labels.  The FP64 mode's one item kernel stands for the
// testing (ev[3] before it).  With a single grid cell there is nothing to
// activate: k_diff emits the items.
// blocks of the item kernel for a one-cell roadmap: one per item, at most
// kGrid (the rows of statistics and re-test regions past the grid stay zero:
// their readers clear them after every update)
unsigned fixed_items_grid(const RmDev &rm)
{
    return (unsigned)std::max<int64_t>(1, std::min<int64_t>(kGrid, rm.items_cap));
}

int plan(const RmDev &rm, Node out[7])
{
    int n = 0;
    const bool single = rm.ncells == 1;
    void *const diff_fn = rm.D == 3 ? (void *)k_diff<3> : (void *)k_diff<2>;
    if (rm.mixed) {
        out[n++] = {diff_fn, dim3(1), 0, 1, 2};
        // with every round tested inline there is nothing to share out
        const bool share = rm.inline_rounds != kInlineAll;
        // one grid cell: its items are fixed, and blocks past them would only
        // start and stop (with pair listing every block writes its list's
        // count, so the whole grid runs)
        const unsigned grid = single && !share ? fixed_items_grid(rm) : kGrid;
        out[n++] = {fn(rm, 0), dim3(grid), 1, 3, share ? 3 : 4};
        if (share) out[n++] = {fn(rm, 1), dim3(kGrid), 1, 4, 4};
        out[n++] = {fn(rm, 2), dim3(kFp64Grid), 1, 5, 5};
    } else {
        out[n++] = {diff_fn, dim3(1), 0, 1, 3};
        out[n++] = {fn(rm, 3), dim3(single ? fixed_items_grid(rm) : kGrid), 1, 4, 5};
    }
    out[n++] = {(void *)k_labels, dim3(rm.ntiles + 1), 4, 6, 6};
    return n;
}

// kernel arguments of one node (storage for the values lives in `Args`)
struct Args {
    RmDev r;
    const rgg_box *ob, *nb;
    uint8_t *lab;
    int64_t *gray;
    int64_t cap;
    rgg_update_result *res;
    int zero = 0;
    void *diff[3], *one[1], *write[6];
    Args(const RmDev &rm, const UpdateArgs &a)
        : r(rm), ob(a.old_b), nb(a.new_b), lab(a.labels), gray(a.gray), cap(a.gray_cap), res(a.res),
          diff{&r, (void *)&ob, (void *)&nb}, one{&r},
          write{&r, &lab, &gray, &cap, &res, &zero}
    {
    }
    Args(const Args &) = delete;
    void **of(int kind)
    {
        return kind == 0 ? diff : (kind == 4 ? write : one);
    }
    dim3 block(int kind) const { return dim3(kind == 0 ? kDiffBlock : kBlock); }
};

}  // namespace

hipError_t launch_update(const RmDev &rm, const UpdateArgs &a, hipStream_t s, hipEvent_t *ev)
{
    if (rm.chunk < 1 || rm.chunk > kItemCap) return hipErrorInvalidValue;   // at most kSlots edges of an item per thread
    Node nodes[7];
    const int n = plan(rm, nodes);
    Args args(rm, a);
    hipError_t err;
    if (ev && (err = hipEventRecord(ev[0], s)) != hipSuccess) return err;
    for (int k = 0; k < n; ++k) {
        const Node &nd = nodes[k];
        if ((err = hipLaunchKernel(nd.fn, nd.grid, args.block(nd.kind), args.of(nd.kind), 0, s)) != hipSuccess)
            return err;
        if (ev && nd.ev0 >= 0)
            for (int m = nd.ev0; m <= nd.ev1; ++m)
                if ((err = hipEventRecord(ev[m], s)) != hipSuccess) return err;
    }
    return hipSuccess;
}

int item_edges_max() { return kItemCap; }

__global__ void __launch_bounds__(kBlock) k_cell_slots(RmDev rm, int4 *out, int64_t n)
{
    const int64_t k = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (k >= n) return;
    const int e = rm.cell_edges[k];
    const float4 *aabb = reinterpret_cast<const float4 *>(rm.aabb);
    const int jfix = rm.p_fixed ? rm.p_fixed / rm.B : 0;
    int j0, J;
    if (jfix) {
        J = jfix;
        j0 = (int)(uint32_t)((int64_t)e * jfix);
    } else {
        const int64_t s0 = rm.soff[e];
        j0 = (int)(uint32_t)(s0 / rm.B);
        J = (int)((rm.soff[e + 1] - s0) / rm.B);
    }
    out[k] = make_int4(e, __float_as_int(aabb[2 * (int64_t)e].w), j0, J);
}

hipError_t fill_cell_slots(const RmDev &rm, int4 *out, int64_t n, hipStream_t s)
{
    if (n <= 0) return hipSuccess;
    k_cell_slots<<<dim3((unsigned)((n + kBlock - 1) / kBlock)), dim3(kBlock), 0, s>>>(rm, out, n);
    return hipGetLastError();
}

hipError_t test_blocks_resident(int D, int device, int *out)
{
    int per_cu = 0, n_cu = 0;
    hipError_t e = D == 3 ? hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, k_pairs<3, 0>, kBlock, 0)
                          : hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, k_pairs<2, 0>, kBlock, 0);
    if (e != hipSuccess) return e;
    if ((e = hipDeviceGetAttribute(&n_cu, hipDeviceAttributeMultiprocessorCount, device)) != hipSuccess) return e;
    *out = per_cu * n_cu;
    return hipSuccess;
}

hipError_t item_blocks_resident(int D, int device, int *out)
{
    int per_cu = 0, n_cu = 0;
    hipError_t e = D == 3 ? hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, k_item32<3, 0>, kBlock, 0)
                          : hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, k_item32<2, 0>, kBlock, 0);
    if (e != hipSuccess) return e;
    if ((e = hipDeviceGetAttribute(&n_cu, hipDeviceAttributeMultiprocessorCount, device)) != hipSuccess) return e;
    *out = per_cu * n_cu;
    return hipSuccess;
}

hipError_t launch_labels(const RmDev &rm, const UpdateArgs &a, hipStream_t s)
{
    k_count<<<rm.ntiles, kBlock, 0, s>>>(rm);
    hipError_t err = hipGetLastError();
    if (err != hipSuccess) return err;
    k_write<<<rm.ntiles, kBlock, 0, s>>>(rm, a.labels, a.gray, a.gray_cap, a.res, 1);
    return hipGetLastError();
}

hipError_t add_update_nodes(hipGraph_t g, const RmDev &rm, const UpdateArgs &a, hipGraphNode_t dep,
                            hipGraphNode_t *last)
{
    if (rm.chunk < 1 || rm.chunk > kItemCap) return hipErrorInvalidValue;
    Node nodes[7];
    const int n = plan(rm, nodes);
    Args args(rm, a);   // hipGraphAddKernelNode copies the argument values
    hipGraphNode_t prev = dep;
    for (int k = 0; k < n; ++k) {
        hipKernelNodeParams p = {};
        p.func = nodes[k].fn;
        p.gridDim = nodes[k].grid;
        p.blockDim = args.block(nodes[k].kind);
        p.sharedMemBytes = 0;
        p.kernelParams = args.of(nodes[k].kind);
        p.extra = nullptr;
        hipGraphNode_t node;
        hipError_t err = hipGraphAddKernelNode(&node, g, prev ? &prev : nullptr, prev ? 1 : 0, &p);
        if (err != hipSuccess) return err;
        prev = node;
    }
    *last = prev;
    return hipSuccess;
}

namespace {

// Copies the request table from pinned host memory into device memory: the
// device reads the host rows itself, so a batched launch needs no copy
// engine (whose hand-over to the kernels' queue costs more than the copy).
// One word per thread: every read of host memory is in flight at once.
static_assert(sizeof(BatchReq) % 4 == 0, "request rows are copied as 32-bit words");

// The kernels of a batched update in order, each handed to `emit(fn, grid,
// block, args)` (a graph-node adder or a stream launcher).  With `h_tab`
// (pinned host rows) the diff kernel copies them to `tab`.
// `after(stage)` follows each kernel: 0 diff, 1 cells, 3 item, 4 binary64
// pass, 5 labels (count and write).
template <typename Emit, typename After>
hipError_t batch_kernels(Emit emit, After after, const BatchReq *tab, const BatchReq *h_tab, const int32_t *grp,
                         int n, const BatchGroup *groups, int n_groups, bool any_grid, int n_tiles, int n_wtiles)
{
    const BatchReq *t = tab;
    int nn = n;
    hipError_t err;
    BatchReq *t_dst = const_cast<BatchReq *>(tab);
    const BatchReq *t_src = h_tab;
    void *a_first[] = {(void *)&t_dst, (void *)&t_src};
    if ((err = emit((void *)k_diff_batch, dim3(n), dim3(kDiffBlock), a_first)) != hipSuccess) return err;
    void *a_diff[] = {(void *)&t};
    if ((err = after(0)) != hipSuccess) return err;
    void *a_tn[] = {(void *)&t, (void *)&nn};
    // the grid roadmaps' cells are activated by the diff kernel itself
    if (any_grid && (err = after(1)) != hipSuccess) return err;
    for (int k = 0; k < n_groups; ++k) {
        const BatchGroup &gr = groups[k];
        const int32_t *gp = grp + gr.off;
        int cnt = gr.count;
        void *a_item[] = {(void *)&t, (void *)&gp, (void *)&cnt};
        void *fn = gr.D == 3 ? (gr.mixed ? (void *)k_item32_batch<3> : (void *)k_item64_batch<3>)
                             : (gr.mixed ? (void *)k_item32_batch<2> : (void *)k_item64_batch<2>);
        if ((err = emit(fn, dim3(kBatchItemGrid), dim3(kBlock), a_item)) != hipSuccess) return err;
        if ((err = after(3)) != hipSuccess) return err;
        if (gr.mixed) {
            void *a_fp[] = {(void *)&t, (void *)&gp};
            void *fp = gr.D == 3 ? (void *)k_fp64_batch<3> : (void *)k_fp64_batch<2>;
            if ((err = emit(fp, dim3(kFp64BatchGrid * cnt), dim3(kBlock), a_fp)) != hipSuccess) return err;
            if ((err = after(4)) != hipSuccess) return err;
        }
    }
    if ((err = emit((void *)k_count_batch, dim3(n_tiles), dim3(kBlock), a_tn)) != hipSuccess) return err;
    if ((err = emit((void *)k_write_batch, dim3(n_wtiles), dim3(kBlock), a_tn)) != hipSuccess) return err;
    return after(5);
}

}  // namespace

hipError_t add_batch_nodes(hipGraph_t g, const BatchReq *tab, const BatchReq *h_tab, const int32_t *grp, int n,
                           const BatchGroup *groups, int n_groups, bool any_grid, int n_tiles,
                           int n_wtiles, hipGraphNode_t dep, hipGraphNode_t *last)
{
    hipGraphNode_t prev = dep;
    auto add = [&](void *fn, dim3 grid, dim3 block, void **args) -> hipError_t {
        hipKernelNodeParams p = {};
        p.func = fn;
        p.gridDim = grid;
        p.blockDim = block;
        p.sharedMemBytes = 0;
        p.kernelParams = args;
        p.extra = nullptr;
        hipGraphNode_t node;
        hipError_t err = hipGraphAddKernelNode(&node, g, prev ? &prev : nullptr, prev ? 1 : 0, &p);
        if (err == hipSuccess) prev = node;
        return err;
    };
    auto none = [](int) { return hipSuccess; };
    hipError_t err = batch_kernels(add, none, tab, h_tab, grp, n, groups, n_groups, any_grid, n_tiles, n_wtiles);
    if (err == hipSuccess) *last = prev;
    return err;
}

// The request table of rgg_update_batch_noalloc.  Host code never passes the
// array's name to a kernel or a copy: it uses the address that
// batch_scratch_address returns for the current device.
static __device__ __align__(256) unsigned char scratch[kBatchScratchBytes];

hipError_t batch_scratch_address(void **ptr)
{
    *ptr = nullptr;
    return hipGetSymbolAddress(ptr, HIP_SYMBOL(scratch));
}

hipError_t launch_batch(hipStream_t s, const BatchReq *tab, const BatchReq *h_tab, const int32_t *grp, int n,
                        const BatchGroup *groups, int n_groups, bool any_grid, int n_tiles, int n_wtiles,
                        BatchTiming *timing)
{
    auto launch = [&](void *fn, dim3 grid, dim3 block, void **args) -> hipError_t {
        return hipLaunchKernel(fn, grid, block, args, 0, s);
    };
    if (!timing) {
        auto none = [](int) { return hipSuccess; };
        return batch_kernels(launch, none, tab, h_tab, grp, n, groups, n_groups, any_grid, n_tiles, n_wtiles);
    }
    timing->n = 0;
    auto mark = [&](int stage) -> hipError_t {
        if (timing->n >= BatchTiming::kMax) return hipErrorInvalidValue;
        timing->stage[timing->n] = stage;
        return hipEventRecord(timing->ev[1 + timing->n++], s);
    };
    hipError_t err = hipEventRecord(timing->ev[0], s);
    if (err != hipSuccess) return err;
    return batch_kernels(launch, mark, tab, h_tab, grp, n, groups, n_groups, any_grid, n_tiles, n_wtiles);
}

}  // namespace rgg
