// Device-side layout of a resident roadmap and the launch interface of the
// update pipeline.  Internal to librgg (shared by kernels.hip and api.cpp).
#pragma once

#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

#include "rgg.h"

namespace rgg {

// Control block of one roadmap, in device memory.  k_diff resets it at the
// start of every update; later kernels of the same update read it.
struct Ctl {
    int32_t status;        // RGG_OK / RGG_E_INVALID_ARG / RGG_E_STATE_MISMATCH
    int32_t n_chg;         // changed (box, sign) entries
    int32_t n_items;       // (cell, chunk) work items of the grid scan
    int32_t n_df;          // items left whole to the binary64 pass (their list's length)
    int32_t label_ticket;  // next tile of the one-pass label kernel (dispatch order)
    int32_t claim;         // items claimed past the static ones by a batched item
                           // launch (the counter of its group's first request)
};

// One changed obstacle entry: the box a slot held before (sign -1) or holds
// now (sign +1).  In each chunk of 512 slots, the old boxes' entries come
// first (in slot order), then the new boxes'.
struct alignas(16) ChgEntry {
    // the first 32 bytes are what the binary32 kernels stage: two 16-byte loads
    float lo32[3], hi32[3];    // outward-rounded binary32 copy
    float sbox;                // largest |coordinate| of the binary32 copy
    int32_t sign;
    double lo[3], hi[3];       // exact box (unused axes zero)
    int32_t c0[3], c1[3];      // inclusive grid-cell range; empty when c0 > c1
};
static_assert(offsetof(ChgEntry, sbox) == 24 && offsetof(ChgEntry, sign) == 28 && alignof(ChgEntry) == 16,
              "the binary32 part of an entry is two aligned 16-byte words");

// Everything a kernel needs about a roadmap, passed by value.
struct RmDev {
    int32_t D, B, mixed, chunk;
    int64_t E, M;
    float band_rel;
    int32_t ntiles;            // label tiles of kLabelTile edges
    int32_t p_fixed;           // sphere samples per edge when every edge has the same count, else 0
    int32_t test_slots;        // blocks of the pair testing resident at once on the device
    // approximations (see HostGeometry for the layouts)
    const int64_t *soff;
    const float *samp32;
    const double *samp64;
    const float *cap32;
    const double *cap64;
    const float *aabb;
    const float *rad2_32;      // [B] r_i^2 rounded to binary32
    const double *rad64;       // [B]
    // the second forms of Sec. 4.2: bit kModeObb, an oriented box per body
    // intersected with the capsules (outer); bit kModeSplines, shortcut
    // splines instead of the copies (inner)
    int32_t mode;
    int32_t nbody;             // robot bodies (1, or the arm's links)
    const double *obb64;       // [E][nbody][2D + D*D] centre, axes (rows), half-extents
    const unsigned long long *body_sph;   // [nbody] spheres of each body (bit i: sphere i)
    const int32_t *sseg;       // [E*B + 1] first spline segment of (edge, sphere)
    const float *seg32;        // [segments][2D + 1] spline segments: A, B, rho
    const double *seg64;
    // grid
    int32_t gdim[3];
    int32_t pad0;
    double gorg[3];
    double ginv;
    int64_t ncells;
    const int32_t *cell_start;
    const int32_t *cell_edges;
    // per slot of the cell lists (grid roadmaps; null with one cell): the
    // edge, the bits of its box's largest |coordinate|, its first
    // configuration / B and its configurations per sphere, so an item's
    // edges come in one contiguous 16-byte load per slot instead of a
    // gather through the edge id
    const int4 *cell_slot;
    int64_t items_cap;
    // block-local slab masks (binary32): slab of x on axis d is
    // clamp(floor((x - sl_org[d]) * sl_inv[d]), 0, slabs_of(D) - 1)
    float sl_org[3];
    float pad2;
    float sl_inv[3];
    int32_t pad4;
    // state and per-update scratch
    int2 *cnt;                 // [E] (outer, inner) counters
    uint32_t *cell_bits;       // [ceil(ncells/32)] touched cells, zero between updates
    rgg_box *resident;         // [M] obstacle slots
    ChgEntry *chg;             // [2M]
    int2 *items;               // [items_cap] (cell, chunk)
    int2 *rc;                  // [kStatBlocks][rc_cap] (edge, entry) pairs each block of
                               // the FP32 item kernel leaves to the binary64 re-test
    int32_t *rc_cnt;           // [kStatBlocks]
    int32_t rc_cap;
    int32_t *df;               // [items_cap] items left whole to the binary64 pass (an
                               // item block's re-test region was full), ctl->n_df of them
    // the FP32 mode's pair listing and pair testing
    int32_t pl_cap;            // pairs each listing block may leave for the pair testing
    int32_t inline_rounds;     // pair rounds of an item its listing block tests before it
                               // lists the rest (kInlineAll: every round, no pair testing)
    int2 *pl;                  // [kStatBlocks][pl_cap] (edge, entry) pairs
    int32_t *pl_cnt;           // [kStatBlocks] pairs each listing block left
    int2 *rt;                  // [kStatBlocks][rt_cap(pl_cap)] pairs each share left to the
                               // binary64 re-test (a share holds at most that many pairs)
    int32_t *rt_cnt;           // [kStatBlocks]
    int32_t *tile_cnt;         // [ntiles] gray edges per label tile
    unsigned long long *tile_state;   // [ntiles] look-back words of the one-pass label
                                      // kernel: flag (bits 62-63) | gray count
    unsigned long long *blk_stats;   // [kStats][kStatBlocks] statistics rows (the first
                                     // kStatRows in use), cleared by each update's fold
    Ctl *ctl;
};

constexpr int kModeObb = 1;
constexpr int kModeSplines = 2;
__host__ __device__ constexpr int obb_words(int D) { return 2 * D + D * D; }

// per-block statistics rows: pairs, pairs whose outer approximation met,
// re-tested pairs, bytes of the testing kernels, grid entries scanned,
// candidate edges, bytes of the pair listing, bytes of the binary64 pass
constexpr int kStats = 8;
constexpr int kStatPairBytes = 3, kStatItemBytes = 6, kStatFp64Bytes = 7;
constexpr int kStatBlocks = 2048;  // blocks of the item kernels
constexpr int kStatRows = 256;     // rows of blk_stats in use: item and pair-share blocks add
                                   // to row blockIdx & 255 (atomics), binary64 blocks to their own
constexpr int kMaxSlots = 4096;    // 2*slots changed entries at most

constexpr int kLocalCells = 512;   // uint4 words of the item kernel's slab masks (at most)
// Slabs per axis of the item kernel's block-local slab masks.
__host__ __device__ constexpr int slabs_of(int D) { return D == 3 ? 80 : 128; }
constexpr int kCopyStride3 = 4;    // values per sample copy in 3-D (xyz + pad)
constexpr int kCopyStride2 = 2;    // in 2-D
constexpr int kRcCap = 1024;       // default re-test pairs one item-kernel block may queue
constexpr int kPairListCap = 512;  // pairs one listing block may hand to the pair testing
constexpr int kInlineAll = 0x7fffffff;   // inline_rounds: every round tested by the listing block
// Capacity of a share's re-test region: a share holds at most one round
// (kPairCap pairs) or, when the shares span every statistics block, at most
// one listing block's capacity.
__host__ __device__ constexpr int32_t rt_cap_of(int32_t pl_cap) { return pl_cap > 256 ? pl_cap : 256; }
constexpr int kLabelTile = 4096;   // edges per block of the label kernels

struct UpdateArgs {
    const rgg_box *old_b;
    const rgg_box *new_b;
    uint8_t *labels;           // may be null
    int64_t *gray;             // may be null
    int64_t gray_cap;
    rgg_update_result *res;
};

// One request of a batched update: the roadmap's device view, the update's
// arguments, and the request's first label tile in the batch's tile range.
struct BatchReq {
    RmDev rm;
    UpdateArgs a;
    int32_t tile0;             // first count tile (ntiles per request)
    int32_t wtile0;            // first write tile (ntiles + 1 per request)
};

constexpr int kMaxBatch = 256;     // requests per batched launch

// Fixed device scratch of rgg_update_batch_noalloc: one batched update's
// request table (kMaxBatch rows) followed by its row list.  The array lives
// in the library's code object, one copy per device, so that entry point
// allocates nothing.
constexpr size_t kBatchTableBytes = (sizeof(BatchReq) * kMaxBatch + 255) / 256 * 256;
constexpr size_t kBatchScratchBytes = kBatchTableBytes + sizeof(int32_t) * kMaxBatch;
static_assert(kBatchScratchBytes <= 121 * 1024, "the documented size of the fixed request table");
// Device address of that scratch on the current device (hipGetSymbolAddress).
hipError_t batch_scratch_address(void **ptr);

// The kernels of a batched update of distinct roadmaps, appended to `g` as a
// chain after `dep` (may be null); *last receives the final node.  `tab` is
// the device table of the n requests (groups of one kernel variant listed in
// `grp`, sorted), `n_tiles`/`n_wtiles` the totals of the tile ranges.
struct BatchGroup {
    int32_t D, mixed, off, count;  // requests grp[off .. off + count)
};
hipError_t add_batch_nodes(hipGraph_t g, const BatchReq *tab, const BatchReq *h_tab, const int32_t *grp, int n,
                           const BatchGroup *groups, int n_groups, bool any_grid, int n_tiles,
                           int n_wtiles, hipGraphNode_t dep, hipGraphNode_t *last);
// Events of a timed batched launch: ev[0] before the first kernel, ev[1 + k]
// after kernel k, whose stage (0 diff, 1 cells, 3 item, 4 binary64 pass,
// 5 labels) is stage[k]; n kernels were marked.
struct BatchTiming {
    static constexpr int kMax = 16;
    hipEvent_t ev[kMax + 1];
    int stage[kMax];
    int n;
};
// The same kernels launched on `s` (timed when `timing` is non-null).
hipError_t launch_batch(hipStream_t s, const BatchReq *tab, const BatchReq *h_tab, const int32_t *grp, int n,
                        const BatchGroup *groups, int n_groups, bool any_grid, int n_tiles, int n_wtiles,
                        BatchTiming *timing = nullptr);

// Full validation of listed edges (rgg_validate): the robot, each edge's
// motion parameters and chord-deviation bounds, and the resident slots.
constexpr int kValMaxActive = 512;   // unknown sub-intervals per level, at most
constexpr int kValBoxes = 64;        // candidate boxes staged in LDS per page

struct VRobot {
    int32_t kind, B, L, dof;
    double base[2];
    double pos[64 * 3];        // SE2 [B][2], SE3 [B][3], arm [B]
    double rad[64];
    double len[32];
    int32_t link[64];
};

struct ValDev {
    int32_t D, B, dof, vstride;      // vstride = 2 dof + 3
    int64_t E, M;
    const VRobot *rob;
    const double *motion;      // [E][vstride]: a[dof], b[dof] (SE3: short-arc sign), turn, half, sin_half
    const double *delta;       // [E][B] chord-deviation bounds
    const double *cap64;       // [E][2D+1][B] capsules (their chords bound the search)
    const rgg_box *resident;   // [M]
};

// Queues the validation of ids[0 .. n) (n capped by count->n_gray when
// count is non-null, and zero when count->status is not RGG_OK) on `s`.
// When labels is non-null, each validated edge's entry becomes GREEN (FREE)
// or RED (COLLIDES, UNRESOLVED).  verdict, level and witness may be null.
hipError_t launch_validate(const ValDev &v, const int64_t *ids, int64_t n, const rgg_update_result *count,
                           int32_t max_level, int32_t max_active, uint8_t *verdict, int32_t *level,
                           double *witness, uint8_t *labels, hipStream_t s);

// Queues the kernels of one update on `s`.  When `ev` is non-null, ev[0..6]
// are recorded before, between and after the stages (diff, cells, grid scan,
// classify, re-test, labels).
hipError_t launch_update(const RmDev &rm, const UpdateArgs &a, hipStream_t s, hipEvent_t *ev);

// Appends the same kernels to `g` as a chain; `dep` (may be null) is the
// node they wait for, *last receives the final node.
hipError_t add_update_nodes(hipGraph_t g, const RmDev &rm, const UpdateArgs &a, hipGraphNode_t dep,
                            hipGraphNode_t *last);

// Recomputes labels and the gray list from the counters regardless of the
// last update's status (used by rgg_labels / rgg_gray_list).
hipError_t launch_labels(const RmDev &rm, const UpdateArgs &a, hipStream_t s);

// Edges a work item of the classify kernels may hold (at most two per thread).
int item_edges_max();
// Fills rm.cell_slot (n = the cell lists' length) from the roadmap's edge
// boxes and sample offsets, on stream s.
hipError_t fill_cell_slots(const RmDev &rm, int4 *out, int64_t n, hipStream_t s);
// Blocks of the binary32 item kernel for dimension D resident on `device` at
// once (blocks per CU times CUs).
hipError_t item_blocks_resident(int D, int device, int *out);
// blocks of the FP32 pair testing resident at once (RmDev::test_slots)
hipError_t test_blocks_resident(int D, int device, int *out);

}  // namespace rgg
