// C ABI of librgg (declared in include/rgg.h).
#include <hip/hip_runtime.h>
#include <math.h>
#include <stdarg.h>
#include <stdio.h>
#include <string.h>

#include <algorithm>
#include <array>
#include <chrono>
#include <functional>
#include <map>
#include <mutex>
#include <memory>
#include <string>
#include <thread>
#include <vector>

#include "rgg.h"
#include "rgg_device.h"
#include "rgg_internal.h"
#include "api_internal.h"

static_assert(rgg::local_slabs(2) == rgg::slabs_of(2) && rgg::local_slabs(3) == rgg::slabs_of(3),
              "slab counts of host and device");
static_assert(rgg::kCopyStride3 == 4 && rgg::kCopyStride2 == 2, "sample layout of host and device");

using namespace rgg;

namespace {
thread_local std::string g_err;
}  // namespace

namespace rgg {

rgg_status fail(rgg_status st, const char *fmt, ...)
{
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    g_err = buf;
    return st;
}

rgg_status hip_fail(hipError_t e, const char *what)
{
    return fail(RGG_E_DEVICE, "%s: %s", what, hipGetErrorString(e));
}

}  // namespace rgg

namespace {

int host_threads(int requested)
{
    if (requested > 0) return std::min(requested, 64);
    unsigned n = std::thread::hardware_concurrency();
    return (int)std::max(1u, std::min(n, 16u));
}

constexpr int32_t kChunk = 256;   // edges per grid work item by default (one per thread)

// Puts `grid` (built for work items of `chunk` edges) in place of the
// roadmap's current grid, if any.  The new arrays are allocated first, so a
// failure leaves the old grid in use.  The caller makes sure no queued work
// still reads the old arrays.
rgg_status install_grid(rgg_roadmap *rm, const HostGrid &grid, int32_t chunk)
{
    RmDev &dv = rm->dv;
    const int64_t ncells = (int64_t)grid.dim[0] * grid.dim[1] * grid.dim[2];
    const size_t ncw = (size_t)((ncells + 31) / 32);
    int32_t *cstart = nullptr, *cedges = nullptr, *df = nullptr;
    uint32_t *bits = nullptr;
    int2 *items = nullptr;
    int4 *cslot = nullptr;
    auto undo = [&](rgg_status s) {
        rm->release(cstart);
        rm->release(cedges);
        rm->release(bits);
        rm->release(df);
        rm->release(items);
        rm->release(cslot);
        return s;
    };
    rgg_status st;
    if ((st = rm->upload(&cstart, grid.start.data(), grid.start.size(), "grid starts")) != RGG_OK) return undo(st);
    if ((st = rm->upload(&cedges, grid.edges.data(), grid.edges.size(), "grid lists")) != RGG_OK) return undo(st);
    if ((st = rm->alloc(&bits, ncw, "cell marks")) != RGG_OK) return undo(st);
    if ((st = rm->alloc(&df, (size_t)std::max<int64_t>(grid.items_cap, 1), "deferred items")) != RGG_OK)
        return undo(st);
    if (ncells == 1) {
        // the one cell's work items never change: (0, h) for every chunk h
        std::vector<int2> fixed((size_t)grid.items_cap);
        for (int64_t h = 0; h < grid.items_cap; ++h) fixed[(size_t)h] = make_int2(0, (int32_t)h);
        if ((st = rm->upload(&items, fixed.data(), fixed.size(), "grid items")) != RGG_OK) return undo(st);
    } else if ((st = rm->alloc(&items, (size_t)grid.items_cap, "grid items")) != RGG_OK) {
        return undo(st);
    }
    hipError_t e = hipMemset(bits, 0, 4 * std::max<size_t>(ncw, 1));
    if (e != hipSuccess) return undo(hip_fail(e, "clear marks"));
    if (ncells > 1 && !grid.edges.empty()) {
        // the cell lists' slots with each edge's box size and sample range
        const int64_t n = (int64_t)grid.edges.size();
        if ((st = rm->alloc(&cslot, (size_t)n, "grid slots")) != RGG_OK) return undo(st);
        RmDev view = dv;
        view.cell_edges = cedges;
        if ((e = fill_cell_slots(view, cslot, n, nullptr)) != hipSuccess) return undo(hip_fail(e, "grid slots"));
        if ((e = hipStreamSynchronize(nullptr)) != hipSuccess) return undo(hip_fail(e, "grid slots"));
    }
    rm->release(dv.cell_start);
    rm->release(dv.cell_edges);
    rm->release(dv.cell_bits);
    rm->release(dv.df);
    rm->release(dv.items);
    rm->release(dv.cell_slot);
    dv.cell_start = cstart;
    dv.cell_edges = cedges;
    dv.cell_slot = cslot;
    dv.cell_bits = bits;
    dv.df = df;
    dv.items = items;
    dv.chunk = chunk;
    for (int d = 0; d < 3; ++d) {
        dv.gdim[d] = grid.dim[d];
        dv.gorg[d] = grid.org[d];
        dv.sl_org[d] = grid.sl_org[d];
        dv.sl_inv[d] = grid.sl_inv[d];
    }
    dv.ginv = grid.inv;
    dv.ncells = ncells;
    dv.items_cap = grid.items_cap;
    rgg_roadmap_info &in = rm->info;
    for (int d = 0; d < 3; ++d) in.grid_cells[d] = grid.dim[d];
    in.cell_size = grid.cell;
    in.grid_entries = (int64_t)grid.edges.size();
    in.item_edges = chunk;
    return RGG_OK;
}

constexpr int kTuneMaxStates = 64;

// One roadmap under tuning: its edge boxes on the host (for candidate
// grids), its configuration before tuning, and device copies of the state a
// (the resident one) and of the states b_i it is moved to and back from.
struct TuneSubject {
    rgg_roadmap *rm = nullptr;
    HostGeometry g;
    double mean_ext = 0.0;
    double cur_cell = -1.0;     // < 0: one cell
    int32_t cur_chunk = 0;
    int n_b = 0;
    rgg_box *d_states = nullptr;            // [(1 + n_b) * M]
    rgg_update_result *d_res = nullptr;     // [2 * n_b]
    std::vector<int64_t> gray_ref;          // gray counts of the first candidate
    ~TuneSubject()
    {
        if (d_states) (void)hipFree(d_states);
        if (d_res) (void)hipFree(d_res);
    }
    // the update a -> b_i (to == true) or b_i -> a
    UpdateArgs args(int i, bool to) const
    {
        const int64_t M = rm->dv.M;
        const rgg_box *a = d_states, *bi = d_states + (size_t)(1 + i) * M;
        return {to ? a : bi, to ? bi : a, rm->d_labels, rm->d_gray, rm->dv.E, d_res + 2 * i + (to ? 0 : 1)};
    }
};

// Waits for the roadmap's queued work, checks that `a` is its resident state
// (bit for bit, as an update checks it, so that the round trips end where
// they start) and stages the states on the device.
rgg_status tune_subject(rgg_roadmap *rm, const rgg_box *a, int n_b, const rgg_box *const *bs, TuneSubject *t)
{
    const int64_t M = rm->dv.M, E = rm->dv.E;
    if (rm->wait_ev) HIP_OR_FAIL(hipEventSynchronize(rm->wait_ev), "wait for the previous update");
    HIP_OR_FAIL(hipStreamSynchronize(rm->stream), "roadmap stream");
    if (M > 0) {
        std::vector<rgg_box> cur((size_t)M);
        HIP_OR_FAIL(hipMemcpy(cur.data(), rm->dv.resident, sizeof(rgg_box) * M, hipMemcpyDeviceToHost),
                    "read obstacle slots");
        if (memcmp(cur.data(), a, sizeof(rgg_box) * M) != 0)
            return fail(RGG_E_STATE_MISMATCH, "obstacles_a differs from the resident obstacle slots");
    }
    t->rm = rm;
    t->n_b = n_b;
    t->g.D = rm->dv.D;
    t->g.E = E;
    t->g.aabb.resize((size_t)std::max<int64_t>(E, 1) * kAabbStride);
    if (E > 0)
        HIP_OR_FAIL(hipMemcpy(t->g.aabb.data(), rm->dv.aabb, sizeof(float) * (size_t)E * kAabbStride,
                              hipMemcpyDeviceToHost),
                    "read edge boxes");
    double ext_sum = 0.0;
    for (int64_t e = 0; e < E; ++e) {
        const float *b = t->g.aabb.data() + e * kAabbStride;
        double ext = 0.0;
        for (int d = 0; d < t->g.D; ++d) ext = std::max(ext, (double)b[4 + d] - (double)b[d]);
        ext_sum += ext;
    }
    t->mean_ext = E > 0 ? ext_sum / (double)E : 0.0;
    t->cur_cell = rm->dv.ncells == 1 ? -1.0 : rm->info.cell_size;
    t->cur_chunk = rm->dv.chunk;
    HIP_OR_FAIL(hipMalloc(&t->d_states, sizeof(rgg_box) * std::max<int64_t>(1, (1 + n_b) * M)), "tuning states");
    HIP_OR_FAIL(hipMalloc(&t->d_res, sizeof(rgg_update_result) * 2 * n_b), "tuning results");
    if (M > 0) {
        HIP_OR_FAIL(hipMemcpy(t->d_states, a, sizeof(rgg_box) * M, hipMemcpyHostToDevice), "upload boxes");
        for (int i = 0; i < n_b; ++i)
            HIP_OR_FAIL(hipMemcpy(t->d_states + (size_t)(1 + i) * M, bs[i], sizeof(rgg_box) * M, hipMemcpyHostToDevice),
                        "upload boxes");
    }
    return RGG_OK;
}

// A candidate work decomposition: items of `chunk` edges and grid cells of
// `factor` times the roadmap's mean edge extent (factor < 0: one cell;
// factor == 0: each roadmap's configuration before tuning).
struct TuneCand {
    double factor;
    int32_t chunk;
};

rgg_status tune_apply(TuneSubject &t, const TuneCand &c)
{
    double cell = -1.0;
    int32_t chunk = c.chunk;
    if (c.factor == 0.0) {
        cell = t.cur_cell;
        chunk = t.cur_chunk;
    } else if (c.factor > 0.0 && t.mean_ext > 0.0 && std::isfinite(c.factor * t.mean_ext)) {
        cell = c.factor * t.mean_ext;
    }
    HostGrid grid;
    std::string err;
    rgg_status st = build_grid(t.g, cell, chunk, &grid, &err);
    if (st != RGG_OK) return fail(st, "%s", err.c_str());
    return install_grid(t.rm, grid, chunk);
}

// Times every candidate with `run(count)` (count round trips of `per_rt`
// updates each) after one untimed round trip, checks that the gray counts
// never change, and keeps the fastest (candidate 0, the configuration before
// tuning, unless another is at least 3% faster).  `refresh` (optional) runs
// after each change of configuration.
template <typename Run>
rgg_status tune_search(std::vector<TuneSubject *> &subj, hipStream_t s, int reps, int per_rt, Run &&run,
                       bool per_batch, rgg_tune_report *report,
                       const std::function<rgg_status()> &refresh = nullptr,
                       const std::vector<TuneCand> &extra = {})
{
    std::vector<TuneCand> cands = {{0.0, 0}};
    for (int32_t chunk : {512, 256, 128, 64})
        for (double f : {-1.0, 1.0, 2.0, 4.0, 8.0}) cands.push_back({f, chunk});
    for (const TuneCand &c : extra) cands.push_back(c);
    if ((int)cands.size() > RGG_TUNE_MAX_CANDIDATES) cands.resize(RGG_TUNE_MAX_CANDIDATES);
    struct Ev {
        hipEvent_t e0 = nullptr, e1 = nullptr;
        ~Ev()
        {
            if (e0) (void)hipEventDestroy(e0);
            if (e1) (void)hipEventDestroy(e1);
        }
    } ev;
    HIP_OR_FAIL(hipEventCreate(&ev.e0), "hipEventCreate");
    HIP_OR_FAIL(hipEventCreate(&ev.e1), "hipEventCreate");
    std::vector<double> us(cands.size(), 0.0);
    rgg_status st;
    auto apply = [&](const TuneCand &c) -> rgg_status {
        for (TuneSubject *t : subj)
            if ((st = tune_apply(*t, c)) != RGG_OK) return st;
        return refresh ? refresh() : RGG_OK;
    };
    for (size_t k = 0; k < cands.size(); ++k) {
        if ((st = apply(cands[k])) != RGG_OK) return st;
        if ((st = run(1)) != RGG_OK) return st;
        HIP_OR_FAIL(hipEventRecord(ev.e0, s), "hipEventRecord");
        if ((st = run(reps)) != RGG_OK) return st;
        HIP_OR_FAIL(hipEventRecord(ev.e1, s), "hipEventRecord");
        HIP_OR_FAIL(hipEventSynchronize(ev.e1), "tuning run");
        float ms = 0.0f;
        HIP_OR_FAIL(hipEventElapsedTime(&ms, ev.e0, ev.e1), "hipEventElapsedTime");
        us[k] = 1e3 * (double)ms / ((double)reps * per_rt);
        for (size_t j = 0; j < subj.size(); ++j) {
            TuneSubject &t = *subj[j];
            std::vector<rgg_update_result> r((size_t)(2 * t.n_b));
            HIP_OR_FAIL(hipMemcpy(r.data(), t.d_res, sizeof(rgg_update_result) * r.size(), hipMemcpyDeviceToHost),
                        "read results");
            for (size_t i = 0; i < r.size(); ++i)
                if (r[i].status != RGG_OK)
                    return fail(r[i].status, "roadmap %zu: a state to tune on holds an invalid box", j);
            if (k == 0) {
                t.gray_ref.resize(r.size());
                for (size_t i = 0; i < r.size(); ++i) t.gray_ref[i] = r[i].n_gray;
            } else {
                for (size_t i = 0; i < r.size(); ++i)
                    if (r[i].n_gray != t.gray_ref[i])
                        return fail(RGG_E_DEVICE, "roadmap %zu: candidate %zu changed a gray count (%lld vs %lld)", j,
                                    k, (long long)r[i].n_gray, (long long)t.gray_ref[i]);
            }
        }
    }
    size_t best = 0;
    for (size_t k = 1; k < cands.size(); ++k)
        if (us[k] < us[best]) best = k;
    if (us[best] > 0.97 * us[0]) best = 0;
    if ((st = apply(cands[best])) != RGG_OK) return st;
    if (report) {
        *report = rgg_tune_report{};
        report->n_candidates = (int32_t)cands.size();
        const rgg_roadmap *rm0 = subj[0]->rm;
        report->item_edges = rm0->dv.chunk;
        report->cell_size = per_batch ? (cands[best].factor < 0 ? INFINITY : cands[best].factor) : rm0->info.cell_size;
        for (int d = 0; d < 3; ++d) report->grid_cells[d] = per_batch ? 0 : rm0->info.grid_cells[d];
        report->us_per_update = us[best];
        report->us_before = us[0];
        for (size_t k = 0; k < cands.size(); ++k) {
            const bool cur = cands[k].factor == 0.0;
            report->cand_item_edges[k] = cur ? (per_batch ? 0 : subj[0]->cur_chunk) : cands[k].chunk;
            double cell = cands[k].factor < 0 ? INFINITY : cands[k].factor * (per_batch ? 1.0 : subj[0]->mean_ext);
            if (cur) cell = per_batch ? 0.0 : (subj[0]->cur_cell < 0 ? INFINITY : subj[0]->cur_cell);
            report->cand_cell_size[k] = cell;
            report->cand_us[k] = us[k];
        }
    }
    return RGG_OK;
}

}  // namespace

struct rgg_graph {
    int device = 0;
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    std::vector<rgg_roadmap *> roadmaps;
};

struct rgg_batch {
    static constexpr int kRing = 8;   // host request tables in flight
    int device = 0;
    int n = 0;
    std::vector<rgg_roadmap *> rms;   // request order
    std::vector<int32_t> order;       // request index of each table row
    BatchReq *d_tab = nullptr;        // [n] rows, grouped by kernel variant
    int32_t *d_grp = nullptr;         // [n] row indices, grouped
    BatchReq *h_tab[kRing] = {};      // pinned
    hipEvent_t done[kRing] = {};      // end of the launch that used the slot
    bool used[kRing] = {};
    int ring = 0;
    // one captured graph per ring slot: its first kernel copies that slot's
    // host table
    hipGraph_t graph[kRing] = {};
    hipGraphExec_t exec[kRing] = {};
    std::vector<BatchGroup> groups;
    bool any_grid = false;
    int tiles = 0, wtiles = 0;
    // stage timing (rgg_batch_timing_*)
    bool timing = false;
    std::vector<BatchTiming> t_pool, t_pending;
    double ms_acc[6] = {0, 0, 0, 0, 0, 0};
    int64_t timed = 0;

    ~rgg_batch()
    {
        hipSetDevice(device);
        for (int k = 0; k < kRing; ++k)
            if (done[k] && used[k]) hipEventSynchronize(done[k]);
        for (auto *v : {&t_pool, &t_pending})
            for (BatchTiming &t : *v)
                for (hipEvent_t e : t.ev) hipEventDestroy(e);
        // the roadmaps' last updates have completed: nothing left to wait for
        for (rgg_roadmap *rm : rms) {
            for (int k = 0; k < kRing; ++k)
                if (rm->wait_ev == done[k]) rm->wait_ev = nullptr;
            rm->holders--;
        }
        for (int k = 0; k < kRing; ++k) {
            if (done[k]) hipEventDestroy(done[k]);
            if (h_tab[k]) hipHostFree(h_tab[k]);
        }
        for (int k = 0; k < kRing; ++k) {
            if (exec[k]) hipGraphExecDestroy(exec[k]);
            if (graph[k]) hipGraphDestroy(graph[k]);
        }
        if (d_tab) hipFree(d_tab);
        if (d_grp) hipFree(d_grp);
    }
};

// (Re)builds the batch's graphs, one per ring slot: the slot's table copy,
// then the batch's kernels.  The kernels depend on whether any roadmap uses
// a grid, so tuning rebuilds them.
static rgg_status build_batch_graphs(rgg_batch *b)
{
    for (int k = 0; k < rgg_batch::kRing; ++k) {
        if (b->exec[k]) (void)hipGraphExecDestroy(b->exec[k]);
        if (b->graph[k]) (void)hipGraphDestroy(b->graph[k]);
        b->exec[k] = nullptr;
        b->graph[k] = nullptr;
        HIP_OR_FAIL(hipGraphCreate(&b->graph[k], 0), "hipGraphCreate");
        hipGraphNode_t last = nullptr;
        HIP_OR_FAIL(add_batch_nodes(b->graph[k], b->d_tab, b->h_tab[k], b->d_grp, b->n, b->groups.data(),
                                    (int)b->groups.size(), b->any_grid, b->tiles, b->wtiles, nullptr, &last),
                    "hipGraphAddKernelNode");
        HIP_OR_FAIL(hipGraphInstantiate(&b->exec[k], b->graph[k], nullptr, nullptr, 0), "hipGraphInstantiate");
    }
    return RGG_OK;
}

extern "C" {

const char *rgg_last_error(void) { return g_err.c_str(); }

const char *rgg_version(void) { return "librgg 0.1 (gfx950)"; }

rgg_status rgg_context_create(int device, rgg_context **out)
{
    if (!out) return fail(RGG_E_INVALID_ARG, "null output pointer");
    int n = 0;
    HIP_OR_FAIL(hipGetDeviceCount(&n), "hipGetDeviceCount");
    if (device < 0 || device >= n) return fail(RGG_E_INVALID_ARG, "device %d out of range (%d devices)", device, n);
    HIP_OR_FAIL(hipSetDevice(device), "hipSetDevice");
    // the fixed scratch of rgg_update_batch_noalloc: each device holds its
    // own copy of the array, at its own address, found with that device
    // current
    void *scratch = nullptr;
    HIP_OR_FAIL(batch_scratch_address(&scratch), "hipGetSymbolAddress(batch scratch)");
    if (!scratch) return fail(RGG_E_DEVICE, "the batch scratch has no device address");
    *out = new rgg_context{device, scratch};
    return RGG_OK;
}

void rgg_context_destroy(rgg_context *ctx) { delete ctx; }

namespace {

// What a roadmap's device state is built from besides its geometry and grid.
struct RoadmapParams {
    int64_t M;                 // obstacle slots
    bool mixed;                // binary32 tests with the binary64 re-test
    double band_rel;           // as rgg_build_opts.band_rel
    int32_t retest_capacity;   // as rgg_build_opts.retest_capacity
    int32_t chunk;             // edges per work item
    int32_t pair_list_capacity;   // as rgg_build_opts.pair_list_capacity
    int32_t inline_rounds;        // RmDev::inline_rounds (resolved: 0..2^20 or kInlineAll)
};

// RmDev::inline_rounds for rgg_build_opts.inline_rounds
int32_t inline_rounds_of(int32_t opt)
{
    if (opt == RGG_INLINE_ALL) return kInlineAll;
    return opt == RGG_INLINE_NONE ? 0 : opt;
}

rgg_status hip_ok(hipError_t e, const char *what) { return e == hipSuccess ? RGG_OK : hip_fail(e, what); }

// Device bytes make_roadmap allocates for g, grid and p (each array at least
// one element, as rgg_roadmap::alloc gives it).
int64_t device_bytes_needed(const HostGeometry &g, const HostGrid &grid, const RoadmapParams &p)
{
    int64_t total = 0;
    auto add = [&](size_t count, size_t size) { total += (int64_t)(std::max<size_t>(1, count) * size); };
    const int64_t E = g.E, M = p.M;
    const int B = g.B;
    add(g.soff.size(), 8);
    add(g.samp.size(), 8);
    add(g.cap.size(), 8);
    add(g.aabb.size(), 4);
    add((size_t)B, 8);
    add((size_t)B, 4);
    if (p.mixed) {
        add(g.samp.size(), 4);
        add(g.cap.size(), 4);
    }
    if (!g.obb.empty()) {
        add(g.obb.size(), 8);
        add((size_t)g.n_bodies, 8);
    }
    if (!g.sseg.empty()) {
        add(g.sseg.size(), 4);
        add(g.seg.size(), 8);
        if (p.mixed) add(g.seg.size(), 4);
    }
    const int64_t ncells = (int64_t)grid.dim[0] * grid.dim[1] * grid.dim[2];
    add(grid.start.size(), 4);
    add(grid.edges.size(), 4);
    if (ncells > 1 && !grid.edges.empty()) add(grid.edges.size(), sizeof(int4));
    add((size_t)((ncells + 31) / 32), 4);
    add((size_t)std::max<int64_t>(grid.items_cap, 1), 4);
    add((size_t)grid.items_cap, sizeof(int2));
    const int64_t ntiles = std::max<int64_t>(1, (E + kLabelTile - 1) / kLabelTile);
    const int32_t rc_cap = p.retest_capacity > 0 ? p.retest_capacity : kRcCap;
    add((size_t)E, sizeof(int2));
    add((size_t)M, sizeof(rgg_box));
    add((size_t)(2 * M), sizeof(ChgEntry));
    add((size_t)kStatBlocks * rc_cap, sizeof(int2));
    add((size_t)kStatBlocks, 4);
    if (p.mixed) {
        add((size_t)kStatBlocks, 4);
        if (p.inline_rounds != kInlineAll) {
            const int32_t pl_cap = p.pair_list_capacity > 0 ? p.pair_list_capacity : kPairListCap;
            add((size_t)kStatBlocks * pl_cap, sizeof(int2));
            add((size_t)kStatBlocks * rt_cap_of(pl_cap), sizeof(int2));
            add((size_t)kStatBlocks, 4);
        }
    }
    add((size_t)kStatBlocks * kStats, 8);
    add((size_t)ntiles + 1, 4);
    add((size_t)ntiles, 8);
    add(1, sizeof(Ctl));
    add((size_t)(2 * M), sizeof(rgg_box));
    add(1, sizeof(rgg_update_result));
    add((size_t)E, 1);
    add((size_t)E, 8);
    add(1, sizeof(VRobot));
    add(g.motion.size(), 8);
    add(g.delta.size(), 8);
    return total;
}

// Admission of a roadmap by device memory: refused, before anything is
// allocated, when its arrays would exceed `budget` bytes (0: the free device
// memory) or the free device memory.
rgg_status admit_roadmap(int64_t need, int64_t budget)
{
    size_t free_b = 0, total_b = 0;
    HIP_OR_FAIL(hipMemGetInfo(&free_b, &total_b), "hipMemGetInfo");
    const int64_t allowed = budget > 0 ? std::min<int64_t>(budget, (int64_t)free_b) : (int64_t)free_b;
    if (need > allowed)
        return fail(RGG_E_OUT_OF_MEMORY, "the roadmap needs %lld bytes of device memory; %lld allowed (%s)",
                    (long long)need, (long long)allowed,
                    budget > 0 && budget <= (int64_t)free_b ? "mem_budget" : "free device memory");
    return RGG_OK;
}

// Device arrays, scratch and state of a roadmap from its host geometry and
// grid.  resident and cnt (may be null) are the obstacle slots and counters
// to start from; otherwise every slot is ABSENT and every counter zero.  On
// failure nothing is left allocated.
rgg_status make_roadmap(rgg_context *ctx, const HostGeometry &g, const HostGrid &grid, const RoadmapParams &p,
                        const rgg_box *resident, const int2 *cnt, rgg_roadmap **out)
{
    rgg_status st;
    auto *rm = new rgg_roadmap();
    rm->ctx = ctx;
    rm->device = ctx->device;
    const int64_t E = g.E, M = p.M;
    const int D = g.D, B = g.B;
    const bool mixed = p.mixed;
    RmDev &dv = rm->dv;
    dv.D = D;
    dv.B = B;
    dv.mixed = mixed ? 1 : 0;
    dv.E = E;
    dv.M = M;
    dv.band_rel = (float)(p.band_rel > 0.0 ? p.band_rel : 1e-5);
    if (std::isinf(p.band_rel)) dv.band_rel = INFINITY;
    dv.ntiles = (int32_t)std::max<int64_t>(1, (E + kLabelTile - 1) / kLabelTile);
    dv.p_fixed = 0;
    if (E > 0) {
        const int64_t p0 = g.soff[1] - g.soff[0];
        bool same = p0 <= INT32_MAX;
        for (int64_t e = 1; e < E && same; ++e) same = g.soff[e + 1] - g.soff[e] == p0;
        if (same) dv.p_fixed = (int32_t)p0;
    }
    auto guard = [&](rgg_status s) {
        if (s != RGG_OK) delete rm;
        return s;
    };

    // approximations: binary64 always (the re-test and the FP64 mode read it),
    // binary32 copies for the FP32 mode
    const size_t nsamp = g.samp.size(), ncap = g.cap.size();
    int64_t *soff;
    double *samp64, *cap64, *rad64;
    float *aabb, *rad2;
    if ((st = rm->upload(&soff, g.soff.data(), g.soff.size(), "sample offsets")) != RGG_OK) return guard(st);
    if ((st = rm->upload(&samp64, g.samp.data(), nsamp, "binary64 samples")) != RGG_OK) return guard(st);
    if ((st = rm->upload(&cap64, g.cap.data(), ncap, "binary64 capsules")) != RGG_OK) return guard(st);
    if ((st = rm->upload(&aabb, g.aabb.data(), g.aabb.size(), "edge boxes")) != RGG_OK) return guard(st);
    if ((st = rm->upload(&rad64, g.radius.data(), (size_t)B, "radii")) != RGG_OK) return guard(st);
    std::vector<float> r2((size_t)B);
    for (int i = 0; i < B; ++i) r2[i] = (float)(g.radius[i] * g.radius[i]);
    if ((st = rm->upload(&rad2, r2.data(), (size_t)B, "radii^2")) != RGG_OK) return guard(st);
    dv.soff = soff;
    dv.samp64 = samp64;
    dv.cap64 = cap64;
    dv.aabb = aabb;
    dv.rad64 = rad64;
    dv.rad2_32 = rad2;
    if (mixed) {
        std::vector<float> tmp;
        float *s32, *c32;
        try {
            tmp.resize(std::max(nsamp, ncap));
        } catch (const std::bad_alloc &) {
            return guard(fail(RGG_E_OUT_OF_MEMORY, "host memory for binary32 copies"));
        }
        for (size_t i = 0; i < nsamp; ++i) tmp[i] = (float)g.samp[i];
        if ((st = rm->upload(&s32, tmp.data(), nsamp, "binary32 samples")) != RGG_OK) return guard(st);
        for (size_t i = 0; i < ncap; ++i) tmp[i] = (float)g.cap[i];
        if ((st = rm->upload(&c32, tmp.data(), ncap, "binary32 capsules")) != RGG_OK) return guard(st);
        dv.samp32 = s32;
        dv.cap32 = c32;
    }
    // the second forms (Sec. 4.2), when built
    dv.mode = (g.obb.empty() ? 0 : kModeObb) | (g.sseg.empty() ? 0 : kModeSplines);
    dv.nbody = g.n_bodies;
    if (!g.obb.empty()) {
        std::vector<unsigned long long> bs((size_t)g.n_bodies, 0ull);
        for (int i = 0; i < B; ++i) bs[g.body[i]] |= 1ull << i;
        double *o64;
        unsigned long long *d_bs;
        if ((st = rm->upload(&o64, g.obb.data(), g.obb.size(), "oriented boxes")) != RGG_OK) return guard(st);
        if ((st = rm->upload(&d_bs, bs.data(), bs.size(), "body spheres")) != RGG_OK) return guard(st);
        dv.obb64 = o64;
        dv.body_sph = d_bs;
    }
    if (!g.sseg.empty()) {
        if (g.sseg.back() > (int64_t)INT32_MAX)
            return guard(fail(RGG_E_OUT_OF_MEMORY, "%lld spline segments; at most 2^31 - 1", (long long)g.sseg.back()));
        std::vector<int32_t> off(g.sseg.begin(), g.sseg.end());
        int32_t *d_off;
        double *g64;
        if ((st = rm->upload(&d_off, off.data(), off.size(), "spline offsets")) != RGG_OK) return guard(st);
        if ((st = rm->upload(&g64, g.seg.data(), g.seg.size(), "binary64 spline segments")) != RGG_OK)
            return guard(st);
        dv.sseg = d_off;
        dv.seg64 = g64;
        if (mixed) {
            std::vector<float> tmp(g.seg.size());
            for (size_t i = 0; i < g.seg.size(); ++i) tmp[i] = (float)g.seg[i];
            float *g32;
            if ((st = rm->upload(&g32, tmp.data(), tmp.size(), "binary32 spline segments")) != RGG_OK)
                return guard(st);
            dv.seg32 = g32;
        }
    }
    if ((st = install_grid(rm, grid, p.chunk)) != RGG_OK) return guard(st);
    // state and scratch
    std::vector<rgg_box> absent((size_t)M);
    for (auto &b : absent)
        for (int k = 0; k < 3; ++k) {
            b.lo[k] = 1.0;
            b.hi[k] = -1.0;
        }
    if ((st = rm->alloc(&dv.cnt, (size_t)E, "counters")) != RGG_OK) return guard(st);
    if ((st = rm->upload(&dv.resident, resident ? resident : absent.data(), (size_t)M, "obstacle slots")) != RGG_OK)
        return guard(st);
    if ((st = rm->alloc(&dv.chg, (size_t)(2 * M), "changed entries")) != RGG_OK) return guard(st);
    dv.rc_cap = p.retest_capacity > 0 ? p.retest_capacity : kRcCap;
    if ((st = rm->alloc(&dv.rc, (size_t)kStatBlocks * dv.rc_cap, "re-test regions")) != RGG_OK) return guard(st);
    if ((st = rm->alloc(&dv.rc_cnt, (size_t)kStatBlocks, "re-test counts")) != RGG_OK) return guard(st);
    if (mixed) {
        dv.pl_cap = p.pair_list_capacity > 0 ? p.pair_list_capacity : kPairListCap;
        dv.inline_rounds = p.inline_rounds;
        int slots = 0;
        const hipError_t he = test_blocks_resident(dv.D, ctx->device, &slots);
        if (he != hipSuccess) return guard(hip_fail(he, "occupancy query"));
        dv.test_slots = slots;
        // the listing kernel writes its blocks' pair counts in every form;
        // the lists and the shares' re-test regions exist only with listing
        if ((st = rm->alloc(&dv.pl_cnt, (size_t)kStatBlocks, "pair list counts")) != RGG_OK) return guard(st);
        if (dv.inline_rounds != kInlineAll) {
            if ((st = rm->alloc(&dv.pl, (size_t)kStatBlocks * dv.pl_cap, "pair lists")) != RGG_OK) return guard(st);
            if ((st = rm->alloc(&dv.rt, (size_t)kStatBlocks * rt_cap_of(dv.pl_cap), "share re-test regions")) !=
                RGG_OK)
                return guard(st);
            if ((st = rm->alloc(&dv.rt_cnt, (size_t)kStatBlocks, "share re-test counts")) != RGG_OK) return guard(st);
        }
    }
    if ((st = rm->alloc(&dv.blk_stats, (size_t)kStatBlocks * kStats, "statistics")) != RGG_OK) return guard(st);
    if ((st = rm->alloc(&dv.tile_cnt, (size_t)dv.ntiles + 1, "tile counts")) != RGG_OK) return guard(st);
    if ((st = rm->alloc(&dv.tile_state, (size_t)dv.ntiles, "tile states")) != RGG_OK) return guard(st);
    if ((st = rm->alloc(&dv.ctl, 1, "control block")) != RGG_OK) return guard(st);
    if ((st = rm->alloc(&rm->d_stage, (size_t)(2 * M), "box staging")) != RGG_OK) return guard(st);
    if ((st = rm->alloc(&rm->d_res, 1, "result")) != RGG_OK) return guard(st);
    if ((st = rm->alloc(&rm->d_labels, (size_t)E, "labels")) != RGG_OK) return guard(st);
    if ((st = rm->alloc(&rm->d_gray, (size_t)E, "gray list")) != RGG_OK) return guard(st);
    // full validation
    {
        static_assert(sizeof(((VRobot *)nullptr)->pos) == sizeof(double) * kMaxSpheres * 3 &&
                          sizeof(((VRobot *)nullptr)->len) == sizeof(double) * kMaxLinks,
                      "VRobot holds the largest robot");
        VRobot hr = {};
        hr.kind = g.kind;
        hr.B = B;
        hr.L = g.L;
        hr.dof = g.dof;
        hr.base[0] = g.rob_base[0];
        hr.base[1] = g.rob_base[1];
        for (size_t k = 0; k < g.rob_pos.size(); ++k) hr.pos[k] = g.rob_pos[k];
        for (int i = 0; i < B; ++i) {
            hr.rad[i] = g.radius[i];
            hr.link[i] = i < (int)g.rob_link.size() ? g.rob_link[i] : 0;
        }
        for (size_t k = 0; k < g.rob_len.size(); ++k) hr.len[k] = g.rob_len[k];
        ValDev &vd = rm->val;
        VRobot *d_rob;
        double *d_mot, *d_del;
        if ((st = rm->upload(&d_rob, &hr, 1, "validation robot")) != RGG_OK) return guard(st);
        if ((st = rm->upload(&d_mot, g.motion.data(), g.motion.size(), "edge motions")) != RGG_OK) return guard(st);
        if ((st = rm->upload(&d_del, g.delta.data(), g.delta.size(), "chord deviations")) != RGG_OK) return guard(st);
        vd.D = D;
        vd.B = B;
        vd.dof = g.dof;
        vd.vstride = 2 * g.dof + 3;
        vd.E = E;
        vd.M = M;
        vd.rob = d_rob;
        vd.motion = d_mot;
        vd.delta = d_del;
        vd.cap64 = cap64;
        vd.resident = dv.resident;
    }
    if (cnt && E > 0)
        st = hip_ok(hipMemcpy(dv.cnt, cnt, sizeof(int2) * E, hipMemcpyHostToDevice), "restore counters");
    else
        st = hip_ok(hipMemset(dv.cnt, 0, sizeof(int2) * std::max<int64_t>(E, 1)), "clear counters");
    if (st != RGG_OK) return guard(st);
    if ((st = hip_ok(hipMemset(dv.ctl, 0, sizeof(Ctl)), "clear control")) != RGG_OK) return guard(st);
    if ((st = hip_ok(hipMemset(dv.tile_state, 0, sizeof(unsigned long long) * dv.ntiles), "clear tile states")) != RGG_OK) return guard(st);
    if ((st = hip_ok(hipMemset(dv.rc_cnt, 0, sizeof(int32_t) * kStatBlocks), "clear re-test counts")) != RGG_OK) return guard(st);
    if (mixed) {
        if ((st = hip_ok(hipMemset(dv.pl_cnt, 0, sizeof(int32_t) * kStatBlocks), "clear pair list counts")) != RGG_OK)
            return guard(st);
        if (dv.rt_cnt &&
            (st = hip_ok(hipMemset(dv.rt_cnt, 0, sizeof(int32_t) * kStatBlocks), "clear share re-test counts")) !=
                RGG_OK)
            return guard(st);
    }
    if ((st = hip_ok(hipMemset(dv.blk_stats, 0, sizeof(unsigned long long) * kStatBlocks * kStats), "clear statistics")) != RGG_OK) return guard(st);
    if ((st = hip_ok(hipMemset(rm->d_labels, 0, std::max<int64_t>(E, 1)), "clear labels")) != RGG_OK) return guard(st);
    if ((st = hip_ok(hipHostMalloc((void **)&rm->h_stage, sizeof(rgg_box) * std::max<int64_t>(2 * M, 1)), "pinned staging")) != RGG_OK) return guard(st);
    if ((st = hip_ok(hipHostMalloc((void **)&rm->h_res, sizeof(rgg_update_result)), "pinned result")) != RGG_OK) return guard(st);
    if ((st = hip_ok(hipStreamCreateWithFlags(&rm->stream, hipStreamNonBlocking), "stream")) != RGG_OK) return guard(st);
    if ((st = hip_ok(hipEventCreateWithFlags(&rm->done, hipEventDisableTiming), "event")) != RGG_OK) return guard(st);
    if ((st = hip_ok(hipDeviceSynchronize(), "build upload")) != RGG_OK) return guard(st);

    rgg_roadmap_info &in = rm->info;
    in.n_edges = E;
    in.n_slots = M;
    in.dim = D;
    in.n_spheres = B;
    in.n_sphere_samples = g.soff.back();
    *out = rm;
    return RGG_OK;
}

}  // namespace

rgg_status rgg_build(rgg_context *ctx, const rgg_roadmap_desc *rd, const rgg_robot *robot,
                     const rgg_build_opts *opts, rgg_roadmap **out)
{
    if (!ctx || !out) return fail(RGG_E_INVALID_ARG, "null context or output pointer");
    std::string err;
    rgg_status st = validate_build_inputs(rd, robot, opts, &err);
    if (st != RGG_OK) return fail(st, "%s", err.c_str());
    auto t0 = std::chrono::steady_clock::now();
    HIP_OR_FAIL(hipSetDevice(ctx->device), "hipSetDevice");

    HostGeometry g;
    st = build_geometry(rd, robot, opts, 0, rd->n_edges, host_threads(opts->host_threads), &g, &err);
    if (st != RGG_OK) return fail(st, "%s", err.c_str());
    if (g.B > 0 && g.soff.back() / g.B > (int64_t)UINT32_MAX)
        return fail(RGG_E_INVALID_ARG, "%lld configurations over all edges; at most 2^32 - 1",
                    (long long)(g.soff.back() / g.B));
    const int32_t chunk = opts->item_edges > 0 ? opts->item_edges : kChunk;
    HostGrid grid;
    st = build_grid(g, opts->cell_size, chunk, &grid, &err);
    if (st != RGG_OK) return fail(st, "%s", err.c_str());

    const RoadmapParams p = {opts->n_obstacle_slots, opts->precision == RGG_PREC_FP32_RECHECK, opts->band_rel,
                             opts->retest_capacity, chunk, opts->pair_list_capacity,
                             inline_rounds_of(opts->inline_rounds)};
    if ((st = admit_roadmap(device_bytes_needed(g, grid, p), opts->mem_budget)) != RGG_OK) return st;
    rgg_roadmap *rm = nullptr;
    if ((st = make_roadmap(ctx, g, grid, p, nullptr, nullptr, &rm)) != RGG_OK) return st;
    rm->info.build_seconds = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
    *out = rm;
    return RGG_OK;
}

rgg_status rgg_destroy(rgg_roadmap *rm)
{
    if (!rm) return fail(RGG_E_INVALID_ARG, "null roadmap");
    delete rm;
    return RGG_OK;
}

rgg_status rgg_roadmap_info_get(rgg_roadmap *rm, rgg_roadmap_info *out)
{
    if (!rm || !out) return fail(RGG_E_INVALID_ARG, "null argument");
    *out = rm->info;
    return RGG_OK;
}

}  // extern "C"

namespace rgg {

// Orders this update after the roadmap's previous one when the streams differ.
rgg_status order_after_previous(rgg_roadmap *rm, hipStream_t s)
{
    if (rm->wait_ev && rm->last_stream != s)
        HIP_OR_FAIL(hipStreamWaitEvent(s, rm->wait_ev, 0), "hipStreamWaitEvent");
    return RGG_OK;
}

rgg_status finish_update(rgg_roadmap *rm, hipStream_t s)
{
    HIP_OR_FAIL(hipEventRecord(rm->done, s), "hipEventRecord");
    rm->wait_ev = rm->done;
    rm->last_stream = s;
    return RGG_OK;
}

}  // namespace rgg

namespace {

rgg_status enqueue(rgg_roadmap *rm, hipStream_t s, const UpdateArgs &a)
{
    rgg_status st = order_after_previous(rm, s);
    if (st != RGG_OK) return st;
    hipEvent_t *ev = nullptr;
    if (rm->timing) {
        if (rm->pool.empty()) {
            std::array<hipEvent_t, 7> set;
            for (auto &e : set) HIP_OR_FAIL(hipEventCreate(&e), "hipEventCreate");
            rm->pool.push_back(set);
        }
        rm->pending.push_back(rm->pool.back());
        rm->pool.pop_back();
        ev = rm->pending.back().data();
    }
    HIP_OR_FAIL(launch_update(rm->dv, a, s, ev), "update launch");
    return finish_update(rm, s);
}

}  // namespace

extern "C" {

rgg_status rgg_update_async(rgg_roadmap *rm, void *stream, int64_t m, const rgg_box *d_old,
                            const rgg_box *d_new, uint8_t *d_labels, int64_t *d_gray,
                            int64_t gray_cap, rgg_update_result *d_result)
{
    if (!rm) return fail(RGG_E_INVALID_ARG, "null roadmap");
    if (m != rm->dv.M) return fail(RGG_E_INVALID_ARG, "m = %lld but the roadmap has %lld slots", (long long)m, (long long)rm->dv.M);
    if (m > 0 && (!d_old || !d_new)) return fail(RGG_E_INVALID_ARG, "null box arrays");
    if (!d_result) return fail(RGG_E_INVALID_ARG, "null result pointer");
    if (gray_cap < 0) return fail(RGG_E_INVALID_ARG, "negative gray_cap");
    HIP_OR_FAIL(hipSetDevice(rm->device), "hipSetDevice");
    UpdateArgs a = {d_old, d_new, d_labels, d_gray, d_gray ? gray_cap : 0, d_result};
    return enqueue(rm, (hipStream_t)stream, a);
}

rgg_status rgg_update(rgg_roadmap *rm, int64_t m, const rgg_box *obstacles_old,
                      const rgg_box *obstacles_new, uint8_t *labels, int64_t *gray,
                      int64_t gray_cap, int64_t *n_gray, rgg_update_result *result)
{
    if (!rm) return fail(RGG_E_INVALID_ARG, "null roadmap");
    const int64_t M = rm->dv.M, E = rm->dv.E;
    if (m != M) return fail(RGG_E_INVALID_ARG, "m = %lld but the roadmap has %lld slots", (long long)m, (long long)M);
    if (m > 0 && (!obstacles_old || !obstacles_new)) return fail(RGG_E_INVALID_ARG, "null box arrays");
    if (gray && gray_cap < 0) return fail(RGG_E_INVALID_ARG, "negative gray_cap");
    HIP_OR_FAIL(hipSetDevice(rm->device), "hipSetDevice");
    hipStream_t s = rm->stream;
    if (M > 0) {
        memcpy(rm->h_stage, obstacles_old, sizeof(rgg_box) * M);
        memcpy(rm->h_stage + M, obstacles_new, sizeof(rgg_box) * M);
        rgg_status st = order_after_previous(rm, s);
        if (st != RGG_OK) return st;
        HIP_OR_FAIL(hipMemcpyAsync(rm->d_stage, rm->h_stage, sizeof(rgg_box) * 2 * M, hipMemcpyHostToDevice, s), "upload boxes");
    }
    UpdateArgs a = {rm->d_stage, rm->d_stage + M, rm->d_labels, rm->d_gray, E, rm->d_res};
    rgg_status st = enqueue(rm, s, a);
    if (st != RGG_OK) return st;
    HIP_OR_FAIL(hipMemcpyAsync(rm->h_res, rm->d_res, sizeof(rgg_update_result), hipMemcpyDeviceToHost, s), "read result");
    HIP_OR_FAIL(hipStreamSynchronize(s), "update");
    const rgg_update_result r = *rm->h_res;
    if (result) *result = r;
    if (r.status != RGG_OK) {
        return fail(r.status, r.status == RGG_E_STATE_MISMATCH
                                  ? "obstacles_old differs from the resident obstacle slots"
                                  : "non-finite or out-of-range box coordinate");
    }
    if (labels && E > 0) HIP_OR_FAIL(hipMemcpy(labels, rm->d_labels, (size_t)E, hipMemcpyDeviceToHost), "read labels");
    if (gray) {
        int64_t k = std::min(r.n_gray, gray_cap);
        if (k > 0) HIP_OR_FAIL(hipMemcpy(gray, rm->d_gray, sizeof(int64_t) * k, hipMemcpyDeviceToHost), "read gray list");
    }
    if (n_gray) *n_gray = r.n_gray;
    if (gray && r.n_gray > gray_cap)
        return fail(RGG_E_CAPACITY, "gray list has %lld edges, capacity %lld", (long long)r.n_gray, (long long)gray_cap);
    return RGG_OK;
}

static rgg_status check_validate_args(rgg_roadmap *rm, int64_t n, int32_t *max_level, int32_t *max_active)
{
    if (!rm) return fail(RGG_E_INVALID_ARG, "null roadmap");
    if (n < 0) return fail(RGG_E_INVALID_ARG, "negative edge count");
    if (*max_level == 0) *max_level = RGG_VALIDATE_DEFAULT_LEVELS;
    if (*max_active == 0) *max_active = RGG_VALIDATE_DEFAULT_ACTIVE;
    if (*max_level < 0 || *max_level > 30) return fail(RGG_E_INVALID_ARG, "max_level must be 0..30");
    if (*max_active < 1 || *max_active > kValMaxActive) return fail(RGG_E_INVALID_ARG, "max_active must be 0..512");
    return RGG_OK;
}

rgg_status rgg_validate_async(rgg_roadmap *rm, void *stream, const int64_t *d_ids, int64_t n,
                              const rgg_update_result *d_count, int32_t max_level, int32_t max_active,
                              uint8_t *d_verdict, int32_t *d_level, double *d_witness, uint8_t *d_labels)
{
    rgg_status st = check_validate_args(rm, n, &max_level, &max_active);
    if (st != RGG_OK) return st;
    if (n > 0 && (!d_ids || (!d_verdict && !d_labels)))
        return fail(RGG_E_INVALID_ARG, "null ids, or neither verdicts nor labels requested");
    HIP_OR_FAIL(hipSetDevice(rm->device), "hipSetDevice");
    hipStream_t s = (hipStream_t)stream;
    if ((st = order_after_previous(rm, s)) != RGG_OK) return st;
    HIP_OR_FAIL(launch_validate(rm->val, d_ids, n, d_count, max_level, max_active, d_verdict, d_level, d_witness,
                                d_labels, s),
                "validate launch");
    return finish_update(rm, s);
}

rgg_status rgg_validate(rgg_roadmap *rm, const int64_t *ids, int64_t n, int32_t max_level, int32_t max_active,
                        uint8_t *verdict, int32_t *level, double *witness)
{
    rgg_status st = check_validate_args(rm, n, &max_level, &max_active);
    if (st != RGG_OK) return st;
    if (n == 0) return RGG_OK;
    if (!ids || !verdict) return fail(RGG_E_INVALID_ARG, "null array");
    for (int64_t i = 0; i < n; ++i)
        if (ids[i] < 0 || ids[i] >= rm->dv.E)
            return fail(RGG_E_INVALID_ARG, "ids[%lld] = %lld is not an edge", (long long)i, (long long)ids[i]);
    HIP_OR_FAIL(hipSetDevice(rm->device), "hipSetDevice");
    hipStream_t s = rm->stream;
    // one device block: ids, then verdicts, levels and witnesses
    const size_t b_ids = sizeof(int64_t) * n, b_wit = sizeof(double) * n, b_lev = sizeof(int32_t) * n;
    char *d = nullptr;
    HIP_OR_FAIL(hipMalloc((void **)&d, b_ids + b_wit + b_lev + (size_t)n), "validation buffers");
    int64_t *d_ids = (int64_t *)d;
    double *d_wit = (double *)(d + b_ids);
    int32_t *d_lev = (int32_t *)(d + b_ids + b_wit);
    uint8_t *d_ver = (uint8_t *)(d + b_ids + b_wit + b_lev);
    auto run = [&]() -> rgg_status {
        rgg_status r = order_after_previous(rm, s);
        if (r != RGG_OK) return r;
        HIP_OR_FAIL(hipMemcpyAsync(d_ids, ids, b_ids, hipMemcpyHostToDevice, s), "upload ids");
        HIP_OR_FAIL(launch_validate(rm->val, d_ids, n, nullptr, max_level, max_active, d_ver, d_lev, d_wit, nullptr,
                                    s),
                    "validate launch");
        if ((r = finish_update(rm, s)) != RGG_OK) return r;
        HIP_OR_FAIL(hipMemcpyAsync(verdict, d_ver, (size_t)n, hipMemcpyDeviceToHost, s), "read verdicts");
        if (level) HIP_OR_FAIL(hipMemcpyAsync(level, d_lev, b_lev, hipMemcpyDeviceToHost, s), "read levels");
        if (witness) HIP_OR_FAIL(hipMemcpyAsync(witness, d_wit, b_wit, hipMemcpyDeviceToHost, s), "read witnesses");
        HIP_OR_FAIL(hipStreamSynchronize(s), "validate");
        return RGG_OK;
    };
    st = run();
    if (st != RGG_OK) (void)hipStreamSynchronize(s);
    (void)hipFree(d);
    return st;
}

static rgg_status refresh_labels(rgg_roadmap *rm, rgg_update_result *r)
{
    HIP_OR_FAIL(hipSetDevice(rm->device), "hipSetDevice");
    hipStream_t s = rm->stream;
    rgg_status st = order_after_previous(rm, s);
    if (st != RGG_OK) return st;
    UpdateArgs a = {nullptr, nullptr, rm->d_labels, rm->d_gray, rm->dv.E, rm->d_res};
    HIP_OR_FAIL(launch_labels(rm->dv, a, s), "label launch");
    HIP_OR_FAIL(hipMemcpyAsync(rm->h_res, rm->d_res, sizeof(rgg_update_result), hipMemcpyDeviceToHost, s), "read result");
    HIP_OR_FAIL(hipStreamSynchronize(s), "labels");
    st = finish_update(rm, s);
    *r = *rm->h_res;
    return st;
}

rgg_status rgg_labels(rgg_roadmap *rm, uint8_t *out)
{
    if (!rm || (!out && rm->dv.E > 0)) return fail(RGG_E_INVALID_ARG, "null argument");
    rgg_update_result r;
    rgg_status st = refresh_labels(rm, &r);
    if (st != RGG_OK) return st;
    if (rm->dv.E > 0) HIP_OR_FAIL(hipMemcpy(out, rm->d_labels, (size_t)rm->dv.E, hipMemcpyDeviceToHost), "read labels");
    return RGG_OK;
}

rgg_status rgg_gray_list(rgg_roadmap *rm, int64_t *out, int64_t cap, int64_t *n)
{
    if (!rm || !n || cap < 0 || (cap > 0 && !out)) return fail(RGG_E_INVALID_ARG, "bad argument");
    rgg_update_result r;
    rgg_status st = refresh_labels(rm, &r);
    if (st != RGG_OK) return st;
    *n = r.n_gray;
    int64_t k = std::min(r.n_gray, cap);
    if (k > 0) HIP_OR_FAIL(hipMemcpy(out, rm->d_gray, sizeof(int64_t) * k, hipMemcpyDeviceToHost), "read gray list");
    return r.n_gray > cap ? fail(RGG_E_CAPACITY, "gray list has %lld edges, capacity %lld", (long long)r.n_gray, (long long)cap) : RGG_OK;
}

rgg_status rgg_timing_enable(rgg_roadmap *rm, int32_t on)
{
    if (!rm) return fail(RGG_E_INVALID_ARG, "null roadmap");
    rm->timing = on != 0;
    return RGG_OK;
}

rgg_status rgg_timing_read(rgg_roadmap *rm, double ms[6], int64_t *n_updates)
{
    if (!rm || !ms) return fail(RGG_E_INVALID_ARG, "null argument");
    HIP_OR_FAIL(hipSetDevice(rm->device), "hipSetDevice");
    for (auto &set : rm->pending) {
        HIP_OR_FAIL(hipEventSynchronize(set[6]), "hipEventSynchronize");
        for (int k = 0; k < 6; ++k) {
            float t = 0.0f;
            HIP_OR_FAIL(hipEventElapsedTime(&t, set[k], set[k + 1]), "hipEventElapsedTime");
            rm->ms_acc[k] += t;
        }
        rm->timed++;
        rm->pool.push_back(set);
    }
    rm->pending.clear();
    for (int k = 0; k < 6; ++k) {
        ms[k] = rm->ms_acc[k];
        rm->ms_acc[k] = 0.0;
    }
    if (n_updates) *n_updates = rm->timed;
    rm->timed = 0;
    return RGG_OK;
}

rgg_status rgg_graph_create(rgg_context *ctx, int32_t n, const rgg_update_req *reqs, rgg_graph **out)
{
    if (!ctx || !out || n < 1 || !reqs) return fail(RGG_E_INVALID_ARG, "bad argument");
    for (int32_t k = 0; k < n; ++k) {
        const rgg_update_req &q = reqs[k];
        if (!q.rm || q.m != q.rm->dv.M || (q.m > 0 && (!q.d_old || !q.d_new)) || !q.d_result || q.gray_cap < 0)
            return fail(RGG_E_INVALID_ARG, "bad request %d", k);
        if (q.rm->device != ctx->device) return fail(RGG_E_INVALID_ARG, "request %d is on another device", k);
    }
    HIP_OR_FAIL(hipSetDevice(ctx->device), "hipSetDevice");
    auto *g = new rgg_graph();
    g->device = ctx->device;
    hipError_t e = hipGraphCreate(&g->graph, 0);
    if (e != hipSuccess) {
        delete g;
        return hip_fail(e, "hipGraphCreate");
    }
    std::map<rgg_roadmap *, hipGraphNode_t> tail;
    for (int32_t k = 0; k < n; ++k) {
        const rgg_update_req &q = reqs[k];
        UpdateArgs a = {q.d_old, q.d_new, q.d_labels, q.d_gray, q.d_gray ? q.gray_cap : 0, q.d_result};
        hipGraphNode_t dep = tail.count(q.rm) ? tail[q.rm] : nullptr, last = nullptr;
        e = add_update_nodes(g->graph, q.rm->dv, a, dep, &last);
        if (e != hipSuccess) {
            hipGraphDestroy(g->graph);
            delete g;
            return hip_fail(e, "hipGraphAddKernelNode");
        }
        tail[q.rm] = last;
    }
    for (auto &kv : tail) g->roadmaps.push_back(kv.first);
    e = hipGraphInstantiate(&g->exec, g->graph, nullptr, nullptr, 0);
    if (e != hipSuccess) {
        hipGraphDestroy(g->graph);
        delete g;
        return hip_fail(e, "hipGraphInstantiate");
    }
    for (rgg_roadmap *rm : g->roadmaps) rm->holders++;   // the nodes hold its arrays
    *out = g;
    return RGG_OK;
}

rgg_status rgg_graph_launch(rgg_graph *g, void *stream)
{
    if (!g) return fail(RGG_E_INVALID_ARG, "null graph");
    HIP_OR_FAIL(hipSetDevice(g->device), "hipSetDevice");
    hipStream_t s = (hipStream_t)stream;
    for (rgg_roadmap *rm : g->roadmaps) {
        rgg_status st = order_after_previous(rm, s);
        if (st != RGG_OK) return st;
    }
    HIP_OR_FAIL(hipGraphLaunch(g->exec, s), "hipGraphLaunch");
    for (rgg_roadmap *rm : g->roadmaps) {
        rgg_status st = finish_update(rm, s);
        if (st != RGG_OK) return st;
    }
    return RGG_OK;
}

rgg_status rgg_graph_destroy(rgg_graph *g)
{
    if (!g) return fail(RGG_E_INVALID_ARG, "null graph");
    hipSetDevice(g->device);
    if (g->exec) hipGraphExecDestroy(g->exec);
    if (g->graph) hipGraphDestroy(g->graph);
    for (rgg_roadmap *rm : g->roadmaps) rm->holders--;
    delete g;
    return RGG_OK;
}

rgg_status rgg_batch_create(rgg_context *ctx, int32_t n, rgg_roadmap *const *rms, rgg_batch **out)
{
    if (!ctx || !out || !rms) return fail(RGG_E_INVALID_ARG, "null argument");
    if (n < 1 || n > kMaxBatch) return fail(RGG_E_INVALID_ARG, "n = %d, allowed 1..%d", n, kMaxBatch);
    std::map<rgg_roadmap *, int> seen;
    for (int32_t k = 0; k < n; ++k) {
        if (!rms[k]) return fail(RGG_E_INVALID_ARG, "roadmap %d is null", k);
        if (rms[k]->device != ctx->device) return fail(RGG_E_INVALID_ARG, "roadmap %d is on another device", k);
        if (seen.count(rms[k])) return fail(RGG_E_INVALID_ARG, "roadmap %d repeats roadmap %d", k, seen[rms[k]]);
        seen[rms[k]] = k;
        if (rms[k]->dv.chunk < 1 || rms[k]->dv.chunk > item_edges_max())
            return fail(RGG_E_INVALID_ARG, "roadmap %d has work items of %d edges", k, rms[k]->dv.chunk);
        if (rms[k]->dv.mode != 0)
            return fail(RGG_E_UNSUPPORTED, "roadmap %d uses the oriented boxes or splines; batches take the "
                        "capsule and copy forms", k);
    }
    HIP_OR_FAIL(hipSetDevice(ctx->device), "hipSetDevice");
    std::unique_ptr<rgg_batch> b(new rgg_batch());
    b->device = ctx->device;
    b->n = n;
    b->rms.assign(rms, rms + n);
    for (rgg_roadmap *rm : b->rms) rm->holders++;   // released by ~rgg_batch
    // table rows grouped by kernel variant (dimension, precision)
    std::vector<BatchGroup> &groups = b->groups;
    for (int D = 2; D <= 3; ++D)
        for (int mixed = 0; mixed <= 1; ++mixed) {
            BatchGroup g = {D, mixed, (int32_t)b->order.size(), 0};
            for (int32_t k = 0; k < n; ++k)
                if (rms[k]->dv.D == D && rms[k]->dv.mixed == mixed) {
                    b->order.push_back(k);
                    ++g.count;
                }
            if (g.count) groups.push_back(g);
        }
    for (int32_t k = 0; k < n; ++k) {
        b->any_grid = b->any_grid || rms[k]->dv.ncells > 1;
        b->tiles += rms[k]->dv.ntiles;
        b->wtiles += rms[k]->dv.ntiles + 1;
    }
    std::vector<int32_t> grp(n);
    for (int32_t k = 0; k < n; ++k) grp[k] = k;   // rows are already grouped
    HIP_OR_FAIL(hipMalloc(&b->d_tab, sizeof(BatchReq) * n), "batch table");
    HIP_OR_FAIL(hipMalloc(&b->d_grp, sizeof(int32_t) * n), "batch groups");
    HIP_OR_FAIL(hipMemcpy(b->d_grp, grp.data(), sizeof(int32_t) * n, hipMemcpyHostToDevice), "batch groups");
    for (int k = 0; k < rgg_batch::kRing; ++k) {
        HIP_OR_FAIL(hipHostMalloc((void **)&b->h_tab[k], sizeof(BatchReq) * n, hipHostMallocDefault), "pinned table");
        HIP_OR_FAIL(hipEventCreateWithFlags(&b->done[k], hipEventDisableTiming), "hipEventCreate");
    }
    rgg_status st = build_batch_graphs(b.get());
    if (st != RGG_OK) return st;
    *out = b.release();
    return RGG_OK;
}

static rgg_status batch_launch(rgg_batch *b, const rgg_update_req *reqs, void *stream, bool graph)
{
    if (!b || !reqs) return fail(RGG_E_INVALID_ARG, "null argument");
    for (int k = 0; k < b->n; ++k) {
        const rgg_update_req &q = reqs[k];
        if (q.rm != b->rms[k]) return fail(RGG_E_INVALID_ARG, "request %d names another roadmap than the batch", k);
        if (q.m != q.rm->dv.M || (q.m > 0 && (!q.d_old || !q.d_new)) || !q.d_result || q.gray_cap < 0)
            return fail(RGG_E_INVALID_ARG, "bad request %d", k);
    }
    HIP_OR_FAIL(hipSetDevice(b->device), "hipSetDevice");
    hipStream_t s = (hipStream_t)stream;
    // a free host table: its previous copy has completed
    const int slot = b->ring;
    b->ring = (b->ring + 1) % rgg_batch::kRing;
    if (b->used[slot]) HIP_OR_FAIL(hipEventSynchronize(b->done[slot]), "hipEventSynchronize");
    BatchReq *h = b->h_tab[slot];
    int tile = 0, wtile = 0;
    for (int row = 0; row < b->n; ++row) {
        const rgg_update_req &q = reqs[b->order[row]];
        BatchReq &t = h[row];
        t.rm = q.rm->dv;
        t.a = {q.d_old, q.d_new, q.d_labels, q.d_gray, q.d_gray ? q.gray_cap : 0, q.d_result};
        t.tile0 = tile;
        t.wtile0 = wtile;
        tile += q.rm->dv.ntiles;
        wtile += q.rm->dv.ntiles + 1;
    }
    for (rgg_roadmap *rm : b->rms) {
        rgg_status st = order_after_previous(rm, s);
        if (st != RGG_OK) return st;
    }
    BatchTiming *tm = nullptr;
    if (b->timing && !graph) {
        if (b->t_pool.empty()) {
            BatchTiming t = {};
            for (hipEvent_t &e : t.ev) HIP_OR_FAIL(hipEventCreate(&e), "hipEventCreate");
            b->t_pool.push_back(t);
        }
        b->t_pending.push_back(b->t_pool.back());
        b->t_pool.pop_back();
        tm = &b->t_pending.back();
    }
    if (graph)
        HIP_OR_FAIL(hipGraphLaunch(b->exec[slot], s), "hipGraphLaunch");
    else
        HIP_OR_FAIL(launch_batch(s, b->d_tab, h, b->d_grp, b->n, b->groups.data(), (int)b->groups.size(),
                                 b->any_grid, b->tiles, b->wtiles, tm),
                    "batch launch");
    HIP_OR_FAIL(hipEventRecord(b->done[slot], s), "hipEventRecord");
    b->used[slot] = true;
    for (rgg_roadmap *rm : b->rms) {   // one event stands for every roadmap's update
        rm->wait_ev = b->done[slot];
        rm->last_stream = s;
    }
    return RGG_OK;
}

rgg_status rgg_batch_launch(rgg_batch *b, const rgg_update_req *reqs, void *stream)
{
    return batch_launch(b, reqs, stream, false);
}

rgg_status rgg_batch_launch_graph(rgg_batch *b, const rgg_update_req *reqs, void *stream)
{
    return batch_launch(b, reqs, stream, true);
}

rgg_status rgg_batch_timing_enable(rgg_batch *b, int32_t on)
{
    if (!b) return fail(RGG_E_INVALID_ARG, "null batch");
    b->timing = on != 0;
    return RGG_OK;
}

rgg_status rgg_batch_timing_read(rgg_batch *b, double ms[6], int64_t *n_launches)
{
    if (!b) return fail(RGG_E_INVALID_ARG, "null batch");
    HIP_OR_FAIL(hipSetDevice(b->device), "hipSetDevice");
    for (BatchTiming &t : b->t_pending) {
        HIP_OR_FAIL(hipEventSynchronize(t.ev[t.n]), "hipEventSynchronize");
        for (int k = 0; k < t.n; ++k) {
            float m = 0.0f;
            HIP_OR_FAIL(hipEventElapsedTime(&m, t.ev[k], t.ev[k + 1]), "hipEventElapsedTime");
            b->ms_acc[t.stage[k]] += m;
        }
        b->timed++;
        b->t_pool.push_back(t);
    }
    b->t_pending.clear();
    if (ms)
        for (int k = 0; k < 6; ++k) ms[k] = b->ms_acc[k];
    if (n_launches) *n_launches = b->timed;
    for (double &m : b->ms_acc) m = 0.0;
    b->timed = 0;
    return RGG_OK;
}

rgg_status rgg_batch_destroy(rgg_batch *b)
{
    if (!b) return fail(RGG_E_INVALID_ARG, "null batch");
    delete b;
    return RGG_OK;
}

rgg_status rgg_update_batch(rgg_context *ctx, int32_t n, const rgg_update_req *reqs, void *stream)
{
    if (!ctx || !reqs || n < 1 || n > kMaxBatch) return fail(RGG_E_INVALID_ARG, "bad argument");
    std::vector<rgg_roadmap *> rms(n);
    for (int32_t k = 0; k < n; ++k) rms[k] = reqs[k].rm;
    rgg_batch *b = nullptr;
    rgg_status st = rgg_batch_create(ctx, n, rms.data(), &b);
    if (st != RGG_OK) return st;
    st = rgg_batch_launch(b, reqs, stream);
    if (st == RGG_OK) {
        hipError_t e = hipStreamSynchronize((hipStream_t)stream);
        if (e != hipSuccess) st = hip_fail(e, "batched update");
    }
    rgg_batch_destroy(b);
    return st;
}

rgg_status rgg_update_batch_noalloc(rgg_context *ctx, int32_t n, const rgg_update_req *reqs, void *stream)
{
    if (!ctx || !reqs) return fail(RGG_E_INVALID_ARG, "null argument");
    if (n < 1 || n > kMaxBatch)
        return fail(RGG_E_INVALID_ARG, "n = %d, allowed 1..%d (the size of the fixed request table)", n, kMaxBatch);
    for (int32_t k = 0; k < n; ++k) {
        const rgg_update_req &q = reqs[k];
        if (!q.rm) return fail(RGG_E_INVALID_ARG, "request %d names no roadmap", k);
        if (q.rm->device != ctx->device) return fail(RGG_E_INVALID_ARG, "roadmap %d is on another device", k);
        for (int32_t j = 0; j < k; ++j)
            if (reqs[j].rm == q.rm) return fail(RGG_E_INVALID_ARG, "request %d repeats the roadmap of request %d", k, j);
        if (q.rm->dv.chunk < 1 || q.rm->dv.chunk > item_edges_max())
            return fail(RGG_E_INVALID_ARG, "roadmap %d has work items of %d edges", k, q.rm->dv.chunk);
        if (q.rm->dv.mode != 0)
            return fail(RGG_E_UNSUPPORTED, "roadmap %d uses the oriented boxes or splines; batches take the "
                        "capsule and copy forms", k);
        if (q.m != q.rm->dv.M || (q.m > 0 && (!q.d_old || !q.d_new)) || !q.d_result || q.gray_cap < 0)
            return fail(RGG_E_INVALID_ARG, "bad request %d", k);
    }
    HIP_OR_FAIL(hipSetDevice(ctx->device), "hipSetDevice");
    hipStream_t s = (hipStream_t)stream;
    // The host side of the table is static too; the lock also keeps calls of
    // this process from overlapping on the device scratch, which every
    // context of the device shares.
    static std::mutex mu;
    static BatchReq h_tab[kMaxBatch];
    static int32_t h_grp[kMaxBatch];
    std::lock_guard<std::mutex> lock(mu);
    BatchReq *d_tab = (BatchReq *)ctx->batch_scratch;
    int32_t *d_grp = (int32_t *)((char *)ctx->batch_scratch + kBatchTableBytes);
    // rows grouped by kernel variant (dimension, precision), as rgg_batch_create
    BatchGroup groups[4];
    int n_groups = 0, row = 0, tile = 0, wtile = 0;
    bool any_grid = false;
    for (int D = 2; D <= 3; ++D)
        for (int mixed = 0; mixed <= 1; ++mixed) {
            BatchGroup g = {D, mixed, row, 0};
            for (int32_t k = 0; k < n; ++k) {
                const rgg_update_req &q = reqs[k];
                if (q.rm->dv.D != D || q.rm->dv.mixed != mixed) continue;
                BatchReq &t = h_tab[row];
                t.rm = q.rm->dv;
                t.a = {q.d_old, q.d_new, q.d_labels, q.d_gray, q.d_gray ? q.gray_cap : 0, q.d_result};
                t.tile0 = tile;
                t.wtile0 = wtile;
                tile += q.rm->dv.ntiles;
                wtile += q.rm->dv.ntiles + 1;
                any_grid = any_grid || q.rm->dv.ncells > 1;
                h_grp[row] = row;
                ++row;
                ++g.count;
            }
            if (g.count) groups[n_groups++] = g;
        }
    for (int32_t k = 0; k < n; ++k) {
        rgg_status st = order_after_previous(reqs[k].rm, s);
        if (st != RGG_OK) return st;
    }
    HIP_OR_FAIL(hipMemcpyAsync(d_tab, h_tab, sizeof(BatchReq) * n, hipMemcpyHostToDevice, s), "copy batch table");
    HIP_OR_FAIL(hipMemcpyAsync(d_grp, h_grp, sizeof(int32_t) * n, hipMemcpyHostToDevice, s), "copy batch rows");
    HIP_OR_FAIL(launch_batch(s, d_tab, nullptr, d_grp, n, groups, n_groups, any_grid, tile, wtile), "batch launch");
    for (int32_t k = 0; k < n; ++k) {
        rgg_status st = finish_update(reqs[k].rm, s);
        if (st != RGG_OK) return st;
    }
    // the next call rewrites the static tables
    HIP_OR_FAIL(hipStreamSynchronize(s), "batched update");
    return RGG_OK;
}

rgg_status rgg_tune(rgg_roadmap *rm, int64_t m, const rgg_box *obstacles_a, int32_t n_b,
                    const rgg_box *obstacles_b, int32_t reps, rgg_tune_report *report)
{
    if (!rm) return fail(RGG_E_INVALID_ARG, "null roadmap");
    const int64_t M = rm->dv.M;
    if (m != M) return fail(RGG_E_INVALID_ARG, "m = %lld but the roadmap has %lld slots", (long long)m, (long long)M);
    if (n_b < 1 || n_b > kTuneMaxStates) return fail(RGG_E_INVALID_ARG, "n_b = %d, allowed 1..%d", n_b, kTuneMaxStates);
    if (M > 0 && (!obstacles_a || !obstacles_b)) return fail(RGG_E_INVALID_ARG, "null box arrays");
    if (reps < 0 || reps > 1000) return fail(RGG_E_INVALID_ARG, "reps = %d, allowed 0..1000", reps);
    if (reps == 0) reps = 5;
    if (rm->holders.load() > 0)
        return fail(RGG_E_BUSY, "the roadmap is held by a graph, a batch or a server request");
    HIP_OR_FAIL(hipSetDevice(rm->device), "hipSetDevice");
    std::vector<const rgg_box *> bs((size_t)n_b);
    for (int i = 0; i < n_b; ++i) bs[(size_t)i] = obstacles_b + (size_t)i * M;
    TuneSubject t;
    rgg_status st = tune_subject(rm, obstacles_a, n_b, bs.data(), &t);
    if (st != RGG_OK) return st;
    hipStream_t s = rm->stream;
    // every state b_i is visited from a and left back to a
    auto run = [&](int count) -> rgg_status {
        for (int r = 0; r < count; ++r)
            for (int i = 0; i < n_b; ++i) {
                HIP_OR_FAIL(launch_update(rm->dv, t.args(i, true), s, nullptr), "update launch");
                HIP_OR_FAIL(launch_update(rm->dv, t.args(i, false), s, nullptr), "update launch");
            }
        return RGG_OK;
    };
    // one cell with items sized so that their count fills 1, 2 or 3 rounds
    // of the resident item blocks exactly
    std::vector<TuneCand> extra;
    int resident = 0;
    HIP_OR_FAIL(item_blocks_resident(rm->dv.D, rm->device, &resident), "occupancy query");
    for (int rounds = 1; rounds <= 3 && resident > 0; ++rounds) {
        const int64_t chunk = (rm->dv.E + (int64_t)rounds * resident - 1) / ((int64_t)rounds * resident);
        if (chunk >= 32 && chunk <= item_edges_max() && chunk != 512 && chunk != 256 && chunk != 128 && chunk != 64)
            extra.push_back({-1.0, (int32_t)chunk});
    }
    std::vector<TuneSubject *> subj = {&t};
    st = tune_search(subj, s, reps, 2 * n_b, run, false, report, nullptr, extra);
    if (st != RGG_OK) return st;
    return finish_update(rm, s);
}

rgg_status rgg_batch_tune(rgg_batch *b, const rgg_box *const *obstacles_a, const rgg_box *const *obstacles_b,
                          int32_t reps, rgg_tune_report *report)
{
    if (!b || !obstacles_a || !obstacles_b) return fail(RGG_E_INVALID_ARG, "null argument");
    if (reps < 0 || reps > 1000) return fail(RGG_E_INVALID_ARG, "reps = %d, allowed 0..1000", reps);
    if (reps == 0) reps = 5;
    for (int k = 0; k < b->n; ++k) {
        if (b->rms[k]->dv.M > 0 && (!obstacles_a[k] || !obstacles_b[k]))
            return fail(RGG_E_INVALID_ARG, "null box arrays for roadmap %d", k);
        if (b->rms[k]->holders.load() != 1)
            return fail(RGG_E_BUSY, "roadmap %d is also held by another graph, batch or server request", k);
    }
    HIP_OR_FAIL(hipSetDevice(b->device), "hipSetDevice");
    for (int k = 0; k < rgg_batch::kRing; ++k)
        if (b->used[k]) HIP_OR_FAIL(hipEventSynchronize(b->done[k]), "batch launches");
    std::vector<std::unique_ptr<TuneSubject>> subj((size_t)b->n);
    std::vector<TuneSubject *> ptrs((size_t)b->n);
    for (int k = 0; k < b->n; ++k) {
        subj[(size_t)k].reset(new TuneSubject());
        rgg_status st = tune_subject(b->rms[k], obstacles_a[k], 1, &obstacles_b[k], subj[(size_t)k].get());
        if (st != RGG_OK) return fail(st, "roadmap %d: %s", k, rgg_last_error());
        ptrs[(size_t)k] = subj[(size_t)k].get();
    }
    hipStream_t s = b->rms[0]->stream;
    // request tables of the two directions, in the batch's row order
    std::vector<BatchReq> fwd((size_t)b->n), back((size_t)b->n);
    BatchReq *d_fwd = nullptr, *d_back = nullptr;
    struct Free {
        BatchReq **p[2];
        ~Free()
        {
            for (auto q : p)
                if (*q) (void)hipFree(*q);
        }
    } fr{{&d_fwd, &d_back}};
    HIP_OR_FAIL(hipMalloc(&d_fwd, sizeof(BatchReq) * b->n), "tuning tables");
    HIP_OR_FAIL(hipMalloc(&d_back, sizeof(BatchReq) * b->n), "tuning tables");
    auto fill = [&]() -> rgg_status {
        int tile = 0, wtile = 0;
        for (int row = 0; row < b->n; ++row) {
            const int k = b->order[row];
            rgg_roadmap *rm = b->rms[k];
            fwd[(size_t)row] = {rm->dv, subj[(size_t)k]->args(0, true), tile, wtile};
            back[(size_t)row] = {rm->dv, subj[(size_t)k]->args(0, false), tile, wtile};
            tile += rm->dv.ntiles;
            wtile += rm->dv.ntiles + 1;
        }
        b->any_grid = false;
        for (rgg_roadmap *rm : b->rms) b->any_grid = b->any_grid || rm->dv.ncells > 1;
        HIP_OR_FAIL(hipMemcpy(d_fwd, fwd.data(), sizeof(BatchReq) * b->n, hipMemcpyHostToDevice), "tuning tables");
        HIP_OR_FAIL(hipMemcpy(d_back, back.data(), sizeof(BatchReq) * b->n, hipMemcpyHostToDevice), "tuning tables");
        return RGG_OK;
    };
    auto run = [&](int count) -> rgg_status {
        for (int r = 0; r < count; ++r)
            for (BatchReq *tab : {d_fwd, d_back})
                HIP_OR_FAIL(launch_batch(s, tab, nullptr, b->d_grp, b->n, b->groups.data(), (int)b->groups.size(), b->any_grid,
                                         b->tiles, b->wtiles),
                            "batch launch");
        return RGG_OK;
    };
    rgg_status st = tune_search(ptrs, s, reps, 2, run, true, report, fill);
    // whatever happened, the launches follow the roadmaps' grids as they now
    // are; the captured graph's kernels depend on whether any uses a grid
    b->any_grid = false;
    for (rgg_roadmap *rm : b->rms) b->any_grid = b->any_grid || rm->dv.ncells > 1;
    const rgg_status sg = build_batch_graphs(b);
    if (st != RGG_OK) return st;
    if (sg != RGG_OK) return sg;
    for (rgg_roadmap *rm : b->rms) {
        st = finish_update(rm, s);
        if (st != RGG_OK) return st;
    }
    return RGG_OK;
}

}  // extern "C"

namespace {

// Roadmap files: a header, the binary64 geometry, the state, and an FNV-1a
// 64-bit checksum of every preceding byte.  Host byte order.
constexpr char kMagic[8] = {'R', 'G', 'G', 'M', 'A', 'P', '0', '1'};
constexpr uint32_t kFileVersion = 4;

struct FileHeader {
    char magic[8];
    uint32_t version;
    int32_t D, B, mixed, chunk, retest_capacity;
    int64_t E, M;
    float band_rel;
    int32_t one_cell;
    double cell;
    int64_t n_samp, n_cap;
};

struct Fnv {
    uint64_t h = 0xcbf29ce484222325ull;   // FNV-1a 64-bit offset basis
    void add(const void *p, size_t n)
    {
        const unsigned char *b = static_cast<const unsigned char *>(p);
        for (size_t i = 0; i < n; ++i) h = (h ^ b[i]) * 0x100000001b3ull;   // FNV 64-bit prime
    }
};

struct FileOut {
    FILE *f = nullptr;
    Fnv sum;
    bool ok = true;
    ~FileOut()
    {
        if (f) fclose(f);
    }
    void put(const void *p, size_t n)
    {
        if (!ok || n == 0) return;
        sum.add(p, n);
        ok = fwrite(p, 1, n, f) == n;
    }
};

struct FileIn {
    FILE *f = nullptr;
    Fnv sum;
    bool ok = true;
    ~FileIn()
    {
        if (f) fclose(f);
    }
    void get(void *p, size_t n)
    {
        if (!ok || n == 0) return;
        ok = fread(p, 1, n, f) == n;
        if (ok) sum.add(p, n);
    }
};

// What a roadmap file holds, read back on the host.
struct LoadedFile {
    FileHeader h;
    int32_t pl_cap = 0;        // pair-list capacity (0 in the FP64 mode)
    int32_t inline_rounds = 0; // RmDev::inline_rounds (0 in the FP64 mode)
    HostGeometry g;
    std::vector<rgg_box> resident;
    std::vector<int2> cnt;
};

template <typename T>
rgg_status read_back(std::vector<T> *v, const T *d, size_t n, const char *what)
{
    try {
        v->resize(n);
    } catch (const std::bad_alloc &) {
        return fail(RGG_E_OUT_OF_MEMORY, "host memory for %s", what);
    }
    if (n) HIP_OR_FAIL(hipMemcpy(v->data(), d, sizeof(T) * n, hipMemcpyDeviceToHost), what);
    return RGG_OK;
}

}  // namespace

extern "C" {

rgg_status rgg_save(rgg_roadmap *rm, const char *path)
{
    if (!rm || !path) return fail(RGG_E_INVALID_ARG, "null argument");
    if (rm->holders.load() > 0)
        return fail(RGG_E_BUSY, "the roadmap is held by a graph, a batch or a server request");
    HIP_OR_FAIL(hipSetDevice(rm->device), "hipSetDevice");
    if (rm->wait_ev) HIP_OR_FAIL(hipEventSynchronize(rm->wait_ev), "wait for the previous update");
    HIP_OR_FAIL(hipStreamSynchronize(rm->stream), "roadmap stream");
    const RmDev &dv = rm->dv;
    const int64_t E = dv.E, M = dv.M;
    std::vector<int64_t> soff;
    std::vector<double> samp, cap, rad;
    std::vector<float> aabb;
    std::vector<rgg_box> resident;
    std::vector<int2> cnt;
    rgg_status st;
    if ((st = read_back(&soff, dv.soff, (size_t)(E + 1), "sample offsets")) != RGG_OK) return st;
    const int64_t n_samp = (int64_t)copy_stride(dv.D) * soff.back();
    const int64_t n_cap = E * (2 * dv.D + 1) * dv.B;
    if ((st = read_back(&samp, dv.samp64, (size_t)n_samp, "samples")) != RGG_OK) return st;
    if ((st = read_back(&cap, dv.cap64, (size_t)n_cap, "capsules")) != RGG_OK) return st;
    if ((st = read_back(&rad, dv.rad64, (size_t)dv.B, "radii")) != RGG_OK) return st;
    if ((st = read_back(&aabb, dv.aabb, (size_t)(E * kAabbStride), "edge boxes")) != RGG_OK) return st;
    if ((st = read_back(&resident, dv.resident, (size_t)M, "obstacle slots")) != RGG_OK) return st;
    if ((st = read_back(&cnt, dv.cnt, (size_t)E, "counters")) != RGG_OK) return st;
    const ValDev &vd = rm->val;
    std::vector<VRobot> vrob;
    std::vector<double> vmot, vdel;
    if ((st = read_back(&vrob, vd.rob, 1, "validation robot")) != RGG_OK) return st;
    if ((st = read_back(&vmot, vd.motion, (size_t)(E * vd.vstride), "edge motions")) != RGG_OK) return st;
    if ((st = read_back(&vdel, vd.delta, (size_t)(E * dv.B), "chord deviations")) != RGG_OK) return st;
    // the second forms, when built
    std::vector<double> obb, seg;
    std::vector<int32_t> sseg32;
    if (dv.mode & kModeObb)
        if ((st = read_back(&obb, dv.obb64, (size_t)(E * dv.nbody * obb_words(dv.D)), "oriented boxes")) != RGG_OK)
            return st;
    if (dv.mode & kModeSplines) {
        if ((st = read_back(&sseg32, dv.sseg, (size_t)(E * dv.B + 1), "spline offsets")) != RGG_OK) return st;
        if ((st = read_back(&seg, dv.seg64, (size_t)sseg32.back() * (2 * dv.D + 1), "spline segments")) != RGG_OK)
            return st;
    }
    std::vector<int64_t> sseg(sseg32.begin(), sseg32.end());
    FileHeader h = {};
    memcpy(h.magic, kMagic, sizeof kMagic);
    h.version = kFileVersion;
    h.D = dv.D;
    h.B = dv.B;
    h.mixed = dv.mixed;
    h.chunk = dv.chunk;
    h.retest_capacity = dv.rc_cap;
    h.E = E;
    h.M = M;
    h.band_rel = dv.band_rel;
    h.one_cell = std::isfinite(rm->info.cell_size) ? 0 : 1;
    h.cell = rm->info.cell_size;
    h.n_samp = n_samp;
    h.n_cap = n_cap;
    FileOut out;
    out.f = fopen(path, "wb");
    if (!out.f) return fail(RGG_E_INVALID_ARG, "cannot open %s for writing", path);
    out.put(&h, sizeof h);
    out.put(soff.data(), sizeof(int64_t) * soff.size());
    out.put(samp.data(), sizeof(double) * samp.size());
    out.put(cap.data(), sizeof(double) * cap.size());
    out.put(rad.data(), sizeof(double) * rad.size());
    out.put(aabb.data(), sizeof(float) * aabb.size());
    out.put(resident.data(), sizeof(rgg_box) * resident.size());
    out.put(cnt.data(), sizeof(int2) * cnt.size());
    out.put(vrob.data(), sizeof(VRobot));
    out.put(vmot.data(), sizeof(double) * vmot.size());
    out.put(vdel.data(), sizeof(double) * vdel.size());
    const int32_t forms[4] = {dv.mode, dv.nbody, dv.pl_cap, dv.inline_rounds};
    out.put(forms, sizeof forms);
    out.put(obb.data(), sizeof(double) * obb.size());
    out.put(sseg.data(), sizeof(int64_t) * sseg.size());
    out.put(seg.data(), sizeof(double) * seg.size());
    const uint64_t sum = out.sum.h;
    out.put(&sum, sizeof sum);
    const bool flushed = out.ok && fflush(out.f) == 0;
    const bool closed = fclose(out.f) == 0;
    out.f = nullptr;
    if (!flushed || !closed) return fail(RGG_E_INVALID_ARG, "writing %s failed", path);
    return RGG_OK;
}

// Reads and checks a roadmap file (host only): everything rgg_load needs
// before it touches the device.
static rgg_status read_roadmap_file(const char *path, LoadedFile *L)
{
    FileHeader &h = L->h;
    HostGeometry &g = L->g;
    std::vector<rgg_box> &resident = L->resident;
    std::vector<int2> &cnt = L->cnt;
    FileIn in;
    in.f = fopen(path, "rb");
    if (!in.f) return fail(RGG_E_INVALID_ARG, "cannot open %s", path);
    in.get(&h, sizeof h);
    if (!in.ok || memcmp(h.magic, kMagic, sizeof kMagic) != 0) return fail(RGG_E_INVALID_ARG, "%s is not a roadmap file", path);
    if (h.version != kFileVersion) return fail(RGG_E_INVALID_ARG, "roadmap file version %u, expected %u", h.version, kFileVersion);
    if ((h.D != 2 && h.D != 3) || h.B < 1 || h.B > kMaxSpheres || h.E < 0 || h.E > INT32_MAX || h.M < 0 ||
        h.M > 4096 || h.chunk < 1 || h.chunk > 512 || h.retest_capacity < 1 ||
        h.retest_capacity > (1 << 20) || !(h.band_rel > 0.0f) || h.n_cap != h.E * (2 * h.D + 1) * h.B || h.n_samp < 0)
        return fail(RGG_E_INVALID_ARG, "%s: inconsistent header", path);
    g.D = h.D;
    g.B = h.B;
    g.E = h.E;
    try {
        g.soff.resize((size_t)(h.E + 1));
        in.get(g.soff.data(), sizeof(int64_t) * g.soff.size());
        if (!in.ok || g.soff[0] != 0 || (int64_t)copy_stride(h.D) * g.soff.back() != h.n_samp)
            return fail(RGG_E_INVALID_ARG, "%s: inconsistent sample offsets", path);
        // each edge holds whole configurations, as many as a build can give
        // (a zero count would leave the copy tests without a stride)
        for (int64_t e = 0; e < h.E; ++e) {
            const int64_t P = g.soff[(size_t)e + 1] - g.soff[(size_t)e];
            if (P < kMinEdgeConfigs * h.B || P > kMaxEdgeConfigs * h.B || P % h.B != 0)
                return fail(RGG_E_INVALID_ARG, "%s: inconsistent sample offsets", path);
        }
        g.samp.resize((size_t)h.n_samp);
        g.cap.resize((size_t)h.n_cap);
        g.radius.resize((size_t)h.B);
        g.aabb.resize((size_t)h.E * kAabbStride);
    } catch (const std::bad_alloc &) {
        return fail(RGG_E_OUT_OF_MEMORY, "host memory for %s", path);
    }
    try {
        resident.resize((size_t)h.M);
        cnt.resize((size_t)h.E);
    } catch (const std::bad_alloc &) {
        return fail(RGG_E_OUT_OF_MEMORY, "host memory for %s", path);
    }
    in.get(g.samp.data(), sizeof(double) * g.samp.size());
    in.get(g.cap.data(), sizeof(double) * g.cap.size());
    in.get(g.radius.data(), sizeof(double) * g.radius.size());
    in.get(g.aabb.data(), sizeof(float) * g.aabb.size());
    in.get(resident.data(), sizeof(rgg_box) * resident.size());
    in.get(cnt.data(), sizeof(int2) * cnt.size());
    VRobot vr;
    in.get(&vr, sizeof vr);
    if (!in.ok) return fail(RGG_E_INVALID_ARG, "%s is truncated", path);
    const int want_dof = vr.kind == RGG_SE2 ? 3 : (vr.kind == RGG_SE3 ? 7 : vr.L);
    bool robot_ok = (vr.kind == RGG_SE2 || vr.kind == RGG_SE3 || vr.kind == RGG_PLANAR_ARM) &&
                    (vr.kind == RGG_SE3 ? 3 : 2) == h.D && vr.B == h.B && vr.dof == want_dof &&
                    (vr.kind != RGG_PLANAR_ARM || (vr.L >= 1 && vr.L <= kMaxLinks));
    for (int i = 0; robot_ok && vr.kind == RGG_PLANAR_ARM && i < vr.B; ++i)
        robot_ok = vr.link[i] >= 0 && vr.link[i] < vr.L;
    if (!robot_ok) return fail(RGG_E_INVALID_ARG, "%s: inconsistent robot", path);
    g.kind = vr.kind;
    g.dof = vr.dof;
    g.L = vr.kind == RGG_PLANAR_ARM ? vr.L : 0;
    const int per = vr.kind == RGG_SE2 ? 2 : (vr.kind == RGG_SE3 ? 3 : 1);
    g.rob_pos.assign(vr.pos, vr.pos + vr.B * per);
    g.rob_link.assign(vr.link, vr.link + vr.B);
    g.rob_len.assign(vr.len, vr.len + g.L);
    g.rob_base[0] = vr.base[0];
    g.rob_base[1] = vr.base[1];
    try {
        g.motion.resize((size_t)(h.E * (2 * vr.dof + 3)));
        g.delta.resize((size_t)(h.E * h.B));
    } catch (const std::bad_alloc &) {
        return fail(RGG_E_OUT_OF_MEMORY, "host memory for %s", path);
    }
    in.get(g.motion.data(), sizeof(double) * g.motion.size());
    in.get(g.delta.data(), sizeof(double) * g.delta.size());
    // the second forms: mode bits and body count, then the boxes and splines
    // and the pair-list capacity and inline rounds of the FP32 mode
    int32_t forms[4] = {0, 0, 0, 0};
    in.get(forms, sizeof forms);
    if (!in.ok) return fail(RGG_E_INVALID_ARG, "%s is truncated", path);
    const int nb = vr.kind == RGG_PLANAR_ARM ? vr.L : 1;
    if ((forms[0] & ~(kModeObb | kModeSplines)) != 0 || forms[1] != nb || forms[2] < 0 ||
        forms[2] > (1 << 20) || (forms[3] != kInlineAll && (forms[3] < 0 || forms[3] > (1 << 20))))
        return fail(RGG_E_INVALID_ARG, "%s: inconsistent approximation forms", path);
    L->pl_cap = forms[2];
    L->inline_rounds = forms[3];
    g.n_bodies = nb;
    g.body.assign((size_t)h.B, 0);
    g.body_has.assign((size_t)nb, 0);
    for (int i = 0; i < h.B; ++i) {
        g.body[i] = vr.kind == RGG_PLANAR_ARM ? vr.link[i] : 0;
        g.body_has[g.body[i]] = 1;
    }
    try {
        if (forms[0] & kModeObb) {
            g.obb.resize((size_t)(h.E * nb * obb_stride(h.D)));
            in.get(g.obb.data(), sizeof(double) * g.obb.size());
        }
        if (forms[0] & kModeSplines) {
            g.sseg.resize((size_t)(h.E * h.B + 1));
            in.get(g.sseg.data(), sizeof(int64_t) * g.sseg.size());
            if (!in.ok) return fail(RGG_E_INVALID_ARG, "%s is truncated", path);
            // each sphere keeps between 0 and n segments (n + 1 configurations)
            bool ok = g.sseg[0] == 0;
            for (int64_t e = 0; ok && e < h.E; ++e) {
                const int64_t n = (g.soff[(size_t)e + 1] - g.soff[(size_t)e]) / h.B - 1;
                for (int i = 0; ok && i < h.B; ++i) {
                    const int64_t k = g.sseg[(size_t)(e * h.B + i + 1)] - g.sseg[(size_t)(e * h.B + i)];
                    ok = k >= 0 && k <= n;
                }
            }
            if (!ok || g.sseg.back() > (int64_t)INT32_MAX)
                return fail(RGG_E_INVALID_ARG, "%s: inconsistent spline offsets", path);
            g.seg.resize((size_t)(g.sseg.back() * (2 * h.D + 1)));
            in.get(g.seg.data(), sizeof(double) * g.seg.size());
        }
    } catch (const std::bad_alloc &) {
        return fail(RGG_E_OUT_OF_MEMORY, "host memory for %s", path);
    }
    const uint64_t want = in.sum.h;
    uint64_t sum = 0;
    if (in.ok) in.get(&sum, sizeof sum);
    if (!in.ok) return fail(RGG_E_INVALID_ARG, "%s is truncated", path);
    if (sum != want) return fail(RGG_E_INVALID_ARG, "%s: checksum mismatch", path);
    return RGG_OK;
}

rgg_status rgg_load(rgg_context *ctx, const char *path, rgg_roadmap **out)
{
    if (!ctx || !path || !out) return fail(RGG_E_INVALID_ARG, "null argument");
    auto t0 = std::chrono::steady_clock::now();
    LoadedFile L;
    rgg_status rs = read_roadmap_file(path, &L);
    if (rs != RGG_OK) return rs;
    const FileHeader &h = L.h;
    const HostGeometry &g = L.g;
    HIP_OR_FAIL(hipSetDevice(ctx->device), "hipSetDevice");
    HostGrid grid;
    std::string err;
    rgg_status st = build_grid(g, h.one_cell ? -1.0 : h.cell, h.chunk, &grid, &err);
    if (st != RGG_OK) return fail(st, "%s", err.c_str());
    const RoadmapParams p = {h.M, h.mixed != 0, (double)h.band_rel, h.retest_capacity, h.chunk, L.pl_cap,
                             L.inline_rounds};
    if ((st = admit_roadmap(device_bytes_needed(g, grid, p), 0)) != RGG_OK) return st;
    rgg_roadmap *rm = nullptr;
    if ((st = make_roadmap(ctx, g, grid, p, L.resident.data(), L.cnt.data(), &rm)) != RGG_OK) return st;
    rm->info.build_seconds = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
    *out = rm;
    return RGG_OK;
}

rgg_status rgg_debug_read_file(const char *path, int64_t *n_edges)
{
    if (!path) return fail(RGG_E_INVALID_ARG, "null argument");
    LoadedFile L;
    rgg_status st = read_roadmap_file(path, &L);
    if (st != RGG_OK) return st;
    if (n_edges) *n_edges = L.h.E;
    return RGG_OK;
}

rgg_status rgg_debug_second_forms(const rgg_roadmap_desc *rd, const rgg_robot *robot,
                                  const rgg_build_opts *opts, int64_t e0, int64_t e1, double *obb,
                                  int64_t *n_segments, double *segments)
{
    std::string err;
    rgg_status st = validate_build_inputs(rd, robot, opts, &err);
    if (st != RGG_OK) return fail(st, "%s", err.c_str());
    if (e0 < 0 || e1 < e0 || e1 > rd->n_edges) return fail(RGG_E_INVALID_ARG, "bad edge range");
    HostGeometry g;
    st = build_geometry(rd, robot, opts, e0, e1, host_threads(opts->host_threads), &g, &err);
    if (st != RGG_OK) return fail(st, "%s", err.c_str());
    if (obb && !g.obb.empty()) memcpy(obb, g.obb.data(), sizeof(double) * g.obb.size());
    if (!g.sseg.empty()) {
        const int64_t n = g.E * g.B;
        if (n_segments)
            for (int64_t k = 0; k < n; ++k) n_segments[k] = g.sseg[k + 1] - g.sseg[k];
        if (segments) memcpy(segments, g.seg.data(), sizeof(double) * g.seg.size());
    }
    return RGG_OK;
}

rgg_status rgg_debug_geometry(const rgg_roadmap_desc *rd, const rgg_robot *robot,
                              const rgg_build_opts *opts, int64_t e0, int64_t e1, int64_t *n_configs,
                              double *centres, double *capsule, float *aabb)
{
    std::string err;
    rgg_status st = validate_build_inputs(rd, robot, opts, &err);
    if (st != RGG_OK) return fail(st, "%s", err.c_str());
    if (e0 < 0 || e1 < e0 || e1 > rd->n_edges || !n_configs) return fail(RGG_E_INVALID_ARG, "bad edge range");
    HostGeometry g;
    st = build_geometry(rd, robot, opts, e0, e1, host_threads(opts->host_threads), &g, &err);
    if (st != RGG_OK) return fail(st, "%s", err.c_str());
    const int D = g.D, B = g.B;
    int64_t row = 0;
    for (int64_t k = 0; k < g.E; ++k) {
        const int64_t P = g.soff[k + 1] - g.soff[k];
        n_configs[k] = P / B;
        if (centres) {
            const int S = copy_stride(D);
            const double *blk = g.samp.data() + S * g.soff[k];
            const int64_t J = P / B;   // block layout [B][J][S] -> rows (j, i)
            for (int64_t j = 0; j < J; ++j)
                for (int i = 0; i < B; ++i)
                    for (int d = 0; d < D; ++d)
                        centres[(row + j * B + i) * D + d] = blk[(i * J + j) * S + d];
        }
        row += P;
        if (capsule) {
            const double *cp = g.cap.data() + k * (2 * D + 1) * B;
            for (int i = 0; i < B; ++i)
                for (int f = 0; f < 2 * D + 1; ++f) capsule[(k * B + i) * (2 * D + 1) + f] = cp[f * B + i];
        }
        if (aabb)
            for (int d = 0; d < 3; ++d) {
                aabb[k * 6 + d] = g.aabb[k * kAabbStride + d];
                aabb[k * 6 + 3 + d] = g.aabb[k * kAabbStride + 4 + d];
            }
    }
    return RGG_OK;
}

}  // extern "C"
