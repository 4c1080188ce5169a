// C ABI of librgg (declared in include/rgg.h).
#include <hip/hip_runtime.h>
#include <math.h>
#include <stdarg.h>
#include <stdio.h>
#include <string.h>

#include <algorithm>
#include <array>
#include <chrono>
#include <map>
#include <memory>
#include <string>
#include <thread>
#include <vector>

#include "rgg.h"
#include "rgg_device.h"
#include "rgg_internal.h"
#include "api_internal.h"

static_assert(rgg::kLocalGridCells == rgg::kLocalCells, "pruning-grid size of host and device");
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

constexpr int32_t kChunk = 256;   // edges per grid work item

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
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    std::vector<BatchGroup> groups;
    bool any_grid = false;
    int tiles = 0, wtiles = 0;

    ~rgg_batch()
    {
        hipSetDevice(device);
        for (int k = 0; k < kRing; ++k)
            if (done[k] && used[k]) hipEventSynchronize(done[k]);
        // the roadmaps' last updates have completed: nothing left to wait for
        for (rgg_roadmap *rm : rms)
            for (int k = 0; k < kRing; ++k)
                if (rm->wait_ev == done[k]) rm->wait_ev = nullptr;
        for (int k = 0; k < kRing; ++k) {
            if (done[k]) hipEventDestroy(done[k]);
            if (h_tab[k]) hipHostFree(h_tab[k]);
        }
        if (exec) hipGraphExecDestroy(exec);
        if (graph) hipGraphDestroy(graph);
        if (d_tab) hipFree(d_tab);
        if (d_grp) hipFree(d_grp);
    }
};

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
    *out = new rgg_context{device};
    return RGG_OK;
}

void rgg_context_destroy(rgg_context *ctx) { delete ctx; }

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
    HostGrid grid;
    st = build_grid(g, opts->cell_size, kChunk, &grid, &err);
    if (st != RGG_OK) return fail(st, "%s", err.c_str());

    auto *rm = new rgg_roadmap();
    rm->ctx = ctx;
    rm->device = ctx->device;
    const int64_t E = g.E, M = opts->n_obstacle_slots;
    const int D = g.D, B = g.B;
    const bool mixed = opts->precision == RGG_PREC_FP32_RECHECK;
    RmDev &dv = rm->dv;
    dv.D = D;
    dv.B = B;
    dv.mixed = mixed ? 1 : 0;
    dv.chunk = kChunk;
    dv.E = E;
    dv.M = M;
    dv.band_rel = (float)(opts->band_rel > 0.0 ? opts->band_rel : 1e-5);
    if (std::isinf(opts->band_rel)) dv.band_rel = INFINITY;
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
    // grid
    for (int d = 0; d < 3; ++d) {
        dv.gdim[d] = grid.dim[d];
        dv.gorg[d] = grid.org[d];
    }
    dv.ginv = grid.inv;
    for (int d = 0; d < 3; ++d) {
        dv.lg_org[d] = grid.lg_org[d];
        dv.lg_dim[d] = grid.lg_dim[d];
    }
    dv.lg_inv = grid.lg_inv;
    dv.ncells = (int64_t)grid.dim[0] * grid.dim[1] * grid.dim[2];
    dv.items_cap = grid.items_cap;
    int32_t *cstart, *cedges;
    if ((st = rm->upload(&cstart, grid.start.data(), grid.start.size(), "grid starts")) != RGG_OK) return guard(st);
    if ((st = rm->upload(&cedges, grid.edges.data(), grid.edges.size(), "grid lists")) != RGG_OK) return guard(st);
    dv.cell_start = cstart;
    dv.cell_edges = cedges;
    // state and scratch
    std::vector<rgg_box> absent((size_t)M);
    for (auto &b : absent)
        for (int k = 0; k < 3; ++k) {
            b.lo[k] = 1.0;
            b.hi[k] = -1.0;
        }
    const size_t ncw = (size_t)((dv.ncells + 31) / 32);
    if ((st = rm->alloc(&dv.cnt, (size_t)E, "counters")) != RGG_OK) return guard(st);
    if ((st = rm->alloc(&dv.cell_bits, ncw, "cell marks")) != RGG_OK) return guard(st);
    if ((st = rm->upload(&dv.resident, absent.data(), (size_t)M, "obstacle slots")) != RGG_OK) return guard(st);
    if ((st = rm->alloc(&dv.chg, (size_t)(2 * M), "changed entries")) != RGG_OK) return guard(st);
    dv.rc_cap = opts->retest_capacity > 0 ? opts->retest_capacity : kRcCap;
    dv.df_cap = (int32_t)((grid.items_cap + kStatBlocks - 1) / kStatBlocks);
    if ((st = rm->alloc(&dv.rc, (size_t)kStatBlocks * dv.rc_cap, "re-test regions")) != RGG_OK) return guard(st);
    if ((st = rm->alloc(&dv.rc_cnt, (size_t)kStatBlocks, "re-test counts")) != RGG_OK) return guard(st);
    if ((st = rm->alloc(&dv.df, (size_t)kStatBlocks * dv.df_cap, "deferred items")) != RGG_OK) return guard(st);
    if ((st = rm->alloc(&dv.df_cnt, (size_t)kStatBlocks, "deferred counts")) != RGG_OK) return guard(st);
    if (dv.ncells == 1) {
        // the one cell's work items never change: (0, chunk) for every chunk
        std::vector<int2> items((size_t)grid.items_cap);
        for (int64_t h = 0; h < grid.items_cap; ++h) items[(size_t)h] = make_int2(0, (int32_t)h);
        if ((st = rm->upload(&dv.items, items.data(), items.size(), "grid items")) != RGG_OK) return guard(st);
    } else if ((st = rm->alloc(&dv.items, (size_t)grid.items_cap, "grid items")) != RGG_OK) {
        return guard(st);
    }
    if ((st = rm->alloc(&dv.blk_stats, (size_t)kStatBlocks * kStats, "statistics")) != RGG_OK) return guard(st);
    if ((st = rm->alloc(&dv.tile_cnt, (size_t)dv.ntiles + 1, "tile counts")) != RGG_OK) return guard(st);
    if ((st = rm->alloc(&dv.ctl, 1, "control block")) != RGG_OK) return guard(st);
    if ((st = rm->alloc(&rm->d_stage, (size_t)(2 * M), "box staging")) != RGG_OK) return guard(st);
    if ((st = rm->alloc(&rm->d_res, 1, "result")) != RGG_OK) return guard(st);
    if ((st = rm->alloc(&rm->d_labels, (size_t)E, "labels")) != RGG_OK) return guard(st);
    if ((st = rm->alloc(&rm->d_gray, (size_t)E, "gray list")) != RGG_OK) return guard(st);
    HIP_OR_FAIL(hipMemset(dv.cnt, 0, sizeof(int2) * std::max<int64_t>(E, 1)), "clear counters");
    HIP_OR_FAIL(hipMemset(dv.cell_bits, 0, 4 * std::max<size_t>(ncw, 1)), "clear marks");
    HIP_OR_FAIL(hipMemset(dv.ctl, 0, sizeof(Ctl)), "clear control");
    HIP_OR_FAIL(hipMemset(dv.rc_cnt, 0, sizeof(int32_t) * kStatBlocks), "clear re-test counts");
    HIP_OR_FAIL(hipMemset(dv.df_cnt, 0, sizeof(int32_t) * kStatBlocks), "clear deferred counts");
    HIP_OR_FAIL(hipMemset(dv.blk_stats, 0, sizeof(unsigned long long) * kStatBlocks * kStats), "clear statistics");
    HIP_OR_FAIL(hipMemset(rm->d_labels, 0, std::max<int64_t>(E, 1)), "clear labels");
    HIP_OR_FAIL(hipHostMalloc((void **)&rm->h_stage, sizeof(rgg_box) * std::max<int64_t>(2 * M, 1)), "pinned staging");
    HIP_OR_FAIL(hipHostMalloc((void **)&rm->h_res, sizeof(rgg_update_result)), "pinned result");
    HIP_OR_FAIL(hipStreamCreateWithFlags(&rm->stream, hipStreamNonBlocking), "stream");
    HIP_OR_FAIL(hipEventCreateWithFlags(&rm->done, hipEventDisableTiming), "event");
    HIP_OR_FAIL(hipDeviceSynchronize(), "build upload");

    rgg_roadmap_info &in = rm->info;
    in.n_edges = E;
    in.n_slots = M;
    in.dim = D;
    in.n_spheres = B;
    in.n_sphere_samples = g.soff.back();
    for (int d = 0; d < 3; ++d) in.grid_cells[d] = grid.dim[d];
    in.cell_size = grid.cell;
    in.grid_entries = (int64_t)grid.edges.size();
    in.build_seconds = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
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
        if (rms[k]->dv.chunk != kChunk) return fail(RGG_E_INVALID_ARG, "roadmap %d has an unexpected chunk", k);
    }
    HIP_OR_FAIL(hipSetDevice(ctx->device), "hipSetDevice");
    std::unique_ptr<rgg_batch> b(new rgg_batch());
    b->device = ctx->device;
    b->n = n;
    b->rms.assign(rms, rms + n);
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
    HIP_OR_FAIL(hipGraphCreate(&b->graph, 0), "hipGraphCreate");
    hipGraphNode_t last = nullptr;
    HIP_OR_FAIL(add_batch_nodes(b->graph, b->d_tab, b->d_grp, n, groups.data(), (int)groups.size(), b->any_grid,
                                b->tiles, b->wtiles, nullptr, &last),
                "hipGraphAddKernelNode");
    HIP_OR_FAIL(hipGraphInstantiate(&b->exec, b->graph, nullptr, nullptr, 0), "hipGraphInstantiate");
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
    HIP_OR_FAIL(hipMemcpyAsync(b->d_tab, h, sizeof(BatchReq) * b->n, hipMemcpyHostToDevice, s), "copy batch table");
    if (graph)
        HIP_OR_FAIL(hipGraphLaunch(b->exec, s), "hipGraphLaunch");
    else
        HIP_OR_FAIL(launch_batch(s, b->d_tab, b->d_grp, b->n, b->groups.data(), (int)b->groups.size(), b->any_grid,
                                 b->tiles, b->wtiles),
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
