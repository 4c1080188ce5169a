// Request server of librgg: continuous batching of roadmap updates.
//
// Submitters queue requests (the obstacle boxes are copied at once).  One
// worker thread owns every HIP call of the server:
//   * it completes finished batches (an event per stream slot), releasing
//     their pool space and publishing each request's result and latency;
//   * while a stream slot is free it forms the next batch from the queue in
//     submission order: at most one request per roadmap, a request only when
//     its boxes fit the free pool space, and never a request of a roadmap
//     whose earlier request is still queued;
//   * it stages the boxes (pinned host -> device pool), the request table,
//     launches the batch's stage kernels and copies the results back.
// Requests of one roadmap in different batches are ordered on the device by
// the roadmap's last-update event, so a new batch may start while earlier
// ones still run.
#include <hip/hip_runtime.h>
#include <string.h>

#include <algorithm>
#include <chrono>
#include <condition_variable>
#include <deque>
#include <map>
#include <mutex>
#include <thread>
#include <unordered_map>
#include <vector>

#include "api_internal.h"

using namespace rgg;

namespace {

using Clock = std::chrono::steady_clock;

constexpr int64_t kAlign = 256;

int64_t round_up(int64_t x) { return (x + kAlign - 1) / kAlign * kAlign; }

// First-fit allocator over [0, size) of the device pool.
struct PoolMap {
    std::map<int64_t, int64_t> free_;   // offset -> length
    explicit PoolMap(int64_t size) { free_[0] = size; }
    int64_t take(int64_t n)
    {
        for (auto it = free_.begin(); it != free_.end(); ++it) {
            if (it->second < n) continue;
            const int64_t off = it->first, len = it->second;
            free_.erase(it);
            if (len > n) free_[off + n] = len - n;
            return off;
        }
        return -1;
    }
    void give(int64_t off, int64_t n)
    {
        auto it = free_.emplace(off, n).first;
        auto nx = std::next(it);
        if (nx != free_.end() && it->first + it->second == nx->first) {
            it->second += nx->second;
            free_.erase(nx);
        }
        if (it != free_.begin()) {
            auto pv = std::prev(it);
            if (pv->first + pv->second == it->first) {
                pv->second += it->second;
                free_.erase(it);
            }
        }
    }
};

struct Pending {
    uint64_t ticket;
    rgg_roadmap *rm;
    std::vector<rgg_box> boxes;   // old then new, 2m
    uint8_t *d_labels;
    int64_t *d_gray;
    int64_t gray_cap;
    bool validate;
    uint8_t *d_verdict;
    Clock::time_point submitted;
    Clock::time_point launched;   // its batch was queued on the device
    int64_t bytes;                // pool bytes
};

struct Ticket {
    int state = 0;                // 0 queued, 1 running, 2 done
    rgg_update_result res = {};
    rgg_request_timing timing = {};
};

struct Slot {
    hipStream_t s = nullptr;
    hipEvent_t ev = nullptr;
    bool busy = false;
    BatchReq *d_tab = nullptr, *h_tab = nullptr;
    int32_t *d_grp = nullptr;
    rgg_update_result *d_res = nullptr, *h_res = nullptr;
    std::vector<Pending> reqs;    // in table-row order
    std::vector<int64_t> offs;    // pool offset of each request
};

}  // namespace

struct rgg_server {
    int device = 0;
    rgg_server_opts opts = {};
    char *d_pool = nullptr;
    char *h_pool = nullptr;       // pinned mirror of the pool
    PoolMap pool{0};
    std::vector<Slot> slots;

    std::mutex mu;
    std::condition_variable cv_work, cv_done;
    std::deque<Pending> queue;
    std::unordered_map<uint64_t, Ticket> tickets;
    uint64_t next_ticket = 1;
    bool stopping = false;
    bool closed = false;          // rgg_server_stop has joined the worker
    int pollers = 0;              // threads waiting in rgg_server_poll
    int64_t free_at_start = 0;    // free device bytes when the server started
    std::string worker_error;
    std::thread worker;
    std::vector<rgg_roadmap *> seen;   // roadmaps this server has updated (worker only)
    std::vector<rgg_roadmap *> held;   // roadmaps named by a submitted request (under mu)

    void run();
    bool dispatch(Slot &slot, std::vector<Pending> &batch);
    void complete(Slot &slot);
    void fail_worker(const char *msg);
};

namespace {

void free_server(rgg_server *srv)
{
    hipSetDevice(srv->device);
    for (Slot &sl : srv->slots) {
        if (sl.s) hipStreamSynchronize(sl.s);
        if (sl.ev) hipEventDestroy(sl.ev);
        if (sl.s) hipStreamDestroy(sl.s);
        if (sl.d_tab) hipFree(sl.d_tab);
        if (sl.d_grp) hipFree(sl.d_grp);
        if (sl.d_res) hipFree(sl.d_res);
        if (sl.h_tab) hipHostFree(sl.h_tab);
        if (sl.h_res) hipHostFree(sl.h_res);
    }
    if (srv->d_pool) hipFree(srv->d_pool);
    if (srv->h_pool) hipHostFree(srv->h_pool);
    delete srv;
}

}  // namespace

// Launches one batch on `slot`.  The requests come grouped by kernel variant
// (dimension, precision), their pool offsets in slot.offs.
bool rgg_server::dispatch(Slot &slot, std::vector<Pending> &batch)
{
    std::vector<BatchGroup> groups;
    bool any_grid = false;
    int tiles = 0, wtiles = 0;
    const int n = (int)batch.size();
    for (int r = 0; r < n; ++r) {
        const RmDev &dv = batch[r].rm->dv;
        if (groups.empty() || groups.back().D != dv.D || groups.back().mixed != dv.mixed)
            groups.push_back({dv.D, dv.mixed, r, 0});
        ++groups.back().count;
        any_grid = any_grid || dv.ncells > 1;
        BatchReq &t = slot.h_tab[r];
        const int64_t off = slot.offs[r];
        const int64_t M = dv.M;
        memcpy(h_pool + off, batch[r].boxes.data(), sizeof(rgg_box) * 2 * M);
        const rgg_box *d_old = reinterpret_cast<const rgg_box *>(d_pool + off);
        t.rm = dv;
        t.a = {d_old, d_old + M, batch[r].d_labels, batch[r].d_gray, batch[r].d_gray ? batch[r].gray_cap : 0,
               slot.d_res + r};
        t.tile0 = tiles;
        t.wtile0 = wtiles;
        tiles += dv.ntiles;
        wtiles += dv.ntiles + 1;
    }
    hipStream_t s = slot.s;
    const Clock::time_point launched = Clock::now();
    for (int r = 0; r < n; ++r) {
        batch[r].launched = launched;
        if (order_after_previous(batch[r].rm, s) != RGG_OK) return false;
        const int64_t M = batch[r].rm->dv.M;
        if (M > 0 && hipMemcpyAsync(d_pool + slot.offs[r], h_pool + slot.offs[r], sizeof(rgg_box) * 2 * M,
                                    hipMemcpyHostToDevice, s) != hipSuccess)
            return false;
    }
    // the batch's first kernel copies the slot's pinned table
    if (launch_batch(s, slot.d_tab, slot.h_tab, slot.d_grp, n, groups.data(), (int)groups.size(), any_grid, tiles,
                     wtiles) != hipSuccess)
        return false;
    // non-lazy requests: validate each gray list after the batch, on the
    // same stream, capped by the request's own result
    for (int r = 0; r < n; ++r) {
        const Pending &q = batch[r];
        if (!q.validate || q.gray_cap == 0) continue;
        if (launch_validate(q.rm->val, q.d_gray, q.gray_cap, slot.d_res + r, RGG_VALIDATE_DEFAULT_LEVELS,
                            RGG_VALIDATE_DEFAULT_ACTIVE, q.d_verdict, nullptr, nullptr, q.d_labels, s) != hipSuccess)
            return false;
    }
    if (hipMemcpyAsync(slot.h_res, slot.d_res, sizeof(rgg_update_result) * n, hipMemcpyDeviceToHost, s) != hipSuccess)
        return false;
    if (hipEventRecord(slot.ev, s) != hipSuccess) return false;
    for (int r = 0; r < n; ++r) {
        batch[r].rm->wait_ev = slot.ev;
        batch[r].rm->last_stream = s;
        if (std::find(seen.begin(), seen.end(), batch[r].rm) == seen.end()) seen.push_back(batch[r].rm);
    }
    slot.reqs = std::move(batch);
    slot.busy = true;
    return true;
}

void rgg_server::complete(Slot &slot)
{
    const Clock::time_point now = Clock::now();
    std::lock_guard<std::mutex> lk(mu);
    for (size_t r = 0; r < slot.reqs.size(); ++r) {
        const Pending &q = slot.reqs[r];
        Ticket &t = tickets[q.ticket];
        t.res = slot.h_res[r];
        t.timing.latency_us = std::chrono::duration<double, std::micro>(now - q.submitted).count();
        t.timing.queue_us = std::chrono::duration<double, std::micro>(q.launched - q.submitted).count();
        t.timing.service_us = std::chrono::duration<double, std::micro>(now - q.launched).count();
        t.timing.batch_size = (int32_t)slot.reqs.size();
        t.state = 2;
        pool.give(slot.offs[r], slot.reqs[r].bytes);
    }
    slot.reqs.clear();
    slot.offs.clear();
    slot.busy = false;
    cv_done.notify_all();
}

// Records a worker error and wakes every waiting poller: their tickets will
// not complete, and rgg_server_poll reports the error instead.
void rgg_server::fail_worker(const char *msg)
{
    {
        std::lock_guard<std::mutex> lk(mu);
        worker_error = msg;
        stopping = true;
    }
    cv_done.notify_all();
}

void rgg_server::run()
{
    hipSetDevice(device);
    const int max_batch = opts.max_batch;
    for (;;) {
        // completions
        bool any_busy = false;
        for (Slot &sl : slots) {
            if (!sl.busy) continue;
            const hipError_t q = hipEventQuery(sl.ev);
            if (q == hipSuccess) {
                complete(sl);
            } else if (q != hipErrorNotReady) {
                fail_worker(hipGetErrorString(q));
                return;
            } else {
                any_busy = true;
            }
        }
        // next batch, while a slot is free
        Slot *free_slot = nullptr;
        for (Slot &sl : slots)
            if (!sl.busy) {
                free_slot = &sl;
                break;
            }
        std::vector<Pending> batch;
        {
            std::unique_lock<std::mutex> lk(mu);
            if (!worker_error.empty()) return;
            if (free_slot && !queue.empty()) {
                std::vector<rgg_roadmap *> taken, blocked;
                auto has = [](const std::vector<rgg_roadmap *> &v, rgg_roadmap *r) {
                    return std::find(v.begin(), v.end(), r) != v.end();
                };
                for (auto it = queue.begin(); it != queue.end() && (int)batch.size() < max_batch;) {
                    rgg_roadmap *rm = it->rm;
                    if (has(taken, rm) || has(blocked, rm)) {
                        blocked.push_back(rm);   // keeps this roadmap's order
                        ++it;
                        continue;
                    }
                    const int64_t off = pool.take(it->bytes);
                    if (off < 0) {
                        blocked.push_back(rm);
                        ++it;
                        continue;
                    }
                    free_slot->offs.push_back(off);
                    tickets[it->ticket].state = 1;
                    taken.push_back(rm);
                    batch.push_back(std::move(*it));
                    it = queue.erase(it);
                }
            }
            if (batch.empty()) {
                if (stopping && queue.empty() && !any_busy) return;
                if (!any_busy) {
                    // idle: sleep until a request arrives (or stop)
                    cv_work.wait(lk, [&] { return stopping || !queue.empty(); });
                    continue;
                }
            }
        }
        if (!batch.empty()) {
            // pool offsets were recorded in take order; dispatch sorts the rows,
            // so carry each offset with its request
            std::vector<std::pair<Pending, int64_t>> rows;
            for (size_t r = 0; r < batch.size(); ++r) rows.emplace_back(std::move(batch[r]), free_slot->offs[r]);
            std::stable_sort(rows.begin(), rows.end(), [](const auto &a, const auto &b) {
                const int ka = a.first.rm->dv.D * 2 + a.first.rm->dv.mixed;
                const int kb = b.first.rm->dv.D * 2 + b.first.rm->dv.mixed;
                return ka < kb;
            });
            batch.clear();
            free_slot->offs.clear();
            for (auto &pr : rows) {
                batch.push_back(std::move(pr.first));
                free_slot->offs.push_back(pr.second);
            }
            if (!dispatch(*free_slot, batch)) {
                fail_worker("batch launch failed");
                return;
            }
        } else {
            std::this_thread::yield();   // batches in flight: poll again
        }
    }
}

extern "C" {

rgg_status rgg_server_start(rgg_context *ctx, const rgg_server_opts *opts_in, rgg_server **out)
{
    if (!ctx || !out) return fail(RGG_E_INVALID_ARG, "null argument");
    rgg_server_opts o = opts_in ? *opts_in : rgg_server_opts{};
    if (o.reserved != 0) return fail(RGG_E_INVALID_ARG, "reserved must be 0");
    if (o.n_streams == 0) o.n_streams = 4;
    if (o.max_queue == 0) o.max_queue = 4096;
    if (o.max_batch == 0) o.max_batch = 64;
    HIP_OR_FAIL(hipSetDevice(ctx->device), "hipSetDevice");
    size_t free_b = 0, total_b = 0;
    HIP_OR_FAIL(hipMemGetInfo(&free_b, &total_b), "hipMemGetInfo");
    if (o.pool_bytes == 0) {
        // admission by free device memory: the staging pool that bounds the
        // requests in flight takes 1/64 of what is free now, within
        // [16 MiB, 256 MiB] (256 MiB holds 5,000 requests of 1,000 boxes)
        o.pool_bytes = std::min<int64_t>(std::max<int64_t>((int64_t)(free_b / 64), 16ll << 20), 256ll << 20);
    }
    if (o.pool_bytes > (int64_t)free_b)
        return fail(RGG_E_OUT_OF_MEMORY, "pool of %lld bytes exceeds the %zu bytes of free device memory",
                    (long long)o.pool_bytes, free_b);
    if (o.n_streams < 1 || o.n_streams > 16) return fail(RGG_E_INVALID_ARG, "n_streams must be 1..16");
    if (o.max_queue < 1) return fail(RGG_E_INVALID_ARG, "max_queue must be positive");
    if (o.max_batch < 1 || o.max_batch > kMaxBatch) return fail(RGG_E_INVALID_ARG, "max_batch must be 1..%d", kMaxBatch);
    if (o.pool_bytes < kAlign) return fail(RGG_E_INVALID_ARG, "pool_bytes too small");
    rgg_server *srv = new rgg_server();
    srv->device = ctx->device;
    srv->opts = o;
    srv->free_at_start = (int64_t)free_b;
    srv->pool = PoolMap(round_up(o.pool_bytes));
    auto bail = [&](hipError_t e, const char *what) {
        free_server(srv);
        return hip_fail(e, what);
    };
    hipError_t e;
    if ((e = hipMalloc(&srv->d_pool, round_up(o.pool_bytes))) != hipSuccess) return bail(e, "server pool");
    if ((e = hipHostMalloc((void **)&srv->h_pool, round_up(o.pool_bytes), hipHostMallocDefault)) != hipSuccess)
        return bail(e, "server pinned pool");
    std::vector<int32_t> ident(kMaxBatch);
    for (int k = 0; k < kMaxBatch; ++k) ident[k] = k;   // rows are grouped: group lists are row ranges
    srv->slots.resize(o.n_streams);
    for (Slot &sl : srv->slots) {
        if ((e = hipStreamCreateWithFlags(&sl.s, hipStreamNonBlocking)) != hipSuccess) return bail(e, "server stream");
        if ((e = hipEventCreateWithFlags(&sl.ev, hipEventDisableTiming)) != hipSuccess) return bail(e, "server event");
        if ((e = hipMalloc(&sl.d_tab, sizeof(BatchReq) * kMaxBatch)) != hipSuccess) return bail(e, "server table");
        if ((e = hipMalloc(&sl.d_grp, sizeof(int32_t) * kMaxBatch)) != hipSuccess) return bail(e, "server groups");
        if ((e = hipMalloc(&sl.d_res, sizeof(rgg_update_result) * kMaxBatch)) != hipSuccess) return bail(e, "server results");
        if ((e = hipHostMalloc((void **)&sl.h_tab, sizeof(BatchReq) * kMaxBatch, hipHostMallocDefault)) != hipSuccess)
            return bail(e, "server pinned table");
        if ((e = hipHostMalloc((void **)&sl.h_res, sizeof(rgg_update_result) * kMaxBatch, hipHostMallocDefault)) !=
            hipSuccess)
            return bail(e, "server pinned results");
        if ((e = hipMemcpy(sl.d_grp, ident.data(), sizeof(int32_t) * kMaxBatch, hipMemcpyHostToDevice)) != hipSuccess)
            return bail(e, "server groups");
    }
    srv->worker = std::thread([srv] { srv->run(); });
    *out = srv;
    return RGG_OK;
}

rgg_status rgg_server_submit(rgg_server *srv, const rgg_server_req *req, uint64_t *ticket)
{
    if (!srv || !req || !ticket) return fail(RGG_E_INVALID_ARG, "null argument");
    rgg_roadmap *rm = req->rm;
    if (!rm) return fail(RGG_E_INVALID_ARG, "null roadmap");
    if (rm->device != srv->device) return fail(RGG_E_INVALID_ARG, "roadmap on another device");
    if (rm->dv.mode != 0)
        return fail(RGG_E_UNSUPPORTED, "the server batches roadmaps of the capsule and copy forms only");
    const int64_t M = rm->dv.M;
    if (req->m != M) return fail(RGG_E_INVALID_ARG, "m = %lld but the roadmap has %lld slots", (long long)req->m, (long long)M);
    if (M > 0 && (!req->old_boxes || !req->new_boxes)) return fail(RGG_E_INVALID_ARG, "null box arrays");
    if (req->gray_cap < 0) return fail(RGG_E_INVALID_ARG, "negative gray_cap");
    const int64_t bytes = round_up(std::max<int64_t>(1, (int64_t)sizeof(rgg_box) * 2 * M));
    if (bytes > round_up(srv->opts.pool_bytes))
        return fail(RGG_E_INVALID_ARG, "the request's boxes (%lld bytes) never fit the pool", (long long)bytes);
    Pending p;
    p.rm = rm;
    p.boxes.resize((size_t)(2 * M));
    if (M > 0) {
        memcpy(p.boxes.data(), req->old_boxes, sizeof(rgg_box) * M);
        memcpy(p.boxes.data() + M, req->new_boxes, sizeof(rgg_box) * M);
    }
    if (req->validate && (!req->d_labels || !req->d_gray))
        return fail(RGG_E_INVALID_ARG, "a validated request needs d_labels and d_gray");
    p.d_labels = req->d_labels;
    p.d_gray = req->d_gray;
    p.gray_cap = req->gray_cap;
    p.validate = req->validate != 0;
    p.d_verdict = req->d_verdict;
    p.bytes = bytes;
    {
        std::lock_guard<std::mutex> lk(srv->mu);
        if (!srv->worker_error.empty()) return fail(RGG_E_DEVICE, "server stopped: %s", srv->worker_error.c_str());
        if (srv->stopping) return fail(RGG_E_INVALID_ARG, "server is stopping");
        if ((int64_t)srv->queue.size() >= srv->opts.max_queue) return fail(RGG_E_BUSY, "server queue is full");
        if (std::find(srv->held.begin(), srv->held.end(), rm) == srv->held.end()) {
            srv->held.push_back(rm);
            rm->holders++;   // until rgg_server_stop
        }
        p.ticket = srv->next_ticket++;
        p.submitted = Clock::now();
        srv->tickets[p.ticket] = Ticket();
        *ticket = p.ticket;
        srv->queue.push_back(std::move(p));
    }
    srv->cv_work.notify_one();
    return RGG_OK;
}

rgg_status rgg_server_poll_timing(rgg_server *srv, uint64_t ticket, int32_t wait, int32_t *done,
                                  rgg_update_result *result, rgg_request_timing *timing)
{
    if (!srv || !done) return fail(RGG_E_INVALID_ARG, "null argument");
    std::unique_lock<std::mutex> lk(srv->mu);
    auto it = srv->tickets.find(ticket);
    if (it == srv->tickets.end()) return fail(RGG_E_INVALID_ARG, "unknown ticket %llu", (unsigned long long)ticket);
    if (wait) {
        srv->pollers++;
        srv->cv_done.wait(lk, [&] {
            auto t = srv->tickets.find(ticket);
            return t == srv->tickets.end() || t->second.state == 2 || !srv->worker_error.empty() || srv->closed;
        });
        if (--srv->pollers == 0 && srv->closed) srv->cv_done.notify_all();
    }
    it = srv->tickets.find(ticket);
    if (it == srv->tickets.end()) return fail(RGG_E_INVALID_ARG, "ticket %llu was released", (unsigned long long)ticket);
    if (it->second.state != 2) {
        if (!srv->worker_error.empty()) return fail(RGG_E_DEVICE, "server stopped: %s", srv->worker_error.c_str());
        if (srv->closed) return fail(RGG_E_INVALID_ARG, "server is stopping");
        *done = 0;
        return RGG_OK;
    }
    *done = 1;
    if (result) *result = it->second.res;
    if (timing) *timing = it->second.timing;
    srv->tickets.erase(it);
    return RGG_OK;
}

rgg_status rgg_server_poll(rgg_server *srv, uint64_t ticket, int32_t wait, int32_t *done,
                           rgg_update_result *result, double *latency_us)
{
    rgg_request_timing t = {};
    rgg_status st = rgg_server_poll_timing(srv, ticket, wait, done, result, &t);
    if (st == RGG_OK && *done && latency_us) *latency_us = t.latency_us;
    return st;
}

rgg_status rgg_server_info(rgg_server *srv, rgg_server_opts *opts, int64_t *free_at_start)
{
    if (!srv) return fail(RGG_E_INVALID_ARG, "null server");
    if (opts) *opts = srv->opts;
    if (free_at_start) *free_at_start = srv->free_at_start;
    return RGG_OK;
}

rgg_status rgg_server_stop(rgg_server *srv)
{
    if (!srv) return fail(RGG_E_INVALID_ARG, "null server");
    {
        std::lock_guard<std::mutex> lk(srv->mu);
        srv->stopping = true;
    }
    srv->cv_work.notify_all();
    if (srv->worker.joinable()) srv->worker.join();
    {
        // wake every poller still waiting (their tickets cannot complete after
        // a worker error) and free nothing until the last one has left
        std::unique_lock<std::mutex> lk(srv->mu);
        srv->closed = true;
        srv->cv_done.notify_all();
        srv->cv_done.wait(lk, [&] { return srv->pollers == 0; });
    }
    const std::string err = srv->worker_error;
    hipSetDevice(srv->device);
    for (Slot &sl : srv->slots)
        if (sl.s) hipStreamSynchronize(sl.s);
    // the roadmaps' last updates have completed: their events are the
    // server's, which are about to go
    for (rgg_roadmap *rm : srv->seen)
        for (Slot &sl : srv->slots)
            if (rm->wait_ev == sl.ev) rm->wait_ev = nullptr;
    for (rgg_roadmap *rm : srv->held) rm->holders--;
    free_server(srv);
    if (!err.empty()) return fail(RGG_E_DEVICE, "server worker: %s", err.c_str());
    return RGG_OK;
}

}  // extern "C"
