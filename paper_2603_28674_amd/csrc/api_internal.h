// Host-side objects of librgg shared by the C ABI (api.cpp) and the request
// server (server.cpp).  Internal to the library.
#pragma once

#include <hip/hip_runtime.h>

#include <algorithm>
#include <array>
#include <atomic>
#include <string>
#include <vector>

#include "rgg.h"
#include "rgg_device.h"

namespace rgg {

// Sets the thread's last-error message and returns `st`.
rgg_status fail(rgg_status st, const char *fmt, ...);
rgg_status hip_fail(hipError_t e, const char *what);

#define HIP_OR_FAIL(call, what)                                   \
    do {                                                          \
        hipError_t e__ = (call);                                  \
        if (e__ != hipSuccess) return rgg::hip_fail(e__, what);   \
    } while (0)

}  // namespace rgg

using rgg::fail;
using rgg::hip_fail;

struct rgg_context {
    int device;
    // device address of the library's fixed batch scratch on `device`
    // (rgg_update_batch_noalloc), looked up once when the context opens
    void *batch_scratch = nullptr;
};

struct rgg_roadmap {
    rgg_context *ctx = nullptr;
    int device = 0;
    rgg::RmDev dv = {};
    rgg_roadmap_info info = {};
    std::vector<std::pair<void *, size_t>> allocs;   // device buffers and their sizes
    // graphs, batches and server requests that hold the roadmap's device
    // arrays; its grid is not rebuilt while any do
    std::atomic<int> holders{0};
    hipStream_t stream = nullptr;     // for host-buffer calls
    hipEvent_t done = nullptr;        // end of the most recent single update
    hipEvent_t wait_ev = nullptr;     // event marking the end of the most recent update
                                      // (done, or a batch's event); null = none pending
    hipStream_t last_stream = nullptr;
    // staging for host-buffer updates
    rgg_box *h_stage = nullptr;       // pinned [2M]
    rgg_box *d_stage = nullptr;       // [2M]
    rgg_update_result *h_res = nullptr;   // pinned
    rgg_update_result *d_res = nullptr;
    uint8_t *d_labels = nullptr;      // [E]
    int64_t *d_gray = nullptr;        // [E]
    // full validation: robot, per-edge motions and chord-deviation bounds
    rgg::ValDev val = {};
    // timing
    bool timing = false;
    std::vector<std::array<hipEvent_t, 7>> pool, pending;
    double ms_acc[6] = {0, 0, 0, 0, 0, 0};
    int64_t timed = 0;

    ~rgg_roadmap()
    {
        if (device >= 0) hipSetDevice(device);
        if (wait_ev) hipEventSynchronize(wait_ev);   // the last update, on any stream
        if (stream) hipStreamSynchronize(stream);
        for (auto &set : pool)
            for (auto ev : set) hipEventDestroy(ev);
        for (auto &set : pending)
            for (auto ev : set) hipEventDestroy(ev);
        for (auto &a : allocs) hipFree(a.first);
        if (h_stage) hipHostFree(h_stage);
        if (h_res) hipHostFree(h_res);
        if (done) hipEventDestroy(done);
        if (stream) hipStreamDestroy(stream);
    }

    template <typename T>
    rgg_status alloc(T **p, size_t count, const char *what)
    {
        size_t bytes = std::max<size_t>(1, count) * sizeof(T);   // at least one element
        void *q = nullptr;
        hipError_t e = hipMalloc(&q, bytes);
        if (e != hipSuccess) {
            (void)hipGetLastError();
            return fail(RGG_E_OUT_OF_MEMORY, "device allocation of %zu bytes for %s failed", bytes, what);
        }
        allocs.emplace_back(q, bytes);
        info.device_bytes += (int64_t)bytes;
        *p = (T *)q;
        return RGG_OK;
    }

    // frees a buffer obtained from alloc (null is ignored)
    void release(const void *p)
    {
        if (!p) return;
        for (size_t k = 0; k < allocs.size(); ++k)
            if (allocs[k].first == p) {
                (void)hipFree(allocs[k].first);
                info.device_bytes -= (int64_t)allocs[k].second;
                allocs.erase(allocs.begin() + (std::ptrdiff_t)k);
                return;
            }
    }

    template <typename T>
    rgg_status upload(T **p, const T *src, size_t count, const char *what)
    {
        rgg_status st = alloc(p, count, what);
        if (st != RGG_OK) return st;
        if (count) HIP_OR_FAIL(hipMemcpy(*p, src, count * sizeof(T), hipMemcpyHostToDevice), what);
        return RGG_OK;
    }
};


namespace rgg {

// Stream ordering of a roadmap's updates: the next update waits for the
// previous one when it is queued on another stream.
rgg_status order_after_previous(rgg_roadmap *rm, hipStream_t s);
rgg_status finish_update(rgg_roadmap *rm, hipStream_t s);

}  // namespace rgg
