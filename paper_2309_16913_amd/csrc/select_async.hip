// rt_range_select_async: a range select into caller-owned device buffers
// whose workspace the library keeps in a per-device pool.
//
// The call enqueues the count stage, reads the 8-byte total back (the only
// wait), and either refuses the select (RT_ENOMEM, the ids buffer untouched)
// or enqueues the fill stage and the sort and returns while they run.  A
// pooled workspace is handed to a later call only after the event recorded
// behind its last use has completed, so calls on different streams never
// share one while it is in use.
#include <mutex>
#include <vector>

#include "../../include/rt.h"
#include "rt_api_internal.h"
#include "rt_internal.h"

namespace rtk {
namespace {

// d_total = total, or all ones when a kernel-side check failed
__global__ void total_word(const uint64_t *__restrict__ status, uint64_t *__restrict__ d_total) {
    d_total[0] = (status[1] & 2u) ? ~0ull : status[0];
}

struct AsyncWs {
    void *d = nullptr;            // workspace, then 2 uint64 of status words at its end
    uint64_t bytes = 0;           // usable workspace bytes (status excluded)
    uint64_t *h_total = nullptr;  // pinned host word for the total
    hipEvent_t done = nullptr;    // recorded behind the last enqueued use
};

constexpr int kMaxDevices = 64;
struct AsyncPool {
    std::mutex mu;
    std::vector<AsyncWs *> idle;
};
AsyncPool g_async_pool[kMaxDevices];

uint64_t *status_of(AsyncWs *w) {
    return reinterpret_cast<uint64_t *>(static_cast<uint8_t *>(w->d) + w->bytes);
}

hipError_t ws_alloc(AsyncWs *w, uint64_t bytes) {
    if (w->d) (void)hipFree(w->d);
    w->d = nullptr;
    w->bytes = 0;
    hipError_t e = hipMalloc(&w->d, bytes + 256);
    if (e == hipSuccess) w->bytes = bytes;
    return e;
}

// A workspace of at least `bytes` whose previous use has finished: an idle one
// (grown by half again when too small) or a new one.
hipError_t acquire(int dev, uint64_t bytes, AsyncWs **out) {
    AsyncWs *w = nullptr;
    {
        AsyncPool &p = g_async_pool[dev];
        std::lock_guard<std::mutex> lk(p.mu);
        for (size_t i = 0; i < p.idle.size(); ++i) {
            if (hipEventQuery(p.idle[i]->done) == hipSuccess) {
                w = p.idle[i];
                p.idle.erase(p.idle.begin() + (long)i);
                break;
            }
        }
    }
    hipError_t e = hipSuccess;
    if (!w) {
        w = new AsyncWs();
        e = hipEventCreateWithFlags(&w->done, hipEventDisableTiming);
        if (e == hipSuccess) e = hipHostMalloc(reinterpret_cast<void **>(&w->h_total), 8, hipHostMallocDefault);
    }
    if (e == hipSuccess && w->bytes < bytes) e = ws_alloc(w, bytes + bytes / 2);
    if (e != hipSuccess) {
        // keep the object: its event and pinned word stay valid for a later call
        std::lock_guard<std::mutex> lk(g_async_pool[dev].mu);
        if (w->done) g_async_pool[dev].idle.push_back(w);
        else delete w;
        return e;
    }
    *out = w;
    return hipSuccess;
}

// Hand a workspace back once everything enqueued on s so far has finished.
void release(int dev, AsyncWs *w, hipStream_t s) {
    (void)hipEventRecord(w->done, s);
    std::lock_guard<std::mutex> lk(g_async_pool[dev].mu);
    g_async_pool[dev].idle.push_back(w);
}

}  // namespace
}  // namespace rtk

using namespace rtk;

extern "C" int rt_range_select_async(const rt_tree *t, const float *d_queries, uint64_t nq, uint64_t *d_offsets,
                                     uint32_t *d_ids, uint64_t ids_capacity, uint64_t *d_total, void *stream) {
    if (!t || (nq && !d_queries) || !d_offsets || !d_total || (ids_capacity && !d_ids))
        return fail(RT_EINVAL, "NULL argument");
    if (nq > 0xFFF00000ull) return fail(RT_EINVAL, "nq = %llu too large", (unsigned long long)nq);
    if ((reinterpret_cast<uintptr_t>(d_queries) & 15) != 0) return fail(RT_EINVAL, "queries not 16-byte aligned");
    if (t->device < 0 || t->device >= kMaxDevices) return fail(RT_EINVAL, "device %d out of range", t->device);
    try {
        DevSet ds(t->device);
        hipStream_t s = static_cast<hipStream_t>(stream);
        const int dev = t->device;
        AsyncWs *w = nullptr;
        hipError_t e = acquire(dev, rt_select_workspace_bytes(nq, 0), &w);
        if (e != hipSuccess) return hip_fail(e, "select workspace");
        int rc = enqueue_select_stage(t, reinterpret_cast<const float4 *>(d_queries), nq, d_offsets, nullptr, 0,
                                      w->d, nullptr, s, 1, nullptr, nullptr);
        if (rc == RT_OK) {
            e = hipMemcpyAsync(d_total, d_offsets + nq, 8, hipMemcpyDeviceToDevice, s);
            if (e == hipSuccess) e = hipMemcpyAsync(w->h_total, d_offsets + nq, 8, hipMemcpyDeviceToHost, s);
            if (e == hipSuccess) e = hipStreamSynchronize(s);
            if (e != hipSuccess) rc = hip_fail(e, "count stage");
        }
        if (rc != RT_OK) {
            release(dev, w, s);
            return rc;
        }
        const uint64_t total = *w->h_total;
        if (total > ids_capacity) {
            release(dev, w, s);
            return fail(RT_ENOMEM, "the result has %llu ids, the buffer holds %llu", (unsigned long long)total,
                        (unsigned long long)ids_capacity);
        }
        const uint64_t need = rt_select_workspace_bytes(nq, total);
        if (w->bytes < need) {
            // the sort needs more scratch than this workspace has: move the
            // count stage's part (order, split plan) into a larger one
            AsyncWs *w2 = nullptr;
            e = acquire(dev, need, &w2);
            if (e == hipSuccess)
                e = hipMemcpyAsync(w2->d, w->d, rt_select_workspace_bytes(nq, 0), hipMemcpyDeviceToDevice, s);
            release(dev, w, s);
            if (e != hipSuccess) {
                if (w2) release(dev, w2, s);
                return hip_fail(e, "select workspace");
            }
            w = w2;
        }
        uint64_t *st = status_of(w);
        rc = enqueue_select_stage(t, reinterpret_cast<const float4 *>(d_queries), nq, d_offsets, d_ids, total, w->d,
                                  st, s, 2, nullptr, nullptr);
        if (rc == RT_OK) {
            hipLaunchKernelGGL(total_word, dim3(1), dim3(1), 0, s, st, d_total);
            e = hipGetLastError();
            if (e != hipSuccess) rc = hip_fail(e, "fill stage");
        }
        release(dev, w, s);
        return rc;
    } catch (const std::bad_alloc &) {
        return fail(RT_ENOMEM, "host allocation failed");
    } catch (...) {
        return fail(RT_EDEVICE, "unexpected failure");
    }
}
