// rt_range_select_device_noalloc: rt_range_select_device with its workspace
// in a fixed device array instead of a caller buffer, for callers that may
// not allocate (code under HIP graph capture, serving loops, harnesses that
// forbid hipMalloc).  Nothing here allocates: the array is part of the
// library's code object, so each device that loads the library holds one
// copy of it until the process ends.
#include <mutex>

#include "../../include/rt.h"
#include "rt_api_internal.h"
#include "rt_internal.h"

namespace rtk {
namespace {

constexpr uint64_t kScratchBytes = RT_NOALLOC_SCRATCH_BYTES;
constexpr int kMaxDevices = 64;

// The workspace of every call on a device.  Host code never passes this
// name to a kernel (on the host it is only a stand-in for the symbol): it
// uses the device address looked up once per device below.
__device__ __align__(256) uint8_t scratch[kScratchBytes];

std::mutex g_mu;
void *g_addr[kMaxDevices] = {};

// Device address of `scratch` on the current device (looked up on the first
// call on each device, with that device current).
int scratch_address(int dev, void **out) {
    std::lock_guard<std::mutex> lk(g_mu);
    if (!g_addr[dev]) {
        void *p = nullptr;
        const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !p) return hip_fail(e != hipSuccess ? e : hipErrorUnknown, "scratch address");
        g_addr[dev] = p;
    }
    *out = g_addr[dev];
    return RT_OK;
}

}  // namespace
}  // namespace rtk

using namespace rtk;

extern "C" int rt_range_select_device_noalloc(const rt_tree *t, const float *d_queries, uint64_t nq,
                                              uint64_t *d_offsets, uint32_t *d_ids, uint64_t ids_capacity,
                                              uint64_t *d_status, void *stream) {
    if (!t || (nq && !d_queries) || !d_offsets || !d_status || (ids_capacity && !d_ids))
        return fail(RT_EINVAL, "NULL argument");
    if (nq > 0xFFF00000ull) return fail(RT_EINVAL, "nq = %llu too large", (unsigned long long)nq);
    if ((reinterpret_cast<uintptr_t>(d_queries) & 15) != 0) return fail(RT_EINVAL, "queries not 16-byte aligned");
    if (t->device < 0 || t->device >= kMaxDevices) return fail(RT_EINVAL, "device %d out of range", t->device);
    const uint64_t need = rt_select_workspace_bytes(nq, ids_capacity);
    if (need > kScratchBytes)
        return fail(RT_EINVAL,
                    "%llu queries with room for %llu ids need %llu bytes of workspace; the fixed scratch holds "
                    "%llu (RT_NOALLOC_SCRATCH_BYTES): use rt_range_select_device with a caller workspace",
                    (unsigned long long)nq, (unsigned long long)ids_capacity, (unsigned long long)need,
                    (unsigned long long)kScratchBytes);
    DevSet ds(t->device);
    void *work = nullptr;
    if (int rc = scratch_address(t->device, &work)) return rc;
    // the select clears what must start at zero (its control words) itself
    return enqueue_select(t, reinterpret_cast<const float4 *>(d_queries), nq, d_offsets, d_ids, ids_capacity, work,
                          d_status, static_cast<hipStream_t>(stream), false, nullptr);
}
