// Device-side STR build (placeholder until the device packer lands).
#include "rt_api_internal.h"

extern "C" int rt_build_str_device(const float *d_rects, uint64_t n, uint32_t fanout, uint32_t layout,
                                   void *stream, rt_tree **out) {
    (void)d_rects; (void)n; (void)fanout; (void)layout; (void)stream;
    if (out) *out = nullptr;
    return rtk::fail(RT_EINVAL, "device build not available in this version");
}
