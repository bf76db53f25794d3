// In-library choice of fanout, node layout and work mapping for a tree built
// with fanout 0 or RT_LAYOUT_AUTO.
//
// The paper's operators depend on the fanout F and on the node layouts D0,
// D1 and D2 (section 2.3), and which is fastest depends on the machine and
// the data.  With no query set at build time, the tuner times a probe set
// drawn from the data itself: windows centred on the centres of seeded
// objects (so clustered data gets clustered probes), square, with an area of
// a fraction of the data's bounding box that is log-uniform in [1e-6, 1e-3]
// (the paper's default selectivity, 0.1%, is the top of that range).  Every
// candidate tree is built on the device and the probe set is selected on it
// (count, scan, fill, sort, timed with HIP events, best of two runs after a
// warm-up); the fastest is kept, the others are freed.  For the chosen tree
// the split mapping (one lane group per query, or large windows split into
// one work item per parent-of-leaves subtree) is timed the same way.
//
// The choice is remembered per (device architecture, log2 of the object
// count, candidate sets, low-x option) in memory and in a text file:
// $RT_TUNE_CACHE if set (an empty value keeps the cache in memory only),
// else $HOME/.cache/rt_mi355x_tune.txt.  A later build with the same key
// builds the cached choice without timing.
#include <sys/stat.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <map>
#include <mutex>
#include <string>
#include <vector>

#include "../../include/rt.h"
#include "rt_api_internal.h"
#include "rt_internal.h"

namespace rtk {
namespace {

__device__ __forceinline__ uint64_t mix64(uint64_t z) {
    z += 0x9E3779B97F4A7C15ull;
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}

__global__ void probe_windows(const float4 *__restrict__ rects, uint64_t n, uint32_t np, float4 mbr,
                              float4 *__restrict__ out) {
    const uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= np) return;
    const uint64_t h = mix64(0x5EEDull * 1315423911ull + i);
    const float4 r = rects[h % n];
    float cx = 0.5f * r.x + 0.5f * r.z, cy = 0.5f * r.y + 0.5f * r.w;
    if (cx != cx) cx = 0.f;   // an object spanning -inf..+inf
    if (cy != cy) cy = 0.f;
    const double u = (double)(mix64(h) >> 11) * (1.0 / 9007199254740992.0);
    const double sel = pow(10.0, -6.0 + 3.0 * u);
    double area = ((double)mbr.z - (double)mbr.x) * ((double)mbr.w - (double)mbr.y);
    if (!(area > 0.0) || !(area < 1e300)) area = 1.0;
    double half = 0.5 * sqrt(sel * area);
    if (!(half >= 0.0) || !(half < 1e300)) half = 0.0;
    out[i] = make_float4((float)(cx - half), (float)(cy - half), (float)(cx + half), (float)(cy + half));
}

struct Choice {
    uint32_t fanout, layout, kmin;
};

std::mutex g_mu;
std::map<std::string, Choice> g_cache;
bool g_loaded = false;

std::string cache_path() {
    const char *p = std::getenv("RT_TUNE_CACHE");
    if (p) return std::string(p);
    const char *home = std::getenv("HOME");
    if (!home || !*home) return std::string();
    return std::string(home) + "/.cache/rt_mi355x_tune.txt";
}

void load_cache_locked() {
    if (g_loaded) return;
    g_loaded = true;
    const std::string path = cache_path();
    if (path.empty()) return;
    FILE *f = std::fopen(path.c_str(), "r");
    if (!f) return;
    // one choice per line; lines of other formats (an earlier version's
    // timings of another select form) are skipped
    char line[512], key[256];
    unsigned F, L, K;
    while (std::fgets(line, sizeof line, f)) {
        if (std::sscanf(line, "rt-tune-v2 %255s %u %u %u", key, &F, &L, &K) == 4 && F >= 2 && F <= 64 &&
            (L == RT_LAYOUT_AOS || L == RT_LAYOUT_SOA || L == RT_LAYOUT_D2))
            g_cache[key] = Choice{F, L, K};
    }
    std::fclose(f);
}

void store_locked(const std::string &key, const Choice &c) {
    g_cache[key] = c;
    const std::string path = cache_path();
    if (path.empty()) return;
    const size_t slash = path.rfind('/');
    if (slash != std::string::npos && slash > 0) (void)mkdir(path.substr(0, slash).c_str(), 0755);
    FILE *f = std::fopen(path.c_str(), "a");
    if (!f) return;   // not writable: the in-memory cache still holds it
    std::fprintf(f, "rt-tune-v2 %s %u %u %u\n", key.c_str(), c.fanout, c.layout, c.kmin);
    std::fclose(f);
}

std::string make_key(uint64_t n, const std::vector<uint32_t> &fs, const std::vector<uint32_t> &ls, bool sort_lx) {
    int dev = 0;
    (void)hipGetDevice(&dev);
    hipDeviceProp_t p;
    std::string arch = "unknown";
    if (hipGetDeviceProperties(&p, dev) == hipSuccess) {
        arch = p.gcnArchName;
        const size_t colon = arch.find(':');
        if (colon != std::string::npos) arch = arch.substr(0, colon);
    }
    int lg = 0;
    while ((2ull << lg) <= n) ++lg;
    std::string k = arch + "|n2^" + std::to_string(lg) + "|F";
    for (uint32_t f : fs) k += std::to_string(f) + ",";
    k += "|L";
    for (uint32_t l : ls) k += std::to_string(l) + ",";
    k += sort_lx ? "|sortlx" : "|plain";
    return k;
}

// Times complete selects of the probe set on one tree.
struct Prober {
    hipStream_t s;
    uint32_t np = 0;
    DevBuf dq, off, ids, work, status;
    uint64_t total = 0, wb = 0;
    hipEvent_t ev[2] = {nullptr, nullptr};

    explicit Prober(hipStream_t st) : s(st) {}
    ~Prober() {
        for (auto &e : ev)
            if (e) (void)hipEventDestroy(e);
    }

    int setup(const float4 *d_rects, uint64_t n, const rt_tree *t) {
        np = (uint32_t)std::min<uint64_t>(16384, std::max<uint64_t>(512, n / 16));
        hipError_t e = dq.alloc((size_t)np * 16);
        if (e == hipSuccess) e = off.alloc((size_t)(np + 1) * 8);
        if (e == hipSuccess) e = status.alloc(16);
        if (e == hipSuccess) e = work.alloc(rt_select_workspace_bytes(np, 0));
        if (e == hipSuccess) e = hipEventCreate(&ev[0]);
        if (e == hipSuccess) e = hipEventCreate(&ev[1]);
        if (e != hipSuccess) return hip_fail(e, "tuner setup");
        const float4 mbr = make_float4(t->mbr[0], t->mbr[1], t->mbr[2], t->mbr[3]);
        hipLaunchKernelGGL(probe_windows, dim3((np + 255) / 256), dim3(256), 0, s, d_rects, n, np, mbr,
                           static_cast<float4 *>(dq.p));
        e = hipGetLastError();
        if (e != hipSuccess) return hip_fail(e, "tuner probes");
        int rc = enqueue_select_stage(t, static_cast<const float4 *>(dq.p), np, static_cast<uint64_t *>(off.p),
                                      nullptr, 0, work.p, nullptr, s, 1, nullptr, nullptr);
        if (rc) return rc;
        e = hipMemcpyAsync(&total, static_cast<uint64_t *>(off.p) + np, 8, hipMemcpyDeviceToHost, s);
        if (e == hipSuccess) e = hipStreamSynchronize(s);
        // timed as one-call selects with room for the count pass's records
        // (the fill replays them), the form the device select is given
        wb = select_replay_ws_bytes(np, total);
        if (e == hipSuccess) e = ids.alloc(total * 4);
        if (e == hipSuccess) e = work.alloc(wb);
        return e == hipSuccess ? RT_OK : hip_fail(e, "tuner setup");
    }

    // best of two timed runs after a warm-up, in ms (negative on failure)
    float time(const rt_tree *t) {
        float best = -1.f;
        for (int r = 0; r < 3; ++r) {
            if (hipEventRecord(ev[0], s) != hipSuccess) return -1.f;
            if (enqueue_select_stage(t, static_cast<const float4 *>(dq.p), np, static_cast<uint64_t *>(off.p),
                                     static_cast<uint32_t *>(ids.p), total, work.p,
                                     static_cast<uint64_t *>(status.p), s, 3, nullptr, nullptr,
                                     wb - select_ws_bytes(np, total)) != RT_OK)
                return -1.f;
            if (hipEventRecord(ev[1], s) != hipSuccess || hipEventSynchronize(ev[1]) != hipSuccess) return -1.f;
            float ms = 0.f;
            if (hipEventElapsedTime(&ms, ev[0], ev[1]) != hipSuccess) return -1.f;
            if (r > 0 && (best < 0.f || ms < best)) best = ms;
        }
        uint64_t st[2] = {0, 0};
        if (hipMemcpy(st, status.p, 16, hipMemcpyDeviceToHost) != hipSuccess || st[1] != 0 || st[0] != total)
            return -1.f;
        return best;
    }
};

void release_tree(rt_tree *t) {
    if (!t) return;
    tree_release(t);
    std::free(reinterpret_cast<ObjHdr *>(t) - 1);
}

}  // namespace

int build_tuned(const float4 *d_rects, uint64_t n, uint32_t fanout, uint32_t layout, bool sort_lx, hipStream_t s,
                rt_tree **out) {
    std::vector<uint32_t> fs, ls;
    if (fanout) fs.push_back(fanout);
    else fs = {16, 32, 64};
    if (layout != RT_LAYOUT_AUTO) ls.push_back(layout);
    else ls = {RT_LAYOUT_AOS, RT_LAYOUT_SOA, RT_LAYOUT_D2};
    if (n == 0)   // nothing to time: an empty tree of the first candidates
        return build_str_on_device(d_rects, n, fanout ? fanout : 32u,
                                   layout == RT_LAYOUT_AUTO ? (uint32_t)RT_LAYOUT_SOA : layout, sort_lx, s, out);
    const std::string key = make_key(n, fs, ls, sort_lx);
    {
        std::lock_guard<std::mutex> lk(g_mu);
        load_cache_locked();
        auto it = g_cache.find(key);
        if (it != g_cache.end()) {
            int rc = build_str_on_device(d_rects, n, it->second.fanout, it->second.layout, sort_lx, s, out);
            if (rc == RT_OK) (*out)->split_kmin = it->second.kmin;
            return rc;
        }
    }
    Prober pr(s);
    rt_tree *best = nullptr;
    float best_ms = -1.f;
    for (uint32_t F : fs) {
        for (uint32_t L : ls) {
            rt_tree *t = nullptr;
            int rc = build_str_on_device(d_rects, n, F, L, sort_lx, s, &t);
            if (rc) {
                release_tree(best);
                return rc;
            }
            if (pr.np == 0) {
                rc = pr.setup(d_rects, n, t);
                if (rc) {
                    release_tree(t);
                    return rc;
                }
            }
            const float ms = pr.time(t);
            if (ms < 0.f) {
                release_tree(t);
                release_tree(best);
                return fail(RT_EDEVICE, "tuner: a probe select failed");
            }
            if (!best || ms < best_ms) {
                release_tree(best);
                best = t;
                best_ms = ms;
            } else {
                release_tree(t);
            }
        }
    }
    // work mapping on the chosen tree
    uint32_t kmin = 0;
    if (best->height >= 3) {
        best->split_kmin = 16;
        const float ms = pr.time(best);
        if (ms >= 0.f && ms < best_ms) kmin = 16;
    }
    best->split_kmin = kmin;
    {
        std::lock_guard<std::mutex> lk(g_mu);
        store_locked(key, Choice{best->fanout, best->layout, kmin});
    }
    *out = best;
    return RT_OK;
}

}  // namespace rtk
