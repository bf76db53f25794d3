// Spatial join entry points: level-synchronous traversal of both trees
// (section 4) driven from the host, one frontier of node pairs per level.
//
// Per level: a count pass gives each frontier pair its number of qualifying
// child pairs, a scan turns the counts into output offsets, the host reads
// the total, and a fill pass writes the next frontier (or, at the leaves,
// the (idA << 32 | idB) keys).  The keys are radix sorted into the canonical
// lexicographic order.  Device buffers are kept across levels and across
// calls (a per-device pool of workspaces, grown geometrically), so a join
// allocates only when it outgrows every earlier one on its device.
#include <cstdlib>
#include <cstring>
#include <mutex>
#include <new>
#include <utility>
#include <vector>

#include "pair_sort.h"
#include "rt_api_internal.h"

using namespace rtk;

namespace {

int bits_for(uint64_t maxval) {
    int b = 0;
    while (b < 64 && (maxval >> b)) ++b;
    return b;
}

// Device buffer that only reallocates when it has to grow.
struct Grow {
    DevBuf b;
    uint64_t cap = 0;   // bytes
    hipError_t need(uint64_t bytes) {
        if (bytes <= cap && b.p) return hipSuccess;
        uint64_t c = cap * 2 > bytes ? cap * 2 : bytes;
        if (c < 4096) c = 4096;
        hipError_t e = b.alloc(c);
        cap = e == hipSuccess ? c : 0;
        return e;
    }
    template <class T> T *as() const { return static_cast<T *>(b.p); }
};

struct JoinRun {
    Grow ctrl, fr[2], cnt, off, stmp, keys, ktmp, hist, hscan, rtmp, tacc, lvl, slot;
    uint64_t npairs = 0;
    const uint64_t *sorted = nullptr;   // device, npairs keys
    uint64_t tests = 0;                 // entry-pair predicates at equal levels (counted runs)
    uint64_t test_entries = 0;          // real entries loaded by the tile expansion (counted runs)
    uint64_t test_desc = 0;             // entry-versus-tree predicates of descending pairs
    uint64_t node_pairs = 0;            // node pairs visited over all levels (level-by-level runs)
    bool pairs_done = false;            // the (a, b) words are already written (replay with sort)
    // frontier size of every level in the last join run level by level with
    // host reads (empty: none yet); sizes the grids of the replayed levels
    std::vector<uint64_t> last_levels;
    // the replayed levels' launches as a graph: captured when the same join
    // (same trees, flags, level sizes and buffers) is replayed a second time
    // in a row, relaunched while it stays the same
    std::vector<uint64_t> replay_key, graph_key;
    hipGraph_t graph = nullptr;
    uint64_t *host_tail = nullptr;      // pinned: key count, overflow flag | error word << 32
    hipGraphExec_t graph_exec = nullptr;
};

// Workspaces are pooled per device: a call takes one (or makes one) and
// returns it when done, after its stream has drained, so concurrent calls
// never share buffers.  Pooled device memory is held until the process
// ends (hipFree would stall the device on every call).
constexpr int kMaxDevices = 64;
struct JoinPool {
    std::mutex mu;
    std::vector<JoinRun *> idle;
};
JoinPool g_join_pool[kMaxDevices];

struct PooledRun {
    int dev;
    hipStream_t s;
    JoinRun *w = nullptr;
    PooledRun(int d, hipStream_t st) : dev(d), s(st) {
        JoinPool &p = g_join_pool[dev];
        std::lock_guard<std::mutex> lk(p.mu);
        if (!p.idle.empty()) {
            w = p.idle.back();
            p.idle.pop_back();
        }
        if (!w) w = new JoinRun();
    }
    ~PooledRun() {
        (void)hipStreamSynchronize(s);   // nothing of this call may still use the buffers
        JoinPool &p = g_join_pool[dev];
        std::lock_guard<std::mutex> lk(p.mu);
        p.idle.push_back(w);
    }
};

// Sorts the total keys in w.keys into the canonical order (only the digits
// that can be nonzero).
int sort_keys(const rt_tree *a, const rt_tree *b, uint64_t total, hipStream_t s, JoinRun &w) {
    const int bb = bits_for(b->n_objects ? b->n_objects - 1 : 0);
    const int ba = bits_for(a->n_objects ? a->n_objects - 1 : 0);
    hipError_t e = w.ktmp.need(total * 8);
    if (e != hipSuccess) return hip_fail(e, "join sort");
    uint64_t *src = w.keys.as<uint64_t>(), *tmp = w.ktmp.as<uint64_t>();
    // Up to ~1.5K keys per bucket on average: buckets by the top 11 bits of
    // the key (every key is below 2^(32 + ba)), each sorted in LDS; four
    // launches against the LSD sort's twenty.  Larger results keep the LSD
    // sort (most buckets would exceed the LDS cap).
    if (total <= (uint64_t)kPairBuckets * 1536) {
        e = w.hist.need((kPairSortWords + 4) * 4);
        if (e == hipSuccess) e = launch_pair_bucket_sort(src, total, 21 + ba, tmp, w.hist.as<uint32_t>(), s);
        if (e != hipSuccess) return hip_fail(e, "join sort");
        w.npairs = total;
        w.sorted = tmp;
        return RT_OK;
    }
    // 11-bit digits: 4 passes for two 21-bit ids instead of 6 (each pass
    // costs about the same few launches whatever its width)
    constexpr int kDigit = 11;
    int shifts[16], np = 0;
    for (int sft = 0; sft < bb; sft += kDigit) shifts[np++] = sft;
    for (int sft = 32; sft < 32 + ba; sft += kDigit) shifts[np++] = sft;
    const uint64_t he = radix_hist_elems(total, kDigit);
    e = w.hist.need(he * 4);
    if (e == hipSuccess) e = w.hscan.need((he + 1) * 8);
    if (e == hipSuccess) e = w.rtmp.need(scan_tmp_elems(he) * 8);
    bool in_tmp = false;
    if (e == hipSuccess)
        e = launch_radix_sort_u64(src, tmp, total, shifts, np, w.hist.as<uint32_t>(), w.hscan.as<uint64_t>(),
                                  w.rtmp.as<uint64_t>(), &in_tmp, s, kDigit);
    if (e != hipSuccess) return hip_fail(e, "join sort");
    w.npairs = total;
    w.sorted = in_tmp ? tmp : src;
    return RT_OK;
}

constexpr int kReplayMiss = -1000;   // not an RT_ code: the replay did not fit, run level by level

inline int mode_of(int la, int lb) {
    return la > lb ? JOIN_DESC_A : (lb > la ? JOIN_DESC_B : (la == 0 ? JOIN_EMIT : JOIN_BOTH));
}

inline void descend(int mode, int &la, int &lb) {
    if (mode == JOIN_DESC_A) --la;
    else if (mode == JOIN_DESC_B) --lb;
    else { --la; --lb; }
}

// The levels of the last run replayed without host reads: each level's
// frontier size stays on the device (the scan writes it, clamped to what the
// next level's buffers and grid allow), grids are sized from the last run's
// level sizes plus slack, and the host reads only the key count at the end.
// A level that outgrew those bounds marks the run, which then returns
// kReplayMiss (the caller runs level by level, growing the buffers).
int join_keys_replay(const rt_tree *a, const rt_tree *b, int flags, hipStream_t s, JoinRun &w, uint32_t *d_out,
                     uint64_t out_cap) {
    const std::vector<uint64_t> rec = w.last_levels;
    const size_t H = rec.size();
    if (H == 0) return kReplayMiss;
    const TreeView va = view_of(a), vb = view_of(b);
    hipError_t e = w.lvl.need((H + 2) * 8);
    if (e != hipSuccess) return hip_fail(e, "join setup");
    uint64_t *lv = w.lvl.as<uint64_t>();                      // lv[L]: size of level L (L >= 1); lv[H]: keys
    uint32_t *over = reinterpret_cast<uint32_t *>(lv + H + 1);
    Ctrl *ctrl = w.ctrl.as<Ctrl>();
    // frontier pairs a level can hold in fr[k] and the per-level buffers
    auto level_cap = [&](int k) {
        uint64_t c = w.fr[k].cap / 8;
        c = std::min(c, w.cnt.cap / 4);
        c = std::min(c, w.off.cap / 8 ? w.off.cap / 8 - 1 : 0);
        const uint64_t st = w.stmp.cap / 8;
        c = std::min(c, st > 1 ? (st - 1) * scan_tile_elems() : 0);
        c = std::min(c, w.slot.cap / join_slot_bytes(1));
        return std::min<uint64_t>(c, 0xFFFFFFFFull);
    };
    auto with_slack = [](uint64_t n) { return n + n / 4 + 1024; };
    // When the key buffer is small enough for the bucket sort, the sort and
    // the (a, b) words follow the levels with the key count on the device,
    // so the whole join needs one host read: out receives the words (the
    // caller's buffer, or for a host copy the key buffer, free by then),
    // unless the count exceeds its capacity or a level overflowed.
    const uint64_t kmax = w.keys.cap / 8;
    const bool fused = kmax > 0 && kmax <= (uint64_t)kPairBuckets * 1536;
    uint32_t *out = d_out ? d_out : w.keys.as<uint32_t>();
    const uint64_t cap_out = d_out ? out_cap : kmax;
    const int ba = bits_for(a->n_objects ? a->n_objects - 1 : 0);
    if (fused) {
        e = w.ktmp.need(kmax * 8);
        if (e == hipSuccess) e = w.hist.need((kPairSortWords + 4) * 4);
        if (e != hipSuccess) return hip_fail(e, "join setup");
    }
    // every launch of the replay; RT_OK, kReplayMiss or an error
    auto enqueue = [&](hipStream_t st) -> int {
        hipError_t e2 = launch_zero(ctrl, sizeof(Ctrl), st);
        if (e2 == hipSuccess) e2 = launch_zero(lv, (H + 2) * 8, st);   // and the overflow flag
        if (e2 == hipSuccess) e2 = launch_zero(w.fr[0].b.p, 8, st);   // (root A, root B) = (0, 0)
        if (e2 != hipSuccess) return hip_fail(e2, "join setup");
        int la = (int)a->height - 1, lb = (int)b->height - 1;
        int cur = 0;
        uint64_t lim = 1;   // level 0: the pair of roots
        for (size_t L = 0; L < H; ++L) {
            const int mode = mode_of(la, lb);
            const bool emit = mode == JOIN_EMIT;
            if (emit != (L + 1 == H)) return kReplayMiss;   // not the shape of the last run
            if (lim == 0) return kReplayMiss;
            const uint64_t next_lim =
                emit ? w.keys.cap / 8 : std::min<uint64_t>(with_slack(rec[L + 1]), level_cap(1 - cur));
            const uint64_t *nd = L == 0 ? nullptr : lv + L;
            const uint2 *fr = w.fr[cur].as<uint2>();
            uint64_t *off = w.off.as<uint64_t>();
            uint16_t *slots = w.slot.as<uint16_t>();
            e2 = launch_join_level(va, vb, fr, (uint32_t)lim, nd, mode, false, w.cnt.as<uint32_t>(), nullptr,
                                   nullptr, nullptr, 0, slots, ctrl, flags, nullptr, st);
            if (e2 == hipSuccess)
                e2 = launch_scan_u32_dev(w.cnt.as<uint32_t>(), nd, lim, off, w.stmp.as<uint64_t>(), lv + L + 1,
                                         next_lim, over, st);
            if (e2 == hipSuccess)
                e2 = launch_join_level(va, vb, fr, (uint32_t)lim, nd, mode, true, nullptr, off,
                                       emit ? nullptr : w.fr[1 - cur].as<uint2>(),
                                       emit ? w.keys.as<uint64_t>() : nullptr, next_lim, slots, ctrl, flags,
                                       nullptr, st);
            if (e2 != hipSuccess) return hip_fail(e2, "join level");
            cur = 1 - cur;
            lim = next_lim;
            descend(mode, la, lb);
        }
        if (fused) {
            e2 = launch_pair_bucket_sort(w.keys.as<uint64_t>(), kmax, 21 + ba, w.ktmp.as<uint64_t>(),
                                         w.hist.as<uint32_t>(), st, lv + H);
            if (e2 == hipSuccess)
                e2 = launch_keys_to_pairs_dev(w.ktmp.as<uint64_t>(), lv + H, kmax, cap_out, over, out, st);
            if (e2 != hipSuccess) return hip_fail(e2, "join sort");
        }
        // the error word beside the overflow flag: the status is one read
        e2 = launch_copy_err(ctrl, over + 1, st);
        if (e2 != hipSuccess) return hip_fail(e2, "join status");
        return RT_OK;
    };
    // what the launches depend on: both tree views, the flags, the level
    // sizes of the last run and every buffer's address and size
    std::vector<uint64_t> key;
    auto put = [&key](const void *p, size_t n) {
        const size_t w0 = key.size();
        key.resize(w0 + (n + 7) / 8, 0);
        std::memcpy(key.data() + w0, p, n);
    };
    put(&va, sizeof(va));
    put(&vb, sizeof(vb));
    key.push_back((uint64_t)(uint32_t)flags);
    key.push_back(H);
    key.insert(key.end(), rec.begin(), rec.end());
    for (const Grow *g : {&w.ctrl, &w.lvl, &w.fr[0], &w.fr[1], &w.cnt, &w.off, &w.stmp, &w.slot, &w.keys, &w.ktmp,
                          &w.hist}) {
        key.push_back(reinterpret_cast<uint64_t>(g->b.p));
        key.push_back(g->cap);
    }
    key.push_back(fused);
    key.push_back(reinterpret_cast<uint64_t>(out));
    key.push_back(cap_out);
    if (w.graph_exec && key == w.graph_key) {
        e = hipGraphLaunch(w.graph_exec, s);
        if (e != hipSuccess) return hip_fail(e, "join graph launch");
    } else if (key == w.replay_key) {
        // second replay of the same join in a row: capture it
        if (w.graph_exec) (void)hipGraphExecDestroy(w.graph_exec);
        if (w.graph) (void)hipGraphDestroy(w.graph);
        w.graph_exec = nullptr;
        w.graph = nullptr;
        w.graph_key.clear();
        // a stream of its own for the capture, destroyed right after: a
        // stream kept alive holds one of the process's few hardware queues,
        // which the caller's own streams would then share
        hipStream_t cs = nullptr;
        e = hipStreamCreateWithFlags(&cs, hipStreamNonBlocking);
        if (e == hipSuccess) e = hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal);
        if (e != hipSuccess) {
            if (cs) (void)hipStreamDestroy(cs);
            return hip_fail(e, "join graph capture");
        }
        const int rc = enqueue(cs);
        e = hipStreamEndCapture(cs, &w.graph);
        (void)hipStreamDestroy(cs);
        if (rc != RT_OK) {
            if (w.graph) (void)hipGraphDestroy(w.graph);
            w.graph = nullptr;
            return rc;
        }
        if (e == hipSuccess) e = hipGraphInstantiate(&w.graph_exec, w.graph, nullptr, nullptr, 0);
        if (e != hipSuccess) {
            w.graph_exec = nullptr;
            return hip_fail(e, "join graph capture");
        }
        w.graph_key = key;
        e = hipGraphLaunch(w.graph_exec, s);
        if (e != hipSuccess) return hip_fail(e, "join graph launch");
    } else {
        w.replay_key = key;
        if (int rc = enqueue(s)) return rc;
    }
    if (!w.host_tail) {
        e = hipHostMalloc(reinterpret_cast<void **>(&w.host_tail), 16, hipHostMallocDefault);
        if (e != hipSuccess) {
            w.host_tail = nullptr;
            return hip_fail(e, "join status buffer");
        }
    }
    e = hipMemcpyAsync(w.host_tail, lv + H, 16, hipMemcpyDeviceToHost, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    if (e != hipSuccess) return hip_fail(e, "join status");
    const uint64_t tail[2] = {w.host_tail[0], w.host_tail[1] & 0xFFFFFFFFull};   // key count, overflow flag
    const uint32_t err = (uint32_t)(w.host_tail[1] >> 32);
    if (err) return fail(RT_EDEVICE, "kernel check failed (flags %u)", err);
    if (tail[1] & 1u) return kReplayMiss;
    w.npairs = 0;
    w.sorted = nullptr;
    w.tests = 0;
    if (fused) {
        w.npairs = tail[0];
        w.sorted = w.ktmp.as<uint64_t>();
        w.pairs_done = true;
        return RT_OK;
    }
    return tail[0] ? sort_keys(a, b, tail[0], s, w) : RT_OK;
}

// Runs the join up to the sorted keys on the device; a replay may also write
// the (a, b) words (w.pairs_done): to d_out if not NULL and the pairs fit
// out_cap, else to the key buffer.
int join_keys(const rt_tree *a, const rt_tree *b, int flags, bool count_tests, hipStream_t s, JoinRun &w,
              uint32_t *d_out, uint64_t out_cap) {
    hipError_t e = w.ctrl.need(sizeof(Ctrl));
    if (e != hipSuccess) return hip_fail(e, "join setup");
    w.pairs_done = false;
    if (!count_tests) {
        const int rc = join_keys_replay(a, b, flags, s, w, d_out, out_cap);
        if (rc != kReplayMiss) return rc;
    }
    // level by level, each level's size read on the host
    const TreeView va = view_of(a), vb = view_of(b);
    if (e == hipSuccess) e = w.fr[0].need(8);
    if (e == hipSuccess && count_tests) e = w.tacc.need(kTestSlots * 16 * 8);
    if (e != hipSuccess) return hip_fail(e, "join setup");
    Ctrl *ctrl = w.ctrl.as<Ctrl>();
    unsigned long long *tacc = count_tests ? w.tacc.as<unsigned long long>() : nullptr;
    e = launch_zero(ctrl, sizeof(Ctrl), s);
    if (e == hipSuccess && tacc) e = launch_zero(tacc, kTestSlots * 16 * 8, s);
    if (e == hipSuccess) e = launch_zero(w.fr[0].b.p, 8, s);   // (root A, root B) = (0, 0)
    if (e != hipSuccess) return hip_fail(e, "join setup");
    uint64_t nfr = (a->n_objects && b->n_objects) ? 1 : 0;
    int cur = 0;
    int la = (int)a->height - 1, lb = (int)b->height - 1;
    w.npairs = 0;
    w.sorted = nullptr;
    std::vector<uint64_t> levels;
    while (nfr) {
        levels.push_back(nfr);
        const int mode = mode_of(la, lb);
        e = w.cnt.need(nfr * 4);
        if (e == hipSuccess) e = w.slot.need(join_slot_bytes(nfr));
        if (e == hipSuccess) e = w.off.need((nfr + 1) * 8);
        if (e == hipSuccess) e = w.stmp.need(scan_tmp_elems(nfr) * 8);
        if (e != hipSuccess) return hip_fail(e, "join frontier");
        const uint2 *fr = w.fr[cur].as<uint2>();
        uint64_t *off = w.off.as<uint64_t>();
        uint16_t *slots = w.slot.as<uint16_t>();
        e = launch_join_level(va, vb, fr, (uint32_t)nfr, nullptr, mode, false, w.cnt.as<uint32_t>(), nullptr,
                              nullptr, nullptr, 0, slots, ctrl, flags, tacc, s);
        if (e == hipSuccess) e = launch_scan_u32(w.cnt.as<uint32_t>(), nfr, off, w.stmp.as<uint64_t>(), s);
        uint64_t total = 0;
        if (e == hipSuccess) e = hipMemcpyAsync(&total, off + nfr, 8, hipMemcpyDeviceToHost, s);
        if (e == hipSuccess) e = hipStreamSynchronize(s);
        if (e != hipSuccess) return hip_fail(e, "join count");
        if (total == 0) break;
        if (mode == JOIN_EMIT) {
            e = w.keys.need(total * 8);
            if (e == hipSuccess)
                e = launch_join_level(va, vb, fr, (uint32_t)nfr, nullptr, mode, true, nullptr, off, nullptr,
                                      w.keys.as<uint64_t>(), total, slots, ctrl, flags, nullptr, s);
            if (e != hipSuccess) return hip_fail(e, "join emit");
            const int rc = sort_keys(a, b, total, s, w);
            if (rc) return rc;
            break;
        }
        if (total >= 0xFFFFFFFFull) return fail(RT_ENOMEM, "join frontier too large");
        e = w.fr[1 - cur].need(total * 8);
        if (e == hipSuccess)
            e = launch_join_level(va, vb, fr, (uint32_t)nfr, nullptr, mode, true, nullptr, off,
                                  w.fr[1 - cur].as<uint2>(), nullptr, total, slots, ctrl, flags, nullptr, s);
        if (e != hipSuccess) return hip_fail(e, "join expand");
        cur = 1 - cur;
        nfr = total;
        descend(mode, la, lb);
    }
    Ctrl hc;
    e = hipMemcpyAsync(&hc, ctrl, sizeof(Ctrl), hipMemcpyDeviceToHost, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    if (e != hipSuccess) return hip_fail(e, "join status");
    if (hc.err) return fail(RT_EDEVICE, "kernel check failed (flags %u)", hc.err);
    w.last_levels = levels;
    w.tests = w.test_entries = w.test_desc = 0;
    w.node_pairs = 0;
    for (uint64_t l : levels) w.node_pairs += l;
    if (tacc) {
        std::vector<unsigned long long> h(kTestSlots * 16);
        e = hipMemcpy(h.data(), tacc, h.size() * 8, hipMemcpyDeviceToHost);
        if (e != hipSuccess) return hip_fail(e, "join statistics");
        for (uint32_t k = 0; k < kTestSlots; ++k) {
            w.tests += h[k * 16];
            w.test_entries += h[k * 16 + 1];
            w.test_desc += h[k * 16 + 2];
        }
    }
    return RT_OK;
}

int check_join_args(const rt_tree *a, const rt_tree *b, int32_t *flags) {
    if (!a || !b) return fail(RT_EINVAL, "tree is NULL");
    if (a->device != b->device) return fail(RT_EINVAL, "trees are on different devices");
    if (a->device < 0 || a->device >= kMaxDevices) return fail(RT_EINVAL, "device %d out of range", a->device);
    const bool both_sorted = a->sorted_lx && b->sorted_lx;
    // measured fastest: candidate lists with O3 + O5 + the lower bound on
    // sorted trees, else the full tile (candidate lists without pruning cost
    // more than they save)
    if (*flags == RT_JOIN_DEFAULT) *flags = both_sorted ? (RT_JOIN_O3 | RT_JOIN_O5 | RT_JOIN_LB) : RT_JOIN_TILE;
    if (*flags & ~(RT_JOIN_O3 | RT_JOIN_O4 | RT_JOIN_O5 | RT_JOIN_TILE | RT_JOIN_LB))
        return fail(RT_EINVAL, "unknown join flags 0x%x", (unsigned)*flags);
    if ((*flags & RT_JOIN_TILE) && (*flags & ~RT_JOIN_TILE))
        return fail(RT_EINVAL, "RT_JOIN_TILE cannot be combined with pruning");
    if ((*flags & RT_JOIN_LB) && (*flags & (RT_JOIN_O3 | RT_JOIN_O4 | RT_JOIN_O5)) != (RT_JOIN_O3 | RT_JOIN_O5))
        return fail(RT_EINVAL, "RT_JOIN_LB goes with RT_JOIN_O3 | RT_JOIN_O5 only");
    if ((*flags & (RT_JOIN_O3 | RT_JOIN_O4 | RT_JOIN_O5 | RT_JOIN_LB)) && !both_sorted)
        return fail(RT_EINVAL, "join pruning needs both trees built with RT_BUILD_SORT_LX");
    return RT_OK;
}

}  // namespace

extern "C" int rt_spatial_join(const rt_tree *a, const rt_tree *b, rt_pairs **out) {
    return rt_spatial_join_ex(a, b, RT_JOIN_DEFAULT, out, nullptr);
}

extern "C" int rt_spatial_join_ex(const rt_tree *a, const rt_tree *b, int32_t flags, rt_pairs **out,
                                  uint64_t *tests) {
    if (!out) return fail(RT_EINVAL, "out is NULL");
    *out = nullptr;
    if (tests) *tests = 0;
    int rc = check_join_args(a, b, &flags);
    if (rc) return rc;
    try {
        DevSet ds(a->device);
        hipStream_t s = nullptr;
        PooledRun run(a->device, s);
        JoinRun &w = *run.w;
        rc = join_keys(a, b, flags, tests != nullptr, s, w, nullptr, 0);
        if (rc) return rc;
        if (tests) *tests = w.tests;
        void *mem = obj_alloc(KIND_PAIRS, sizeof(rt_pairs));
        if (!mem) return fail(RT_ENOMEM, "host allocation failed");
        rt_pairs *r = static_cast<rt_pairs *>(mem);
        r->n = w.npairs;
        r->pairs = static_cast<uint32_t *>(std::malloc(w.npairs ? w.npairs * 8 : 8));
        if (!r->pairs) {
            rt_free(r);
            return fail(RT_ENOMEM, "host allocation failed");
        }
        if (w.npairs) {
            // reuse the sort's other buffer for the (a, b) words (where a
            // replay has already written them)
            uint32_t *dp = const_cast<uint32_t *>(reinterpret_cast<const uint32_t *>(
                w.sorted == w.keys.as<uint64_t>() ? w.ktmp.as<uint64_t>() : w.keys.as<uint64_t>()));
            hipError_t e = w.pairs_done ? hipSuccess : launch_keys_to_pairs(w.sorted, w.npairs, dp, s);
            if (e == hipSuccess) e = hipMemcpy(r->pairs, dp, w.npairs * 8, hipMemcpyDeviceToHost);
            if (e != hipSuccess) {
                rt_free(r);
                return hip_fail(e, "copying the pairs");
            }
        }
        *out = r;
        return RT_OK;
    } catch (const std::bad_alloc &) {
        return fail(RT_ENOMEM, "host allocation failed");
    } catch (...) {
        return fail(RT_EDEVICE, "unexpected failure");
    }
}

extern "C" int rt_join_visit_stats(const rt_tree *a, const rt_tree *b, uint64_t *node_pairs, uint64_t *entry_pairs,
                                   uint64_t *entries) {
    if (!node_pairs || !entry_pairs || !entries) return fail(RT_EINVAL, "NULL argument");
    *node_pairs = *entry_pairs = *entries = 0;
    int32_t flags = RT_JOIN_TILE;
    int rc = check_join_args(a, b, &flags);
    if (rc) return rc;
    try {
        DevSet ds(a->device);
        hipStream_t s = nullptr;
        PooledRun run(a->device, s);
        JoinRun &w = *run.w;
        rc = join_keys(a, b, flags, true, s, w, nullptr, 0);
        if (rc) return rc;
        *node_pairs = w.node_pairs;
        *entry_pairs = w.tests + w.test_desc;
        *entries = w.test_entries;
        return RT_OK;
    } catch (const std::bad_alloc &) {
        return fail(RT_ENOMEM, "host allocation failed");
    } catch (...) {
        return fail(RT_EDEVICE, "unexpected failure");
    }
}

extern "C" int rt_spatial_join_device(const rt_tree *a, const rt_tree *b, int32_t flags, uint32_t *d_pairs,
                                      uint64_t capacity, uint64_t *n_pairs, void *stream) {
    if (!n_pairs) return fail(RT_EINVAL, "n_pairs is NULL");
    *n_pairs = 0;
    int rc = check_join_args(a, b, &flags);
    if (rc) return rc;
    if (capacity && !d_pairs) return fail(RT_EINVAL, "d_pairs is NULL with capacity > 0");
    try {
        DevSet ds(a->device);
        hipStream_t s = static_cast<hipStream_t>(stream);
        PooledRun run(a->device, s);
        JoinRun &w = *run.w;
        rc = join_keys(a, b, flags, false, s, w, d_pairs, capacity);
        if (rc) return rc;
        *n_pairs = w.npairs;
        if (w.npairs > capacity)
            return fail(RT_ENOMEM, "join has %llu pairs, capacity %llu", (unsigned long long)w.npairs,
                        (unsigned long long)capacity);
        if (w.pairs_done) return RT_OK;   // written and waited for by the replay
        hipError_t e = launch_keys_to_pairs(w.sorted, w.npairs, d_pairs, s);
        if (e == hipSuccess) e = hipStreamSynchronize(s);
        if (e != hipSuccess) return hip_fail(e, "writing the pairs");
        return RT_OK;
    } catch (const std::bad_alloc &) {
        return fail(RT_ENOMEM, "host allocation failed");
    } catch (...) {
        return fail(RT_EDEVICE, "unexpected failure");
    }
}
