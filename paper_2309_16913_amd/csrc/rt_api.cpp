// C-ABI entry points: validation, device memory, the launch sequences of a
// range select and of a join, result copies, and the tagged rt_free.
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <new>
#include <string>
#include <vector>

#include "../../include/rt.h"
#include "rt_api_internal.h"
#include "rt_internal.h"

using namespace rtk;

// ---------------------------------------------------------------------------
// errors and tagged objects
// ---------------------------------------------------------------------------
static thread_local std::string g_err;

int rtk::fail(int code, const char *fmt, ...) {
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    g_err = buf;
    return code;
}

int rtk::hip_fail(hipError_t e, const char *what) {
    return fail(e == hipErrorOutOfMemory ? RT_ENOMEM : RT_EDEVICE, "%s: %s", what, hipGetErrorString(e));
}

extern "C" const char *rt_last_error(void) { return g_err.c_str(); }
extern "C" const char *rt_version(void) { return "rt-mi355x 1.0 (gfx950)"; }

void *rtk::obj_alloc(uint32_t kind, size_t bytes) {
    void *raw = std::malloc(sizeof(ObjHdr) + bytes);
    if (!raw) return nullptr;
    ObjHdr *h = static_cast<ObjHdr *>(raw);
    h->magic = kObjMagic;
    h->kind = kind;
    std::memset(h + 1, 0, bytes);
    return h + 1;
}

static ObjHdr *hdr_of(void *obj) { return static_cast<ObjHdr *>(obj) - 1; }

void rtk::tree_release(rt_tree *t) {
    if (!t) return;
    int cur = 0;
    (void)hipGetDevice(&cur);
    (void)hipSetDevice(t->device);
    if (t->d_nodes) (void)hipFree(t->d_nodes);
    if (t->d_meta) (void)hipFree(t->d_meta);
    if (t->d_range) (void)hipFree(t->d_range);
    if (t->d_leaf_ids) (void)hipFree(t->d_leaf_ids);
    (void)hipSetDevice(cur);
    t->~rt_tree();
}

extern "C" void rt_free(void *obj) {
    if (!obj) return;
    ObjHdr *h = hdr_of(obj);
    if (h->magic != kObjMagic) return;   // not ours: ignore rather than corrupt memory
    h->magic = 0;
    switch (h->kind) {
    case KIND_TREE:
        tree_release(static_cast<rt_tree *>(obj));
        break;
    case KIND_IDS: {
        rt_ids *r = static_cast<rt_ids *>(obj);
        std::free(r->offsets);
        std::free(r->ids);
        break;
    }
    case KIND_PAIRS:
        std::free(static_cast<rt_pairs *>(obj)->pairs);
        break;
    case KIND_BATCH:
        batch_release(static_cast<rt_batch *>(obj));
        break;
    default:
        break;
    }
    std::free(h);
}

// ---------------------------------------------------------------------------
// helpers
// ---------------------------------------------------------------------------
int rtk::check_rects(const float *r, uint64_t n, const char *what) {
    if (n && !r) return fail(RT_EINVAL, "%s is NULL with n = %llu", what, (unsigned long long)n);
    for (uint64_t i = 0; i < n; ++i) {
        const float *p = r + 4 * i;
        if (std::isnan(p[0]) || std::isnan(p[1]) || std::isnan(p[2]) || std::isnan(p[3]))
            return fail(RT_EINVAL, "%s[%llu] has a NaN coordinate", what, (unsigned long long)i);
        if (!(p[0] <= p[2]) || !(p[1] <= p[3]))
            return fail(RT_EINVAL, "%s[%llu] has low > high", what, (unsigned long long)i);
    }
    return RT_OK;
}

TreeView rtk::view_of(const rt_tree *t) {
    TreeView v;
    v.nodes = static_cast<const uint8_t *>(t->d_nodes);
    v.fanout = t->fanout;
    v.node_bytes = t->node_bytes;
    v.first_leaf = t->first_leaf;
    v.height = t->height;
    v.layout = t->layout;
    v.lookahead = t->lookahead;
    for (int i = 0; i < 4; ++i) v.mbr[i] = t->mbr[i];
    v.range = static_cast<const uint2 *>(t->d_range);
    v.partial_leaf = t->partial_leaf;
    v.partial_cnt = t->partial_cnt;
    v.leaf_ids = static_cast<const uint32_t *>(t->d_leaf_ids);
    return v;
}

DevBuf::~DevBuf() {
    if (p) (void)hipFree(p);
}
hipError_t DevBuf::alloc(size_t bytes) {
    if (p) (void)hipFree(p);
    p = nullptr;
    return hipMalloc(&p, bytes ? bytes : 16);
}

static uint64_t align256(uint64_t b) { return (b + 255) & ~255ull; }

// Split work items granted per select: at most 4 per query (and 65536),
// divided evenly over the kXcds lists.
static uint64_t split_hcap(uint64_t nq) {
    const uint64_t b = nq * 4 > 65536 ? nq * 4 : 65536;
    return (b + kXcds - 1) / kXcds;
}
static uint64_t split_budget(uint64_t nq) { return split_hcap(nq) * kXcds; }

// Workspace layout of a select:
//   Ctrl | counts[nq] | scan tmp | sort lists | query order | slots per query
//   | slot offsets per query | slot counts | slot offsets | split items
//   | slot scan tmp | sort scratch (cap ids, then class-L descriptors)
//   | bulk-copy descriptors (bulk_capacity(cap))
// Everything before the sort scratch depends on nq only, so a workspace for
// (nq, 0) is a prefix of one for (nq, cap).
struct SelWs {
    Ctrl *ctrl;
    uint32_t *counts;
    uint64_t *scan_tmp;
    uint32_t *lists;
    void *order;
    uint32_t *nslots;
    uint64_t *slot_first;
    uint32_t *slot_counts;
    uint64_t *slot_off;
    uint4 *heavy;
    uint64_t *slot_scan_tmp;
    uint32_t *scratch;
    uint64_t nslot_max;
};

static uint64_t sel_ws_bytes(uint64_t nq, uint64_t cap) {
    const uint64_t S = nq + split_budget(nq);
    return align256(sizeof(Ctrl)) + align256(4 * nq) + align256(8 * scan_tmp_elems(nq)) +
           align256(4 * segsort_ws_elems(nq)) + align256(order_ws_bytes(nq)) + align256(4 * nq) +
           align256(8 * (nq + 1)) + align256(4 * S) + align256(8 * (S + 1)) + align256(16 * split_budget(nq)) +
           align256(8 * scan_tmp_elems(S)) + align256(4 * segsort_scratch_elems(cap)) +
           align256(16 * bulk_capacity(cap));
}

// Record arena past the select's own layout: chunks of kRecChunk 16-byte
// records, then one count per chunk.  Sized for cap / 16 + 16 nq records
// (leaf visits with hits and contained subtrees: about cap / 64 at 10M
// rectangles / 1M windows, fanout 64), a third more for chunks closed early
// (a node's records never straddle two chunks), and one chunk per lane group
// that can hold a partly used one at the end of the pass; a count pass that
// needs more sets the overflow flag and the fill walks the tree instead.
uint64_t rtk::rec_arena_bytes(uint64_t nq, uint64_t cap) {
    const uint64_t recs = (cap / 16 + 16 * nq) * 4 / 3;
    const uint64_t groups = (uint64_t)num_cus() * 8 * 16;
    const uint64_t chunks = (recs + kRecChunk - 1) / kRecChunk + (nq < groups ? nq : groups);
    return align256(16 * kRecChunk * chunks) + align256(4 * chunks) + 512;
}

// Chunks of an arena of `bytes` bytes.
uint32_t rtk::rec_chunks_in(uint64_t bytes) {
    const uint64_t per = 16 * kRecChunk + 4;
    const uint64_t c = bytes > 512 ? (bytes - 512) / per : 0;
    return (uint32_t)(c < 0xFFFFFFF0ull ? c : 0xFFFFFFF0ull);
}

uint64_t rtk::select_ws_bytes(uint64_t nq, uint64_t cap) { return sel_ws_bytes(nq, cap); }
uint64_t rtk::select_replay_ws_bytes(uint64_t nq, uint64_t cap) {
    return sel_ws_bytes(nq, cap) + rec_arena_bytes(nq, cap);
}

// The bulk-copy descriptors of a workspace for (nq, cap).
static uint4 *sel_bulk(uint32_t *scratch, uint64_t cap) {
    return reinterpret_cast<uint4 *>(reinterpret_cast<uint8_t *>(scratch) + align256(4 * segsort_scratch_elems(cap)));
}

static SelWs sel_ws(void *w, uint64_t nq) {
    const uint64_t S = nq + split_budget(nq);
    uint8_t *p = static_cast<uint8_t *>(w);
    SelWs s;
    s.nslot_max = S;
    s.ctrl = reinterpret_cast<Ctrl *>(p);
    p += align256(sizeof(Ctrl));
    s.counts = reinterpret_cast<uint32_t *>(p);
    p += align256(4 * nq);
    s.scan_tmp = reinterpret_cast<uint64_t *>(p);
    p += align256(8 * scan_tmp_elems(nq));
    s.lists = reinterpret_cast<uint32_t *>(p);
    p += align256(4 * segsort_ws_elems(nq));
    s.order = p;
    p += align256(order_ws_bytes(nq));
    s.nslots = reinterpret_cast<uint32_t *>(p);
    p += align256(4 * nq);
    s.slot_first = reinterpret_cast<uint64_t *>(p);
    p += align256(8 * (nq + 1));
    s.slot_counts = reinterpret_cast<uint32_t *>(p);
    p += align256(4 * S);
    s.slot_off = reinterpret_cast<uint64_t *>(p);
    p += align256(8 * (S + 1));
    s.heavy = reinterpret_cast<uint4 *>(p);
    p += align256(16 * split_budget(nq));
    s.slot_scan_tmp = reinterpret_cast<uint64_t *>(p);
    p += align256(8 * scan_tmp_elems(S));
    s.scratch = reinterpret_cast<uint32_t *>(p);
    return s;
}

// ---------------------------------------------------------------------------
// build
// ---------------------------------------------------------------------------
extern "C" int rt_build_str(const float *rects, uint64_t n, uint32_t fanout, uint32_t layout, rt_tree **out) {
    if (!out) return fail(RT_EINVAL, "out is NULL");
    *out = nullptr;
    try {
        if (fanout != 0 && (fanout < 2 || fanout > 64)) return fail(RT_EINVAL, "fanout %u not in 2..64", fanout);
        const bool sort_lx = (layout & RT_BUILD_SORT_LX) != 0;
        layout &= ~RT_BUILD_SORT_LX;
        if (layout != RT_LAYOUT_AOS && layout != RT_LAYOUT_SOA && layout != RT_LAYOUT_D2 && layout != RT_LAYOUT_AUTO)
            return fail(RT_EINVAL, "unknown layout %u", layout);
        if (n >= 0xFFFFFFFFull) return fail(RT_EINVAL, "n = %llu does not fit 32-bit ids", (unsigned long long)n);
        int rc = check_rects(rects, n, "rects");
        if (rc) return rc;
        // the build itself runs on the device
        DevBuf d;
        hipError_t e = d.alloc(n ? n * 16 : 16);
        if (e == hipSuccess && n) e = hipMemcpy(d.p, rects, n * 16, hipMemcpyHostToDevice);
        if (e != hipSuccess) return hip_fail(e, "uploading the rectangles");
        if (fanout == 0 || layout == RT_LAYOUT_AUTO)
            return build_tuned(static_cast<const float4 *>(d.p), n, fanout, layout, sort_lx, nullptr, out);
        return build_str_on_device(static_cast<const float4 *>(d.p), n, fanout, layout, sort_lx, nullptr, out);
    } catch (const std::bad_alloc &) {
        return fail(RT_ENOMEM, "host allocation failed");
    } catch (...) {
        return fail(RT_EDEVICE, "unexpected failure");
    }
}

extern "C" int rt_tree_set_lookahead(rt_tree *t, uint32_t on) {
    if (!t) return fail(RT_EINVAL, "tree is NULL");
    if (on > 1) return fail(RT_EINVAL, "lookahead %u is not 0 or 1", on);
    t->lookahead = on;
    return RT_OK;
}

extern "C" int rt_tree_set_bulk_copy(rt_tree *t, uint32_t mode) {
    if (!t) return fail(RT_EINVAL, "tree is NULL");
    if (mode > RT_BULK_OFF) return fail(RT_EINVAL, "bulk-copy mode %u is not 0, 1 or 2", mode);
    t->bulk_copy = mode;
    return RT_OK;
}

extern "C" int rt_select_replay_info(const void *d_work, uint32_t *chunks, uint32_t *overflowed) {
    if (!d_work || !chunks || !overflowed) return fail(RT_EINVAL, "NULL argument");
    Ctrl hc;
    const hipError_t e = hipMemcpy(&hc, d_work, sizeof(Ctrl), hipMemcpyDeviceToHost);
    if (e != hipSuccess) return hip_fail(e, "reading the select's control words");
    *chunks = hc.rec_chunks;
    *overflowed = hc.rec_overflow;
    return RT_OK;
}

extern "C" int rt_tree_set_replay(rt_tree *t, uint32_t on) {
    if (!t) return fail(RT_EINVAL, "tree is NULL");
    if (on > 1) return fail(RT_EINVAL, "replay %u is not 0 or 1", on);
    t->replay = on;
    return RT_OK;
}

extern "C" int rt_tree_set_split(rt_tree *t, uint32_t kmin) {
    if (!t) return fail(RT_EINVAL, "tree is NULL");
    t->split_kmin = kmin;
    return RT_OK;
}

extern "C" int rt_tree_stats(const rt_tree *t, rt_tree_info *info) {
    if (!t || !info) return fail(RT_EINVAL, "NULL argument");
    std::memset(info, 0, sizeof(*info));
    info->n_objects = t->n_objects;
    info->n_entries = t->n_entries;
    info->device_bytes = (uint64_t)t->n_nodes * t->node_bytes;
    info->n_nodes = t->n_nodes;
    info->height = t->height;
    info->fanout = t->fanout;
    info->layout = t->layout;
    info->node_bytes = t->node_bytes;
    info->first_leaf = t->first_leaf;
    info->device = t->device;
    info->flags = t->sorted_lx ? RT_BUILD_SORT_LX : 0u;
    return RT_OK;
}

extern "C" int rt_tree_export(const rt_tree *t, uint32_t *level, uint32_t *count, uint64_t *first, float *lx,
                              float *ly, float *hx, float *hy, uint32_t *ptr) {
    if (!t || !level || !count || !first || !lx || !ly || !hx || !hy || !ptr) return fail(RT_EINVAL, "NULL argument");
    try {
        std::vector<uint8_t> img((size_t)t->n_nodes * t->node_bytes);
        std::vector<uint32_t> meta(t->n_nodes);
        DevSet ds(t->device);
        hipError_t e = hipMemcpy(img.data(), t->d_nodes, img.size(), hipMemcpyDeviceToHost);
        if (e == hipSuccess) e = hipMemcpy(meta.data(), t->d_meta, meta.size() * 4, hipMemcpyDeviceToHost);
        if (e != hipSuccess) return hip_fail(e, "reading the tree back");
        const uint32_t F = t->fanout;
        uint64_t k = 0;
        for (uint32_t u = 0; u < t->n_nodes; ++u) {
            const uint32_t cnt = meta[u] & 0xFFu;
            level[u] = meta[u] >> 8;
            count[u] = cnt;
            first[u] = k;
            const uint8_t *node = img.data() + (size_t)u * t->node_bytes;
            const float *f = reinterpret_cast<const float *>(node);
            const uint32_t *w = reinterpret_cast<const uint32_t *>(node);
            for (uint32_t s = 0; s < cnt; ++s, ++k) {
                if (t->layout == RT_LAYOUT_SOA) {
                    lx[k] = f[s]; ly[k] = f[F + s]; hx[k] = f[2 * F + s]; hy[k] = f[3 * F + s]; ptr[k] = w[4 * F + s];
                } else if (t->layout == RT_LAYOUT_AOS) {
                    lx[k] = f[5 * s]; ly[k] = f[5 * s + 1]; hx[k] = f[5 * s + 2]; hy[k] = f[5 * s + 3]; ptr[k] = w[5 * s + 4];
                } else {
                    lx[k] = f[2 * s]; ly[k] = f[2 * s + 1]; hx[k] = f[2 * F + 2 * s]; hy[k] = f[2 * F + 2 * s + 1];
                    ptr[k] = w[4 * F + s];
                }
            }
            // unused slots must be NaN padding, or the kernels would see them
            for (uint32_t s = cnt; s < F; ++s) {
                float v = t->layout == RT_LAYOUT_SOA ? f[s] : (t->layout == RT_LAYOUT_AOS ? f[5 * s] : f[2 * s]);
                if (!std::isnan(v)) return fail(RT_EDEVICE, "node %u slot %u is not padding", u, s);
            }
        }
        if (k != t->n_entries) return fail(RT_EDEVICE, "entry count mismatch");
        return RT_OK;
    } catch (const std::bad_alloc &) {
        return fail(RT_ENOMEM, "host allocation failed");
    }
}

// ---------------------------------------------------------------------------
// range select
// ---------------------------------------------------------------------------
extern "C" uint64_t rt_select_workspace_bytes(uint64_t nq, uint64_t cap) { return sel_ws_bytes(nq, cap); }
extern "C" uint64_t rt_select_replay_workspace_bytes(uint64_t nq, uint64_t cap) {
    return select_replay_ws_bytes(nq, cap);
}

static int check_nq(uint64_t nq) {
    if (nq > 0xFFF00000ull) return fail(RT_EINVAL, "nq = %llu too large", (unsigned long long)nq);
    return RT_OK;
}

// Split plan of a select on tree t: queries whose walk reaches at least
// t->split_kmin parents-of-leaves nodes run as one work item per such node.
struct SplitCfg {
    bool on = false;
    uint32_t split_first = 0, kmin = 0, budget = 0;
    float min_area = 0.f;
};

static SplitCfg split_cfg(const rt_tree *t, uint64_t nq) {
    SplitCfg c;
    if (t->split_kmin == 0 || t->height < 3 || nq == 0 || t->n_objects == 0) return c;
    c.on = true;
    c.split_first = t->level_start[2];   // first grandparent-of-leaves node
    c.kmin = t->split_kmin;
    c.budget = (uint32_t)split_hcap(nq);   // per list
    // prefilter: a window smaller than 1/64 of the area that kmin full
    // parents-of-leaves cover on average cannot reach kmin of them
    const double area = (double)(t->mbr[2] - t->mbr[0]) * (double)(t->mbr[3] - t->mbr[1]);
    const double per = (double)t->fanout * t->fanout / (double)t->n_objects;
    const double a = area * per * c.kmin / 64.0;
    c.min_area = (area > 0 && area < 1e300 && a < 3e38) ? (float)a : 0.f;
    return c;
}

int rtk::enqueue_select_stage(const rt_tree *t, const float4 *dq, uint64_t nq, uint64_t *d_off, uint32_t *d_ids,
                              uint64_t cap, void *work, uint64_t *d_status, hipStream_t s, int stage,
                              uint32_t *d_counts_out, void *const *events, uint64_t rec_bytes) {
    SelWs w = sel_ws(work, nq);
    if (nq == 0) {   // no launch of an empty grid: offsets = {0}, status = {0, 0}
        hipError_t e = hipSuccess;
        if (stage & 1) {
            e = launch_zero(w.ctrl, sizeof(Ctrl), s);
            if (e == hipSuccess && d_off && !d_counts_out) e = launch_zero(d_off, 8, s);
        }
        if (e == hipSuccess && (stage & 2) && d_status) e = launch_finalize(d_off, 0, cap, w.ctrl, d_status, s);
        return e == hipSuccess ? RT_OK : hip_fail(e, "empty select");
    }
    const TreeView v = view_of(t);
    const SplitCfg sc = d_counts_out ? SplitCfg() : split_cfg(t, nq);
    auto mark = [&](int k) -> hipError_t {
        return events && events[k] ? hipEventRecord(static_cast<hipEvent_t>(events[k]), s) : hipSuccess;
    };
    hipError_t e = hipSuccess;
    SelectPlan plan;
    if (sc.on) {
        plan.slot_first = w.slot_first;
        plan.heavy = w.heavy;
        plan.hcap = sc.budget;
    }
    // records of the count pass (node and leaf indices must leave the two
    // flag bits free), in the rec_bytes after the layout for (nq, cap) in one
    // call, or for (nq, 0) in a separate count stage; the count stage names
    // the arena in the control words, where the fill stage's replay finds it
    const uint32_t rec_nchunks = rec_chunks_in(rec_bytes);
    const bool rec = (stage & 1) && !d_counts_out && t->replay && rec_nchunks > 0 && t->n_nodes < (1u << 30);
    if (rec) {
        uint8_t *base = static_cast<uint8_t *>(work) + sel_ws_bytes(nq, stage == 1 ? 0 : cap);
        plan.rec = reinterpret_cast<uint4 *>(base);
        plan.rec_count = reinterpret_cast<uint32_t *>(base + align256(16ull * kRecChunk * rec_nchunks));
        plan.rec_nchunks = rec_nchunks;
    }
    if (stage & 1) {   // count stage: ctrl, order, split, count pass, offsets
        uint32_t *counts = d_counts_out ? d_counts_out : (sc.on ? w.slot_counts : w.counts);
        e = launch_zero(w.ctrl, sizeof(Ctrl), s);
        if (e == hipSuccess && rec) e = launch_set_rec(w.ctrl, plan, s);
        if (e == hipSuccess) e = mark(0);
        const uint64_t *order = nullptr;
        if (e == hipSuccess && nq >= kOrderMinQueries)
            e = launch_query_order(dq, (uint32_t)nq, t->mbr, w.order, &order, s);
        plan.order = order;
        if (sc.on) {
            if (e == hipSuccess)
                e = launch_split(v, dq, (uint32_t)nq, 0, sc.split_first, sc.kmin, sc.budget, sc.min_area, w.nslots,
                                 nullptr, nullptr, order, w.ctrl, s);
            if (e == hipSuccess) e = launch_scan_u32(w.nslots, nq, w.slot_first, w.scan_tmp, s);
            // phase 1 walks the XCD slices again: reset their counters
            if (e == hipSuccess) e = launch_zero(w.ctrl->xwork[2], sizeof(w.ctrl->xwork[2]), s);
            if (e == hipSuccess)
                e = launch_split(v, dq, (uint32_t)nq, 1, sc.split_first, sc.kmin, sc.budget, sc.min_area, nullptr,
                                 w.slot_first, w.heavy, order, w.ctrl, s);
            if (e == hipSuccess) e = launch_zero(w.slot_counts, 4 * w.nslot_max, s);
        }
        if (e == hipSuccess)
            e = launch_select_pass(v, dq, (uint32_t)nq, SEL_COUNT, counts, nullptr, nullptr, 0, w.ctrl, 0, plan,
                                   (uint32_t)nq, s);
        if (e == hipSuccess) e = mark(1);
        if (d_counts_out || e != hipSuccess) return e == hipSuccess ? RT_OK : hip_fail(e, "count pass");
        if (sc.on) {
            e = launch_scan_u32(w.slot_counts, w.nslot_max, w.slot_off, w.slot_scan_tmp, s);
            if (e == hipSuccess) e = launch_gather_offsets(w.slot_first, w.slot_off, (uint32_t)nq, d_off, s);
        } else {
            e = launch_scan_u32(w.counts, nq, d_off, w.scan_tmp, s);
        }
        if (e == hipSuccess) e = mark(2);
        if (e != hipSuccess) return hip_fail(e, "count stage");
    }
    if (stage & 2) {   // fill stage: fill pass, sort, status
        // the processing order written by the count stage is still in the workspace
        if (nq >= kOrderMinQueries) plan.order = query_order_result(w.order, nq);
        const uint64_t *fo = sc.on ? w.slot_off : d_off;
        const uint32_t no = sc.on ? (uint32_t)w.nslot_max : (uint32_t)nq;
        // on large trees long contained runs go to the bulk copy after the pass
        if (t->bulk_copy == RT_BULK_ON || (t->bulk_copy == RT_BULK_AUTO && t->n_objects >= kBulkMinObjects)) {
            const uint64_t bcap = bulk_capacity(cap);
            plan.bulk = sel_bulk(w.scratch, cap);
            plan.bulk_cap = (uint32_t)(bcap < 0xFFFFFFFFull ? bcap : 0xFFFFFFFFull);
        }
        // replay the count pass's records (a separate fill stage cannot know
        // whether its count stage made any: the replay checks); the walk then
        // runs only if there were none or they overflowed
        if (rec || stage == 2) {
            e = launch_replay(v, fo, no, d_ids, cap, w.ctrl, s);
            plan.fill_guard = 1;
        }
        if (e == hipSuccess)
            e = launch_select_pass(v, dq, (uint32_t)nq, SEL_FILL, nullptr, fo, d_ids, cap, w.ctrl, 1, plan, no, s);
        if (e == hipSuccess && plan.bulk)
            e = launch_bulk_copy(static_cast<const uint32_t *>(t->d_leaf_ids), plan.bulk, plan.bulk_cap, d_ids, w.ctrl,
                                 s);
        if (e == hipSuccess) e = mark(3);
        if (e == hipSuccess)
            e = launch_segsort(d_off, nq, d_ids, w.scratch, cap, w.lists, t->n_objects, nullptr, s);
        if (e == hipSuccess) e = mark(4);
        if (e == hipSuccess && d_status) e = launch_finalize(d_off, nq, cap, w.ctrl, d_status, s);
        if (e != hipSuccess) return hip_fail(e, "fill stage");
    }
    return RT_OK;
}

int rtk::enqueue_select(const rt_tree *t, const float4 *dq, uint64_t nq, uint64_t *d_off, uint32_t *d_ids,
                        uint64_t cap, void *work, uint64_t *d_status, hipStream_t s, bool count_only,
                        uint32_t *d_counts_out, void *const *events, uint64_t rec_bytes) {
    return enqueue_select_stage(t, dq, nq, d_off, d_ids, cap, work, d_status, s, count_only ? 1 : 3,
                                count_only ? d_counts_out : nullptr, events, count_only ? 0 : rec_bytes);
}

extern "C" int rt_range_select_device_timed(const rt_tree *t, const float *d_queries, uint64_t nq,
                                            uint64_t *d_offsets, uint32_t *d_ids, uint64_t cap, void *d_work,
                                            uint64_t work_bytes, uint64_t *d_status, void *stream,
                                            void *const *events) {
    if (!t || (nq && !d_queries) || !d_offsets || !d_work || !d_status || (cap && !d_ids))
        return fail(RT_EINVAL, "NULL argument");
    if (int rc = check_nq(nq)) return rc;
    if (work_bytes < sel_ws_bytes(nq, cap)) return fail(RT_EINVAL, "workspace too small");
    if ((reinterpret_cast<uintptr_t>(d_queries) & 15) != 0) return fail(RT_EINVAL, "queries not 16-byte aligned");
    DevSet ds(t->device);
    return enqueue_select(t, reinterpret_cast<const float4 *>(d_queries), nq, d_offsets, d_ids, cap, d_work,
                          d_status, static_cast<hipStream_t>(stream), false, nullptr, events,
                          work_bytes - sel_ws_bytes(nq, cap));
}

extern "C" int rt_range_select_device(const rt_tree *t, const float *d_queries, uint64_t nq, uint64_t *d_offsets,
                                      uint32_t *d_ids, uint64_t cap, void *d_work, uint64_t work_bytes,
                                      uint64_t *d_status, void *stream) {
    return rt_range_select_device_timed(t, d_queries, nq, d_offsets, d_ids, cap, d_work, work_bytes, d_status,
                                        stream, nullptr);
}

// The two stages of rt_range_select_device as separate calls (the server
// sizes and places each batch's output between them).
static int check_stage_args(const rt_tree *t, const float *d_queries, uint64_t nq, const void *d_offsets,
                            const void *d_work) {
    if (!t || (nq && !d_queries) || !d_offsets || !d_work) return fail(RT_EINVAL, "NULL argument");
    if (int rc = check_nq(nq)) return rc;
    if ((reinterpret_cast<uintptr_t>(d_queries) & 15) != 0) return fail(RT_EINVAL, "queries not 16-byte aligned");
    return RT_OK;
}

extern "C" int rt_range_select_device_count(const rt_tree *t, const float *d_queries, uint64_t nq,
                                            uint64_t *d_offsets, void *d_work, uint64_t work_bytes, void *stream) {
    if (int rc = check_stage_args(t, d_queries, nq, d_offsets, d_work)) return rc;
    if (work_bytes < sel_ws_bytes(nq, 0)) return fail(RT_EINVAL, "workspace too small");
    DevSet ds(t->device);
    // the workspace past the count stage's own layout holds its records
    return enqueue_select_stage(t, reinterpret_cast<const float4 *>(d_queries), nq, d_offsets, nullptr, 0, d_work,
                                nullptr, static_cast<hipStream_t>(stream), 1, nullptr, nullptr,
                                work_bytes - sel_ws_bytes(nq, 0));
}

extern "C" int rt_range_select_device_fill(const rt_tree *t, const float *d_queries, uint64_t nq,
                                           uint64_t *d_offsets, uint32_t *d_ids, uint64_t cap, void *d_work,
                                           uint64_t work_bytes, uint64_t *d_status, void *stream) {
    if (int rc = check_stage_args(t, d_queries, nq, d_offsets, d_work)) return rc;
    if (!d_status || (cap && !d_ids)) return fail(RT_EINVAL, "NULL argument");
    if (work_bytes < sel_ws_bytes(nq, cap)) return fail(RT_EINVAL, "workspace too small");
    DevSet ds(t->device);
    return enqueue_select_stage(t, reinterpret_cast<const float4 *>(d_queries), nq, d_offsets, d_ids, cap, d_work,
                                d_status, static_cast<hipStream_t>(stream), 2, nullptr, nullptr);
}

extern "C" int rt_range_count_device(const rt_tree *t, const float *d_queries, uint64_t nq, uint32_t *d_counts,
                                     void *d_work, uint64_t work_bytes, void *stream) {
    if (!t || (nq && !d_queries) || !d_counts || !d_work) return fail(RT_EINVAL, "NULL argument");
    if (int rc = check_nq(nq)) return rc;
    if (work_bytes < sel_ws_bytes(nq, 0)) return fail(RT_EINVAL, "workspace too small");
    if ((reinterpret_cast<uintptr_t>(d_queries) & 15) != 0) return fail(RT_EINVAL, "queries not 16-byte aligned");
    DevSet ds(t->device);
    return enqueue_select(t, reinterpret_cast<const float4 *>(d_queries), nq, nullptr, nullptr, 0, d_work, nullptr,
                          static_cast<hipStream_t>(stream), true, d_counts, nullptr);
}

int rtk::make_ids(uint64_t nq, uint64_t total, rt_ids **out) {
    void *mem = obj_alloc(KIND_IDS, sizeof(rt_ids));
    if (!mem) return fail(RT_ENOMEM, "host allocation failed");
    rt_ids *r = static_cast<rt_ids *>(mem);
    r->nq = nq;
    r->offsets = static_cast<uint64_t *>(std::malloc((nq + 1) * 8));
    r->ids = static_cast<uint32_t *>(std::malloc(total ? total * 4 : 4));
    if (!r->offsets || !r->ids) {
        rt_free(r);
        return fail(RT_ENOMEM, "host allocation failed");
    }
    r->offsets[0] = 0;
    *out = r;
    return RT_OK;
}

extern "C" int rt_range_select(const rt_tree *t, const float *queries, uint64_t nq, rt_ids **out) {
    if (!out) return fail(RT_EINVAL, "out is NULL");
    *out = nullptr;
    if (!t) return fail(RT_EINVAL, "tree is NULL");
    try {
        if (int rc = check_nq(nq)) return rc;
        if (int rc = check_rects(queries, nq, "queries")) return rc;
        DevSet ds(t->device);
        if (nq == 0) return make_ids(0, 0, out);
        DevBuf dq, doff, work, dids;
        hipError_t e = dq.alloc(nq * 16);
        if (e == hipSuccess) e = doff.alloc((nq + 1) * 8);
        if (e == hipSuccess) e = work.alloc(sel_ws_bytes(nq, 0));
        if (e == hipSuccess) e = hipMemcpy(dq.p, queries, nq * 16, hipMemcpyHostToDevice);
        if (e != hipSuccess) return hip_fail(e, "select setup");
        // count stage, then size the output exactly and run the fill stage
        SelWs w = sel_ws(work.p, nq);
        hipStream_t s = nullptr;
        int rc = enqueue_select_stage(t, static_cast<const float4 *>(dq.p), nq, static_cast<uint64_t *>(doff.p),
                                      nullptr, 0, work.p, nullptr, s, 1, nullptr, nullptr);
        if (rc) return rc;
        uint64_t total = 0;
        e = hipMemcpy(&total, static_cast<uint64_t *>(doff.p) + nq, 8, hipMemcpyDeviceToHost);
        if (e != hipSuccess) return hip_fail(e, "count pass");
        DevBuf work2;
        e = dids.alloc(total * 4);
        if (e == hipSuccess) e = work2.alloc(sel_ws_bytes(nq, total));
        if (e == hipSuccess) e = hipMemcpy(work2.p, work.p, sel_ws_bytes(nq, 0), hipMemcpyDeviceToDevice);
        if (e != hipSuccess) return hip_fail(e, "allocating the result");
        w = sel_ws(work2.p, nq);
        rc = enqueue_select_stage(t, static_cast<const float4 *>(dq.p), nq, static_cast<uint64_t *>(doff.p),
                                  static_cast<uint32_t *>(dids.p), total, work2.p, nullptr, s, 2, nullptr, nullptr);
        if (rc) return rc;
        Ctrl hc;
        e = hipMemcpy(&hc, w.ctrl, sizeof(Ctrl), hipMemcpyDeviceToHost);
        if (e != hipSuccess) return hip_fail(e, "fill pass");
        if (hc.err) return fail(RT_EDEVICE, "kernel check failed (flags %u)", hc.err);
        rt_ids *r = nullptr;
        if (int rc = make_ids(nq, total, &r)) return rc;
        e = hipMemcpy(r->offsets, doff.p, (nq + 1) * 8, hipMemcpyDeviceToHost);
        if (e == hipSuccess && total) e = hipMemcpy(r->ids, dids.p, total * 4, hipMemcpyDeviceToHost);
        if (e != hipSuccess) {
            rt_free(r);
            return hip_fail(e, "copying the result");
        }
        *out = r;
        return RT_OK;
    } catch (const std::bad_alloc &) {
        return fail(RT_ENOMEM, "host allocation failed");
    } catch (...) {
        return fail(RT_EDEVICE, "unexpected failure");
    }
}

extern "C" int rt_select_visit_stats(const rt_tree *t, const float *queries, uint64_t nq, uint64_t *vnodes,
                                     uint64_t *ventries, uint64_t *vcontained) {
    if (!t || !vnodes || !ventries) return fail(RT_EINVAL, "NULL argument");
    *vnodes = *ventries = 0;
    if (vcontained) *vcontained = 0;
    if (int rc = check_nq(nq)) return rc;
    if (int rc = check_rects(queries, nq, "queries")) return rc;
    if (nq == 0) return RT_OK;
    DevSet ds(t->device);
    DevBuf dq, work;
    hipError_t e = dq.alloc(nq * 16);
    if (e == hipSuccess) e = work.alloc(sel_ws_bytes(nq, 0));
    if (e == hipSuccess) e = hipMemcpy(dq.p, queries, nq * 16, hipMemcpyHostToDevice);
    SelWs w = sel_ws(work.p, nq);
    if (e == hipSuccess) e = launch_zero(w.ctrl, sizeof(Ctrl), nullptr);
    if (e == hipSuccess)
        e = launch_select_pass(view_of(t), static_cast<const float4 *>(dq.p), (uint32_t)nq, SEL_STATS, w.counts,
                               nullptr, nullptr, 0, w.ctrl, 2, SelectPlan(), (uint32_t)nq, nullptr);
    Ctrl hc;
    if (e == hipSuccess) e = hipMemcpy(&hc, w.ctrl, sizeof(Ctrl), hipMemcpyDeviceToHost);
    if (e != hipSuccess) return hip_fail(e, "visit statistics");
    if (hc.err) return fail(RT_EDEVICE, "kernel check failed (flags %u)", hc.err);
    *vnodes = hc.stats[0];
    *ventries = hc.stats[1];
    if (vcontained) *vcontained = hc.stats[2];
    return RT_OK;
}
