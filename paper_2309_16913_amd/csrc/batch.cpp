// Batched range select over many independent trees.
//
// rt_batch_create copies every instance's queries to the device, orders each
// tree's queries by the Morton code of their centres, builds per-XCD work
// lists of (tree, query-chunk) items (trees by decreasing estimated cost, so
// the long items start early and the tail stays short; a tree's items on one
// XCD unless it is large), runs one
// count pass to size the output pool, and captures the whole select -- zero
// the counters, persistent count pass, scan, persistent fill pass, segmented
// sort, status -- into one HIP graph.  rt_batch_run replays that graph.
// rt_batch_run_plain does the same work as one launch sequence per tree, in
// order, with no persistence and no graph: the baseline the batched form is
// measured against.
#include <algorithm>
#include <cmath>
#include <cstdlib>
#include <cstring>
#include <new>
#include <numeric>
#include <vector>

#include "rt_api_internal.h"

using namespace rtk;

struct rt_batch {
    int device = 0;
    uint32_t ntrees = 0, nitems = 0, wave_words = 0;
    uint64_t total_q = 0, cap = 0;
    bool last_plain = false;
    std::vector<const rt_tree *> trees;
    std::vector<uint64_t> q_begin, nq, id_base, id_count, plain_begin;
    void *d_trees = nullptr, *d_items = nullptr, *d_q = nullptr, *d_counts = nullptr, *d_off = nullptr;
    void *d_ids = nullptr, *d_scratch = nullptr, *d_ctrl = nullptr, *d_scan = nullptr, *d_status = nullptr;
    void *d_plain_off = nullptr, *d_lists = nullptr;
    void *d_qrange = nullptr;   // per query: its tree's object count (the bound of its ids)
    void *d_qorder = nullptr;   // per position of a tree's processing order: the local query index
    void *d_list_begin = nullptr;   // kXcds + 1 item list bounds
    void *d_qtree = nullptr;        // per query: its tree's index
    void *d_rec = nullptr;          // record arena of the recording count pass
    uint32_t rec_nchunks = 0;
    bool replay = true;             // the graph's fill replays the count pass's records
    uint64_t id_range = 0;   // largest object count of the batch's trees
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
};

void rtk::batch_release(rt_batch *b) {
    if (!b) return;
    DevSet ds(b->device);
    if (b->exec) (void)hipGraphExecDestroy(b->exec);
    if (b->graph) (void)hipGraphDestroy(b->graph);
    void *bufs[] = {b->d_trees, b->d_items, b->d_q,    b->d_counts, b->d_off,       b->d_ids,
                    b->d_scratch, b->d_ctrl, b->d_scan, b->d_status, b->d_plain_off, b->d_lists,
                    b->d_qrange, b->d_qorder, b->d_list_begin, b->d_qtree, b->d_rec};
    for (void *p : bufs)
        if (p) (void)hipFree(p);
    b->~rt_batch();
}

static hipError_t dmalloc(void **p, size_t bytes) { return hipMalloc(p, bytes ? bytes : 16); }

// The record arena as the kernels take it (rec = NULL: no records).
static BatchRec batch_rec(const rt_batch *b) {
    BatchRec r;
    if (!b->replay || !b->d_rec || !b->rec_nchunks) return r;
    for (const rt_tree *t : b->trees)
        if (t->n_nodes >= (1u << 30)) return r;   // node indices must leave the flag bits free
    r.rec = static_cast<uint4 *>(b->d_rec);
    r.rec_count = reinterpret_cast<uint32_t *>(static_cast<uint8_t *>(b->d_rec) +
                                               ((16ull * kRecChunk * b->rec_nchunks + 255) & ~255ull));
    r.rec_nchunks = b->rec_nchunks;
    return r;
}

// Persistent count pass (recording with rp.rec) + scan over all instances' queries.
static hipError_t enqueue_count_scan(rt_batch *b, hipStream_t s, const BatchRec &rp = BatchRec()) {
    Ctrl *ctrl = static_cast<Ctrl *>(b->d_ctrl);
    hipError_t e = launch_zero(ctrl, sizeof(Ctrl), s);
    if (e == hipSuccess)
        e = launch_batch_pass(static_cast<BatchTree *>(b->d_trees), static_cast<BatchItem *>(b->d_items),
                              static_cast<const uint32_t *>(b->d_list_begin), b->nitems,
                              static_cast<const uint32_t *>(b->d_qorder), static_cast<float4 *>(b->d_q), SEL_COUNT,
                              static_cast<uint32_t *>(b->d_counts), nullptr, nullptr, 0, b->total_q, ctrl, 0,
                              b->wave_words, rp, s);
    if (e == hipSuccess)
        e = launch_scan_u32(static_cast<uint32_t *>(b->d_counts), b->total_q, static_cast<uint64_t *>(b->d_off),
                            static_cast<uint64_t *>(b->d_scan), s);
    return e;
}

static hipError_t enqueue_all(rt_batch *b, hipStream_t s) {
    BatchRec rp = batch_rec(b);
    hipError_t e = enqueue_count_scan(b, s, rp);
    Ctrl *ctrl = static_cast<Ctrl *>(b->d_ctrl);
    if (e == hipSuccess && rp.rec) {   // replay the records; the walk runs only if they overflowed
        e = launch_batch_replay(static_cast<BatchTree *>(b->d_trees), static_cast<const uint32_t *>(b->d_qtree), rp,
                                static_cast<uint64_t *>(b->d_off), b->total_q, static_cast<uint32_t *>(b->d_ids),
                                b->cap, ctrl, s);
        rp.fill_guard = 1;
    }
    if (e == hipSuccess)
        e = launch_batch_pass(static_cast<BatchTree *>(b->d_trees), static_cast<BatchItem *>(b->d_items),
                              static_cast<const uint32_t *>(b->d_list_begin), b->nitems,
                              static_cast<const uint32_t *>(b->d_qorder), static_cast<float4 *>(b->d_q), SEL_FILL,
                              static_cast<uint32_t *>(b->d_counts), static_cast<uint64_t *>(b->d_off),
                              static_cast<uint32_t *>(b->d_ids), b->cap, b->total_q, ctrl, 1, b->wave_words, rp, s);
    if (e == hipSuccess)
        e = launch_segsort(static_cast<uint64_t *>(b->d_off), b->total_q, static_cast<uint32_t *>(b->d_ids),
                           static_cast<uint32_t *>(b->d_scratch), b->cap, static_cast<uint32_t *>(b->d_lists),
                           b->id_range, static_cast<const uint32_t *>(b->d_qrange), s);
    if (e == hipSuccess)
        e = launch_finalize(static_cast<uint64_t *>(b->d_off), b->total_q, b->cap, ctrl,
                            static_cast<uint64_t *>(b->d_status), s);
    return e;
}

// (Re)capture the whole select into the batch's graph.
static hipError_t capture(rt_batch *b) {
    if (b->exec) (void)hipGraphExecDestroy(b->exec);
    if (b->graph) (void)hipGraphDestroy(b->graph);
    b->exec = nullptr;
    b->graph = nullptr;
    hipStream_t cs = nullptr;
    hipError_t e = hipStreamCreateWithFlags(&cs, hipStreamNonBlocking);
    if (e == hipSuccess) e = hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal);
    if (e == hipSuccess) {
        hipError_t e2 = enqueue_all(b, cs);
        e = hipStreamEndCapture(cs, &b->graph);
        if (e2 != hipSuccess) e = e2;
    }
    if (e == hipSuccess) e = hipGraphInstantiate(&b->exec, b->graph, nullptr, nullptr, 0);
    if (cs) (void)hipStreamDestroy(cs);
    return e;
}

extern "C" int rt_batch_create(const rt_tree *const *trees, uint32_t ntrees, const float *const *queries,
                               const uint64_t *nq, uint64_t ids_capacity, rt_batch **out) {
    if (!out) return fail(RT_EINVAL, "out is NULL");
    *out = nullptr;
    if (ntrees && (!trees || !queries || !nq)) return fail(RT_EINVAL, "NULL argument");
    try {
        int dev = 0;
        (void)hipGetDevice(&dev);
        uint64_t total = 0;
        for (uint32_t i = 0; i < ntrees; ++i) {
            if (!trees[i]) return fail(RT_EINVAL, "tree %u is NULL", i);
            if (trees[i]->device != dev) return fail(RT_EINVAL, "tree %u is not on the current device", i);
            if (int rc = check_rects(queries[i], nq[i], "queries")) return rc;
            total += nq[i];
        }
        if (total > 0xFFF00000ull) return fail(RT_EINVAL, "too many queries");
        void *mem = obj_alloc(KIND_BATCH, sizeof(rt_batch));
        if (!mem) return fail(RT_ENOMEM, "host allocation failed");
        rt_batch *b = new (mem) rt_batch();
        auto bail = [&](int rc) {
            rt_free(b);
            return rc;
        };
        b->device = dev;
        b->ntrees = ntrees;
        b->total_q = total;
        b->trees.assign(trees, trees + ntrees);
        b->q_begin.resize(ntrees);
        b->nq.assign(nq, nq + ntrees);
        // descriptors and work items
        std::vector<BatchTree> bt(ntrees);
        struct Cand {
            BatchItem it;
            double cost;
        };
        std::vector<std::vector<Cand>> per_tree(ntrees);
        std::vector<double> tree_cost(ntrees, 0.0);
        std::vector<float> hq((size_t)total * 4);
        std::vector<uint32_t> hrange((size_t)total), horder((size_t)total), htree((size_t)total);
        std::vector<uint64_t> code;
        uint64_t qb = 0;
        for (uint32_t i = 0; i < ntrees; ++i) {
            const rt_tree *t = trees[i];
            bt[i].t = view_of(t);
            bt[i].q_begin = qb;
            bt[i].nq = (uint32_t)nq[i];
            bt[i].stack_cap = stack_bound(t->height, t->fanout);
            b->q_begin[i] = qb;
            b->id_range = std::max<uint64_t>(b->id_range, t->n_objects);
            const uint32_t G = group_width(t->fanout);
            b->wave_words = std::max(b->wave_words, (64 / G) * bt[i].stack_cap);
            if (nq[i]) std::memcpy(hq.data() + 4 * qb, queries[i], nq[i] * 16);
            std::fill(hrange.begin() + qb, hrange.begin() + qb + nq[i],
                      (uint32_t)std::min<uint64_t>(t->n_objects, 0xFFFFFFFFull));
            std::fill(htree.begin() + qb, htree.begin() + qb + nq[i], i);
            // processing order: Morton code of the window centres on a
            // 65536 x 65536 grid over the tree's MBR (only the order of the
            // work depends on it)
            const double mw = (double)t->mbr[2] - t->mbr[0], mh = (double)t->mbr[3] - t->mbr[1];
            const bool grid = mw > 0 && mh > 0 && mw < 1e300 && mh < 1e300;
            code.resize(nq[i]);
            for (uint64_t k = 0; k < nq[i]; ++k) {
                const float *w = queries[i] + 4 * k;
                uint64_t c = 0;
                if (grid) {
                    double cx = ((0.5 * w[0] + 0.5 * w[2]) - t->mbr[0]) / mw * 65535.0;
                    double cy = ((0.5 * w[1] + 0.5 * w[3]) - t->mbr[1]) / mh * 65535.0;
                    cx = cx > 0 ? (cx < 65535.0 ? cx : 65535.0) : 0.0;   // NaN -> 0
                    cy = cy > 0 ? (cy < 65535.0 ? cy : 65535.0) : 0.0;
                    const uint32_t ix = (uint32_t)cx, iy = (uint32_t)cy;
                    for (int bit = 0; bit < 16; ++bit)
                        c |= (uint64_t)((ix >> bit) & 1u) << (2 * bit) | (uint64_t)((iy >> bit) & 1u) << (2 * bit + 1);
                }
                code[k] = (c << 32) | k;
            }
            std::sort(code.begin(), code.end());
            for (uint64_t k = 0; k < nq[i]; ++k) horder[qb + k] = (uint32_t)(code[k] & 0xFFFFFFFFu);
            // chunks of 8 queries per group in that order; cost ~ expected
            // hits + per-query path length (window area as a fraction of the
            // tree's MBR)
            const uint32_t chunk = 8 * (64 / G);
            const double area = grid ? mw * mh : 1.0;
            for (uint64_t q0 = 0; q0 < nq[i]; q0 += chunk) {
                const uint64_t q1 = std::min<uint64_t>(nq[i], q0 + chunk);
                double c = 0;
                for (uint64_t k = q0; k < q1; ++k) {
                    const float *w = queries[i] + 4 * horder[qb + k];
                    double a = (double)(w[2] - w[0]) * (double)(w[3] - w[1]) / area;
                    if (!(a < 1.0)) a = 1.0;
                    c += a * (double)t->n_objects / t->fanout + t->height;
                }
                per_tree[i].push_back({BatchItem{i, (uint32_t)q0, (uint32_t)q1, 0u}, c});
                tree_cost[i] += c;
            }
            qb += nq[i];
        }
        // XCD lists: trees by decreasing cost; a tree costing more than half
        // of an XCD's fair share is cut into kXcds runs of its order (one per
        // XCD), every other tree goes whole to the least loaded XCD
        double all = 0;
        for (double c : tree_cost) all += c;
        std::vector<uint32_t> by_cost(ntrees);
        std::iota(by_cost.begin(), by_cost.end(), 0u);
        std::stable_sort(by_cost.begin(), by_cost.end(),
                         [&](uint32_t x, uint32_t y) { return tree_cost[x] > tree_cost[y]; });
        std::vector<std::vector<BatchItem>> lists(kXcds);
        std::vector<double> load(kXcds, 0.0);
        for (uint32_t i : by_cost) {
            const auto &its = per_tree[i];
            if (its.empty()) continue;
            if (tree_cost[i] > 0.5 * all / kXcds && its.size() >= kXcds) {
                double acc = 0;
                for (const Cand &c : its) {
                    const uint32_t x = std::min<uint32_t>(kXcds - 1, (uint32_t)(acc / tree_cost[i] * kXcds));
                    lists[x].push_back(c.it);
                    load[x] += c.cost;
                    acc += c.cost;
                }
            } else {
                const uint32_t x = (uint32_t)(std::min_element(load.begin(), load.end()) - load.begin());
                for (const Cand &c : its) lists[x].push_back(c.it);
                load[x] += tree_cost[i];
            }
        }
        std::vector<BatchItem> items;
        std::vector<uint32_t> list_begin(kXcds + 1, 0);
        for (uint32_t x = 0; x < kXcds; ++x) {
            list_begin[x] = (uint32_t)items.size();
            items.insert(items.end(), lists[x].begin(), lists[x].end());
        }
        list_begin[kXcds] = (uint32_t)items.size();
        b->nitems = (uint32_t)items.size();

        hipError_t e = dmalloc(&b->d_trees, bt.size() * sizeof(BatchTree));
        if (e == hipSuccess) e = dmalloc(&b->d_items, items.size() * sizeof(BatchItem));
        if (e == hipSuccess) e = dmalloc(&b->d_q, total * 16);
        if (e == hipSuccess) e = dmalloc(&b->d_counts, total * 4);
        if (e == hipSuccess) e = dmalloc(&b->d_off, (total + 1) * 8);
        if (e == hipSuccess) e = dmalloc(&b->d_ctrl, sizeof(Ctrl));
        if (e == hipSuccess) e = dmalloc(&b->d_scan, scan_tmp_elems(std::max<uint64_t>(total, 1)) * 8);
        if (e == hipSuccess) e = dmalloc(&b->d_status, 16);
        if (e == hipSuccess) e = dmalloc(&b->d_lists, segsort_ws_elems(std::max<uint64_t>(total, 1)) * 4);
        if (e == hipSuccess) e = dmalloc(&b->d_qrange, std::max<uint64_t>(total, 1) * 4);
        if (e == hipSuccess) e = dmalloc(&b->d_qorder, std::max<uint64_t>(total, 1) * 4);
        if (e == hipSuccess) e = dmalloc(&b->d_list_begin, (kXcds + 1) * 4);
        if (e == hipSuccess) e = dmalloc(&b->d_qtree, std::max<uint64_t>(total, 1) * 4);
        uint64_t plain_total = 0;
        b->plain_begin.resize(ntrees);
        for (uint32_t i = 0; i < ntrees; ++i) {
            b->plain_begin[i] = plain_total;
            plain_total += nq[i] + 1;
        }
        if (e == hipSuccess) e = dmalloc(&b->d_plain_off, plain_total * 8);
        if (e == hipSuccess) e = hipMemcpy(b->d_trees, bt.data(), bt.size() * sizeof(BatchTree), hipMemcpyHostToDevice);
        if (e == hipSuccess && !items.empty())
            e = hipMemcpy(b->d_items, items.data(), items.size() * sizeof(BatchItem), hipMemcpyHostToDevice);
        if (e == hipSuccess && total) e = hipMemcpy(b->d_q, hq.data(), total * 16, hipMemcpyHostToDevice);
        if (e == hipSuccess && total)
            e = hipMemcpy(b->d_qrange, hrange.data(), total * 4, hipMemcpyHostToDevice);
        if (e == hipSuccess && total)
            e = hipMemcpy(b->d_qorder, horder.data(), total * 4, hipMemcpyHostToDevice);
        if (e == hipSuccess && total) e = hipMemcpy(b->d_qtree, htree.data(), total * 4, hipMemcpyHostToDevice);
        if (e == hipSuccess)
            e = hipMemcpy(b->d_list_begin, list_begin.data(), (kXcds + 1) * 4, hipMemcpyHostToDevice);
        if (e != hipSuccess) return bail(hip_fail(e, "batch setup"));

        // one eager count pass: output size and the per-instance bases
        e = enqueue_count_scan(b, nullptr);
        std::vector<uint64_t> off(total + 1);
        if (e == hipSuccess) e = hipMemcpy(off.data(), b->d_off, (total + 1) * 8, hipMemcpyDeviceToHost);
        if (e != hipSuccess) return bail(hip_fail(e, "batch sizing"));
        b->id_base.resize(ntrees);
        b->id_count.resize(ntrees);
        for (uint32_t i = 0; i < ntrees; ++i) {
            b->id_base[i] = off[b->q_begin[i]];
            b->id_count[i] = off[b->q_begin[i] + nq[i]] - off[b->q_begin[i]];
        }
        b->cap = ids_capacity ? ids_capacity : off[total];
        e = dmalloc(&b->d_ids, b->cap * 4);
        if (e == hipSuccess) e = dmalloc(&b->d_scratch, segsort_scratch_elems(b->cap) * 4);
        // the record arena for the count pass inside the graph
        const uint64_t rb = rec_arena_bytes(total, b->cap);
        if (e == hipSuccess) e = dmalloc(&b->d_rec, rb);
        b->rec_nchunks = rec_chunks_in(rb);
        if (e != hipSuccess) return bail(hip_fail(e, "batch output pool"));

        // capture the whole select into a graph
        e = capture(b);
        if (e != hipSuccess) return bail(hip_fail(e, "batch graph capture"));
        *out = b;
        return RT_OK;
    } catch (const std::bad_alloc &) {
        return fail(RT_ENOMEM, "host allocation failed");
    } catch (...) {
        return fail(RT_EDEVICE, "unexpected failure");
    }
}

extern "C" int rt_batch_set_replay(rt_batch *b, uint32_t on) {
    if (!b) return fail(RT_EINVAL, "batch is NULL");
    if (on > 1) return fail(RT_EINVAL, "replay %u is not 0 or 1", on);
    DevSet ds(b->device);
    b->replay = on != 0;
    const hipError_t e = capture(b);
    return e == hipSuccess ? RT_OK : hip_fail(e, "batch graph capture");
}

extern "C" int rt_batch_replay_info(rt_batch *b, uint32_t *chunks, uint32_t *overflowed) {
    if (!b || !chunks || !overflowed) return fail(RT_EINVAL, "NULL argument");
    DevSet ds(b->device);
    Ctrl hc;
    hipError_t e = hipDeviceSynchronize();
    if (e == hipSuccess) e = hipMemcpy(&hc, b->d_ctrl, sizeof(Ctrl), hipMemcpyDeviceToHost);
    if (e != hipSuccess) return hip_fail(e, "batch replay info");
    *chunks = b->last_plain ? 0u : hc.rec_chunks;
    *overflowed = b->last_plain ? 0u : hc.rec_overflow;
    return RT_OK;
}

extern "C" int rt_batch_run(rt_batch *b, void *stream) {
    if (!b) return fail(RT_EINVAL, "batch is NULL");
    DevSet ds(b->device);
    b->last_plain = false;
    hipError_t e = hipGraphLaunch(b->exec, static_cast<hipStream_t>(stream));
    return e == hipSuccess ? RT_OK : hip_fail(e, "graph launch");
}

extern "C" int rt_batch_run_plain(rt_batch *b, void *stream) {
    if (!b) return fail(RT_EINVAL, "batch is NULL");
    DevSet ds(b->device);
    b->last_plain = true;
    hipStream_t s = static_cast<hipStream_t>(stream);
    Ctrl *ctrl = static_cast<Ctrl *>(b->d_ctrl);
    uint32_t *ids = static_cast<uint32_t *>(b->d_ids);
    uint32_t *scratch = static_cast<uint32_t *>(b->d_scratch);
    hipError_t e = launch_zero(ctrl, sizeof(Ctrl), s);
    for (uint32_t i = 0; i < b->ntrees && e == hipSuccess; ++i) {
        const uint64_t n = b->nq[i];
        if (!n) continue;
        const TreeView v = view_of(b->trees[i]);
        const float4 *q = static_cast<float4 *>(b->d_q) + b->q_begin[i];
        uint32_t *counts = static_cast<uint32_t *>(b->d_counts) + b->q_begin[i];
        uint64_t *off = static_cast<uint64_t *>(b->d_plain_off) + b->plain_begin[i];
        const uint64_t base = b->id_base[i], cnt = b->id_count[i];
        const uint64_t cap = base < b->cap ? std::min<uint64_t>(cnt, b->cap - base) : 0;
        e = launch_zero(ctrl->work, sizeof(ctrl->work), s);
        if (e == hipSuccess) e = launch_zero(ctrl->xwork, sizeof(ctrl->xwork) + sizeof(ctrl->hwork), s);
        if (e == hipSuccess) e = launch_select_pass(v, q, (uint32_t)n, SEL_COUNT, counts, nullptr, nullptr, 0, ctrl, 0, SelectPlan(),
                                                    (uint32_t)n, s);
        if (e == hipSuccess) e = launch_scan_u32(counts, n, off, static_cast<uint64_t *>(b->d_scan), s);
        if (e == hipSuccess)
            e = launch_select_pass(v, q, (uint32_t)n, SEL_FILL, counts, off, ids + base, cap, ctrl, 1, SelectPlan(),
                                   (uint32_t)n, s);
        if (e == hipSuccess)
            e = launch_segsort(off, n, ids + base, scratch + base, cap, static_cast<uint32_t *>(b->d_lists),
                               b->trees[i]->n_objects, nullptr, s);
    }
    return e == hipSuccess ? RT_OK : hip_fail(e, "plain batch launches");
}

extern "C" int rt_batch_status(rt_batch *b, uint64_t *total, uint64_t *flags) {
    if (!b || !total || !flags) return fail(RT_EINVAL, "NULL argument");
    DevSet ds(b->device);
    hipError_t e = hipDeviceSynchronize();
    if (b->last_plain) {
        // the totals the plain launches computed, tree by tree (each tree's
        // output range was sized by the creation-time count pass)
        Ctrl hc;
        if (e == hipSuccess) e = hipMemcpy(&hc, b->d_ctrl, sizeof(Ctrl), hipMemcpyDeviceToHost);
        uint64_t t = 0, over = 0;
        for (uint32_t i = 0; i < b->ntrees && e == hipSuccess; ++i) {
            if (!b->nq[i]) continue;
            uint64_t last = 0;
            e = hipMemcpy(&last, static_cast<uint64_t *>(b->d_plain_off) + b->plain_begin[i] + b->nq[i], 8,
                          hipMemcpyDeviceToHost);
            t += last;
            if (last > b->id_count[i] || b->id_base[i] + last > b->cap) over = 1;
        }
        if (e != hipSuccess) return hip_fail(e, "batch status");
        *total = t;
        *flags = (hc.err ? 2u : 0u) | over;
        return RT_OK;
    }
    uint64_t st[2] = {0, 0};
    if (e == hipSuccess) e = hipMemcpy(st, b->d_status, 16, hipMemcpyDeviceToHost);
    if (e != hipSuccess) return hip_fail(e, "batch status");
    *total = st[0];
    *flags = st[1];
    return RT_OK;
}

extern "C" int rt_batch_result(rt_batch *b, uint32_t i, rt_ids **out) {
    if (!out) return fail(RT_EINVAL, "out is NULL");
    *out = nullptr;
    if (!b || i >= b->ntrees) return fail(RT_EINVAL, "bad batch or index");
    try {
        DevSet ds(b->device);
        hipError_t e = hipDeviceSynchronize();
        const uint64_t n = b->nq[i];
        std::vector<uint64_t> off(n + 1);
        if (e == hipSuccess) {
            if (b->last_plain)
                e = hipMemcpy(off.data(), static_cast<uint64_t *>(b->d_plain_off) + b->plain_begin[i], (n + 1) * 8,
                              hipMemcpyDeviceToHost);
            else
                e = hipMemcpy(off.data(), static_cast<uint64_t *>(b->d_off) + b->q_begin[i], (n + 1) * 8,
                              hipMemcpyDeviceToHost);
        }
        if (e != hipSuccess) return hip_fail(e, "batch result");
        const uint64_t base = b->last_plain ? 0 : off[0];
        const uint64_t cnt = off[n] - off[0];
        const uint64_t at = b->last_plain ? b->id_base[i] : off[0];
        if (at + cnt > b->cap) return fail(RT_ENOMEM, "result exceeded the output pool");
        rt_ids *r = nullptr;
        if (int rc = make_ids(n, cnt, &r)) return rc;
        for (uint64_t k = 0; k <= n; ++k) r->offsets[k] = off[k] - base;
        if (cnt) e = hipMemcpy(r->ids, static_cast<uint32_t *>(b->d_ids) + at, cnt * 4, hipMemcpyDeviceToHost);
        if (e != hipSuccess) {
            rt_free(r);
            return hip_fail(e, "batch result");
        }
        *out = r;
        return RT_OK;
    } catch (const std::bad_alloc &) {
        return fail(RT_ENOMEM, "host allocation failed");
    }
}

extern "C" int rt_range_select_batch(const rt_tree *const *trees, uint32_t ntrees, const float *const *queries,
                                     const uint64_t *nq, rt_ids **out) {
    if (!out) return fail(RT_EINVAL, "out is NULL");
    for (uint32_t i = 0; i < ntrees; ++i) out[i] = nullptr;
    rt_batch *b = nullptr;
    if (int rc = rt_batch_create(trees, ntrees, queries, nq, 0, &b)) return rc;
    int rc = rt_batch_run(b, nullptr);
    uint64_t total = 0, flags = 0;
    if (!rc) rc = rt_batch_status(b, &total, &flags);
    if (!rc && flags) rc = fail(flags & 1 ? RT_ENOMEM : RT_EDEVICE, "batch kernels reported flags %llu",
                                (unsigned long long)flags);
    for (uint32_t i = 0; i < ntrees && !rc; ++i) rc = rt_batch_result(b, i, &out[i]);
    if (rc)
        for (uint32_t i = 0; i < ntrees; ++i) {
            rt_free(out[i]);
            out[i] = nullptr;
        }
    rt_free(b);
    return rc;
}
