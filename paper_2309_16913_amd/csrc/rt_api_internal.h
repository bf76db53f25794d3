// Host-side internals shared by the C-ABI translation units.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

#include "../../include/rt.h"
#include "rt_internal.h"

struct rt_tree {
    int device = 0;
    uint32_t fanout = 0, layout = 0, height = 0, n_nodes = 0, first_leaf = 0, node_bytes = 0;
    uint64_t n_objects = 0, n_entries = 0;
    float mbr[4] = {0, 0, 0, 0};
    uint32_t level_start[33] = {0};   // first node index of each level (0 = leaves)
    uint32_t sorted_lx = 0;           // 1: every node's entries ascend in low x
    uint32_t lookahead = 0;           // 1: select loads the next node ahead after a leaf
    uint32_t bulk_copy = 0;           // RT_BULK_AUTO / ON / OFF: deferral of long contained runs
    uint32_t replay = 1;              // 1: one-call selects replay the count pass's records
    uint32_t split_kmin = 0;          // mapping: split queries reaching >= this many
                                      // parents-of-leaves (0 = one group per query)
    void *d_nodes = nullptr;   // n_nodes * node_bytes
    void *d_meta = nullptr;    // n_nodes uint32: count | level << 8
    void *d_range = nullptr;   // n_nodes uint2: leaves [x, y) under the node
    void *d_leaf_ids = nullptr;   // n_objects uint32: the leaves' ids, leaf after leaf
    uint32_t partial_leaf = 0xFFFFFFFFu, partial_cnt = 0;   // the leaf with < F entries, if any
};

namespace rtk {

constexpr uint32_t kObjMagic = 0x52544f42u;   // "RTOB"
enum : uint32_t { KIND_TREE = 1, KIND_IDS = 2, KIND_PAIRS = 3, KIND_BATCH = 4 };

// Every object handed out through the ABI is preceded by this header so that
// rt_free can tell what it is.
struct alignas(16) ObjHdr {
    uint32_t magic;
    uint32_t kind;
    uint64_t pad;
};

int fail(int code, const char *fmt, ...);
int hip_fail(hipError_t e, const char *what);
void *obj_alloc(uint32_t kind, size_t bytes);
void tree_release(rt_tree *t);
void batch_release(rt_batch *b);
int check_rects(const float *r, uint64_t n, const char *what);
TreeView view_of(const rt_tree *t);
// STR bulk load of n device rectangles (validated again on the device) on
// stream s; returns after the build has finished.
int build_str_on_device(const float4 *d_rects, uint64_t n, uint32_t fanout, uint32_t layout, bool sort_lx,
                        hipStream_t s, rt_tree **out);
// fanout 0 and/or layout RT_LAYOUT_AUTO: build every candidate, time a probe
// select on each and keep the fastest (choice cached per key).
int build_tuned(const float4 *d_rects, uint64_t n, uint32_t fanout, uint32_t layout, bool sort_lx, hipStream_t s,
                rt_tree **out);
int make_ids(uint64_t nq, uint64_t total, rt_ids **out);
// stage bit 1: count stage (order, split, count pass, offsets); bit 2: fill
// stage (fill pass, sort, status).  d_counts_out: count-only mode.
// rec_bytes: workspace bytes past the select's own layout for (nq, cap) that
// may hold the count pass's records (both stages in one call only; 0: none).
int enqueue_select_stage(const rt_tree *t, const float4 *dq, uint64_t nq, uint64_t *d_off, uint32_t *d_ids,
                         uint64_t cap, void *work, uint64_t *d_status, hipStream_t s, int stage,
                         uint32_t *d_counts_out, void *const *events, uint64_t rec_bytes = 0);
int enqueue_select(const rt_tree *t, const float4 *dq, uint64_t nq, uint64_t *d_off, uint32_t *d_ids,
                   uint64_t cap, void *work, uint64_t *d_status, hipStream_t s, bool count_only,
                   uint32_t *d_counts_out, void *const *events = nullptr, uint64_t rec_bytes = 0);
// Workspace bytes of a select for (nq, cap) without and with room for the
// records of the count pass.
uint64_t select_ws_bytes(uint64_t nq, uint64_t cap);
uint64_t select_replay_ws_bytes(uint64_t nq, uint64_t cap);
// Record arena for nq queries and cap ids (records, then one count per
// chunk), and the chunks an arena of `bytes` holds.
uint64_t rec_arena_bytes(uint64_t nq, uint64_t cap);
uint32_t rec_chunks_in(uint64_t bytes);

// Owning device buffer.
struct DevBuf {
    void *p = nullptr;
    DevBuf() = default;
    DevBuf(const DevBuf &) = delete;
    DevBuf &operator=(const DevBuf &) = delete;
    ~DevBuf();
    hipError_t alloc(size_t bytes);
};

// Make a device current for a scope.
struct DevSet {
    int prev = 0;
    explicit DevSet(int dev) {
        (void)hipGetDevice(&prev);
        if (prev != dev) (void)hipSetDevice(dev);
    }
    ~DevSet() {
        int cur = 0;
        (void)hipGetDevice(&cur);
        if (cur != prev) (void)hipSetDevice(prev);
    }
};

}  // namespace rtk
