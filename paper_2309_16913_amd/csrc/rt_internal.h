// Internal declarations shared by the library's host code and HIP kernels.
#pragma once

#include <hip/hip_runtime.h>

#include <cstddef>
#include <cstdint>

namespace rtk {

enum : uint32_t { LAYOUT_AOS = 0, LAYOUT_SOA = 1, LAYOUT_D2 = 3 };

// A device tree as the kernels see it.  Nodes are numbered breadth first from
// the root (node 0), so every node with index >= first_leaf is a leaf and the
// children of every internal node are contiguous (entry e points at the
// node's first child + e).  A node is 20*F bytes; unused entry slots of a
// partly filled node hold NaN rectangles, which fail every comparison and so
// never qualify.
struct TreeView {
    const uint8_t *nodes;
    uint32_t fanout;
    uint32_t node_bytes;
    uint32_t first_leaf;
    uint32_t height;
    uint32_t layout;
    uint32_t lookahead;      // 1: select loads the next node ahead after a leaf
    float mbr[4];            // MBR of the whole tree (root node)
    // per node the range [x, y) of leaves under it (leaves under a node are
    // contiguous); the one leaf with fewer than F entries (kNoNode if none)
    // and its entry count
    const uint2 *range;
    uint32_t partial_leaf, partial_cnt;
    // the object ids of all leaves, leaf after leaf in node order without
    // padding: leaf l's ids start at leaf_start(l), so the leaves of any
    // contiguous leaf range hold one contiguous run of ids
    const uint32_t *leaf_ids;
};
constexpr uint32_t kNoNode = 0xFFFFFFFFu;

constexpr uint32_t kXcds = 8;          // MI355X: 8 XCDs; workgroup i runs on XCD i % 8

// Objects under a node whose leaves are [r.x, r.y): F per leaf, less the
// missing entries of the one leaf that is not full.
__device__ __forceinline__ uint32_t subtree_objects(const TreeView &t, uint2 r) {
    uint32_t c = (r.y - r.x) * t.fanout;
    if (t.partial_leaf >= r.x && t.partial_leaf < r.y) c -= t.fanout - t.partial_cnt;
    return c;
}

// Position of leaf l's first id in TreeView::leaf_ids (l may be one past the
// last leaf: then the object count).
__device__ __forceinline__ uint64_t leaf_start(const TreeView &t, uint32_t l) {
    uint64_t s = (uint64_t)(l - t.first_leaf) * t.fanout;
    if (t.partial_leaf != kNoNode && l > t.partial_leaf) s -= t.fanout - t.partial_cnt;
    return s;
}

// Nontemporal store of an id (written once, read back only by the sort):
// it leaves L2 and the Infinity Cache to the tree nodes.
__device__ __forceinline__ void put_id(uint32_t *p, uint32_t v) { __builtin_nontemporal_store(v, p); }

// Records of the count pass are written once and read once by the fill
// stage: both bypass the caches, which keep the tree nodes.
typedef uint32_t rec_vec __attribute__((ext_vector_type(4)));
__device__ __forceinline__ void put_rec(uint4 *p, uint32_t a, uint32_t b, uint32_t c, uint32_t d) {
    rec_vec v = {a, b, c, d};
    __builtin_nontemporal_store(v, reinterpret_cast<rec_vec *>(p));
}
__device__ __forceinline__ uint4 get_rec(const uint4 *p) {
    const rec_vec v = __builtin_nontemporal_load(reinterpret_cast<const rec_vec *>(p));
    return make_uint4(v.x, v.y, v.z, v.w);
}

// Copy the ids of a run of contained leaves [l0, l1) -- one contiguous run
// of TreeView::leaf_ids -- to out[pos, pos + n) with the G lanes of a group
// (e = lane in the group).  Loads and stores are both aligned to G-id
// chunks of their own array: load chunk m holds ids m*G - sm + lane, store
// chunk k writes ids k*G - dm + lane (sm, dm: the misalignment of source and
// destination in ids), so every load instruction reads whole cache lines and
// every store instruction writes whole 64-byte granules.  A store chunk takes
// its ids from two consecutive load chunks, rotated by dl = (sm - dm) mod G
// lanes (two lane permutes).  Each round loads U+1 chunks and stores U, so a
// short run costs one memory round trip.  Returns n; writes nothing and sets
// *bad if the run would pass `end` (the caller's range).
template <uint32_t U>   // store chunks per round
__device__ __forceinline__ uint64_t copy_leaf_run(const TreeView &t, uint32_t l0, uint32_t l1,
                                                  uint32_t *__restrict__ out, uint64_t pos, uint64_t end, uint32_t e,
                                                  uint32_t G, bool *bad) {
    const uint64_t s0 = leaf_start(t, l0);
    const uint64_t n = leaf_start(t, l1) - s0;
    if (pos + n > end) {
        *bad = true;
        return n;
    }
    const uint32_t *__restrict__ src = t.leaf_ids + s0;
    uint32_t *__restrict__ dst = out + pos;
    const int64_t sm = (int64_t)((reinterpret_cast<uintptr_t>(src) >> 2) & (G - 1));
    const int64_t dm = (int64_t)((reinterpret_cast<uintptr_t>(dst) >> 2) & (G - 1));
    const int64_t o = sm >= dm ? 0 : -1;                          // first load chunk of store chunk 0
    const uint32_t dl = (uint32_t)(sm - dm + (sm >= dm ? 0 : (int64_t)G));   // rotation, in [0, G)
    const uint32_t from = ((threadIdx.x & 63u) - e) + ((e + dl) & (G - 1));  // wave lane to read
    const bool upper = e + dl >= G;                                // from the second load chunk
    const int64_t nk = ((int64_t)n + dm + G - 1) / G;              // store chunks
    for (int64_t k = 0; k < nk; k += U) {
        uint32_t L[U + 1];
#pragma unroll
        for (uint32_t u = 0; u <= U; ++u) {
            const int64_t j = (k + o + u) * (int64_t)G - sm + e;
            L[u] = (j >= 0 && j < (int64_t)n) ? src[j] : 0u;
        }
#pragma unroll
        for (uint32_t u = 0; u < U; ++u) {
            const uint32_t a = (uint32_t)__shfl((int)L[u], (int)from);
            const uint32_t b = (uint32_t)__shfl((int)L[u + 1], (int)from);
            const int64_t j = (k + u) * (int64_t)G - dm + e;
            if (j >= 0 && j < (int64_t)n) put_id(dst + j, upper ? b : a);
        }
    }
    return n;
}

// Kernel-side status words at the start of every workspace.
struct Ctrl {
    uint32_t work[8];        // work-queue counters (one per pass)
    uint32_t err;            // internal error flags
    uint32_t bulk_n;         // long contained runs deferred to the bulk copy (descriptors appended)
    uint32_t bulk_taken;     // descriptors taken by the bulk copy
    uint32_t rec_chunks;     // record chunks taken by the count pass
    uint32_t rec_overflow;   // 1: the record arena filled up (the fill walks the tree)
    uint32_t rec_nchunks;    // the count pass's record arena (0: it recorded nothing); set by the
    uint32_t pad[2];         // count stage, read by the fill stage's replay, which may be a
    uint4 *rec_base;         // separate call
    uint32_t *rec_count;
    uint64_t stats[4];       // visit statistics
    // per-pass, per-XCD query counters, one 128-byte cache line each
    uint32_t xwork[3][kXcds][32];
    // split work items live in kXcds lists (by the XCD slice of their query)
    uint32_t hwork[3][kXcds][32];    // per-pass grab counters per list
    uint32_t hlist[kXcds][32];       // items per list
    uint32_t budget_used[kXcds][32]; // items granted per list
};

constexpr uint32_t kErrStack = 1u;     // traversal stack would overflow
constexpr uint32_t kErrBounds = 2u;    // an output write would fall outside its range
constexpr uint32_t kErrInput = 4u;     // invalid rectangle found on the device

// Long contained runs are deferred to a bulk copy only on trees whose leaf-id
// array (4 bytes per object) is too large to stay in the last-level caches
// beside the output: measured on the 10M-rectangle tree the fill pass copies
// them faster in place (3.66 against 4.43 ms, fanout 64), on a 50M one the
// deferral wins (12.9 against 9.2 ms, fanout 32).
constexpr uint64_t kBulkMinObjects = 1ull << 25;
constexpr uint32_t kBulkMin = 2048;     // shortest run handed to the bulk copy
constexpr uint32_t kBulkChunk = 8192;   // ids per bulk-copy descriptor
// Descriptors a fill pass can append for an output of cap ids: a deferred
// run of n >= kBulkMin ids takes ceil(n / kBulkChunk) <= n / kBulkMin of them.
inline uint64_t bulk_capacity(uint64_t cap) { return cap / kBulkMin + 1; }

// Hand the contained leaves [l0, l1) (n ids of the leaf-id array from
// leaf_start(l0)) to the bulk copy: the group's leader reserves
// ceil(n / kBulkChunk) descriptors and the group's lanes write them.  The
// list is sized so that it cannot fill up (the deferred runs are disjoint
// ranges of the output); if it did, the reserved slots that exist get empty
// descriptors and *bad is set.  lead = the wave lane of the group's lane 0.
// Returns n; sets *bad (writes nothing) if the run would pass `end`.
__device__ __forceinline__ uint64_t defer_leaf_run(const TreeView &t, uint32_t l0, uint32_t l1, uint32_t *out,
                                                   uint64_t pos, uint64_t end, uint32_t e, uint32_t G, uint32_t lead,
                                                   uint4 *bulk, uint32_t bulk_cap, Ctrl *ctrl, bool *bad) {
    const uint64_t s0 = leaf_start(t, l0);
    const uint64_t n = leaf_start(t, l1) - s0;
    if (pos + n > end) {
        *bad = true;
        return n;
    }
    const uint32_t nd = (uint32_t)((n + kBulkChunk - 1) / kBulkChunk);
    uint32_t base = 0;
    if (e == 0) base = atomicAdd(&ctrl->bulk_n, nd);
    base = (uint32_t)__shfl((int)base, (int)lead);
    const bool fits = (uint64_t)base + nd <= bulk_cap;
    for (uint32_t k = e; k < nd; k += G) {
        if (base + k >= bulk_cap) break;
        const uint64_t off = (uint64_t)k * kBulkChunk;
        const uint64_t dst = pos + off;
        const uint32_t len = fits ? (uint32_t)min((uint64_t)kBulkChunk, n - off) : 0u;
        bulk[base + k] = make_uint4((uint32_t)(s0 + off), (uint32_t)dst, (uint32_t)(dst >> 32), len);
    }
    if (!fits) *bad = true;
    return n;
}

// Traversal stack bound for a depth-first walk that pops one node and pushes
// its qualifying children: (h-1)(F-1)+1 entries.
inline uint32_t stack_bound(uint32_t height, uint32_t fanout) {
    return height <= 1 ? 1u : (height - 1) * (fanout - 1) + 1;
}

inline uint32_t group_width(uint32_t fanout) {
    return fanout <= 16 ? 16u : (fanout <= 32 ? 32u : 64u);
}

// ---- select -------------------------------------------------------------
enum SelectMode : int { SEL_COUNT = 0, SEL_FILL = 1, SEL_STATS = 2 };

// How a traversal pass finds its work.
//   order       NULL or nq 64-bit keys whose low 32 bits list the queries in
//               processing order; XCD x takes the x-th eighth first.
//   slot_first  NULL (query q writes output slot q) or nq+1 offsets: query q
//               owns slots [slot_first[q], slot_first[q+1]).
//   heavy       split work items {query, subtree root, slot, 0} in kXcds
//               lists of hcap entries (list x: queries of order slice x,
//               length in Ctrl::hlist[x]); handed out before whole queries,
//               XCD x draining list x first.
struct SelectPlan {
    const uint64_t *order = nullptr;
    const uint64_t *slot_first = nullptr;
    const uint4 *heavy = nullptr;
    uint32_t hcap = 0;
    // fill pass: contained runs of at least kBulkMin ids are not copied by
    // the traversal but appended here as descriptors {leaf-id offset, output
    // position low, high, length <= kBulkChunk} for the bulk copy that
    // follows the pass (NULL: every run is copied in place)
    uint4 *bulk = nullptr;
    uint32_t bulk_cap = 0;
    // count pass: every leaf with hits and every contained subtree is also
    // recorded in chunks of kRecChunk records {output slot, position in the
    // slot, leaf node (| kRecHi: entries 32..63) or kRecRun | first leaf,
    // hit mask or end leaf}; rec_count[c] = records in chunk c.  The fill
    // stage replays them instead of walking the tree (NULL: no records).
    uint4 *rec = nullptr;
    uint32_t *rec_count = nullptr;
    uint32_t rec_nchunks = 0;
    // fill pass: run only if the count pass made no records or they
    // overflowed (the replay wrote everything otherwise)
    uint32_t fill_guard = 0;
};

constexpr uint32_t kRecChunk = 256;          // records per chunk a lane group takes
// records a lane group collects in LDS before storing them (128 measured no
// faster for groups of 64 lanes)
constexpr uint32_t kRecBuf = 64;
constexpr uint32_t kRecRun = 0x80000000u;    // record of a contained leaf range
constexpr uint32_t kRecHi = 0x40000000u;     // leaf record of entries 32..63
constexpr uint32_t kRecDead = 0xFFFFFFFEu;   // the group's chunk state after an overflow



// One traversal pass (persistent grid).  counts/offsets are indexed by output
// slot; noffsets = number of slots (offsets[noffsets] = total).
hipError_t launch_select_pass(const TreeView &t, const float4 *q, uint32_t nq, int mode,
                              uint32_t *counts, const uint64_t *offsets, uint32_t *ids,
                              uint64_t ids_capacity, Ctrl *ctrl, uint32_t work_slot,
                              const SelectPlan &plan, uint32_t noffsets, hipStream_t s);

// Split pre-pass (phase 0: slots per query; phase 1: work items).  Queries
// are taken in the plan's order with the same XCD slices as the passes;
// hcap: items per list (the budget of each list).
hipError_t launch_split(const TreeView &t, const float4 *q, uint32_t nq, int phase, uint32_t split_parent,
                        uint32_t kmin, uint32_t hcap, float min_area, uint32_t *nslots,
                        const uint64_t *slot_first, uint4 *heavy, const uint64_t *order, Ctrl *ctrl,
                        hipStream_t s);
hipError_t launch_gather_offsets(const uint64_t *slot_first, const uint64_t *slot_off, uint32_t nq,
                                 uint64_t *offsets, hipStream_t s);

// Query order for locality: 64-bit keys (Morton code of the window center
// over the tree's MBR) << 32 | query index, sorted.  tmp: 2*nq uint64 plus
// radix temporaries (order_ws_bytes).  *sorted receives the sorted keys.
uint64_t order_ws_bytes(uint64_t nq);
const uint64_t *query_order_result(const void *ws, uint64_t nq);   // where the sorted keys end up
hipError_t launch_query_order(const float4 *q, uint32_t nq, const float *mbr, void *ws,
                              const uint64_t **sorted, hipStream_t s);
constexpr uint32_t kOrderMinQueries = 8192;   // smaller batches keep input order

// Bulk copy of the long contained runs a fill pass deferred (descriptors in
// bulk[0 .. min(ctrl->bulk_n, bulk_cap))) into ids: persistent grid, one block
// per descriptor at a time.  Enqueue right after that fill pass.
// Store the plan's record arena in the control words (after they are zeroed).
hipError_t launch_set_rec(Ctrl *ctrl, const SelectPlan &plan, hipStream_t s);
// Replay of the count pass's records (arena named in the control words):
// writes every recorded hit and contained leaf range at offsets[slot] +
// position; does nothing if the count pass made no records, they overflowed,
// or the result does not fit.
hipError_t launch_replay(const TreeView &t, const uint64_t *offsets, uint32_t noffsets, uint32_t *ids,
                         uint64_t ids_capacity, Ctrl *ctrl, hipStream_t s);

hipError_t launch_bulk_copy(const uint32_t *leaf_ids, const uint4 *bulk, uint32_t bulk_cap, uint32_t *ids,
                            Ctrl *ctrl, hipStream_t s);

// ---- scan, sort ---------------------------------------------------------
// Exclusive scan of n uint32 into n+1 uint64 (out[n] = total).  tmp needs
// scan_tmp_elems(n) uint64.
uint64_t scan_tmp_elems(uint64_t n);
uint64_t scan_tile_elems();   // elements per scan tile: scan_tmp_elems(n) = ceil(n / that) + 1
hipError_t launch_scan_u32(const uint32_t *in, uint64_t n, uint64_t *out, uint64_t *tmp,
                           hipStream_t s);
// The same with the count on the device: *n_dev <= n_max elements (tmp needs
// scan_tmp_elems(n_max)).  If next is not NULL, min(total, next_cap) is stored
// in *next and *over gets bit 0 when the total exceeds next_cap.
hipError_t launch_scan_u32_dev(const uint32_t *in, const uint64_t *n_dev, uint64_t n_max, uint64_t *out,
                               uint64_t *tmp, uint64_t *next, uint64_t next_cap, uint32_t *over, hipStream_t s);

// Sort every CSR segment ascending.  scratch: segsort_scratch_elems(capacity)
// uint32 (segments longer than one LDS tile are bucketed through it); ws:
// segsort_ws_elems(nq) uint32;
// id_range: every id is below it (the object count); seg_range (NULL, or nq
// entries): the bound of each segment's ids when segments come from trees of
// different sizes.  Skips all work if offsets[nq] > capacity.
uint64_t segsort_ws_elems(uint64_t nq);
uint64_t segsort_scratch_elems(uint64_t capacity);
hipError_t launch_segsort(const uint64_t *offsets, uint64_t nq, uint32_t *ids, uint32_t *scratch,
                          uint64_t capacity, uint32_t *ws, uint64_t id_range, const uint32_t *seg_range,
                          hipStream_t s);
inline int id_bits_for(uint64_t n_objects) {
    int b = 0;
    const uint64_t m = n_objects ? n_objects - 1 : 0;
    while (b < 64 && (m >> b)) ++b;
    return b;
}

// LSD radix sort of n uint64 keys over the listed digit positions, digits of
// digit_bits (8 or 11) bits.  Result ends in keys (if even number of passes)
// or tmp; returns which via *in_tmp.  hist needs radix_hist_elems(n,
// digit_bits) uint32, hscan that + 1 uint64 plus scan_tmp_elems of it.
uint64_t radix_hist_elems(uint64_t n, int digit_bits = 8);
hipError_t launch_radix_sort_u64(uint64_t *keys, uint64_t *tmp, uint64_t n, const int *shifts,
                                 int npasses, uint32_t *hist, uint64_t *hscan, uint64_t *stmp,
                                 bool *in_tmp, hipStream_t s, int digit_bits = 8);

// Status finalizer: status[0] = offsets[nq], status[1] = flags.
hipError_t launch_finalize(const uint64_t *offsets, uint64_t nq, uint64_t capacity,
                           const Ctrl *ctrl, uint64_t *status, hipStream_t s);

hipError_t launch_zero(void *p, uint64_t bytes, hipStream_t s);

// ---- join ---------------------------------------------------------------
enum JoinMode : int { JOIN_BOTH = 0, JOIN_EMIT = 1, JOIN_DESC_A = 2, JOIN_DESC_B = 3 };
// expansion variants (same values as the public RT_JOIN_* flags): outer
// slicing, one-to-many / many-to-many inner shrinking (need nodes sorted by
// low x), or the full Fa x Fb tile without candidate lists
enum JoinFlags : int { JOIN_O3 = 1, JOIN_O4 = 2, JOIN_O5 = 4, JOIN_TILE = 8, JOIN_LB = 16 };
// tests_acc (NULL: not counted): the count pass (fill = false) of the
// candidate kernels adds the number of pair predicates it evaluates to
// tests_acc[(pair % kTestSlots) * 16]; the sum over the slots is the total.
constexpr uint32_t kTestSlots = 256;
// nfr_dev (if not NULL): the frontier size on the device, at most nfr (the
// grid is sized for nfr).  The fill pass writes no output index at or past
// out_cap (the caller detects that case from the scan's total).  slots (NULL,
// or join_slot_bytes(nfr) of device memory, the same for the count and the
// fill pass of a level): hit records that spare the candidate kernels'
// fill pass the tests of pairs with few hits.
uint64_t join_slot_bytes(uint64_t nfr);
hipError_t launch_join_level(const TreeView &a, const TreeView &b, const uint2 *frontier,
                             uint32_t nfr, const uint64_t *nfr_dev, int mode, bool fill, uint32_t *counts,
                             const uint64_t *offsets, uint2 *next, uint64_t *keys, uint64_t out_cap,
                             uint16_t *slots, Ctrl *ctrl, int flags, unsigned long long *tests_acc, hipStream_t s);
hipError_t launch_keys_to_pairs(const uint64_t *keys, uint64_t n, uint32_t *pairs, hipStream_t s);

// ---- batch --------------------------------------------------------------
struct BatchTree {
    TreeView t;
    uint64_t q_begin;        // first global query index of this tree
    uint32_t nq;
    uint32_t stack_cap;
};
struct BatchItem {           // a chunk of one tree's queries
    uint32_t tree;
    uint32_t q0, q1;         // positions [q0, q1) in the tree's processing order
    uint32_t pad;
};
// Work items in kXcds lists (list x = items[list_begin[x] .. list_begin[x+1])),
// drained first by the blocks of XCD x; qorder[q_begin + position] = local
// query index (each tree's queries in the Morton order of their centres).
// rec (count pass): record arena as SelectPlan::rec / rec_count / rec_nchunks,
// with global query indices as output slots (NULL: no records).  fill_guard
// (fill pass): run only if the count pass's records overflowed.
struct BatchRec {
    uint4 *rec = nullptr;
    uint32_t *rec_count = nullptr;
    uint32_t rec_nchunks = 0;
    uint32_t fill_guard = 0;
};
hipError_t launch_batch_pass(const BatchTree *trees, const BatchItem *items, const uint32_t *list_begin,
                             uint32_t nitems, const uint32_t *qorder, const float4 *q, int mode, uint32_t *counts,
                             const uint64_t *offsets, uint32_t *ids, uint64_t capacity, uint64_t total_q, Ctrl *ctrl,
                             uint32_t work_slot, uint32_t wave_words, const BatchRec &rec, hipStream_t s);
// Replay of a recording batch count pass; qtree[global query] = its tree.
hipError_t launch_batch_replay(const BatchTree *trees, const uint32_t *qtree, const BatchRec &rec,
                               const uint64_t *offsets, uint64_t total_q, uint32_t *ids, uint64_t capacity,
                               Ctrl *ctrl, hipStream_t s);

int num_cus();

}  // namespace rtk
