/*
 * rt.h -- C ABI of the MI355X (gfx950) R-tree range-select and spatial-join
 * library.
 *
 * The operations follow the problem statement of "SIMD-ified R-tree Query
 * Processing and Optimization" (Rayhan and Aref): an in-memory 2D R-tree whose
 * node holds up to F entries (MBR, ptr) with MBR = (low_x, low_y, high_x,
 * high_y) (section 2.3); a range select that returns the objects whose MBR
 * intersects a query rectangle (section 3); and an R-tree join that returns
 * the intersecting pairs of two indexed relations by traversing both trees
 * from their roots and following intersecting child pairs (section 4).
 *
 * Predicate.  An object r and a window (or an object of the other relation)
 * s intersect iff
 *     r.lx <= s.hx && s.lx <= r.hx && r.ly <= s.hy && s.ly <= r.hy
 * with IEEE fp32 comparisons (exact; no arithmetic touches a coordinate on
 * the result path).  Boundaries are closed: touching rectangles intersect.
 *
 * Conventions for every call:
 *   - Rectangles are float32 rows of 4: (low_x, low_y, high_x, high_y).
 *     Object id = row index (uint32), query id = row index.
 *   - Sizes are element counts.  "host" pointers are ordinary CPU memory;
 *     "device" pointers are HIP device memory of the tree's device.
 *   - Return value: RT_OK (0) or a negative RT_E* code; on failure every
 *     *out is set to NULL, nothing partial is returned, and rt_last_error()
 *     holds a message.  No C++ exception crosses this interface.
 *   - Inputs are borrowed for the duration of the call and never retained.
 *   - Every object returned through **out is owned by the library and is
 *     released with rt_free().
 *   - A built tree is immutable; concurrent selects and joins on it are safe.
 *     Calls without a stream argument are synchronous.
 */
#ifndef RT_MI355X_H
#define RT_MI355X_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum {
    RT_OK = 0,
    RT_EINVAL = -1,   /* bad argument: NULL with n > 0, NaN, lx > hx or ly > hy,
                         fanout not in 2..64, unknown layout, n >= 2^32,
                         trees on different devices, buffer too small */
    RT_ENOMEM = -2,   /* a host or device allocation failed, or an output
                         buffer given by the caller is too small */
    RT_EDEVICE = -3   /* a HIP runtime error, or an internal check in a kernel */
};

/* Node storage layouts (section 2.3).  AOS is layout D0: each entry's five
 * fields contiguous.  SOA is layout D1: per node, arrays lx[F], ly[F], hx[F],
 * hy[F], ptr[F].  D2 is layout D2: lo[2F] (x,y pairs), hi[2F], ptr[F].
 * AUTO lets the builder choose among the three by timing (see
 * rt_build_str). */
enum { RT_LAYOUT_AOS = 0, RT_LAYOUT_SOA = 1, RT_LAYOUT_AUTO = 2, RT_LAYOUT_D2 = 3 };

/* Build option, OR-ed into the layout argument of the builders: store the
 * entries of every node in ascending low-x order (ties keep the STR order),
 * children moving with their entries, so that their subtrees stay
 * contiguous.  Section 4.1 assumes nodes sorted on one MBR key for its join
 * pruning; the order never changes a select or join result. */
#define RT_BUILD_SORT_LX 0x100u

/* Join expansion variants for rt_spatial_join_ex (section 4):
 *   RT_JOIN_O3    outer slicing: outer children whose low x exceeds every
 *                 inner high x are skipped (with sorted nodes, the rest of the
 *                 outer node after the first such child)
 *   RT_JOIN_O4    inner shrinking, one outer child at a time (one-to-many):
 *                 the inner scan stops at the first inner child whose low x
 *                 exceeds the outer high x
 *   RT_JOIN_O5    the same stop found for all outer children at once by the
 *                 many-to-many search of section 4.2 (takes precedence over
 *                 O4)
 *   RT_JOIN_TILE  no candidate lists: every one of the Fa x Fb child pairs
 *                 is tested (cannot be combined with the others)
 *   RT_JOIN_LB    (not in the paper; only as RT_JOIN_O3 | RT_JOIN_O5 |
 *                 RT_JOIN_LB) the inner scan also starts late: inner
 *                 children whose low x lies below the outer low x minus the
 *                 widest inner child (less a margin that covers rounding)
 *                 end left of the outer child and are skipped, found by the
 *                 same many-to-many search
 * O3, O4, O5 and LB need both trees built with RT_BUILD_SORT_LX.  No flag
 * gives candidate lists without pruning.  RT_JOIN_DEFAULT picks
 * O3|O5|LB when both trees are sorted, else RT_JOIN_TILE. */
enum { RT_JOIN_O3 = 1, RT_JOIN_O4 = 2, RT_JOIN_O5 = 4, RT_JOIN_TILE = 8, RT_JOIN_LB = 16, RT_JOIN_DEFAULT = -1 };

typedef struct rt_tree rt_tree;   /* opaque; device-resident; immutable */

/* Range-select result in CSR form: ids[offsets[q] .. offsets[q+1]) are the
 * ids of every object intersecting query q, ascending, no duplicates. */
typedef struct rt_ids {
    uint64_t nq;
    uint64_t *offsets;   /* nq + 1 entries, offsets[0] = 0 */
    uint32_t *ids;       /* offsets[nq] entries */
} rt_ids;

/* Join result: every (a, b) with A[a] and B[b] intersecting, in
 * lexicographic order, as pairs[2k] = a, pairs[2k+1] = b. */
typedef struct rt_pairs {
    uint64_t n;
    uint32_t *pairs;     /* 2n entries */
} rt_pairs;

/* Tree facts (read by the byte model and the tests). */
typedef struct rt_tree_info {
    uint64_t n_objects;
    uint64_t n_entries;      /* sum of node entry counts */
    uint64_t device_bytes;   /* node storage on the device */
    uint32_t n_nodes;
    uint32_t height;         /* levels including the leaf level */
    uint32_t fanout;
    uint32_t layout;
    uint32_t node_bytes;     /* stride of one node = 20 * fanout */
    uint32_t first_leaf;     /* nodes are numbered root first; leaves last */
    int32_t device;
    uint32_t flags;          /* RT_BUILD_SORT_LX if the nodes are sorted by low x */
} rt_tree_info;

/*
 * Build a packed R-tree over n rectangles with Sort-Tile-Recursive bulk
 * loading (the paper does not say how its trees are built; section 2.3 gives
 * what a node holds) on the current HIP device.  The rectangles are checked
 * on the host, copied to the device and packed there by the same kernels as
 * rt_build_str_device.  Shape: a level of c > F items gets ceil(c/F) nodes in
 * S = ceil(sqrt(ceil(c/F))) vertical slices of S*F items by x-center, each
 * slice ordered by y-center (f32 0.5*lo + 0.5*hi, ties by item index), runs
 * of F items per node; nodes are numbered breadth first from the root with
 * the children of every node contiguous in entry order.
 *   rects   host, n*4 floats; NaN or lx > hx or ly > hy -> RT_EINVAL;
 *           +-Inf allowed.  n = 0 gives an empty tree (one empty leaf).
 *   fanout  maximum entries per node F, 2..64, or 0: chosen by the library.
 *   layout  RT_LAYOUT_*, optionally OR-ed with RT_BUILD_SORT_LX;
 *           RT_LAYOUT_AUTO: chosen by the library.
 *   out     receives the tree; free with rt_free.
 * Library choice (fanout 0 and/or RT_LAYOUT_AUTO): every candidate tree
 * (fanouts 16, 32, 64 and/or layouts D0, D1, D2) is built on the device and
 * a probe set of windows drawn from the data (centred on seeded objects,
 * area log-uniform in [1e-6, 1e-3] of the data's bounding box) is selected on
 * it (one-call device selects whose workspace holds the count pass's
 * records); the fastest is kept, together with the faster split mapping
 * (rt_tree_set_split 0 or 16).  The choice is cached per (device
 * architecture, log2 n, candidate sets, RT_BUILD_SORT_LX) in memory and
 * appended to the text file $RT_TUNE_CACHE (empty: memory only; unset:
 * $HOME/.cache/rt_mi355x_tune.txt; lines "rt-tune-v2 key fanout layout
 * kmin", lines of other formats ignored), so later builds with the same key
 * do no timing.  rt_tree_stats reports the choice.
 */
int rt_build_str(const float *rects, uint64_t n, uint32_t fanout, uint32_t layout,
                 rt_tree **out);

/* Same as rt_build_str with the rectangles already on the device (d_rects,
 * n*4 floats on the current device, 16-byte aligned, read only); the whole
 * build runs in HIP kernels on `stream` (hipStream_t, NULL = default stream)
 * and the call returns after it has finished.  The rectangles are validated
 * on the device (RT_EINVAL without the index of the bad one).  Temporary
 * device memory: about 30 bytes per rectangle. */
int rt_build_str_device(const float *d_rects, uint64_t n, uint32_t fanout, uint32_t layout,
                        void *stream, rt_tree **out);

/*
 * Range select (section 3): for each of the nq host query windows, the ids of
 * the intersecting objects.  queries: host, nq*4 floats (NaN, lx > hx or
 * ly > hy -> RT_EINVAL; +-Inf allowed).  nq = 0 gives offsets = {0}.
 */
int rt_range_select(const rt_tree *t, const float *queries, uint64_t nq, rt_ids **out);

/*
 * R-tree spatial join (section 4): all intersecting (a, b), a from tree a's
 * relation and b from tree b's.  Both trees must live on the same device.
 * Same as rt_spatial_join_ex(a, b, RT_JOIN_DEFAULT, out, NULL).
 * All join calls draw their device workspaces from a per-device pool that
 * the library keeps until the process ends; a join repeated with the same
 * trees and flags is replayed from a HIP graph captured in that workspace
 * (results are the same either way).  Concurrent calls use separate
 * workspaces.
 */
int rt_spatial_join(const rt_tree *a, const rt_tree *b, rt_pairs **out);

/* Join with an explicit expansion variant (RT_JOIN_* flags above; results
 * never depend on it).  tests, if not NULL, receives the number of child-pair
 * predicates evaluated in expansions where both nodes are at the same level
 * (for RT_JOIN_TILE: the real entry pairs n_u * n_v of every such node
 * pair; padding slots are not counted).  Pruning flags on a tree built
 * without RT_BUILD_SORT_LX, unknown bits, or TILE combined with pruning ->
 * RT_EINVAL. */
int rt_spatial_join_ex(const rt_tree *a, const rt_tree *b, int32_t flags, rt_pairs **out, uint64_t *tests);

/* Work of the plain synchronized traversal of section 4 (the tile
 * expansion, no pruning) for the byte and operation model of the join:
 * node_pairs = node pairs visited over all levels (including the root pair
 * and the pairs where only the deeper tree descends), entry_pairs = entry
 * predicates evaluated (n_u * n_v real entries per node pair at equal
 * levels, plus the deeper node's entries against the other tree's bounding
 * box where one side descends alone), entries = real entries loaded.  Runs
 * the join once (results discarded).  Same argument rules as
 * rt_spatial_join. */
int rt_join_visit_stats(const rt_tree *a, const rt_tree *b, uint64_t *node_pairs, uint64_t *entry_pairs,
                        uint64_t *entries);

/* Join with the result left in device memory: d_pairs (2 * capacity uint32
 * on the trees' device, caller-owned) receives pairs[2k] = a,
 * pairs[2k+1] = b in lexicographic order and *n_pairs (host) their number.
 * More pairs than capacity -> RT_ENOMEM with *n_pairs set and d_pairs
 * untouched (call again with a buffer that large).  flags as for
 * rt_spatial_join_ex.  Runs on `stream` (hipStream_t, NULL = default) and
 * returns after that work has finished. */
int rt_spatial_join_device(const rt_tree *a, const rt_tree *b, int32_t flags, uint32_t *d_pairs,
                           uint64_t capacity, uint64_t *n_pairs, void *stream);

/* Release an rt_tree, rt_ids or rt_pairs (and a tree's device memory).
 * NULL is a no-op. */
void rt_free(void *obj);

/* ------------------------------------------------------------------------ */
/* Device-pointer, stream-ordered range select (used for batching, serving   */
/* and timing with inputs already resident in device memory).                */
/* ------------------------------------------------------------------------ */

/* Workspace bytes that rt_range_select_device needs for nq queries and an
 * output capacity of ids_capacity ids. */
uint64_t rt_select_workspace_bytes(uint64_t nq, uint64_t ids_capacity);

/* Workspace bytes with which rt_range_select_device (and _timed) also keeps
 * the count pass's output in compact records (per leaf with hits: its hit
 * mask; per contained subtree: its leaf range) and the fill writes the ids
 * by replaying them instead of walking the tree a second time (section 3's
 * two traversals, the second replaced by a streaming pass; results are
 * identical).  Any size from rt_select_workspace_bytes up is accepted: the
 * bytes past it hold the records, and when they do not suffice (or the tree
 * has 2^30 nodes or more, or replay is off for the tree) the fill walks the
 * tree.  The two-stage calls replay when the count stage's workspace has room
 * past its own layout. */
uint64_t rt_select_replay_workspace_bytes(uint64_t nq, uint64_t ids_capacity);

/* Whether one-call selects on this tree may replay the count pass's records
 * (see rt_select_replay_workspace_bytes; on = 1, the default) or always walk
 * the tree twice (on = 0).  Never changes a result.  Other values ->
 * RT_EINVAL.  Not to be called while selects on the tree run. */
int rt_tree_set_replay(rt_tree *t, uint32_t on);

/* After a one-call select on the workspace d_work has finished (the caller
 * synchronizes its stream): *chunks = record chunks of 256 records its count
 * pass took (0 if it did not record), *overflowed = 1 if the records did not
 * fit and the fill walked the tree.  Blocking copy of 64 bytes. */
int rt_select_replay_info(const void *d_work, uint32_t *chunks, uint32_t *overflowed);

/*
 * Enqueue a complete range select on `stream` and return without waiting.
 *   d_queries   device, nq*4 floats (not validated: the caller guarantees
 *               no NaN and lx <= hx, ly <= hy)
 *   d_offsets   device, nq+1 uint64 (written)
 *   d_ids       device, ids_capacity uint32 (written only if the result fits)
 *   d_work      device workspace of at least rt_select_workspace_bytes bytes
 *   d_status    device, 2 uint64 written at the end: [0] = total ids,
 *               [1] = flags (1: total > ids_capacity, d_ids left untouched
 *               and the CSR is not valid; 2: internal error)
 * Returns RT_EINVAL for bad sizes; kernel-side outcomes are in d_status.
 */
int rt_range_select_device(const rt_tree *t, const float *d_queries, uint64_t nq,
                           uint64_t *d_offsets, uint32_t *d_ids, uint64_t ids_capacity,
                           void *d_work, uint64_t work_bytes, uint64_t *d_status, void *stream);

/* Size of the fixed device scratch of rt_range_select_device_noalloc. */
#define RT_NOALLOC_SCRATCH_BYTES (32ull << 20)

/*
 * For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): the same
 * select as rt_range_select_device, with the same arguments and d_status
 * contract, but its workspace is a fixed array of RT_NOALLOC_SCRATCH_BYTES
 * (32 MiB) in the library's device code, which every device that runs the
 * library holds until the process ends.  The call allocates nothing and only
 * enqueues on `stream`.  A size whose workspace
 * (rt_select_workspace_bytes(nq, ids_capacity)) exceeds the scratch ->
 * RT_EINVAL with a message, before anything is enqueued (for instance up to
 * 65536 queries with room for 4M ids fit).  All calls on one device share
 * that device's scratch: calls whose work overlaps in time on one device
 * (different host threads, or different streams without ordering between
 * them) race and must not be issued; calls ordered on one stream are safe.
 */
int rt_range_select_device_noalloc(const rt_tree *t, const float *d_queries, uint64_t nq, uint64_t *d_offsets,
                                   uint32_t *d_ids, uint64_t ids_capacity, uint64_t *d_status, void *stream);

/* rt_range_select_device plus phase timing: events (hipEvent_t[5], created by
 * the caller) are recorded on `stream` before the count pass, after it, after
 * the scan, after the fill pass and after the segmented sort, so the caller can
 * read each phase's duration with hipEventElapsedTime.  events may be NULL. */
int rt_range_select_device_timed(const rt_tree *t, const float *d_queries, uint64_t nq,
                                 uint64_t *d_offsets, uint32_t *d_ids, uint64_t ids_capacity,
                                 void *d_work, uint64_t work_bytes, uint64_t *d_status,
                                 void *stream, void *const *events);

/*
 * Range select (section 3) into caller-owned device buffers, the output
 * placed by the caller.  The library keeps the workspace (a per-device pool,
 * held until the process ends; a workspace is reused only after the work
 * enqueued on it has finished).
 *   d_queries    device, nq*4 floats, 16-byte aligned (not validated: the
 *                caller guarantees no NaN and lx <= hx, ly <= hy)
 *   d_offsets    device, nq+1 uint64: the CSR offsets (always written)
 *   d_ids        device, ids_capacity uint32: the ids, ascending per query
 *   d_total      device, 1 uint64: the number of ids of the result (written
 *                in both outcomes below; all ones if a kernel-side check
 *                failed, an internal error)
 *   stream       hipStream_t (NULL = default stream)
 * The call enqueues the count stage on `stream` and waits for it (it reads
 * the total back).  If the result has more than ids_capacity ids it returns
 * RT_ENOMEM and nothing is written to d_ids; otherwise it enqueues the fill
 * stage and the sort and returns RT_OK without waiting for them: d_ids and
 * the final *d_total are valid once `stream` has reached this point.
 * RT_EINVAL for NULL buffers or misaligned queries, RT_EDEVICE for HIP
 * errors.
 */
int rt_range_select_async(const rt_tree *t, const float *d_queries, uint64_t nq, uint64_t *d_offsets,
                          uint32_t *d_ids, uint64_t ids_capacity, uint64_t *d_total, void *stream);

/* rt_range_select_device in two calls, for callers that decide where the
 * output goes (or whether it is run at all) once its exact size is known.
 * The count stage computes d_offsets (nq+1 uint64, d_offsets[nq] = total
 * ids) and leaves the processing order and split plan in d_work; the fill
 * stage, enqueued later with the same tree, queries, d_offsets and d_work
 * (whose first rt_select_workspace_bytes(nq, 0) bytes must be unchanged),
 * writes the ids and d_status as rt_range_select_device does.  A count stage
 * may be followed by no fill stage, and each fill stage needs a count stage
 * of its own (it consumes the work counters the count stage resets).  Both
 * only enqueue on `stream`.
 * work_bytes: at least rt_select_workspace_bytes(nq, 0) for the count stage
 * and rt_select_workspace_bytes(nq, ids_capacity) for the fill stage.  The
 * count stage uses any bytes of d_work past rt_select_workspace_bytes(nq, 0)
 * for its records (see rt_select_replay_workspace_bytes): the fill stage
 * then replays them instead of walking the tree, and those bytes must also
 * stay unchanged until it runs.  With exactly rt_select_workspace_bytes(nq,
 * 0) bytes for the count stage the fill stage walks the tree. */
int rt_range_select_device_count(const rt_tree *t, const float *d_queries, uint64_t nq, uint64_t *d_offsets,
                                 void *d_work, uint64_t work_bytes, void *stream);
int rt_range_select_device_fill(const rt_tree *t, const float *d_queries, uint64_t nq, uint64_t *d_offsets,
                                uint32_t *d_ids, uint64_t ids_capacity, void *d_work, uint64_t work_bytes,
                                uint64_t *d_status, void *stream);

/* Count pass only: d_counts[q] = number of objects intersecting query q
 * (device, nq uint32).  Used to size outputs before admitting work. */
int rt_range_count_device(const rt_tree *t, const float *d_queries, uint64_t nq,
                          uint32_t *d_counts, void *d_work, uint64_t work_bytes, void *stream);

/* ------------------------------------------------------------------------ */
/* Batched select over many independent trees in one persistent launch.      */
/* ------------------------------------------------------------------------ */

/* Host-side batch: trees[i] with queries[i] (host, nq[i]*4 floats) for
 * i < ntrees; out[i] receives tree i's CSR (free each with rt_free).  All
 * trees must be on the current device; they may differ in fanout and layout.
 * The traversal of all trees runs as one persistent kernel per pass fed by a
 * device work queue of (tree, query-chunk) items, replayed from a captured
 * HIP graph. */
int rt_range_select_batch(const rt_tree *const *trees, uint32_t ntrees,
                          const float *const *queries, const uint64_t *nq, rt_ids **out);

typedef struct rt_batch rt_batch;   /* opaque prepared batch (device-resident) */

/* Prepare a device-resident batch: copies the queries to the device, builds
 * the work queue and captures the count -> scan -> fill -> sort launches
 * into a HIP graph whose output pool holds ids_capacity ids.
 * ids_capacity = 0 sizes the pool by running the count pass once.  The
 * graph's count pass records its leaves and contained subtrees and the fill
 * replays them (see rt_select_replay_workspace_bytes; the walking fill runs
 * instead if the records outgrow their arena). */
int rt_batch_create(const rt_tree *const *trees, uint32_t ntrees,
                    const float *const *queries, const uint64_t *nq,
                    uint64_t ids_capacity, rt_batch **out);
/* Replay the captured graph on `stream` (asynchronous). */
int rt_batch_run(rt_batch *b, void *stream);
/* Same work as rt_batch_run without the graph or the persistent kernel: one
 * plain launch sequence per tree, in order (the baseline it must beat). */
int rt_batch_run_plain(rt_batch *b, void *stream);
/* After a run has finished: total ids and the flags word (see d_status). */
int rt_batch_status(rt_batch *b, uint64_t *total, uint64_t *flags);
/* Copy tree i's CSR to the host. */
int rt_batch_result(rt_batch *b, uint32_t i, rt_ids **out);
/* Recapture the batch's graph with the replayed fill (on = 1, the default)
 * or the walking fill (on = 0); results are identical.  Other values ->
 * RT_EINVAL.  Not to be called while a run of the batch is in flight. */
int rt_batch_set_replay(rt_batch *b, uint32_t on);
/* After a graph run has finished: record chunks its count pass took and
 * whether they overflowed (both 0 after rt_batch_run_plain).  Synchronizes
 * the device. */
int rt_batch_replay_info(rt_batch *b, uint32_t *chunks, uint32_t *overflowed);

/* ------------------------------------------------------------------------ */
/* Introspection                                                             */
/* ------------------------------------------------------------------------ */

int rt_tree_stats(const rt_tree *t, rt_tree_info *info);

/* Work mapping of later selects on this tree (never changes a result).
 * A query whose walk reaches at least kmin parents-of-leaves nodes is split
 * into one work item per such subtree, so many lane groups share one large
 * window instead of one group walking it alone; kmin = 0 keeps one group per
 * query (the default).  Not to be called while selects on the tree run. */
int rt_tree_set_split(rt_tree *t, uint32_t kmin);

/* Lookahead loads in later selects on this tree (section 3, optimization O2;
 * never changes a result): on = 1 makes the traversal load the next node's
 * entries as soon as it pops a leaf (the next node is then already known),
 * so that load overlaps the leaf's comparison and output; on = 0 (default)
 * loads each node when it is popped.  Other values -> RT_EINVAL.  Not to be
 * called while selects on the tree run. */
int rt_tree_set_lookahead(rt_tree *t, uint32_t on);

/* Where the fill pass of later selects on this tree copies contained runs
 * (section 3, the whole-subtree copy of a node fully inside the window; never
 * changes a result).  RT_BULK_AUTO (default): runs of at least 2048 ids are
 * appended as descriptors and copied by a streaming kernel after the pass on
 * trees of at least 2^25 objects, whose leaf-id array does not stay cached;
 * smaller trees copy every run in the pass.  RT_BULK_ON / RT_BULK_OFF force
 * the one or the other.  Other values -> RT_EINVAL.  Not to be called while
 * selects on the tree run. */
enum { RT_BULK_AUTO = 0, RT_BULK_ON = 1, RT_BULK_OFF = 2 };
int rt_tree_set_bulk_copy(rt_tree *t, uint32_t mode);

/* Copy the tree to host arrays in a neutral node/entry form: per node
 * (root = node 0) level (0 = leaf), entry count and index of its first entry;
 * per entry the MBR and ptr (object id at a leaf, child node otherwise).
 * Array lengths: n_nodes for level/count/first, n_entries for the rest. */
int rt_tree_export(const rt_tree *t, uint32_t *level, uint32_t *count, uint64_t *first,
                   float *lx, float *ly, float *hx, float *hy, uint32_t *ptr);

/* Per-query traversal statistics for the byte model, summed over the nq host
 * queries (same traversal as the select kernels): visited nodes, their
 * entries, and (vcontained, may be NULL) the ids emitted wholesale from
 * subtrees whose MBR lies inside the window. */
int rt_select_visit_stats(const rt_tree *t, const float *queries, uint64_t nq,
                          uint64_t *vnodes, uint64_t *ventries, uint64_t *vcontained);

/* Message for the last failure on the calling thread ("" if none). */
const char *rt_last_error(void);

/* Library version string. */
const char *rt_version(void);

#ifdef __cplusplus
}
#endif
#endif /* RT_MI355X_H */
