// Range-select traversal kernels for gfx950.
//
// One query is handled by a group of G lanes (G = 16, 32 or 64, the smallest
// power of two >= F), so a wave64 runs 64/G queries side by side.  Lane e of a
// group owns entry e of the node being visited.  Per visited node:
//   1. the query window sits in registers, the same in all lanes of the group
//      (the paper broadcasts the query into vector registers once per query,
//      section 3 step 1);
//   2. each lane loads its entry's MBR -- for the SoA layout D1 the group's
//      loads of lx[], ly[], hx[], hy[] are four coalesced 4F-byte reads
//      (section 3 step 2);
//   3. the four fp32 comparisons give a per-lane hit; __ballot turns the hits
//      of the wave into a 64-bit mask and the group takes its G bits (the
//      SIMD compare-to-bitmask of section 3 step 3);
//   4. at an internal node the qualifying children are pushed onto the group's
//      stack in LDS at base + rank (rank = popcount of the mask below the
//      lane), the GPU form of the masked compress-store into the queue
//      (section 3 step 4, and the recursion-free traversal O1).  Nodes are
//      numbered breadth first with the children of a node contiguous, so a
//      child index is the node's first child + the entry slot; only that one
//      pointer is read per internal node.  At a leaf the
//      group counts its hits (count pass) or writes the object ids at the
//      query's output cursor + rank (fill pass).
// The stack is depth-first (a LIFO of node ids) so its size stays bounded by
// (h-1)(F-1)+1 entries instead of a whole tree level.
//
// Work distribution: the grid is persistent; a group that empties its stack
// takes the next query index from a device counter (the count pass two at a
// time, see grab_chunk).  Both passes walk the same
// tree with the same predicate, so the fill pass writes exactly the count
// pass's number of ids for every query.
#include "rt_internal.h"

namespace rtk {

template <int LAYOUT>
__device__ __forceinline__ void load_entry(const uint8_t *__restrict__ node, uint32_t F, uint32_t e,
                                           float &lx, float &ly, float &hx, float &hy) {
    if constexpr (LAYOUT == LAYOUT_SOA) {
        const float *f = reinterpret_cast<const float *>(node);
        lx = f[e];
        ly = f[F + e];
        hx = f[2 * F + e];
        hy = f[3 * F + e];
    } else if constexpr (LAYOUT == LAYOUT_AOS) {
        const float *f = reinterpret_cast<const float *>(node) + 5 * e;
        lx = f[0];
        ly = f[1];
        hx = f[2];
        hy = f[3];
    } else {
        const float2 *lo = reinterpret_cast<const float2 *>(node);
        const float2 a = lo[e];
        const float2 b = lo[F + e];
        lx = a.x;
        ly = a.y;
        hx = b.x;
        hy = b.y;
    }
}

template <int LAYOUT>
__device__ __forceinline__ uint32_t load_ptr(const uint8_t *__restrict__ node, uint32_t F, uint32_t e) {
    const uint32_t *u = reinterpret_cast<const uint32_t *>(node);
    if constexpr (LAYOUT == LAYOUT_AOS) return u[5 * e + 4];
    return u[4 * F + e];
}

// Next query for a group leader.  The processing order is cut into eight
// slices; a block on XCD `home` drains slice `home` first (the queries of a
// slice are close in space, so they share tree nodes in that XCD's L2), then
// the following slices in turn.  `visited` counts the slices found empty.
// Returns nq when everything has been handed out.
__device__ __forceinline__ uint32_t grab_query(Ctrl *ctrl, uint32_t slot, uint32_t nq, const uint64_t *order,
                                               uint32_t home, uint32_t &visited, uint32_t *slice = nullptr,
                                               bool look_first = false) {
    while (visited < kXcds) {
        const uint32_t x = (home + visited) % kXcds;
        const uint32_t b0 = (uint32_t)(((uint64_t)x * nq) / kXcds);
        const uint32_t b1 = (uint32_t)(((uint64_t)(x + 1) * nq) / kXcds);
        // look_first (grids sized independently of the work, where most
        // groups of a small batch are idle): read another XCD's counter
        // before taking from it.  A drained slice's counter only grows, so a
        // read that shows it drained is final and the atomic, which thousands
        // of idle groups would otherwise queue on, is skipped.  Otherwise the
        // read would only add a round trip per steal.
        if (look_first && visited > 0 &&
            __hip_atomic_load(&ctrl->xwork[slot][x][0], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) >= b1 - b0) {
            visited += 1;
            continue;
        }
        const uint32_t k = atomicAdd(&ctrl->xwork[slot][x][0], 1u);
        if (k < b1 - b0) {
            if (slice) *slice = x;
            return order ? (uint32_t)order[b0 + k] : b0 + k;
        }
        visited += 1;
    }
    return nq;
}

// Work unit of a pass: a query started at the root, or -- for a query split
// into subtrees -- one (query, subtree root) item.  `oslot` is the output
// slot (count pass: index into counts; fill pass: index into offsets).
struct Unit {
    uint32_t q, node, oslot;
};

// Next split item for a group leader (split items are the long ones and go
// first), or q = nq when every list is drained.
__device__ __forceinline__ Unit next_split_item(Ctrl *ctrl, uint32_t slot, uint32_t nq, const SelectPlan &plan,
                                                uint32_t home, uint32_t &hvisited) {
    while (hvisited < kXcds) {
        const uint32_t x = (home + hvisited) % kXcds;
        const uint32_t nh = ctrl->hlist[x][0];
        if (hvisited > 0 &&
            __hip_atomic_load(&ctrl->hwork[slot][x][0], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) >= nh) {
            hvisited += 1;
            continue;
        }
        const uint32_t k = atomicAdd(&ctrl->hwork[slot][x][0], 1u);
        if (k < nh) {
            const uint4 it = plan.heavy[(uint64_t)x * plan.hcap + k];
            return Unit{it.x, it.y, it.z};
        }
        hvisited += 1;
    }
    return Unit{nq, 0u, 0u};
}

// Whole queries are handed out K at a time: one atomic on the slice counter
// takes K consecutive positions of the processing order, and the group loads
// their query indices and windows in one round (lane i holds the i-th).  The
// slice counters are single addresses that every group of an XCD updates, and
// their atomics are serialized: with one query per atomic the count pass (a
// few nodes per query) waits on them.  The fill pass keeps K = 1: its queries
// take longer, and a group holding several of them widens the XCD's front in
// the processing order, which costs L2 hits.  Returns the number taken (0:
// all handed out) and the first position in *p0.
template <uint32_t K>
__device__ __forceinline__ uint32_t grab_chunk(Ctrl *ctrl, uint32_t slot, uint32_t nq, uint32_t home,
                                               uint32_t &visited, bool look_first, uint32_t *p0) {
    while (visited < kXcds) {
        const uint32_t x = (home + visited) % kXcds;
        const uint32_t b0 = (uint32_t)(((uint64_t)x * nq) / kXcds);
        const uint32_t b1 = (uint32_t)(((uint64_t)(x + 1) * nq) / kXcds);
        if (look_first && visited > 0 &&
            __hip_atomic_load(&ctrl->xwork[slot][x][0], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) >= b1 - b0) {
            visited += 1;
            continue;
        }
        const uint32_t k = atomicAdd(&ctrl->xwork[slot][x][0], K);
        if (k < b1 - b0) {
            *p0 = b0 + k;
            return min(K, b1 - b0 - k);
        }
        visited += 1;
    }
    return 0;
}

__device__ __forceinline__ uint64_t shfl_u64(uint64_t v, int src) {
    const uint32_t lo = (uint32_t)__shfl((int)(uint32_t)v, src);
    const uint32_t hi = (uint32_t)__shfl((int)(uint32_t)(v >> 32), src);
    return ((uint64_t)hi << 32) | lo;
}

// LA = 1: lookahead (section 3, optimization O2, as a load issued one node
// ahead).  A leaf pushes nothing, so after popping a leaf the next node to be
// visited is already on top of the stack; its entries are loaded right away,
// while the leaf is compared and written out, and the next iteration uses
// them without waiting for a fresh load.  After an internal node the next
// node is one of its children, decided only by the comparison, so nothing is
// loaded ahead there.
// EXT = 1, fill pass: contained runs of at least kBulkMin ids are appended
// to the plan's descriptor list for the bulk copy instead of being copied in
// the pass.  EXT = 1, count pass: every leaf with hits and every contained
// subtree is also written to the plan's record arena, which the fill stage
// replays instead of walking the tree again.
constexpr uint32_t kCountChunk = 2;
// Contained runs of at most this many leaves are copied from the leaves' own
// ptr arrays (layouts D1, D2: a leaf's ids are 4F contiguous bytes of its
// node, and those nodes are the ones neighbouring queries read), longer ones
// from the leaf-id array -- except with 64-entry nodes, where every run is
// copied from the leaves' nodes (measured at 10M rectangles / 1M windows:
// fill 3.65 ms from the nodes, 4.22 ms through the array; with 32-entry
// nodes 5.29 vs 4.85 ms).
constexpr uint32_t kNodeCopyLeaves = 4;

template <int G, int LAYOUT, int MODE, int LA, int EXT>
__global__ void __launch_bounds__(256)
select_kernel(TreeView t, const float4 *__restrict__ qs, uint32_t nq, uint32_t *__restrict__ counts,
              const uint64_t *__restrict__ offsets, uint32_t *__restrict__ ids, uint64_t cap,
              Ctrl *__restrict__ ctrl, uint32_t slot, uint32_t stack_cap, SelectPlan plan, uint32_t noffsets) {
    extern __shared__ uint32_t smem[];
    if constexpr (MODE == SEL_FILL) {
        if (offsets[noffsets] > cap) return;   // result does not fit: leave ids untouched
        if (plan.fill_guard && ctrl->rec_nchunks && !ctrl->rec_overflow) return;   // the replay wrote everything
    }
    const uint32_t lane = threadIdx.x & 63u;
    const uint32_t e = lane & (G - 1);
    const uint32_t gbase = lane & ~(uint32_t)(G - 1);
    uint32_t *stk = smem + (threadIdx.x / G) * stack_cap;
    const uint32_t F = t.fanout;
    const uint64_t gmask = (G == 64) ? ~0ull : ((1ull << G) - 1ull);
    const uint64_t below = (e == 0) ? 0ull : (~0ull >> (64 - e));

    // XCD-relative cursor over the eight slices of the processing order
    const uint32_t home = blockIdx.x % kXcds;
    uint32_t visited = 0;
    uint32_t hvisited = plan.heavy ? 0u : kXcds;
    // the group's chunk of whole queries: lane i < cn holds query cq, its
    // window cw and output slot cs (kNoNode: split); ci = next to start
    // (and, fill pass, its output range [cpos, cend))
    uint32_t cn = 0, ci = 0, cq = 0, cs = 0;
    float4 cw = make_float4(0.f, 0.f, 0.f, 0.f);
    uint64_t cpos = 0, cend = 0;
    uint32_t oslot = 0;
    bool have = false, done = false;
    uint32_t sp = 0;
    float4 q = make_float4(0.f, 0.f, 0.f, 0.f);
    uint64_t pos = 0, end = 0;
    uint64_t vnodes = 0, ventries = 0, vcont = 0;
    // lookahead registers: the node loaded ahead and this lane's entry of it
    uint32_t pf_node = kNoNode, pf_ref = 0;
    float pf_lx = 0.f, pf_ly = 0.f, pf_hx = 0.f, pf_hy = 0.f;
    // recording count pass: records collect in the group's LDS buffer (after
    // the stacks) and go out kRecBuf at a time to the group's current chunk
    // of the arena (rchunk, rcnt records used).  Stores and loads share one
    // completion counter, so a store issued before a node load delays the
    // wait for that load: batching the stores keeps such waits rare.
    uint32_t rchunk = kNoNode, rcnt = 0, nbuf = 0;
    uint4 *rbuf = reinterpret_cast<uint4 *>(smem + ((256 / G) * stack_cap + 3u) / 4u * 4u) + (threadIdx.x / G) * kRecBuf;
    auto rec_flush = [&]() {   // group-uniform
        if (nbuf == 0) return;
        __builtin_amdgcn_wave_barrier();
        if (rchunk != kRecDead && (rchunk == kNoNode || rcnt + nbuf > kRecChunk)) {
            if (rchunk != kNoNode && e == 0) plan.rec_count[rchunk] = rcnt;
            uint32_t c = 0;
            if (e == 0) c = atomicAdd(&ctrl->rec_chunks, 1u);
            c = (uint32_t)__shfl((int)c, (int)gbase);
            if (c < plan.rec_nchunks) {
                rchunk = c;
                rcnt = 0;
            } else {
                if (e == 0) atomicOr(&ctrl->rec_overflow, 1u);
                rchunk = kRecDead;
            }
        }
        if (rchunk < kRecDead) {
            for (uint32_t i = e; i < nbuf; i += G) {
                const uint4 v = rbuf[i];
                put_rec(plan.rec + (size_t)rchunk * kRecChunk + rcnt + i, v.x, v.y, v.z, v.w);
            }
            rcnt += nbuf;
        }
        nbuf = 0;
        __builtin_amdgcn_wave_barrier();
    };

    while (true) {
        if (!done && sp == 0) {
            if (have) {
                if constexpr (MODE == SEL_COUNT) {
                    if (e == 0) counts[oslot] = (uint32_t)pos;
                }
            }
            Unit u{nq, 0u, 0u};
            bool from_chunk = false;
            if (hvisited < kXcds) {
                if (e == 0) u = next_split_item(ctrl, slot, nq, plan, home, hvisited);
                u.q = __shfl(u.q, (int)gbase);
                u.node = __shfl(u.node, (int)gbase);
                u.oslot = __shfl(u.oslot, (int)gbase);
                hvisited = __shfl(hvisited, (int)gbase);
                if (u.q < nq) q = qs[u.q];
            }
            // whole queries from the group's chunk, skipping split ones
            while (u.q >= nq) {
                if (ci >= cn) {
                    uint32_t p0 = 0, c = 0;
                    if (e == 0)
                        c = grab_chunk<MODE == SEL_FILL ? 1u : kCountChunk>(ctrl, slot, nq, home, visited,
                                                                             plan.heavy != nullptr, &p0);
                    c = __shfl(c, (int)gbase);
                    p0 = __shfl(p0, (int)gbase);
                    visited = __shfl(visited, (int)gbase);
                    if (c == 0) break;
                    cn = c;
                    ci = 0;
                    if (e < c) {
                        cq = plan.order ? (uint32_t)plan.order[p0 + e] : p0 + e;
                        cw = qs[cq];
                        cs = cq;
                        if (plan.slot_first) {
                            const uint64_t s0 = plan.slot_first[cq];
                            cs = plan.slot_first[cq + 1] - s0 == 1 ? (uint32_t)s0 : kNoNode;
                        }
                        if constexpr (MODE == SEL_FILL) {
                            if (cs != kNoNode) {
                                cpos = offsets[cs];
                                cend = offsets[cs + 1];
                            }
                        }
                    }
                }
                const int src = (int)(gbase + ci);
                ci += 1;
                const uint32_t os = __shfl(cs, src);
                if (os == kNoNode) continue;   // split: its items cover it
                u = Unit{(uint32_t)__shfl(cq, src), 0u, os};
                q = make_float4(__shfl(cw.x, src), __shfl(cw.y, src), __shfl(cw.z, src), __shfl(cw.w, src));
                if constexpr (MODE == SEL_FILL) {
                    pos = shfl_u64(cpos, src);
                    end = shfl_u64(cend, src);
                }
                from_chunk = true;
            }
            if (u.q < nq) {
                if constexpr (MODE == SEL_FILL) {
                    if (!from_chunk) {   // a split item
                        pos = offsets[u.oslot];
                        end = offsets[u.oslot + 1];
                    }
                } else {
                    pos = 0;
                }
                oslot = u.oslot;
                have = true;
                stk[0] = u.node;
                sp = 1;
            } else {
                have = false;
                done = true;
            }
        }
        if (__all(done)) break;
        __builtin_amdgcn_wave_barrier();

        uint32_t node = 0;
        if (have) {
            sp -= 1;
            node = stk[sp];
        }
        const uint8_t *nb = t.nodes + (size_t)node * t.node_bytes;
        const bool leaf = node >= t.first_leaf;
        bool hit = false, valid = false;
        uint32_t ref = 0;   // first child (internal node) or this entry's object id (leaf, fill pass)
        float lx = 0.f, ly = 0.f, hx = 0.f, hy = 0.f;
        bool got = false;
        if constexpr (LA != 0) {
            got = have && pf_node == node;
            if (got) {
                lx = pf_lx;
                ly = pf_ly;
                hx = pf_hx;
                hy = pf_hy;
                ref = pf_ref;
            }
        }
        if (have && e < F && !got) {
            // the id / first-child load does not depend on the comparison, so it
            // is in flight together with the coordinate loads
            if (!leaf)
                ref = load_ptr<LAYOUT>(nb, F, 0);
            else if constexpr (MODE == SEL_FILL)
                ref = load_ptr<LAYOUT>(nb, F, e);
            load_entry<LAYOUT>(nb, F, e, lx, ly, hx, hy);
        }
        if constexpr (LA != 0) {
            pf_node = kNoNode;
            if (have && leaf && sp > 0) {
                const uint32_t nx = stk[sp - 1];
                pf_node = nx;
                if (e < F) {
                    const uint8_t *nb2 = t.nodes + (size_t)nx * t.node_bytes;
                    pf_ref = 0;
                    if (nx < t.first_leaf)
                        pf_ref = load_ptr<LAYOUT>(nb2, F, 0);
                    else if constexpr (MODE == SEL_FILL)
                        pf_ref = load_ptr<LAYOUT>(nb2, F, e);
                    load_entry<LAYOUT>(nb2, F, e, pf_lx, pf_ly, pf_hx, pf_hy);
                }
            }
        }
        bool cont = false;
        if (have && e < F) {
            hit = (lx <= q.z) && (q.x <= hx) && (ly <= q.w) && (q.y <= hy);
            if constexpr (MODE == SEL_STATS) valid = (lx == lx);
            // an internal entry whose MBR lies inside the window: every object
            // below it qualifies, so its subtree is taken whole
            cont = hit && !leaf && (q.x <= lx) && (hx <= q.z) && (q.y <= ly) && (hy <= q.w);
        }
        const uint64_t m = (__ballot(hit) >> gbase) & gmask;
        const uint64_t cm = (__ballot(cont) >> gbase) & gmask;
        const uint64_t pm = m & ~cm;   // children to descend into
        const uint32_t n = (uint32_t)__popcll(m);
        const uint32_t rank = (uint32_t)__popcll(m & below);
        if constexpr (MODE == SEL_STATS) {
            const uint64_t vm = (__ballot(valid) >> gbase) & gmask;
            if (have) {
                vnodes += 1;
                ventries += (uint64_t)__popcll(vm);
            }
        }
        if (have) {
            if (leaf) {
                if constexpr (MODE == SEL_FILL) {
                    if (hit) {
                        const uint64_t o = pos + rank;
                        // ids are written once and read back only by the
                        // sort: stores that bypass the caches leave L2 to the
                        // tree nodes (fill pass 4.4 -> 3.8 ms at 10M/1M)
                        if (o < end)
                            put_id(ids + o, ref);
                        else
                            atomicOr(&ctrl->err, kErrBounds);
                    }
                }
                if constexpr (MODE == SEL_COUNT && EXT != 0) {
                    if (n) {   // one record per 32 entries with hits
                        const uint32_t lo = (uint32_t)m, hi = (uint32_t)(m >> 32);
                        const uint32_t k = (lo ? 1u : 0u) + (hi ? 1u : 0u);
                        if (nbuf + k > kRecBuf) rec_flush();
                        if (e == 0 && lo) rbuf[nbuf] = make_uint4(oslot, (uint32_t)pos, node, lo);
                        if (G == 64 && e == 32 && hi)
                            rbuf[nbuf + (lo ? 1u : 0u)] =
                                make_uint4(oslot, (uint32_t)pos + (uint32_t)__popc(lo), node | kRecHi, hi);
                        nbuf += k;
                    }
                }
                pos += n;
            } else {
                // children of a node are contiguous: entry e points at first + e
                const uint32_t first = __shfl(ref, (int)gbase);
                if (cm) {   // group-uniform: contained subtrees
                    if constexpr (MODE == SEL_FILL) {
                        // copy the ids of the contained subtrees' leaves.
                        // Consecutive contained children have consecutive
                        // leaves, so each run of them is one leaf range and
                        // one contiguous run of the tree's leaf-id array.
                        uint64_t todo = cm;
                        bool bad = false;
                        while (todo) {
                            const uint32_t j0 = (uint32_t)__builtin_ctzll(todo);
                            const uint64_t sh = todo >> j0;
                            const uint32_t len = ~sh ? (uint32_t)__builtin_ctzll(~sh) : 64u - j0;
                            todo = (j0 + len >= 64) ? 0ull : (todo & (~0ull << (j0 + len)));
                            const uint32_t l0 = t.range[first + j0].x, l1 = t.range[first + j0 + len - 1].y;
                            if constexpr (EXT != 0) {
                                if (subtree_objects(t, make_uint2(l0, l1)) >= kBulkMin) {
                                    pos += defer_leaf_run(t, l0, l1, ids, pos, end, e, G, gbase, plan.bulk,
                                                          plan.bulk_cap, ctrl, &bad);
                                    continue;
                                }
                            }
                            if (LAYOUT != LAYOUT_AOS && (G == 64 || l1 - l0 <= kNodeCopyLeaves)) {
                                // lane e copies entry e of U leaves at a time
                                const bool hasp = t.partial_leaf >= l0 && t.partial_leaf < l1;
                                constexpr uint32_t U = 4;
                                for (uint32_t lb = l0; lb < l1; lb += U) {
                                    uint32_t v[U];
                                    uint64_t o[U];
#pragma unroll
                                    for (uint32_t u = 0; u < U; ++u) {
                                        const uint32_t lf = lb + u;
                                        o[u] = ~0ull;
                                        v[u] = 0;
                                        if (lf < l1 && e < F && !(hasp && lf == t.partial_leaf && e >= t.partial_cnt)) {
                                            o[u] = pos + (uint64_t)(lf - l0) * F + e -
                                                   ((hasp && lf > t.partial_leaf) ? F - t.partial_cnt : 0u);
                                            v[u] = load_ptr<LAYOUT>(t.nodes + (size_t)lf * t.node_bytes, F, e);
                                        }
                                    }
#pragma unroll
                                    for (uint32_t u = 0; u < U; ++u) {
                                        if (o[u] != ~0ull) {
                                            if (o[u] < end)
                                                __builtin_nontemporal_store(v[u], ids + o[u]);
                                            else
                                                atomicOr(&ctrl->err, kErrBounds);
                                        }
                                    }
                                }
                                pos += subtree_objects(t, make_uint2(l0, l1));
                            } else
                                pos += copy_leaf_run<EXT != 0 ? 2 : 4>(t, l0, l1, ids, pos, end, e, G, &bad);
                        }
                        if (bad && e == 0) atomicOr(&ctrl->err, kErrBounds);
                    } else if constexpr (MODE == SEL_COUNT && EXT != 0) {
                        // one record per contained child: its leaf range, at
                        // the position after the contained children before it
                        const uint2 rg = cont ? t.range[first + e] : make_uint2(0u, 0u);
                        const uint32_t sc = cont ? subtree_objects(t, rg) : 0u;
                        uint32_t inc = sc;
                        for (uint32_t d = 1; d < G; d <<= 1) {
                            const uint32_t x = (uint32_t)__shfl_up((int)inc, d, G);
                            if (e >= d) inc += x;
                        }
                        const uint32_t tot = (uint32_t)__shfl((int)inc, (int)(gbase + G - 1));
                        const uint32_t k = (uint32_t)__popcll(cm);
                        if (nbuf + k > kRecBuf) rec_flush();
                        if (cont)
                            rbuf[nbuf + (uint32_t)__popcll(cm & below)] =
                                make_uint4(oslot, (uint32_t)pos + inc - sc, kRecRun | rg.x, rg.y);
                        nbuf += k;
                        pos += tot;
                    } else {
                        uint32_t sc = cont ? subtree_objects(t, t.range[first + e]) : 0u;
                        for (uint32_t d = 1; d < G; d <<= 1) sc += (uint32_t)__shfl_xor((int)sc, (int)d);
                        pos += sc;
                        if constexpr (MODE == SEL_STATS) vcont += sc;
                    }
                }
                const uint32_t prank = (uint32_t)__popcll(pm & below);
                if (hit && !cont) {
                    if (sp + prank < stack_cap)
                        stk[sp + prank] = first + e;
                    else
                        atomicOr(&ctrl->err, kErrStack);
                }
                sp = min(sp + (uint32_t)__popcll(pm), stack_cap);
            }
        }
        __builtin_amdgcn_wave_barrier();
    }
    if constexpr (MODE == SEL_COUNT && EXT != 0) {
        rec_flush();
        if (e == 0 && rchunk < kRecDead) plan.rec_count[rchunk] = rcnt;
    }
    if constexpr (MODE == SEL_STATS) {
        if (e == 0 && (vnodes | ventries)) {
            atomicAdd((unsigned long long *)&ctrl->stats[0], (unsigned long long)vnodes);
            atomicAdd((unsigned long long *)&ctrl->stats[1], (unsigned long long)ventries);
            atomicAdd((unsigned long long *)&ctrl->stats[2], (unsigned long long)vcont);
        }
    }
}

// Split pre-pass.  Walks only the internal levels above the parents of leaves
// (`split_parent` is the first node of the level above them) and finds the
// parents-of-leaves nodes a query reaches.  PHASE 0 counts them: a query reaching at least
// kmin of them (while the item budget lasts) gets one output slot per such
// node, others one slot.  PHASE 1 (after a scan of the slot counts) writes
// one work item {query, node, slot} per node of every split query.  Both
// phases walk identically, so the items match the counts.
template <int G, int LAYOUT, int PHASE>
__global__ void __launch_bounds__(256)
split_kernel(TreeView t, const float4 *__restrict__ qs, uint32_t nq, uint32_t split_parent, uint32_t kmin,
             uint32_t hcap, float min_area, uint32_t *__restrict__ nslots, const uint64_t *__restrict__ slot_first,
             uint4 *__restrict__ heavy, const uint64_t *__restrict__ order, Ctrl *__restrict__ ctrl,
             uint32_t stack_cap) {
    extern __shared__ uint32_t smem[];
    const uint32_t lane = threadIdx.x & 63u;
    const uint32_t e = lane & (G - 1);
    const uint32_t gbase = lane & ~(uint32_t)(G - 1);
    uint32_t *stk = smem + (threadIdx.x / G) * stack_cap;
    const uint32_t F = t.fanout;
    const uint64_t gmask = (G == 64) ? ~0ull : ((1ull << G) - 1ull);
    const uint64_t below = (e == 0) ? 0ull : (~0ull >> (64 - e));
    uint32_t qi = 0, sp = 0, k = 0, base = 0, slot0 = 0, list = 0;
    bool have = false, done = false;
    float4 q = make_float4(0.f, 0.f, 0.f, 0.f);
    const uint32_t home = blockIdx.x % kXcds;
    uint32_t visited = 0;
    while (true) {
        if (!done && sp == 0) {
            if (have && PHASE == 0 && e == 0) {
                uint32_t ns = 1;
                if (k >= kmin) {
                    const uint32_t old = atomicAdd(&ctrl->budget_used[list][0], k);
                    if (old + k <= hcap) ns = k;
                }
                nslots[qi] = ns;
            }
            have = false;
            uint32_t nxt = 0, b = 0, sl = 0;
            if (e == 0) {
                while (true) {
                    nxt = grab_query(ctrl, 2, nq, order, home, visited, &sl);
                    if (nxt >= nq) break;
                    const float4 w = qs[nxt];
                    if constexpr (PHASE == 0) {
                        // windows too small to reach kmin subtrees keep one slot
                        if (!((w.z - w.x) * (w.w - w.y) >= min_area)) {
                            nslots[nxt] = 1;
                            continue;
                        }
                        break;
                    } else {
                        const uint32_t ns = (uint32_t)(slot_first[nxt + 1] - slot_first[nxt]);
                        if (ns <= 1) continue;
                        b = (uint32_t)(sl * hcap) + atomicAdd(&ctrl->hlist[sl][0], ns);
                        break;
                    }
                }
            }
            nxt = __shfl(nxt, (int)gbase);
            b = __shfl(b, (int)gbase);
            sl = __shfl(sl, (int)gbase);
            if (nxt < nq) {
                qi = nxt;
                list = sl;
                have = true;
                q = qs[qi];
                stk[0] = 0u;
                sp = 1;
                k = 0;
                base = b;
                if constexpr (PHASE == 1) slot0 = (uint32_t)slot_first[qi];
            } else {
                done = true;
            }
        }
        if (__all(done)) break;
        __builtin_amdgcn_wave_barrier();
        uint32_t node = 0;
        if (have) {
            sp -= 1;
            node = stk[sp];
        }
        const uint8_t *nb = t.nodes + (size_t)node * t.node_bytes;
        bool hit = false;
        uint32_t ref = 0;
        if (have && e < F) {
            ref = load_ptr<LAYOUT>(nb, F, 0);
            float lx, ly, hx, hy;
            load_entry<LAYOUT>(nb, F, e, lx, ly, hx, hy);
            hit = (lx <= q.z) && (q.x <= hx) && (ly <= q.w) && (q.y <= hy);
        }
        const uint64_t m = (__ballot(hit) >> gbase) & gmask;
        const uint32_t n = (uint32_t)__popcll(m);
        const uint32_t rank = (uint32_t)__popcll(m & below);
        if (have) {
            // group-uniform test: only nodes above the parents-of-leaves level are
            // ever pushed, so a popped node at or past split_parent (the first
            // grandparent-of-leaves node) has parents of leaves as children
            if (node >= split_parent) {
                // the children are parents of leaves: they are the split nodes
                if constexpr (PHASE == 1) {
                    if (hit) heavy[base + k + rank] = make_uint4(qi, ref + e, slot0 + k + rank, 0u);
                }
                k += n;
            } else {
                if (hit) {
                    if (sp + rank < stack_cap)
                        stk[sp + rank] = ref + e;
                    else
                        atomicOr(&ctrl->err, kErrStack);
                }
                sp = min(sp + n, stack_cap);
            }
        }
        __builtin_amdgcn_wave_barrier();
    }
}

// Bulk copy of deferred contained runs: one block per descriptor at a time;
// stores start at a 64-byte boundary of the destination (the first ids up
// to it are written by the first lanes), so every store instruction writes
// whole granules.
__global__ void __launch_bounds__(256)
bulk_copy_kernel(const uint32_t *__restrict__ leaf_ids, const uint4 *__restrict__ bulk, uint32_t bulk_cap,
                 uint32_t *__restrict__ ids, Ctrl *__restrict__ ctrl) {
    __shared__ uint32_t item;
    const uint32_t nitems = min(ctrl->bulk_n, bulk_cap);
    const uint32_t t = threadIdx.x;
    while (true) {
        if (t == 0) item = atomicAdd(&ctrl->bulk_taken, 1u);
        __syncthreads();
        const uint32_t it = item;
        __syncthreads();
        if (it >= nitems) break;
        const uint4 d = bulk[it];
        const uint32_t *__restrict__ src = leaf_ids + d.x;
        uint32_t *__restrict__ dst = ids + (((uint64_t)d.z << 32) | d.y);
        const uint32_t len = d.w;
        const uint32_t head = min((16u - (uint32_t)((reinterpret_cast<uintptr_t>(dst) >> 2) & 15u)) & 15u, len);
        constexpr uint32_t U = 8;
        const uint32_t hv = t < head ? src[t] : 0u;   // loaded with the first round
        uint32_t k = head;
        do {
            uint32_t v[U];
#pragma unroll
            for (uint32_t u = 0; u < U; ++u) {
                const uint32_t i = k + u * 256 + t;
                v[u] = i < len ? src[i] : 0u;
            }
            if (k == head && t < head) put_id(dst + t, hv);
#pragma unroll
            for (uint32_t u = 0; u < U; ++u) {
                const uint32_t i = k + u * 256 + t;
                if (i < len) put_id(dst + i, v[u]);
            }
            k += 256 * U;
        } while (k < len);
    }
}

// Replay of the recording count pass: persistent blocks take record chunks;
// a chunk's records are staged in LDS with their absolute output positions
// (one offsets lookup per record, all loaded at once), then every half-wave
// takes records 8 apart, RU at a time: a leaf record writes the ids of its
// hit entries (lane l: entry l of the record's 32, at its rank in the hit
// mask), a range record copies the leaves' ids from the leaf-id array
// (measured faster than from the leaves' own ptr arrays: fill 2.81 against
// 4.13 ms at 10M rectangles / 1M windows, fanout 64 SoA).
template <int LAYOUT>
__global__ void __launch_bounds__(256)
replay_kernel(TreeView t, const uint64_t *__restrict__ offsets, uint32_t noffsets, uint32_t *__restrict__ ids,
              uint64_t cap, Ctrl *__restrict__ ctrl) {
    __shared__ uint64_t sbase[kRecChunk], send[kRecChunk];
    __shared__ uint2 sref[kRecChunk];
    const uint32_t nchunks = ctrl->rec_nchunks;
    if (!nchunks || ctrl->rec_overflow || offsets[noffsets] > cap) return;
    const uint4 *__restrict__ rec = ctrl->rec_base;
    const uint32_t *__restrict__ rec_count = ctrl->rec_count;
    const uint32_t nch = min(ctrl->rec_chunks, nchunks);
    const uint32_t th = threadIdx.x, hw = th >> 5, l = th & 31u;
    const uint32_t F = t.fanout;
    // records in flight per half-wave (4: fill 2.89 ms, 8: 2.81 at 10M rectangles / 1M windows, fanout 64
    // SoA; on the 50M-rectangle tree 5.70 against 4.05 ms); half-waves per block
    constexpr uint32_t U = 8, HW = 8;
    for (uint32_t c = blockIdx.x; c < nch; c += gridDim.x) {
        const uint32_t cnt = min(rec_count[c], kRecChunk);
        __syncthreads();   // the previous chunk's records are consumed
        if (th < cnt) {
            const uint4 d = get_rec(rec + (size_t)c * kRecChunk + th);
            sbase[th] = offsets[d.x] + d.y;
            send[th] = offsets[d.x + 1];
            sref[th] = make_uint2(d.z, d.w);
        }
        __syncthreads();
        for (uint32_t r0 = hw; r0 < cnt; r0 += HW * U) {
            uint32_t v[U];
            uint64_t o[U];
#pragma unroll
            for (uint32_t u = 0; u < U; ++u) {
                const uint32_t r = r0 + u * HW;
                o[u] = ~0ull;
                v[u] = 0;
                if (r < cnt) {
                    const uint2 d = sref[r];
                    if (!(d.x & kRecRun) && ((d.y >> l) & 1u)) {
                        const uint32_t node = d.x & ~kRecHi;
                        const uint32_t ent = ((d.x & kRecHi) ? 32u : 0u) + l;
                        v[u] = load_ptr<LAYOUT>(t.nodes + (size_t)node * t.node_bytes, F, ent);
                        o[u] = sbase[r] + (uint32_t)__popc(d.y & ((1u << l) - 1u));
                        if (o[u] >= send[r]) {
                            atomicOr(&ctrl->err, kErrBounds);
                            o[u] = ~0ull;
                        }
                    }
                }
            }
            // a leaf record's ids are a short run next to the runs of the
            // records beside it in the chunk (the same block, the same L2):
            // cached stores let L2 merge their partly written lines, where
            // stores that bypass it write each part to memory on its own
            // (fill 2.83 -> 2.67 ms at 10M rectangles / 1M windows).  Range
            // copies write whole lines and keep the bypassing stores.
#pragma unroll
            for (uint32_t u = 0; u < U; ++u)
                if (o[u] != ~0ull) ids[o[u]] = v[u];
#pragma unroll 1
            for (uint32_t u = 0; u < U; ++u) {
                const uint32_t r = r0 + u * HW;
                if (r >= cnt) break;
                const uint2 d = sref[r];
                if (!(d.x & kRecRun)) continue;
                const uint32_t l0 = d.x & ~kRecRun, l1 = d.y;
                const uint64_t s0 = leaf_start(t, l0);
                const uint64_t n = leaf_start(t, l1) - s0;
                const uint64_t b = sbase[r];
                if (b + n > send[r]) {
                    if (l == 0) atomicOr(&ctrl->err, kErrBounds);
                    continue;
                }
                {
                    const uint32_t *__restrict__ src = t.leaf_ids + s0;
                    constexpr uint32_t RU = 8;   // 16: more registers, fill 4.2 ms
                    for (uint64_t i0 = l; i0 < n; i0 += 32 * RU) {
                        uint32_t w[RU];
#pragma unroll
                        for (uint32_t k = 0; k < RU; ++k) {
                            const uint64_t i = i0 + 32 * k;
                            w[k] = i < n ? src[i] : 0u;
                        }
#pragma unroll
                        for (uint32_t k = 0; k < RU; ++k) {
                            const uint64_t i = i0 + 32 * k;
                            if (i < n) put_id(ids + b + i, w[k]);
                        }
                    }
                }
            }
        }
    }
}

__global__ void set_rec_kernel(Ctrl *ctrl, uint4 *rec, uint32_t *rec_count, uint32_t nchunks) {
    ctrl->rec_base = rec;
    ctrl->rec_count = rec_count;
    ctrl->rec_nchunks = nchunks;
}

hipError_t launch_set_rec(Ctrl *ctrl, const SelectPlan &plan, hipStream_t s) {
    hipLaunchKernelGGL(set_rec_kernel, dim3(1), dim3(1), 0, s, ctrl, plan.rec, plan.rec_count, plan.rec_nchunks);
    return hipGetLastError();
}

hipError_t launch_replay(const TreeView &t, const uint64_t *offsets, uint32_t noffsets, uint32_t *ids,
                         uint64_t cap, Ctrl *ctrl, hipStream_t s) {
    const dim3 grid((uint32_t)num_cus() * 8), block(256);
    if (t.layout == LAYOUT_AOS)
        hipLaunchKernelGGL(replay_kernel<LAYOUT_AOS>, grid, block, 0, s, t, offsets, noffsets, ids, cap, ctrl);
    else if (t.layout == LAYOUT_SOA)
        hipLaunchKernelGGL(replay_kernel<LAYOUT_SOA>, grid, block, 0, s, t, offsets, noffsets, ids, cap, ctrl);
    else
        hipLaunchKernelGGL(replay_kernel<LAYOUT_D2>, grid, block, 0, s, t, offsets, noffsets, ids, cap, ctrl);
    return hipGetLastError();
}

hipError_t launch_bulk_copy(const uint32_t *leaf_ids, const uint4 *bulk, uint32_t bulk_cap, uint32_t *ids, Ctrl *ctrl,
                            hipStream_t s) {
    hipLaunchKernelGGL(bulk_copy_kernel, dim3((uint32_t)num_cus() * 8), dim3(256), 0, s, leaf_ids, bulk, bulk_cap,
                       ids, ctrl);
    return hipGetLastError();
}

int num_cus() {
    static int cus = 0;
    if (!cus) {
        int dev = 0;
        if (hipGetDevice(&dev) != hipSuccess) return 256;
        hipDeviceProp_t p;
        if (hipGetDeviceProperties(&p, dev) != hipSuccess) return 256;
        cus = p.multiProcessorCount > 0 ? p.multiProcessorCount : 256;
    }
    return cus;
}

template <int G, int LAYOUT, int MODE>
static hipError_t launch_g(const TreeView &t, const float4 *q, uint32_t nq, uint32_t *counts,
                           const uint64_t *offsets, uint32_t *ids, uint64_t cap, Ctrl *ctrl,
                           uint32_t slot, const SelectPlan &plan, uint32_t noffsets, hipStream_t s) {
    const uint32_t stack_cap = stack_bound(t.height, t.fanout);
    const uint32_t groups_per_block = 256 / G;
    size_t smem = (size_t)groups_per_block * stack_cap * sizeof(uint32_t);
    if (MODE == SEL_COUNT && plan.rec)   // the groups' record buffers follow the stacks, 16-byte aligned
        smem = (smem + 15) / 16 * 16 + (size_t)groups_per_block * kRecBuf * 16;
    uint64_t want = ((uint64_t)nq + groups_per_block - 1) / groups_per_block;
    uint64_t persistent = (uint64_t)num_cus() * 8;
    uint32_t blocks = (uint32_t)(want < persistent ? want : persistent);
    if (plan.heavy) blocks = (uint32_t)persistent;   // split items add work beyond nq
    blocks = (blocks + kXcds - 1) / kXcds * kXcds;   // every XCD gets blocks
    // the fill pass with deferred contained runs is an instance of its own:
    // the deferral branch costs the in-pass copies registers and time
    // (and the recording count pass likewise)
    const bool la = MODE != SEL_STATS && t.lookahead;
    constexpr int EXT = MODE == SEL_STATS ? 0 : 1;
    if ((MODE == SEL_FILL && plan.bulk) || (MODE == SEL_COUNT && plan.rec)) {
        if (la)
            hipLaunchKernelGGL((select_kernel<G, LAYOUT, MODE, 1, EXT>), dim3(blocks), dim3(256), smem, s,
                               t, q, nq, counts, offsets, ids, cap, ctrl, slot, stack_cap, plan, noffsets);
        else
            hipLaunchKernelGGL((select_kernel<G, LAYOUT, MODE, 0, EXT>), dim3(blocks), dim3(256), smem, s,
                               t, q, nq, counts, offsets, ids, cap, ctrl, slot, stack_cap, plan, noffsets);
    } else if (la)
        hipLaunchKernelGGL((select_kernel<G, LAYOUT, MODE, 1, 0>), dim3(blocks), dim3(256), smem, s, t, q, nq,
                           counts, offsets, ids, cap, ctrl, slot, stack_cap, plan, noffsets);
    else
        hipLaunchKernelGGL((select_kernel<G, LAYOUT, MODE, 0, 0>), dim3(blocks), dim3(256), smem, s, t, q, nq,
                           counts, offsets, ids, cap, ctrl, slot, stack_cap, plan, noffsets);
    return hipGetLastError();
}

template <int G, int LAYOUT, int PHASE>
static hipError_t launch_split_g(const TreeView &t, const float4 *q, uint32_t nq, uint32_t split_first,
                                 uint32_t kmin, uint32_t budget, float min_area, uint32_t *nslots,
                                 const uint64_t *slot_first, uint4 *heavy, const uint64_t *order, Ctrl *ctrl,
                                 hipStream_t s) {
    const uint32_t stack_cap = stack_bound(t.height, t.fanout);
    const uint32_t groups_per_block = 256 / G;
    const size_t smem = (size_t)groups_per_block * stack_cap * sizeof(uint32_t);
    uint64_t want = ((uint64_t)nq + groups_per_block - 1) / groups_per_block;
    uint64_t persistent = (uint64_t)num_cus() * 8;
    uint32_t blocks = (uint32_t)(want < persistent ? want : persistent);
    blocks = (blocks + kXcds - 1) / kXcds * kXcds;
    hipLaunchKernelGGL((split_kernel<G, LAYOUT, PHASE>), dim3(blocks), dim3(256), smem, s, t, q, nq, split_first,
                       kmin, budget, min_area, nslots, slot_first, heavy, order, ctrl, stack_cap);
    return hipGetLastError();
}

template <int G, int LAYOUT>
static hipError_t launch_m(const TreeView &t, const float4 *q, uint32_t nq, int mode, uint32_t *counts,
                           const uint64_t *offsets, uint32_t *ids, uint64_t cap, Ctrl *ctrl,
                           uint32_t slot, const SelectPlan &plan, uint32_t noffsets, hipStream_t s) {
    switch (mode) {
    case SEL_COUNT:
        return launch_g<G, LAYOUT, SEL_COUNT>(t, q, nq, counts, offsets, ids, cap, ctrl, slot, plan, noffsets, s);
    case SEL_FILL:
        return launch_g<G, LAYOUT, SEL_FILL>(t, q, nq, counts, offsets, ids, cap, ctrl, slot, plan, noffsets, s);
    default:
        return launch_g<G, LAYOUT, SEL_STATS>(t, q, nq, counts, offsets, ids, cap, ctrl, slot, plan, noffsets, s);
    }
}

template <int G>
static hipError_t launch_l(const TreeView &t, const float4 *q, uint32_t nq, int mode, uint32_t *counts,
                           const uint64_t *offsets, uint32_t *ids, uint64_t cap, Ctrl *ctrl,
                           uint32_t slot, const SelectPlan &plan, uint32_t noffsets, hipStream_t s) {
    switch (t.layout) {
    case LAYOUT_AOS:
        return launch_m<G, LAYOUT_AOS>(t, q, nq, mode, counts, offsets, ids, cap, ctrl, slot, plan, noffsets, s);
    case LAYOUT_SOA:
        return launch_m<G, LAYOUT_SOA>(t, q, nq, mode, counts, offsets, ids, cap, ctrl, slot, plan, noffsets, s);
    default:
        return launch_m<G, LAYOUT_D2>(t, q, nq, mode, counts, offsets, ids, cap, ctrl, slot, plan, noffsets, s);
    }
}

hipError_t launch_select_pass(const TreeView &t, const float4 *q, uint32_t nq, int mode,
                              uint32_t *counts, const uint64_t *offsets, uint32_t *ids,
                              uint64_t cap, Ctrl *ctrl, uint32_t slot, const SelectPlan &plan,
                              uint32_t noffsets, hipStream_t s) {
    switch (group_width(t.fanout)) {
    case 16:
        return launch_l<16>(t, q, nq, mode, counts, offsets, ids, cap, ctrl, slot, plan, noffsets, s);
    case 32:
        return launch_l<32>(t, q, nq, mode, counts, offsets, ids, cap, ctrl, slot, plan, noffsets, s);
    default:
        return launch_l<64>(t, q, nq, mode, counts, offsets, ids, cap, ctrl, slot, plan, noffsets, s);
    }
}

template <int PHASE>
static hipError_t launch_split_phase(const TreeView &t, const float4 *q, uint32_t nq, uint32_t split_first,
                                     uint32_t kmin, uint32_t budget, float min_area, uint32_t *nslots,
                                     const uint64_t *slot_first, uint4 *heavy, const uint64_t *order, Ctrl *ctrl,
                                     hipStream_t s) {
#define RT_SPLIT(G_, L_) \
    launch_split_g<G_, L_, PHASE>(t, q, nq, split_first, kmin, budget, min_area, nslots, slot_first, heavy, order, \
                                  ctrl, s)
    const uint32_t G = group_width(t.fanout);
    if (t.layout == LAYOUT_AOS) return G == 16 ? RT_SPLIT(16, LAYOUT_AOS) : G == 32 ? RT_SPLIT(32, LAYOUT_AOS) : RT_SPLIT(64, LAYOUT_AOS);
    if (t.layout == LAYOUT_SOA) return G == 16 ? RT_SPLIT(16, LAYOUT_SOA) : G == 32 ? RT_SPLIT(32, LAYOUT_SOA) : RT_SPLIT(64, LAYOUT_SOA);
    return G == 16 ? RT_SPLIT(16, LAYOUT_D2) : G == 32 ? RT_SPLIT(32, LAYOUT_D2) : RT_SPLIT(64, LAYOUT_D2);
#undef RT_SPLIT
}

hipError_t launch_split(const TreeView &t, const float4 *q, uint32_t nq, int phase, uint32_t split_parent,
                        uint32_t kmin, uint32_t hcap, float min_area, uint32_t *nslots, const uint64_t *slot_first,
                        uint4 *heavy, const uint64_t *order, Ctrl *ctrl, hipStream_t s) {
    return phase == 0 ? launch_split_phase<0>(t, q, nq, split_parent, kmin, hcap, min_area, nslots, slot_first,
                                              heavy, order, ctrl, s)
                      : launch_split_phase<1>(t, q, nq, split_parent, kmin, hcap, min_area, nslots, slot_first,
                                              heavy, order, ctrl, s);
}

// offsets[q] = slot_offsets[slot_first[q]] for q <= nq (the CSR of whole
// queries from the CSR of output slots)
__global__ void gather_offsets(const uint64_t *__restrict__ slot_first, const uint64_t *__restrict__ slot_off,
                               uint32_t nq, uint64_t *__restrict__ offsets) {
    for (uint32_t i = blockIdx.x * blockDim.x + threadIdx.x; i <= nq; i += gridDim.x * blockDim.x)
        offsets[i] = slot_off[slot_first[i]];
}

hipError_t launch_gather_offsets(const uint64_t *slot_first, const uint64_t *slot_off, uint32_t nq,
                                 uint64_t *offsets, hipStream_t s) {
    uint32_t blocks = (nq + 256) / 256;
    if (blocks > 4096) blocks = 4096;
    hipLaunchKernelGGL(gather_offsets, dim3(blocks), dim3(256), 0, s, slot_first, slot_off, nq, offsets);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// query order for locality
// ---------------------------------------------------------------------------
__device__ __forceinline__ uint32_t spread16(uint32_t v) {
    v &= 0xFFFFu;
    v = (v | (v << 8)) & 0x00FF00FFu;
    v = (v | (v << 4)) & 0x0F0F0F0Fu;
    v = (v | (v << 2)) & 0x33333333u;
    v = (v | (v << 1)) & 0x55555555u;
    return v;
}

// Morton (Z-order) code of each window center on a 65536 x 65536 grid over
// the tree's MBR.  Only the processing order depends on it; no result does.
__global__ void query_morton(const float4 *__restrict__ q, uint32_t nq, float lx, float ly, float sx, float sy,
                             uint64_t *__restrict__ keys) {
    for (uint32_t i = blockIdx.x * blockDim.x + threadIdx.x; i < nq; i += gridDim.x * blockDim.x) {
        const float4 w = q[i];
        float cx = (0.5f * w.x + 0.5f * w.z - lx) * sx;
        float cy = (0.5f * w.y + 0.5f * w.w - ly) * sy;
        cx = fminf(fmaxf(cx, 0.f), 65535.f);   // NaN -> 0
        cy = fminf(fmaxf(cy, 0.f), 65535.f);
        const uint32_t code = spread16((uint32_t)cx) | (spread16((uint32_t)cy) << 1);
        keys[i] = ((uint64_t)code << 32) | i;
    }
}

static uint64_t al256(uint64_t b) { return (b + 255) & ~255ull; }

// The order sorts on the top 22 bits of the 32-bit Morton code (11 bits per
// axis, a 2048 x 2048 grid over the tree's MBR) in two 11-bit passes; the
// order inside a grid cell does not matter for locality.
constexpr int kOrderDigitBits = 11;

uint64_t order_ws_bytes(uint64_t nq) {
    const uint64_t he = radix_hist_elems(nq, kOrderDigitBits);
    return al256(8 * nq) * 2 + al256(4 * he) + al256(8 * (he + 1)) + al256(8 * scan_tmp_elems(he + 1));
}

hipError_t launch_query_order(const float4 *q, uint32_t nq, const float *mbr, void *ws, const uint64_t **sorted,
                              hipStream_t s) {
    uint8_t *p = static_cast<uint8_t *>(ws);
    uint64_t *keys = reinterpret_cast<uint64_t *>(p);
    p += al256(8 * (uint64_t)nq);
    uint64_t *tmp = reinterpret_cast<uint64_t *>(p);
    p += al256(8 * (uint64_t)nq);
    const uint64_t he = radix_hist_elems(nq, kOrderDigitBits);
    uint32_t *hist = reinterpret_cast<uint32_t *>(p);
    p += al256(4 * he);
    uint64_t *hscan = reinterpret_cast<uint64_t *>(p);
    p += al256(8 * (he + 1));
    uint64_t *stmp = reinterpret_cast<uint64_t *>(p);
    float lx = mbr[0], ly = mbr[1], w = mbr[2] - mbr[0], h = mbr[3] - mbr[1];
    const bool ok = (w > 0.f) && (h > 0.f) && (w < 3.0e38f) && (h < 3.0e38f);
    const float sx = ok ? 65535.f / w : 0.f, sy = ok ? 65535.f / h : 0.f;
    if (!ok) lx = ly = 0.f;
    uint32_t blocks = (nq + 255) / 256;
    if (blocks > 4096) blocks = 4096;
    hipLaunchKernelGGL(query_morton, dim3(blocks), dim3(256), 0, s, q, nq, lx, ly, sx, sy, keys);
    // two passes (an even number): the sorted keys end in the first buffer
    const int shifts[2] = {42, 53};
    bool in_tmp = false;
    hipError_t e =
        launch_radix_sort_u64(keys, tmp, nq, shifts, 2, hist, hscan, stmp, &in_tmp, s, kOrderDigitBits);
    *sorted = keys;
    if (e == hipSuccess && in_tmp) e = hipErrorUnknown;
    return e == hipSuccess ? hipGetLastError() : e;
}

const uint64_t *query_order_result(const void *ws, uint64_t nq) {
    (void)nq;
    return static_cast<const uint64_t *>(ws);
}

}  // namespace rtk
