// Persistent multi-tree range-select pass.
//
// A device work queue holds (tree, query-chunk) items for many independent
// trees that may differ in fanout and node layout.  The items are kept in one
// list per XCD: a tree's items go to one XCD (a large tree's are cut into
// contiguous runs of its processing order, one per XCD), so that each tree's
// nodes are shared in one XCD's L2.  A wave takes one item at a time from its
// XCD's list (then from the others when that is drained), configures its
// lanes into groups of G = group_width(F) lanes for that tree, and runs the
// same per-query depth-first traversal as the single-tree kernel (lanes over
// node entries, __ballot masks, LDS stacks).  Groups of a wave pick the
// item's queries in order with a wave-local ballot, so only one global
// atomic is spent per item; the queries of a tree are visited in the Morton
// order of their centres, so consecutive queries share nodes.
#include "rt_internal.h"

namespace rtk {

template <int LAYOUT>
__device__ __forceinline__ void batch_load(const uint8_t *nb, uint32_t F, uint32_t e, float &lx, float &ly, float &hx,
                                           float &hy) {
    if constexpr (LAYOUT == LAYOUT_SOA) {
        const float *f = reinterpret_cast<const float *>(nb);
        lx = f[e];
        ly = f[F + e];
        hx = f[2 * F + e];
        hy = f[3 * F + e];
    } else if constexpr (LAYOUT == LAYOUT_AOS) {
        const float *f = reinterpret_cast<const float *>(nb) + 5 * e;
        lx = f[0];
        ly = f[1];
        hx = f[2];
        hy = f[3];
    } else {
        const float2 *lo = reinterpret_cast<const float2 *>(nb);
        const float2 a = lo[e], b = lo[F + e];
        lx = a.x;
        ly = a.y;
        hx = b.x;
        hy = b.y;
    }
}

template <int LAYOUT>
__device__ __forceinline__ uint32_t batch_ptr(const uint8_t *nb, uint32_t F, uint32_t e) {
    const uint32_t *u = reinterpret_cast<const uint32_t *>(nb);
    if constexpr (LAYOUT == LAYOUT_AOS) return u[5 * e + 4];
    return u[4 * F + e];
}

// Next item for a wave leader: from XCD `home`'s list first, then from the
// following lists in turn (`visited` counts the lists found drained).
__device__ __forceinline__ uint32_t grab_item(Ctrl *ctrl, uint32_t slot, const uint32_t *list_begin, uint32_t home,
                                              uint32_t &visited) {
    while (visited < kXcds) {
        const uint32_t x = (home + visited) % kXcds;
        const uint32_t b0 = list_begin[x], b1 = list_begin[x + 1];
        // a drained list's counter only grows: a read showing it drained is
        // final, and the atomic that idle waves would queue on is skipped
        if (visited > 0 &&
            __hip_atomic_load(&ctrl->xwork[slot][x][0], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) >= b1 - b0) {
            visited += 1;
            continue;
        }
        const uint32_t k = atomicAdd(&ctrl->xwork[slot][x][0], 1u);
        if (k < b1 - b0) return b0 + k;
        visited += 1;
    }
    return kNoNode;
}

// One work item: the queries [item.q0, item.q1) of one tree's processing
// order, run by the wave's groups of G lanes on a tree of node layout LAYOUT.
template <int MODE, int G, int LAYOUT, int REC>
__device__ __forceinline__ void batch_item(const BatchTree &bt, const BatchItem &item, const uint32_t *__restrict__ qorder,
                                           const float4 *__restrict__ qs, uint32_t *__restrict__ counts,
                                           const uint64_t *__restrict__ offsets, uint32_t *__restrict__ ids,
                                           Ctrl *__restrict__ ctrl, uint32_t *wstk, uint32_t lane,
                                           uint64_t lanes_below, const BatchRec &rp, uint4 *wrec) {
    const TreeView &t = bt.t;
    const uint32_t F = t.fanout;
    const uint32_t e = lane & (G - 1);
    const uint32_t gbase = lane & ~(G - 1);
    const uint64_t gmask = (G == 64) ? ~0ull : ((1ull << G) - 1ull);
    const uint64_t below = (e == 0) ? 0ull : (~0ull >> (64 - e));
    uint32_t *stk = wstk + (lane / G) * bt.stack_cap;
    uint32_t nextq = item.q0;   // wave-uniform
    uint64_t gq = 0;            // global query index of the group's query
    bool have = false, done = false;
    uint32_t sp = 0;
    float4 q = make_float4(0.f, 0.f, 0.f, 0.f);
    uint64_t pos = 0, end = 0;
    // recording count pass: as in the single-tree kernel, records collect in
    // the group's LDS buffer and go out kRecBuf at a time to the group's
    // chunk of the arena; the output slot of a record is the global query
    uint32_t rchunk = kNoNode, rcnt = 0, nbuf = 0;
    uint4 *rbuf = wrec + (lane / G) * kRecBuf;
    auto rec_flush = [&]() {   // group-uniform
        if (nbuf == 0) return;
        __builtin_amdgcn_wave_barrier();
        if (rchunk != kRecDead && (rchunk == kNoNode || rcnt + nbuf > kRecChunk)) {
            if (rchunk != kNoNode && e == 0) rp.rec_count[rchunk] = rcnt;
            uint32_t c = 0;
            if (e == 0) c = atomicAdd(&ctrl->rec_chunks, 1u);
            c = (uint32_t)__shfl((int)c, (int)gbase);
            if (c < rp.rec_nchunks) {
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
                put_rec(rp.rec + (size_t)rchunk * kRecChunk + rcnt + i, v.x, v.y, v.z, v.w);
            }
            rcnt += nbuf;
        }
        nbuf = 0;
        __builtin_amdgcn_wave_barrier();
    };

    while (true) {
        const bool need = !done && sp == 0;
        if (need && have) {
            if constexpr (MODE == SEL_COUNT) {
                if (e == 0) counts[gq] = (uint32_t)pos;
            }
            have = false;
        }
        // leaders of needy groups take consecutive queries of the item
        const uint64_t lead = __ballot(need && e == 0);
        const uint32_t r = (uint32_t)__popcll(lead & lanes_below);
        uint32_t mine = __shfl(nextq + r, (int)gbase);
        nextq += (uint32_t)__popcll(lead);
        if (need) {
            if (mine < item.q1) {
                gq = bt.q_begin + qorder[bt.q_begin + mine];
                have = true;
                q = qs[gq];
                stk[0] = 0u;
                sp = 1;
                if constexpr (MODE == SEL_FILL) {
                    pos = offsets[gq];
                    end = offsets[gq + 1];
                } else {
                    pos = 0;
                }
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
        const bool leaf = node >= t.first_leaf;
        bool hit = false, cont = false;
        uint32_t ref = 0;
        if (have && e < F) {
            if (!leaf)
                ref = batch_ptr<LAYOUT>(nb, F, 0);
            else if constexpr (MODE == SEL_FILL)
                ref = batch_ptr<LAYOUT>(nb, F, e);
            float lx, ly, hx, hy;
            batch_load<LAYOUT>(nb, F, e, lx, ly, hx, hy);
            hit = (lx <= q.z) && (q.x <= hx) && (ly <= q.w) && (q.y <= hy);
            // internal entry inside the window: its subtree is taken whole
            cont = hit && !leaf && (q.x <= lx) && (hx <= q.z) && (q.y <= ly) && (hy <= q.w);
        }
        const uint64_t m = (__ballot(hit) >> gbase) & gmask;
        const uint64_t cm = (__ballot(cont) >> gbase) & gmask;
        const uint64_t pm = m & ~cm;
        const uint32_t n = (uint32_t)__popcll(m);
        const uint32_t rank = (uint32_t)__popcll(m & below);
        if (have) {
            if (leaf) {
                if constexpr (MODE == SEL_FILL) {
                    if (hit) {
                        const uint64_t o = pos + rank;
                        if (o < end)
                            put_id(ids + o, ref);
                        else
                            atomicOr(&ctrl->err, kErrBounds);
                    }
                }
                if constexpr (MODE == SEL_COUNT && REC != 0) {
                    if (n) {   // one record per 32 entries with hits
                        const uint32_t lo = (uint32_t)m, hi = (uint32_t)(m >> 32);
                        const uint32_t k = (lo ? 1u : 0u) + (hi ? 1u : 0u);
                        if (nbuf + k > kRecBuf) rec_flush();
                        if (e == 0 && lo) rbuf[nbuf] = make_uint4((uint32_t)gq, (uint32_t)pos, node, lo);
                        if (G == 64 && e == 32 && hi)
                            rbuf[nbuf + (lo ? 1u : 0u)] =
                                make_uint4((uint32_t)gq, (uint32_t)pos + (uint32_t)__popc(lo), node | kRecHi, hi);
                        nbuf += k;
                    }
                }
                pos += n;
            } else {
                const uint32_t first = __shfl(ref, (int)gbase);
                if (cm) {   // group-uniform: contained subtrees
                    if constexpr (MODE == SEL_FILL) {
                        // one contiguous run of the leaf-id array per run
                        // of consecutive contained children
                        uint64_t todo = cm;
                        bool bad = false;
                        while (todo) {
                            const uint32_t j0 = (uint32_t)__builtin_ctzll(todo);
                            const uint64_t sh = todo >> j0;
                            const uint32_t len = ~sh ? (uint32_t)__builtin_ctzll(~sh) : 64u - j0;
                            todo = (j0 + len >= 64) ? 0ull : (todo & (~0ull << (j0 + len)));
                            const uint32_t l0 = t.range[first + j0].x, l1 = t.range[first + j0 + len - 1].y;
                            pos += copy_leaf_run<4>(t, l0, l1, ids, pos, end, e, G, &bad);
                        }
                        if (bad && e == 0) atomicOr(&ctrl->err, kErrBounds);
                    } else if constexpr (REC != 0) {
                        // one record per contained child: its leaf range
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
                                make_uint4((uint32_t)gq, (uint32_t)pos + inc - sc, kRecRun | rg.x, rg.y);
                        nbuf += k;
                        pos += tot;
                    } else {
                        uint32_t sc = cont ? subtree_objects(t, t.range[first + e]) : 0u;
                        for (uint32_t d = 1; d < G; d <<= 1) sc += (uint32_t)__shfl_xor((int)sc, (int)d);
                        pos += sc;
                    }
                }
                const uint32_t prank = (uint32_t)__popcll(pm & below);
                if (hit && !cont) {
                    if (sp + prank < bt.stack_cap)
                        stk[sp + prank] = first + e;
                    else
                        atomicOr(&ctrl->err, kErrStack);
                }
                sp = min(sp + (uint32_t)__popcll(pm), bt.stack_cap);
            }
        }
        __builtin_amdgcn_wave_barrier();
    }
    if constexpr (MODE == SEL_COUNT && REC != 0) {
        rec_flush();
        if (e == 0 && rchunk < kRecDead) rp.rec_count[rchunk] = rcnt;
    }
}

template <int MODE, int REC>
__global__ void __launch_bounds__(256)
batch_kernel(const BatchTree *__restrict__ trees, const BatchItem *__restrict__ items,
             const uint32_t *__restrict__ list_begin, uint32_t nitems, const uint32_t *__restrict__ qorder,
             const float4 *__restrict__ qs, uint32_t *__restrict__ counts, const uint64_t *__restrict__ offsets,
             uint32_t *__restrict__ ids, uint64_t cap, uint64_t total_q, Ctrl *__restrict__ ctrl, uint32_t slot,
             uint32_t wave_words, BatchRec rp) {
    extern __shared__ uint32_t smem[];
    if constexpr (MODE == SEL_FILL) {
        if (offsets[total_q] > cap) return;
        if (rp.fill_guard && ctrl->rec_overflow == 0) return;   // the replay wrote everything
    }
    const uint32_t lane = threadIdx.x & 63u;
    uint32_t *wstk = smem + (threadIdx.x >> 6) * wave_words;
    // record buffers (recording count pass): after the four waves' stacks,
    // 16-byte aligned, 64 / 16 groups of kRecBuf records per wave
    uint4 *wrec = reinterpret_cast<uint4 *>(smem + (4 * wave_words + 3u) / 4u * 4u) + (threadIdx.x >> 6) * 4 * kRecBuf;
    const uint64_t lanes_below = lane ? (~0ull >> (64 - lane)) : 0ull;
    const uint32_t home = blockIdx.x % kXcds;
    uint32_t visited = 0;

    while (true) {
        uint32_t it = kNoNode;
        if (lane == 0) it = grab_item(ctrl, slot, list_begin, home, visited);
        it = __shfl(it, 0);
        visited = __shfl(visited, 0);
        if (it >= nitems) break;
        const BatchItem item = items[it];
        const BatchTree bt = trees[item.tree];
        const uint32_t G = bt.t.fanout <= 16 ? 16u : (bt.t.fanout <= 32 ? 32u : 64u);
#define RT_ITEM(G_, L_) \
    batch_item<MODE, G_, L_, REC>(bt, item, qorder, qs, counts, offsets, ids, ctrl, wstk, lane, lanes_below, rp, wrec)
        if (bt.t.layout == LAYOUT_SOA) {
            if (G == 16) RT_ITEM(16, LAYOUT_SOA);
            else if (G == 32) RT_ITEM(32, LAYOUT_SOA);
            else RT_ITEM(64, LAYOUT_SOA);
        } else if (bt.t.layout == LAYOUT_AOS) {
            if (G == 16) RT_ITEM(16, LAYOUT_AOS);
            else if (G == 32) RT_ITEM(32, LAYOUT_AOS);
            else RT_ITEM(64, LAYOUT_AOS);
        } else {
            if (G == 16) RT_ITEM(16, LAYOUT_D2);
            else if (G == 32) RT_ITEM(32, LAYOUT_D2);
            else RT_ITEM(64, LAYOUT_D2);
        }
#undef RT_ITEM
    }
}

hipError_t launch_batch_pass(const BatchTree *trees, const BatchItem *items, const uint32_t *list_begin,
                             uint32_t nitems, const uint32_t *qorder, const float4 *q, int mode, uint32_t *counts,
                             const uint64_t *offsets, uint32_t *ids, uint64_t cap, uint64_t total_q, Ctrl *ctrl,
                             uint32_t slot, uint32_t wave_words, const BatchRec &rp, hipStream_t s) {
    // wave_words: largest (64 / G) * stack_cap over the trees (one region per wave)
    size_t smem = (size_t)4 * wave_words * sizeof(uint32_t);
    const bool rec = mode == SEL_COUNT && rp.rec;
    if (rec) smem = (smem + 15) / 16 * 16 + (size_t)4 * 4 * kRecBuf * 16;
    uint32_t blocks = (uint32_t)num_cus() * 8;
    const uint32_t want = (nitems + 3) / 4;
    if (want < blocks) blocks = want ? want : 1;
    blocks = (blocks + kXcds - 1) / kXcds * kXcds;   // every XCD gets blocks
    if (rec)
        hipLaunchKernelGGL((batch_kernel<SEL_COUNT, 1>), dim3(blocks), dim3(256), smem, s, trees, items, list_begin,
                           nitems, qorder, q, counts, offsets, ids, cap, total_q, ctrl, slot, wave_words, rp);
    else if (mode == SEL_COUNT)
        hipLaunchKernelGGL((batch_kernel<SEL_COUNT, 0>), dim3(blocks), dim3(256), smem, s, trees, items, list_begin,
                           nitems, qorder, q, counts, offsets, ids, cap, total_q, ctrl, slot, wave_words, rp);
    else
        hipLaunchKernelGGL((batch_kernel<SEL_FILL, 0>), dim3(blocks), dim3(256), smem, s, trees, items, list_begin,
                           nitems, qorder, q, counts, offsets, ids, cap, total_q, ctrl, slot, wave_words, rp);
    return hipGetLastError();
}

// Replay of the recording batch count pass (records' slots are global query
// indices; qtree gives a query's tree).  As the single-tree replay, with the
// source of each record resolved in the staging step: a leaf record's ptr
// array (address of its first entry and the stride between entries: 20
// bytes in AoS, 4 otherwise), a range record's run of its tree's leaf-id
// array.
__global__ void __launch_bounds__(256)
batch_replay_kernel(const BatchTree *__restrict__ trees, const uint32_t *__restrict__ qtree,
                    const uint4 *__restrict__ rec, const uint32_t *__restrict__ rec_count, uint32_t nchunks,
                    const uint64_t *__restrict__ offsets, uint64_t total_q, uint32_t *__restrict__ ids, uint64_t cap,
                    Ctrl *__restrict__ ctrl) {
    constexpr uint32_t U = 8, HW = 8;
    __shared__ uint64_t ssrc[kRecChunk], sbase[kRecChunk];
    __shared__ uint32_t sinfo[kRecChunk];   // leaf: stride; range: id count
    __shared__ uint32_t smask[kRecChunk];   // leaf: hit mask; range: 0 (and sinfo's top bit set)
    constexpr uint32_t kRange = 0x80000000u;
    if (ctrl->rec_overflow || offsets[total_q] > cap) return;
    const uint32_t nch = min(ctrl->rec_chunks, nchunks);
    const uint32_t th = threadIdx.x, hw = th >> 5, l = th & 31u;
    for (uint32_t c = blockIdx.x; c < nch; c += gridDim.x) {
        const uint32_t cnt = min(rec_count[c], kRecChunk);
        __syncthreads();
        if (th < cnt) {
            const uint4 d = get_rec(rec + (size_t)c * kRecChunk + th);
            const uint64_t b = offsets[d.x] + d.y, en = offsets[d.x + 1];
            const TreeView &t = trees[qtree[d.x]].t;
            uint64_t src = 0;
            uint32_t info = 0, mask = 0;
            if (d.z & kRecRun) {
                const uint64_t s0 = leaf_start(t, d.z & ~kRecRun);
                const uint64_t n = leaf_start(t, d.w) - s0;
                src = reinterpret_cast<uint64_t>(t.leaf_ids + s0);
                info = kRange | (uint32_t)n;
                if (b + n > en || n >= kRange) {
                    atomicOr(&ctrl->err, kErrBounds);
                    info = kRange;
                }
            } else {
                const uint32_t node = d.z & ~kRecHi, half = (d.z & kRecHi) ? 32u : 0u;
                const uint8_t *nb = t.nodes + (size_t)node * t.node_bytes;
                const bool aos = t.layout == LAYOUT_AOS;
                src = reinterpret_cast<uint64_t>(nb + (aos ? 16u + 20u * half : 16u * t.fanout + 4u * half));
                info = aos ? 20u : 4u;
                mask = d.w;
                if (b + (uint32_t)__popc(mask) > en) {
                    atomicOr(&ctrl->err, kErrBounds);
                    mask = 0;
                }
            }
            ssrc[th] = src;
            sbase[th] = b;
            sinfo[th] = info;
            smask[th] = mask;
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
                    const uint32_t mask = smask[r];
                    if ((mask >> l) & 1u) {
                        const uint8_t *p = reinterpret_cast<const uint8_t *>(ssrc[r]) + (size_t)sinfo[r] * l;
                        v[u] = *reinterpret_cast<const uint32_t *>(p);
                        o[u] = sbase[r] + (uint32_t)__popc(mask & ((1u << l) - 1u));
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
                const uint32_t info = sinfo[r];
                if (!(info & kRange)) continue;
                const uint32_t n = info & ~kRange;
                const uint32_t *__restrict__ src = reinterpret_cast<const uint32_t *>(ssrc[r]);
                const uint64_t b = sbase[r];
                for (uint32_t i0 = l; i0 < n; i0 += 32 * U) {
                    uint32_t w[U];
#pragma unroll
                    for (uint32_t k = 0; k < U; ++k) {
                        const uint32_t i = i0 + 32 * k;
                        w[k] = i < n ? src[i] : 0u;
                    }
#pragma unroll
                    for (uint32_t k = 0; k < U; ++k) {
                        const uint32_t i = i0 + 32 * k;
                        if (i < n) put_id(ids + b + i, w[k]);
                    }
                }
            }
        }
    }
}

hipError_t launch_batch_replay(const BatchTree *trees, const uint32_t *qtree, const BatchRec &rp,
                               const uint64_t *offsets, uint64_t total_q, uint32_t *ids, uint64_t cap, Ctrl *ctrl,
                               hipStream_t s) {
    hipLaunchKernelGGL(batch_replay_kernel, dim3((uint32_t)num_cus() * 8), dim3(256), 0, s, trees, qtree, rp.rec,
                       rp.rec_count, rp.rec_nchunks, offsets, total_q, ids, cap, ctrl);
    return hipGetLastError();
}

}  // namespace rtk
