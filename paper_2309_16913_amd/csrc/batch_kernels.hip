// Persistent multi-tree range-select pass.
//
// A device work queue holds (tree, query-chunk) items for many independent
// trees that may differ in fanout and node layout.  Each wave takes one item
// at a time from a global counter, configures its lanes into groups of
// G = group_width(F) lanes for that tree, and runs the same per-query
// depth-first traversal as the single-tree kernel (lanes over node entries,
// __ballot masks, LDS stacks).  Groups of a wave pick the item's queries in
// order with a wave-local ballot, so only one global atomic is spent per
// item.
#include "rt_internal.h"

namespace rtk {

__device__ __forceinline__ void batch_load(const TreeView &t, const uint8_t *nb, uint32_t e, float &lx, float &ly,
                                           float &hx, float &hy) {
    const uint32_t F = t.fanout;
    if (t.layout == LAYOUT_SOA) {
        const float *f = reinterpret_cast<const float *>(nb);
        lx = f[e];
        ly = f[F + e];
        hx = f[2 * F + e];
        hy = f[3 * F + e];
    } else if (t.layout == LAYOUT_AOS) {
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

__device__ __forceinline__ uint32_t batch_ptr(const TreeView &t, const uint8_t *nb, uint32_t e) {
    const uint32_t *u = reinterpret_cast<const uint32_t *>(nb);
    return t.layout == LAYOUT_AOS ? u[5 * e + 4] : u[4 * t.fanout + e];
}

template <int MODE>
__global__ void __launch_bounds__(256)
batch_kernel(const BatchTree *__restrict__ trees, const BatchItem *__restrict__ items, uint32_t nitems,
             const float4 *__restrict__ qs, uint32_t *__restrict__ counts, const uint64_t *__restrict__ offsets,
             uint32_t *__restrict__ ids, uint64_t cap, uint64_t total_q, Ctrl *__restrict__ ctrl, uint32_t slot,
             uint32_t wave_words) {
    extern __shared__ uint32_t smem[];
    if constexpr (MODE == SEL_FILL) {
        if (offsets[total_q] > cap) return;
    }
    const uint32_t lane = threadIdx.x & 63u;
    uint32_t *wstk = smem + (threadIdx.x >> 6) * wave_words;
    const uint64_t lanes_below = lane ? (~0ull >> (64 - lane)) : 0ull;

    while (true) {
        uint32_t it = 0;
        if (lane == 0) it = atomicAdd(&ctrl->work[slot], 1u);
        it = __shfl(it, 0);
        if (it >= nitems) break;
        const BatchItem item = items[it];
        const BatchTree bt = trees[item.tree];
        const TreeView &t = bt.t;
        const uint32_t F = t.fanout;
        const uint32_t G = F <= 16 ? 16u : (F <= 32 ? 32u : 64u);
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
                    gq = bt.q_begin + mine;
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
                    ref = batch_ptr(t, nb, 0);
                else if constexpr (MODE == SEL_FILL)
                    ref = batch_ptr(t, nb, e);
                float lx, ly, hx, hy;
                batch_load(t, nb, e, lx, ly, hx, hy);
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
                                __builtin_nontemporal_store(ref, ids + o);
                            else
                                atomicOr(&ctrl->err, kErrBounds);
                        }
                    }
                    pos += n;
                } else {
                    const uint32_t first = __shfl(ref, (int)gbase);
                    if (cm) {   // group-uniform: contained subtrees
                        if constexpr (MODE == SEL_FILL) {
                            uint64_t todo = cm;
                            while (todo) {   // one run of consecutive contained children at a time
                                const uint32_t j0 = (uint32_t)__builtin_ctzll(todo);
                                const uint64_t sh = todo >> j0;
                                const uint32_t len = ~sh ? (uint32_t)__builtin_ctzll(~sh) : 64u - j0;
                                todo = (j0 + len >= 64) ? 0ull : (todo & (~0ull << (j0 + len)));
                                const uint32_t l0 = t.range[first + j0].x, l1 = t.range[first + j0 + len - 1].y;
                                const bool hasp = t.partial_leaf >= l0 && t.partial_leaf < l1;
                                constexpr uint32_t U = 4;   // leaves in flight per lane
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
                                            v[u] = batch_ptr(t, t.nodes + (size_t)lf * t.node_bytes, e);
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
                            }
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
    }
}

hipError_t launch_batch_pass(const BatchTree *trees, const BatchItem *items, uint32_t nitems, const float4 *q,
                             int mode, uint32_t *counts, const uint64_t *offsets, uint32_t *ids, uint64_t cap,
                             uint64_t total_q, Ctrl *ctrl, uint32_t slot, uint32_t wave_words, hipStream_t s) {
    // wave_words: largest (64 / G) * stack_cap over the trees (one region per wave)
    const size_t smem = (size_t)4 * wave_words * sizeof(uint32_t);
    uint32_t blocks = (uint32_t)num_cus() * 8;
    const uint32_t want = (nitems + 3) / 4;
    if (want < blocks) blocks = want ? want : 1;
    if (mode == SEL_COUNT)
        hipLaunchKernelGGL(batch_kernel<SEL_COUNT>, dim3(blocks), dim3(256), smem, s, trees, items, nitems, q, counts,
                           offsets, ids, cap, total_q, ctrl, slot, wave_words);
    else
        hipLaunchKernelGGL(batch_kernel<SEL_FILL>, dim3(blocks), dim3(256), smem, s, trees, items, nitems, q, counts,
                           offsets, ids, cap, total_q, ctrl, slot, wave_words);
    return hipGetLastError();
}

}  // namespace rtk
