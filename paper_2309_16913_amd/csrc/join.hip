// R-tree join kernels for gfx950: synchronized traversal of two trees.
//
// The paper's join (section 4) starts at both roots and follows every pair of
// intersecting children.  Its vectorized "one to many" form broadcasts one
// outer child MBR and compares it with all inner children at once (section
// 4.1, steps 1-3), then compress-stores the qualifying inner addresses and
// duplicates the outer address beside them (step 4).
//
// On the GPU the pairs of one tree level form a frontier that is processed
// level by level, one wave per node pair.  The wave covers the Fa x Fb tile of
// child pairs 64 at a time: lane l of round r tests outer child i and inner
// child j with r*64 + l = i*Fb + j, so each round compares (64/Fb) outer
// children against all inner children -- the one-to-many comparison, widened
// from one broadcast outer MBR to several.  Qualifying pairs are compacted
// with __ballot + popcount ranks into the next frontier (count pass, scan,
// fill pass) or, at the leaf level, written out as 64-bit (idA << 32 | idB)
// keys, which are then sorted (bucket sort at the end of this file) into the
// canonical pair order.
//
// Trees of unequal height: only the deeper side descends, with each of its
// children tested against the MBR of the whole shallower tree, until both
// sides are at the same level (this can only happen at the roots).
#include "pair_sort.h"
#include "rt_internal.h"

namespace rtk {

constexpr uint32_t kSlotHits = 15;     // hit records kept per pair by the count pass
constexpr uint32_t kSlotStride = 16;   // uint16 per pair (32 bytes)

__device__ __forceinline__ void load_any(const TreeView &t, uint32_t node, uint32_t e, float &lx, float &ly,
                                         float &hx, float &hy) {
    const uint8_t *nb = t.nodes + (size_t)node * t.node_bytes;
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

__device__ __forceinline__ uint32_t ptr_any(const TreeView &t, uint32_t node, uint32_t e) {
    const uint32_t *u = reinterpret_cast<const uint32_t *>(t.nodes + (size_t)node * t.node_bytes);
    return t.layout == LAYOUT_AOS ? u[5 * e + 4] : u[4 * t.fanout + e];
}

// One wave per frontier pair; 4 pairs per block.  tests_acc (count pass
// only, NULL: not counted): per pair, the entry-pair predicates of a pair at
// equal levels (n_u * n_v real entries) are added to slot word 0, the real
// entries loaded (n_u + n_v, or the deeper node's n) to word 1 and the
// entry-versus-tree predicates of a descending pair to word 2.
template <int MODE, bool FILL>
__global__ void __launch_bounds__(256)
join_level_kernel(TreeView A, TreeView B, const uint2 *__restrict__ fr, uint32_t nfr,
                  const uint64_t *__restrict__ nfr_dev, uint32_t *__restrict__ counts,
                  const uint64_t *__restrict__ offsets, uint2 *__restrict__ next, uint64_t *__restrict__ keys,
                  uint64_t out_cap, Ctrl *__restrict__ ctrl, unsigned long long *__restrict__ tests_acc) {
    const uint32_t lane = threadIdx.x & 63u;
    const uint32_t p = blockIdx.x * 4 + (threadIdx.x >> 6);
    if (nfr_dev && *nfr_dev < nfr) nfr = (uint32_t)*nfr_dev;
    if (p >= nfr) return;   // whole wave leaves together
    const uint2 pr = fr[p];
    const uint64_t below = lane ? (~0ull >> (64 - lane)) : 0ull;
    uint64_t pos = 0, end = 0;
    if (FILL) {
        pos = offsets[p];
        end = min(offsets[p + 1], out_cap);
    }
    uint32_t total = 0;

    if constexpr (MODE == JOIN_DESC_A || MODE == JOIN_DESC_B) {
        // Deeper side descends; each child is tested against the shallower
        // tree's MBR.  One round covers a node (F <= 64).
        const TreeView &D = (MODE == JOIN_DESC_A) ? A : B;
        const TreeView &S = (MODE == JOIN_DESC_A) ? B : A;
        const uint32_t node = (MODE == JOIN_DESC_A) ? pr.x : pr.y;
        bool hit = false, real = false;
        if (lane < D.fanout) {
            float lx, ly, hx, hy;
            load_any(D, node, lane, lx, ly, hx, hy);
            hit = (lx <= S.mbr[2]) && (S.mbr[0] <= hx) && (ly <= S.mbr[3]) && (S.mbr[1] <= hy);
            real = lx == lx;   // not a padding slot
        }
        const uint64_t m = __ballot(hit);
        total = (uint32_t)__popcll(m);
        if (!FILL && tests_acc) {
            const uint32_t nd = (uint32_t)__popcll(__ballot(real));
            if (lane == 0) {
                atomicAdd(&tests_acc[(p % kTestSlots) * 16 + 1], (unsigned long long)nd);
                atomicAdd(&tests_acc[(p % kTestSlots) * 16 + 2], (unsigned long long)nd);
            }
        }
        if (FILL && hit) {
            const uint64_t o = pos + (uint64_t)__popcll(m & below);
            const uint32_t c = ptr_any(D, node, lane);
            if (o < end)
                next[o] = (MODE == JOIN_DESC_A) ? make_uint2(c, pr.y) : make_uint2(pr.x, c);
            else if (o < out_cap)
                atomicOr(&ctrl->err, kErrBounds);
        }
    } else {
        const uint32_t Fa = A.fanout, Fb = B.fanout;
        const uint32_t tile = Fa * Fb;
        // lane's (i, j) for round 0 and the per-round advance
        uint32_t i = lane / Fb, j = lane % Fb;
        const uint32_t di = 64 / Fb, dj = 64 % Fb;
        uint32_t real_pairs = 0;
        for (uint32_t base = 0; base < tile; base += 64) {
            const bool in = base + lane < tile;
            bool hit = false, real = false;
            if (in) {
                float alx, aly, ahx, ahy, blx, bly, bhx, bhy;
                load_any(A, pr.x, i, alx, aly, ahx, ahy);
                load_any(B, pr.y, j, blx, bly, bhx, bhy);
                hit = (alx <= bhx) && (blx <= ahx) && (aly <= bhy) && (bly <= ahy);
                real = (alx == alx) && (blx == blx);   // neither is a padding slot
            }
            const uint64_t m = __ballot(hit);
            const uint32_t n = (uint32_t)__popcll(m);
            if (!FILL && tests_acc) real_pairs += (uint32_t)__popcll(__ballot(real));
            if (FILL && hit) {
                const uint64_t o = pos + total + (uint64_t)__popcll(m & below);
                const uint32_t ca = ptr_any(A, pr.x, i), cb = ptr_any(B, pr.y, j);
                if (o < end) {
                    if (MODE == JOIN_EMIT)
                        keys[o] = ((uint64_t)ca << 32) | cb;
                    else
                        next[o] = make_uint2(ca, cb);
                } else if (o < out_cap) {
                    atomicOr(&ctrl->err, kErrBounds);
                }
            }
            total += n;
            i += di;
            j += dj;
            if (j >= Fb) {
                j -= Fb;
                i += 1;
            }
        }
        if (!FILL && tests_acc) {
            float x, y, z, w;
            bool ra = false, rb = false;
            if (lane < Fa) {
                load_any(A, pr.x, lane, x, y, z, w);
                ra = x == x;
            }
            if (lane < Fb) {
                load_any(B, pr.y, lane, x, y, z, w);
                rb = x == x;
            }
            const uint32_t ne = (uint32_t)(__popcll(__ballot(ra)) + __popcll(__ballot(rb)));
            if (lane == 0) {
                atomicAdd(&tests_acc[(p % kTestSlots) * 16], (unsigned long long)real_pairs);
                atomicAdd(&tests_acc[(p % kTestSlots) * 16 + 1], (unsigned long long)ne);
            }
        }
    }
    if (!FILL && lane == 0) counts[p] = total;
}

// ---------------------------------------------------------------------------
// Node-pair expansion over candidate lists (section 4.1 pruning, section 4.2
// many-to-many).  One wave per frontier pair; lane i holds outer child i of
// node u (tree A) and lane j inner child j of node v (tree B) in registers,
// loaded once.  Each outer lane i gets a count f_i of inner candidates, the
// inner children 0..f_i-1:
//   no pruning          f_i = number of inner children
//   O3 (outer slicing)  f_i = 0 unless outer low x <= max inner high x; with
//                       children sorted by low x this keeps a prefix of the
//                       outer node (the first child that fails ends the scan)
//   O4 (one to many)    for each kept outer child, its high x is broadcast and
//                       compared with every inner low x in one ballot; f_i is
//                       the length of the leading run of qualifying children
//   O5 (many to many)   every outer lane searches the sorted inner low x on
//                       its own: gather at n/2, compare, and on a clear bit
//                       record the flip index and step down, else step up,
//                       log2(n)+1 rounds -- the same f_i as O4
// The candidates (i, j < f_i) are then enumerated 64 per round through an
// exclusive scan of f: lane t finds its i by a binary search over the scan
// and j = t - scan[i], fetches both MBRs from their lanes and applies the
// full overlap predicate.
// ---------------------------------------------------------------------------
__device__ __forceinline__ float wave_max(float v) {
    for (int d = 32; d >= 1; d >>= 1) v = fmaxf(v, __shfl_xor(v, d));
    return v;
}

// exclusive prefix sum over the wave; *total receives the sum
__device__ __forceinline__ uint32_t wave_excl_scan(uint32_t v, uint32_t lane, uint32_t *total) {
    uint32_t inc = v;
    for (int d = 1; d < 64; d <<= 1) {
        const uint32_t x = __shfl_up(inc, d);
        if (lane >= (uint32_t)d) inc += x;
    }
    *total = __shfl(inc, 63);
    return inc - v;
}

// slots (if not NULL): kSlotHits hit records (i << 8 | j) per pair, written
// by the count pass; the fill pass of a pair with at most that many hits
// takes its children from there instead of testing the candidates again.
// Every lane searches the values v (lane g holds entry g; entries 0..n-1 are
// sorted so that pred holds on a prefix) for the first entry where pred
// fails, n if none: the many-to-many search of section 4.2 (gather at n/2,
// compare, step by halves, log2(n)+1 rounds), each lane with its own pred.
template <class Pred>
__device__ __forceinline__ uint32_t first_failing(float v_lane, uint32_t n, Pred pred) {
    uint32_t npow = 1, lg = 0;
    while (npow < n) {
        npow <<= 1;
        ++lg;
    }
    int g = (int)(npow >> 1);
    uint32_t flip = npow;
    for (uint32_t it = 0; it <= lg; ++it) {
        const float v = __shfl(v_lane, g & 63);
        const bool in = g >= 0 && (uint32_t)g < npow;
        const bool bit = (uint32_t)g < n && pred(v);
        const int step = (it + 2 <= lg) ? (int)(npow >> (it + 2)) : 1;
        if (in) {
            if (bit) {
                g += step;
            } else {
                flip = (uint32_t)g;
                g -= step;
            }
        }
    }
    return flip;
}

template <int MODE, bool FILL, bool O3, int SHRINK, bool LB>
__global__ void __launch_bounds__(256)
join_cand_kernel(TreeView A, TreeView B, const uint2 *__restrict__ fr, uint32_t nfr,
                 const uint64_t *__restrict__ nfr_dev, uint32_t *__restrict__ counts,
                 const uint64_t *__restrict__ offsets, uint2 *__restrict__ next, uint64_t *__restrict__ keys,
                 uint64_t out_cap, uint16_t *__restrict__ slots, Ctrl *__restrict__ ctrl,
                 unsigned long long *__restrict__ tests_acc) {
    const uint32_t lane = threadIdx.x & 63u;
    const uint32_t p = blockIdx.x * 4 + (threadIdx.x >> 6);
    if (nfr_dev && *nfr_dev < nfr) nfr = (uint32_t)*nfr_dev;
    if (p >= nfr) return;   // whole wave leaves together
    const uint2 pr = fr[p];
    const uint64_t below = lane ? (~0ull >> (64 - lane)) : 0ull;
    if (FILL && slots) {
        const uint64_t pos = offsets[p], end = min(offsets[p + 1], out_cap);
        const uint64_t n = offsets[p + 1] - pos;
        if (n <= kSlotHits) {   // wave-uniform
            if (lane < n) {
                const uint32_t h = slots[(uint64_t)p * kSlotStride + lane];
                const uint32_t ca = ptr_any(A, pr.x, h >> 8), cb = ptr_any(B, pr.y, h & 255u);
                const uint64_t o = pos + lane;
                if (o < end) {
                    if (MODE == JOIN_EMIT)
                        keys[o] = ((uint64_t)ca << 32) | cb;
                    else
                        next[o] = make_uint2(ca, cb);
                }
            }
            return;
        }
    }
    float alx = NAN, aly = NAN, ahx = NAN, ahy = NAN, blx = NAN, bly = NAN, bhx = NAN, bhy = NAN;
    if (lane < A.fanout) load_any(A, pr.x, lane, alx, aly, ahx, ahy);
    if (lane < B.fanout) load_any(B, pr.y, lane, blx, bly, bhx, bhy);
    // unused slots hold NaN and sit after the used ones
    const bool av = alx == alx, bv = blx == blx;
    const uint32_t nb = (uint32_t)__popcll(__ballot(bv));
    bool act = av;
    if (O3) {
        const float m = wave_max(bv ? bhx : -INFINITY);
        act = av && alx <= m;
    }
    uint32_t f = nb;
    if (SHRINK == 4) {
        f = 0;
        uint64_t todo = __ballot(act);
        while (todo) {
            const uint32_t i = (uint32_t)__builtin_ctzll(todo);
            todo &= todo - 1;
            const float h = __shfl(ahx, (int)i);
            const uint64_t q = __ballot(bv && blx <= h);
            const uint32_t stop = ~q ? (uint32_t)__builtin_ctzll(~q) : 64u;
            if (lane == i) f = stop;
        }
    } else if (SHRINK == 5) {
        f = first_failing(blx, nb, [&](float v) { return v <= ahx; });
    }
    // LB (lower bound, not in the paper): inner children are sorted by low
    // x and none is wider than wmax, so one whose low x lies below
    // olx - wmax ends left of the outer child and cannot qualify.  The bound
    // is lowered by a margin far above the rounding of its two subtractions,
    // so no qualifying pair is ever cut; candidates are j in [lo, f).
    uint32_t lo = 0;
    if (LB) {
        const float wmax = wave_max(bv ? bhx - blx : -INFINITY);
        const float thr = (alx - wmax) - (fabsf(alx) + wmax) * 0x1p-20f;
        lo = first_failing(blx, nb, [&](float v) { return v < thr; });
        lo = min(lo, f);
    }
    if (!act) f = lo = 0;
    uint32_t T = 0;
    const uint32_t pre = wave_excl_scan(f - lo, lane, &T);
    const int jbase = (int)lo - (int)pre;   // j = t + jbase of the outer child
    uint64_t pos = 0, end = 0;
    if (FILL) {
        pos = offsets[p];
        end = min(offsets[p + 1], out_cap);
    }
    uint32_t total = 0;
    for (uint32_t base = 0; base < T; base += 64) {
        const uint32_t t = base + lane;
        uint32_t i = 0;
        for (uint32_t sft = 32; sft >= 1; sft >>= 1) {
            const uint32_t c = __shfl(pre, (int)(i + sft));
            if (c <= t) i += sft;
        }
        const uint32_t j = min((uint32_t)((int)t + __shfl(jbase, (int)i)), 63u);
        const float olx = __shfl(alx, (int)i), oly = __shfl(aly, (int)i);
        const float ohx = __shfl(ahx, (int)i), ohy = __shfl(ahy, (int)i);
        const float ilx = __shfl(blx, (int)j), ily = __shfl(bly, (int)j);
        const float ihx = __shfl(bhx, (int)j), ihy = __shfl(bhy, (int)j);
        const bool hit = t < T && (olx <= ihx) && (ilx <= ohx) && (oly <= ihy) && (ily <= ohy);
        const uint64_t m = __ballot(hit);
        if (!FILL && slots && hit) {
            const uint32_t r = total + (uint32_t)__popcll(m & below);
            if (r < kSlotHits) slots[(uint64_t)p * kSlotStride + r] = (uint16_t)((i << 8) | j);
        }
        if (FILL && hit) {
            const uint64_t o = pos + total + (uint64_t)__popcll(m & below);
            const uint32_t ca = ptr_any(A, pr.x, i), cb = ptr_any(B, pr.y, j);
            if (o < end) {
                if (MODE == JOIN_EMIT)
                    keys[o] = ((uint64_t)ca << 32) | cb;
                else
                    next[o] = make_uint2(ca, cb);
            } else if (o < out_cap) {
                atomicOr(&ctrl->err, kErrBounds);
            }
        }
        total += (uint32_t)__popcll(m);
    }
    if (!FILL && lane == 0) {
        counts[p] = total;
        // spread over kTestSlots counters, one 128-byte line each
        if (tests_acc) atomicAdd(&tests_acc[(p % kTestSlots) * 16], (unsigned long long)T);
    }
}

template <int MODE, bool O3, int SHRINK, bool LB = false>
static hipError_t launch_cand(const TreeView &a, const TreeView &b, const uint2 *fr, uint32_t nfr,
                              const uint64_t *nfr_dev, bool fill, uint32_t *counts, const uint64_t *offsets,
                              uint2 *next, uint64_t *keys, uint64_t out_cap, uint16_t *slots, Ctrl *ctrl,
                              unsigned long long *tests_acc, hipStream_t s) {
    const uint32_t blocks = (nfr + 3) / 4;
    if (fill)
        hipLaunchKernelGGL((join_cand_kernel<MODE, true, O3, SHRINK, LB>), dim3(blocks), dim3(256), 0, s, a, b, fr, nfr,
                           nfr_dev, counts, offsets, next, keys, out_cap, slots, ctrl,
                           (unsigned long long *)nullptr);
    else
        hipLaunchKernelGGL((join_cand_kernel<MODE, false, O3, SHRINK, LB>), dim3(blocks), dim3(256), 0, s, a, b, fr,
                           nfr, nfr_dev, counts, offsets, next, keys, out_cap, slots, ctrl, tests_acc);
    return hipGetLastError();
}

template <int MODE>
static hipError_t launch_cand_flags(const TreeView &a, const TreeView &b, const uint2 *fr, uint32_t nfr,
                                    const uint64_t *nd, bool fill, uint32_t *counts, const uint64_t *offsets,
                                    uint2 *next, uint64_t *keys, uint64_t cap, uint16_t *sl, Ctrl *ctrl, int flags,
                                    unsigned long long *ta, hipStream_t s) {
    const bool o3 = flags & JOIN_O3;
    const int sh = (flags & JOIN_O5) ? 5 : ((flags & JOIN_O4) ? 4 : 0);
    if (flags & JOIN_LB) {   // only with O3 + O5 (checked by the caller)
        return launch_cand<MODE, true, 5, true>(a, b, fr, nfr, nd, fill, counts, offsets, next, keys, cap, sl, ctrl,
                                                ta, s);
    }
    if (o3) {
        if (sh == 5)
            return launch_cand<MODE, true, 5>(a, b, fr, nfr, nd, fill, counts, offsets, next, keys, cap, sl, ctrl, ta,
                                              s);
        if (sh == 4)
            return launch_cand<MODE, true, 4>(a, b, fr, nfr, nd, fill, counts, offsets, next, keys, cap, sl, ctrl, ta,
                                              s);
        return launch_cand<MODE, true, 0>(a, b, fr, nfr, nd, fill, counts, offsets, next, keys, cap, sl, ctrl, ta, s);
    }
    if (sh == 5)
        return launch_cand<MODE, false, 5>(a, b, fr, nfr, nd, fill, counts, offsets, next, keys, cap, sl, ctrl, ta, s);
    if (sh == 4)
        return launch_cand<MODE, false, 4>(a, b, fr, nfr, nd, fill, counts, offsets, next, keys, cap, sl, ctrl, ta, s);
    return launch_cand<MODE, false, 0>(a, b, fr, nfr, nd, fill, counts, offsets, next, keys, cap, sl, ctrl, ta, s);
}

template <int MODE>
static hipError_t launch_mode(const TreeView &a, const TreeView &b, const uint2 *fr, uint32_t nfr, const uint64_t *nd,
                              bool fill, uint32_t *counts, const uint64_t *offsets, uint2 *next, uint64_t *keys,
                              uint64_t cap, Ctrl *ctrl, unsigned long long *tests_acc, hipStream_t s) {
    const uint32_t blocks = (nfr + 3) / 4;
    if (fill)
        hipLaunchKernelGGL((join_level_kernel<MODE, true>), dim3(blocks), dim3(256), 0, s, a, b, fr, nfr, nd, counts,
                           offsets, next, keys, cap, ctrl, (unsigned long long *)nullptr);
    else
        hipLaunchKernelGGL((join_level_kernel<MODE, false>), dim3(blocks), dim3(256), 0, s, a, b, fr, nfr, nd,
                           counts, offsets, next, keys, cap, ctrl, tests_acc);
    return hipGetLastError();
}

hipError_t launch_join_level(const TreeView &a, const TreeView &b, const uint2 *frontier, uint32_t nfr,
                             const uint64_t *nd, int mode, bool fill, uint32_t *counts, const uint64_t *offsets,
                             uint2 *next, uint64_t *keys, uint64_t cap, uint16_t *slots, Ctrl *ctrl, int flags,
                             unsigned long long *tests_acc, hipStream_t s) {
    if (nfr == 0) return hipSuccess;
    if (!(flags & JOIN_TILE) && (mode == JOIN_BOTH || mode == JOIN_EMIT)) {
        if (mode == JOIN_BOTH)
            return launch_cand_flags<JOIN_BOTH>(a, b, frontier, nfr, nd, fill, counts, offsets, next, keys, cap,
                                                slots, ctrl, flags, tests_acc, s);
        return launch_cand_flags<JOIN_EMIT>(a, b, frontier, nfr, nd, fill, counts, offsets, next, keys, cap, slots,
                                            ctrl, flags, tests_acc, s);
    }
    switch (mode) {
    case JOIN_BOTH:
        return launch_mode<JOIN_BOTH>(a, b, frontier, nfr, nd, fill, counts, offsets, next, keys, cap, ctrl, tests_acc,
                                      s);
    case JOIN_EMIT:
        return launch_mode<JOIN_EMIT>(a, b, frontier, nfr, nd, fill, counts, offsets, next, keys, cap, ctrl, tests_acc,
                                      s);
    case JOIN_DESC_A:
        return launch_mode<JOIN_DESC_A>(a, b, frontier, nfr, nd, fill, counts, offsets, next, keys, cap, ctrl,
                                        tests_acc, s);
    default:
        return launch_mode<JOIN_DESC_B>(a, b, frontier, nfr, nd, fill, counts, offsets, next, keys, cap, ctrl,
                                        tests_acc, s);
    }
}

uint64_t join_slot_bytes(uint64_t nfr) { return nfr * kSlotStride * sizeof(uint16_t); }

__global__ void keys_to_pairs_kernel(const uint64_t *__restrict__ keys, uint64_t n, uint32_t *__restrict__ pairs) {
    for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (uint64_t)gridDim.x * blockDim.x) {
        const uint64_t k = keys[i];
        pairs[2 * i] = (uint32_t)(k >> 32);
        pairs[2 * i + 1] = (uint32_t)k;
    }
}

// The same with the count on the device (at most n_max): writes nothing if the
// count exceeds capacity or *skip has bit 0 set.
__global__ void keys_to_pairs_dev_kernel(const uint64_t *__restrict__ keys, const uint64_t *__restrict__ n_dev,
                                         uint64_t capacity, const uint32_t *__restrict__ skip,
                                         uint32_t *__restrict__ pairs) {
    const uint64_t n = *n_dev;
    if (n > capacity || (*skip & 1u)) return;
    for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (uint64_t)gridDim.x * blockDim.x) {
        const uint64_t k = keys[i];
        pairs[2 * i] = (uint32_t)(k >> 32);
        pairs[2 * i + 1] = (uint32_t)k;
    }
}

hipError_t launch_keys_to_pairs_dev(const uint64_t *keys, const uint64_t *n_dev, uint64_t n_max, uint64_t capacity,
                                    const uint32_t *skip, uint32_t *pairs, hipStream_t s) {
    uint64_t blocks = (n_max + 255) / 256;
    if (blocks > 8192) blocks = 8192;
    if (blocks == 0) blocks = 1;
    hipLaunchKernelGGL(keys_to_pairs_dev_kernel, dim3((uint32_t)blocks), dim3(256), 0, s, keys, n_dev, capacity, skip,
                       pairs);
    return hipGetLastError();
}

__global__ void copy_err_kernel(const Ctrl *__restrict__ ctrl, uint32_t *__restrict__ dst) { *dst = ctrl->err; }

hipError_t launch_copy_err(const Ctrl *ctrl, uint32_t *dst, hipStream_t s) {
    hipLaunchKernelGGL(copy_err_kernel, dim3(1), dim3(1), 0, s, ctrl, dst);
    return hipGetLastError();
}

hipError_t launch_keys_to_pairs(const uint64_t *keys, uint64_t n, uint32_t *pairs, hipStream_t s) {
    if (n == 0) return hipSuccess;
    uint64_t blocks = (n + 255) / 256;
    if (blocks > 8192) blocks = 8192;
    hipLaunchKernelGGL(keys_to_pairs_kernel, dim3((uint32_t)blocks), dim3(256), 0, s, keys, n, pairs);
    return hipGetLastError();
}

// ---- pair keys: bucket sort by the top digit --------------------------------
constexpr uint32_t kPairTile = 4096;   // keys per block in the scatter (256 x 16)

__global__ void __launch_bounds__(256)
pair_bucket_hist(const uint64_t *__restrict__ keys, uint64_t n, const uint64_t *__restrict__ n_dev, int shift,
                 uint32_t *__restrict__ cnt) {
    __shared__ uint32_t h[kPairBuckets];
    if (n_dev) n = min(n, *n_dev);
    for (uint32_t i = threadIdx.x; i < kPairBuckets; i += blockDim.x) h[i] = 0;
    __syncthreads();
    for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (uint64_t)gridDim.x * blockDim.x)
        atomicAdd(&h[(uint32_t)(keys[i] >> shift)], 1u);
    __syncthreads();
    for (uint32_t i = threadIdx.x; i < kPairBuckets; i += blockDim.x)
        if (h[i]) atomicAdd(&cnt[i], h[i]);
}

// One block of 1024: exclusive scan of the counts into start[0 .. kPairBuckets]
// (start[kPairBuckets] = n) and zeroed cursors.
__global__ void __launch_bounds__(1024)
pair_bucket_scan(const uint32_t *__restrict__ cnt, uint32_t *__restrict__ start, uint32_t *__restrict__ cursor) {
    constexpr uint32_t W = 1024 / 64;
    __shared__ uint32_t wsum[W];
    const uint32_t t = threadIdx.x, lane = t & 63u, w = t >> 6;
    const uint32_t a = cnt[2 * t], b = cnt[2 * t + 1];
    uint32_t inc = a + b;
#pragma unroll
    for (int d = 1; d < 64; d <<= 1) {
        const uint32_t x = __shfl_up(inc, d);
        if ((int)lane >= d) inc += x;
    }
    if (lane == 63) wsum[w] = inc;
    __syncthreads();
    uint32_t base = 0;
    for (uint32_t i = 0; i < w; ++i) base += wsum[i];
    const uint32_t ex = base + inc - (a + b);
    start[2 * t] = ex;
    start[2 * t + 1] = ex + a;
    if (t == 1023) start[kPairBuckets] = ex + a + b;
    cursor[2 * t] = 0;
    cursor[2 * t + 1] = 0;
}

// A block takes a tile of keys: LDS ranks per bucket, one global reservation
// per bucket present in the tile, then every key goes to its bucket.  The
// order inside a bucket is arbitrary (the bucket is sorted next).
__global__ void __launch_bounds__(256)
pair_bucket_scatter(const uint64_t *__restrict__ keys, uint64_t n, const uint64_t *__restrict__ n_dev, int shift,
                    const uint32_t *__restrict__ start, uint32_t *__restrict__ cursor, uint64_t *__restrict__ out) {
    constexpr uint32_t R = kPairTile / 256;
    __shared__ uint32_t c[kPairBuckets];
    if (n_dev) n = min(n, *n_dev);
    for (uint64_t t0 = (uint64_t)blockIdx.x * kPairTile; t0 < n; t0 += (uint64_t)gridDim.x * kPairTile) {
        for (uint32_t i = threadIdx.x; i < kPairBuckets; i += 256) c[i] = 0;
        __syncthreads();
        uint64_t k[R];
        uint32_t rk[R];
#pragma unroll
        for (uint32_t r = 0; r < R; ++r) {
            const uint64_t i = t0 + r * 256 + threadIdx.x;
            k[r] = i < n ? keys[i] : 0ull;
            rk[r] = i < n ? atomicAdd(&c[(uint32_t)(k[r] >> shift)], 1u) : 0u;
        }
        __syncthreads();
        for (uint32_t i = threadIdx.x; i < kPairBuckets; i += 256)
            if (c[i]) c[i] = start[i] + atomicAdd(&cursor[i], c[i]);
        __syncthreads();
#pragma unroll
        for (uint32_t r = 0; r < R; ++r) {
            const uint64_t i = t0 + r * 256 + threadIdx.x;
            if (i < n) out[c[(uint32_t)(k[r] >> shift)] + rk[r]] = k[r];
        }
        __syncthreads();
    }
}

// Bitonic sort of P (a power of two) keys in LDS by the block.
__device__ __forceinline__ void lds_bitonic_u64(uint64_t *buf, uint32_t P) {
    for (uint32_t k = 2; k <= P; k <<= 1) {
        for (uint32_t j = k >> 1; j > 0; j >>= 1) {
            for (uint32_t t = threadIdx.x; t < P / 2; t += blockDim.x) {
                const uint32_t i = ((t & ~(j - 1)) << 1) | (t & (j - 1));
                const uint32_t l = i | j;
                const uint64_t x = buf[i], y = buf[l];
                const bool up = (i & k) == 0;
                if ((x > y) == up) {
                    buf[i] = y;
                    buf[l] = x;
                }
            }
            __syncthreads();
        }
    }
}

// Number of keys in v[0 .. n) below x (v sorted).
__device__ __forceinline__ uint32_t count_below(const uint64_t *v, uint32_t n, uint64_t x) {
    uint32_t lo = 0, hi = n;
    while (lo < hi) {
        const uint32_t mid = (lo + hi) >> 1;
        if (v[mid] < x) lo = mid + 1;
        else hi = mid;
    }
    return lo;
}

// One block per bucket: bitonic sort in LDS over the bucket padded to a power
// of two (keys are distinct; padding with all ones sorts last).  A bucket over
// the LDS cap (ids far from uniform) is sorted in runs of the cap, which are
// then merged pairwise through tmp (the partition's input, free by now) at the
// bucket's own positions: every key finds its place as its index in its run
// plus the number of keys below it in the other run.
__global__ void __launch_bounds__(256)
pair_bucket_sort(uint64_t *__restrict__ keys, uint64_t *__restrict__ tmp, const uint32_t *__restrict__ start) {
    __shared__ uint64_t buf[kPairBucketCap];
    for (uint32_t bk = blockIdx.x; bk < kPairBuckets; bk += gridDim.x) {
        const uint32_t s0 = start[bk], c = start[bk + 1] - s0;
        if (c < 2) continue;
        for (uint32_t r0 = 0; r0 < c; r0 += kPairBucketCap) {
            const uint32_t rc = min(c - r0, kPairBucketCap);
            uint32_t P = 2;
            while (P < rc) P <<= 1;
            for (uint32_t i = threadIdx.x; i < P; i += blockDim.x) buf[i] = i < rc ? keys[s0 + r0 + i] : ~0ull;
            __syncthreads();
            lds_bitonic_u64(buf, P);
            for (uint32_t i = threadIdx.x; i < rc; i += blockDim.x) keys[s0 + r0 + i] = buf[i];
            __syncthreads();
        }
        if (c <= kPairBucketCap) continue;
        uint64_t *src = keys + s0, *dst = tmp + s0;
        for (uint32_t w = kPairBucketCap; w < c; w *= 2) {
            for (uint32_t i = threadIdx.x; i < c; i += blockDim.x) {
                const uint32_t a0 = i / (2 * w) * (2 * w);
                const uint32_t b0 = min(a0 + w, c), b1 = min(a0 + 2 * w, c);
                const uint64_t x = src[i];
                const uint32_t pos = i < b0 ? i + count_below(src + b0, b1 - b0, x)
                                            : (i - b0) + a0 + count_below(src + a0, b0 - a0, x);
                dst[pos] = x;
            }
            __syncthreads();
            uint64_t *t2 = src;
            src = dst;
            dst = t2;
        }
        if (src != keys + s0) {
            for (uint32_t i = threadIdx.x; i < c; i += blockDim.x) keys[s0 + i] = src[i];
            __syncthreads();
        }
    }
}

hipError_t launch_pair_bucket_sort(uint64_t *keys, uint64_t n, int shift, uint64_t *out, uint32_t *ws,
                                   hipStream_t s, const uint64_t *n_dev) {
    if (n == 0) return hipSuccess;
    uint32_t *cnt = ws, *start = ws + kPairBuckets, *cursor = ws + 2 * kPairBuckets + 4;
    hipError_t e = launch_zero(cnt, 4 * kPairBuckets, s);
    if (e != hipSuccess) return e;
    const uint64_t tiles = (n + kPairTile - 1) / kPairTile;
    const uint32_t cus = (uint32_t)num_cus();
    const uint32_t hb = (uint32_t)(tiles < (uint64_t)cus * 4 ? tiles : (uint64_t)cus * 4);
    hipLaunchKernelGGL(pair_bucket_hist, dim3(hb), dim3(256), 0, s, keys, n, n_dev, shift, cnt);
    hipLaunchKernelGGL(pair_bucket_scan, dim3(1), dim3(1024), 0, s, cnt, start, cursor);
    const uint32_t sb = (uint32_t)(tiles < (uint64_t)cus * 8 ? tiles : (uint64_t)cus * 8);
    hipLaunchKernelGGL(pair_bucket_scatter, dim3(sb), dim3(256), 0, s, keys, n, n_dev, shift, start, cursor, out);
    hipLaunchKernelGGL(pair_bucket_sort, dim3(kPairBuckets), dim3(256), 0, s, out, keys, start);
    return hipGetLastError();
}

}  // namespace rtk
