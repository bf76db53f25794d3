// Sort-Tile-Recursive bulk load on the device.
//
// The paper does not say how its trees are built; the library bulk-loads them
// with STR (Leutenegger, Lopez, Edgington 1997).  For a level of c items:
// P = ceil(c / F) nodes and S = ceil(sqrt(P)) vertical slices of S*F items.
// Items are ordered by x-center (ties by item index); the item at x-rank p
// belongs to slice p / (S*F); inside a slice items are ordered by y-center
// (ties by item index); consecutive runs of F items of that packing order
// form the level's nodes (every node full but the last).  The node MBRs are
// the next level's items.  Centers only decide the tree's shape, never a
// result: they are compared as order-preserving integers made from
// 0.5*lo + 0.5*hi with each operation rounded to f32.
//
// The packing order (slice, y, index) is reached with stable LSD radix sorts:
// by (y key, index) first, then stably by slice, where an item's slice comes
// from its x-rank.
//
// Final numbering: breadth first from the root; the children of a node are
// stored contiguously in entry order, levels one after another.  pos[l][k]
// is the place of node k of level l (creation order) inside its level; it is
// computed from the root down: the children of the node stored at place g
// start at the sum of the entry counts of the nodes stored before g.
//
// Optionally (RT_BUILD_SORT_LX) the entries of every node are reordered by
// low x before the placement, which moves the children with their entries.
#include <cmath>
#include <new>
#include <vector>

#include "rt_api_internal.h"

namespace rtk {

// Order-preserving integer of a center.  -0.0 counts as +0.0; a NaN center
// (an item spanning -inf..+inf) counts as larger than every number.
__device__ __forceinline__ uint32_t order_key(float c) {
    if (c != c) return 0xFFFFFFFFu;
    if (c == 0.0f) c = 0.0f;
    const uint32_t u = __float_as_uint(c);
    return (u & 0x80000000u) ? ~u : (u | 0x80000000u);
}

// center, each operation rounded (no contraction into an fma)
__device__ __forceinline__ float center(float lo, float hi) {
    return __fadd_rn(__fmul_rn(0.5f, lo), __fmul_rn(0.5f, hi));
}

__global__ void str_validate(const float4 *__restrict__ r, uint64_t n, uint32_t *__restrict__ flag) {
    uint32_t bad = 0;
    for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (uint64_t)gridDim.x * blockDim.x) {
        const float4 v = r[i];
        const bool nan = (v.x != v.x) || (v.y != v.y) || (v.z != v.z) || (v.w != v.w);
        if (nan || !(v.x <= v.z) || !(v.y <= v.w)) bad = 1;
    }
    if (bad) atomicOr(flag, 1u);
}

// keys[i] = key(center_x or center_y of item i) << 32 | i
__global__ void str_center_keys(const float4 *__restrict__ it, uint32_t c, int axis, uint64_t *__restrict__ keys) {
    for (uint32_t i = blockIdx.x * blockDim.x + threadIdx.x; i < c; i += gridDim.x * blockDim.x) {
        const float4 v = it[i];
        const float m = axis ? center(v.y, v.w) : center(v.x, v.z);
        keys[i] = ((uint64_t)order_key(m) << 32) | i;
    }
}

// xrank[item] = its position in x order
__global__ void str_xrank(const uint64_t *__restrict__ xs, uint32_t c, uint32_t *__restrict__ xrank) {
    for (uint32_t p = blockIdx.x * blockDim.x + threadIdx.x; p < c; p += gridDim.x * blockDim.x)
        xrank[(uint32_t)xs[p]] = p;
}

// keys[q] = slice(item) << 32 | item, items taken in (y key, index) order
__global__ void str_slice_keys(const uint64_t *__restrict__ ys, const uint32_t *__restrict__ xrank, uint32_t c,
                               uint64_t slice, uint64_t *__restrict__ keys) {
    for (uint32_t q = blockIdx.x * blockDim.x + threadIdx.x; q < c; q += gridDim.x * blockDim.x) {
        const uint32_t i = (uint32_t)ys[q];
        keys[q] = ((uint64_t)(xrank[i] / slice) << 32) | i;
    }
}

// Optional low-x order inside every node (one wave per node): each entry's
// rank among its node's entries by (low x, position in the packing order).
// order_in NULL: identity.  order_in may equal order_out.
__global__ void str_sort_runs(const uint64_t *order_in, uint64_t *order_out, const float4 *__restrict__ items,
                              uint32_t c, uint32_t F, uint32_t P) {
    const uint32_t lane = threadIdx.x & 63u;
    const uint32_t k = blockIdx.x * 4 + (threadIdx.x >> 6);
    if (k >= P) return;   // whole wave leaves together
    const uint32_t r0 = k * F;
    const uint32_t cnt = c > r0 ? min(c - r0, F) : 0u;
    uint32_t item = 0, key = 0xFFFFFFFFu;
    if (lane < cnt) {
        item = order_in ? (uint32_t)order_in[r0 + lane] : r0 + lane;
        key = order_key(items[item].x);
    }
    uint32_t rank = 0;
    for (uint32_t e = 0; e < cnt; ++e) {
        const uint32_t ke = __shfl(key, (int)e);
        rank += (ke < key || (ke == key && e < lane)) ? 1u : 0u;
    }
    if (lane < cnt) order_out[r0 + rank] = item;
}

// Node MBRs of a level: node k covers packing positions [kF, min(kF+F, c)).
__global__ void str_mbrs(const float4 *__restrict__ it, const uint64_t *__restrict__ order, uint32_t c, uint32_t F,
                         uint32_t P, float4 *__restrict__ mbr) {
    for (uint32_t k = blockIdx.x * blockDim.x + threadIdx.x; k < P; k += gridDim.x * blockDim.x) {
        float4 m = make_float4(INFINITY, INFINITY, -INFINITY, -INFINITY);
        const uint32_t r0 = k * F, r1 = min(c, r0 + F);
        for (uint32_t r = r0; r < r1; ++r) {
            const float4 v = it[order ? (uint32_t)order[r] : r];
            m.x = v.x < m.x ? v.x : m.x;
            m.y = v.y < m.y ? v.y : m.y;
            m.z = m.z < v.z ? v.z : m.z;
            m.w = m.w < v.w ? v.w : m.w;
        }
        if (r1 == r0) m = make_float4(NAN, NAN, NAN, NAN);
        mbr[k] = m;
    }
}

// Places of level l-1's nodes from the places of level l's nodes.
__global__ void str_child_pos(const uint64_t *__restrict__ order, const uint32_t *__restrict__ pos, uint32_t c,
                              uint32_t F, uint32_t P, uint32_t *__restrict__ child_pos) {
    const uint32_t g_last = pos[P - 1];
    const uint32_t short_by = P * F - c;   // missing entries of the last-created node
    for (uint32_t r = blockIdx.x * blockDim.x + threadIdx.x; r < c; r += gridDim.x * blockDim.x) {
        const uint32_t k = r / F, e = r - k * F;
        const uint32_t g = pos[k];
        const uint32_t item = order ? (uint32_t)order[r] : r;
        child_pos[item] = g * F - (g > g_last ? short_by : 0u) + e;
    }
}

// Write every node of one level in its final place.
__global__ void str_write_level(const uint64_t *__restrict__ order, const float4 *__restrict__ items,
                                const uint32_t *__restrict__ pos, const uint32_t *__restrict__ child_pos, uint32_t c,
                                uint32_t P, uint32_t F, uint32_t layout, uint32_t level, uint32_t first,
                                uint32_t child_first, uint8_t *__restrict__ nodes, uint32_t *__restrict__ meta) {
    const uint64_t total = (uint64_t)P * F;
    for (uint64_t w = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; w < total;
         w += (uint64_t)gridDim.x * blockDim.x) {
        const uint32_t k = (uint32_t)(w / F), e = (uint32_t)(w - (uint64_t)k * F);
        const uint32_t r0 = k * F;
        const uint32_t cnt = c > r0 ? min(c - r0, F) : 0u;
        float4 v = make_float4(NAN, NAN, NAN, NAN);
        uint32_t p = 0xFFFFFFFFu;
        if (e < cnt) {
            const uint32_t item = order ? (uint32_t)order[r0 + e] : r0 + e;
            v = items[item];
            p = level == 0 ? item : child_first + child_pos[item];
        }
        const uint32_t g = first + pos[k];
        uint8_t *node = nodes + (uint64_t)g * (20u * F);
        float *f = reinterpret_cast<float *>(node);
        uint32_t *u = reinterpret_cast<uint32_t *>(node);
        if (layout == LAYOUT_SOA) {
            f[e] = v.x;
            f[F + e] = v.y;
            f[2 * F + e] = v.z;
            f[3 * F + e] = v.w;
            u[4 * F + e] = p;
        } else if (layout == LAYOUT_AOS) {
            f[5 * e + 0] = v.x;
            f[5 * e + 1] = v.y;
            f[5 * e + 2] = v.z;
            f[5 * e + 3] = v.w;
            u[5 * e + 4] = p;
        } else {
            f[2 * e] = v.x;
            f[2 * e + 1] = v.y;
            f[2 * F + 2 * e] = v.z;
            f[2 * F + 2 * e + 1] = v.w;
            u[4 * F + e] = p;
        }
        if (e == 0) meta[g] = cnt | (level << 8);
    }
}

// Leaf ranges: a leaf covers [g, g + 1).  Leaves with fewer than F entries
// are counted in partial[2] and the first one found is reported in
// partial[0..1] = {leaf, count}.  The packer fills every leaf but the last
// one of the level, and the contained-subtree arithmetic of the select
// kernels relies on that (at most one short leaf), so the host refuses a
// tree whose count is above one.
__global__ void str_range_leaves(uint32_t first, uint32_t n, uint32_t F, const uint32_t *__restrict__ meta,
                                 uint2 *__restrict__ range, uint32_t *__restrict__ partial) {
    for (uint32_t i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) {
        const uint32_t g = first + i;
        range[g] = make_uint2(g, g + 1);
        const uint32_t cnt = meta[g] & 0xFFu;
        if (cnt < F) {
            if (atomicAdd(&partial[2], 1u) == 0u) {
                partial[0] = g;
                partial[1] = cnt;
            }
        }
    }
}

// The leaves' object ids, leaf after leaf without padding (leaf l's at
// leaf_start(l)); the short leaf and its count come from partial[0..1].
__global__ void str_leaf_ids(uint32_t first_leaf, uint32_t nleaves, uint32_t F, uint32_t layout,
                             const uint8_t *__restrict__ nodes, const uint32_t *__restrict__ meta,
                             const uint32_t *__restrict__ partial, uint64_t n_objects,
                             uint32_t *__restrict__ leaf_ids) {
    const uint32_t pl = partial[0], pc = partial[1];
    const uint64_t slots = (uint64_t)nleaves * F;
    for (uint64_t i = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x; i < slots;
         i += (uint64_t)gridDim.x * blockDim.x) {
        const uint32_t l = first_leaf + (uint32_t)(i / F), e = (uint32_t)(i % F);
        if (e >= (meta[l] & 0xFFu)) continue;
        uint64_t start = (uint64_t)(l - first_leaf) * F;
        if (pl != kNoNode && l > pl) start -= F - pc;
        const uint32_t *u = reinterpret_cast<const uint32_t *>(nodes + (uint64_t)l * (20u * F));
        if (start + e < n_objects)   // always, unless the packing broke its one-short-leaf rule
            leaf_ids[start + e] = layout == LAYOUT_AOS ? u[5 * e + 4] : u[4 * F + e];
    }
}

// Internal node: its children are contiguous from its first pointer, so its
// leaves run from the first child's first leaf to the last child's end.
__global__ void str_range_up(uint32_t first, uint32_t n, uint32_t F, uint32_t layout,
                             const uint8_t *__restrict__ nodes, const uint32_t *__restrict__ meta,
                             uint2 *__restrict__ range) {
    for (uint32_t i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) {
        const uint32_t g = first + i;
        const uint32_t cnt = meta[g] & 0xFFu;
        const uint32_t *u = reinterpret_cast<const uint32_t *>(nodes + (uint64_t)g * (20u * F));
        const uint32_t c0 = layout == LAYOUT_AOS ? u[4] : u[4 * F];
        range[g] = make_uint2(range[c0].x, range[c0 + cnt - 1].y);
    }
}

static uint32_t grid_for(uint64_t n) {
    uint64_t b = (n + 255) / 256;
    if (b == 0) b = 1;
    return (uint32_t)(b < 16384 ? b : 16384);
}

static uint64_t al(uint64_t b) { return (b + 255) & ~255ull; }

int build_str_on_device(const float4 *d_rects, uint64_t n, uint32_t F, uint32_t layout, bool sort_lx,
                        hipStream_t s, rt_tree **out) {
    // level sizes, leaves first
    std::vector<uint64_t> items, nodes;
    for (uint64_t c = n;;) {
        items.push_back(c);
        const uint64_t P = c > F ? (c + F - 1) / F : 1;
        nodes.push_back(P);
        if (c <= F) break;
        c = P;
    }
    const uint32_t H = (uint32_t)items.size();
    std::vector<uint64_t> first(H);
    uint64_t total = 0;
    for (int l = (int)H - 1; l >= 0; --l) {
        first[l] = total;
        total += nodes[l];
    }
    if (H > 32 || total >= 0xFFFFFFFFull) return fail(RT_EINVAL, "too many nodes");

    // workspace: per level the packing order (levels with more than F items),
    // the node MBRs and node places; sort buffers sized for the leaf level
    std::vector<uint64_t> ord_off(H), mbr_off(H), pos_off(H);
    uint64_t ws = 0;
    for (uint32_t l = 0; l < H; ++l) {
        ord_off[l] = ws;
        ws += (items[l] > F || sort_lx) ? al(8 * items[l] + 8) : 0;
        mbr_off[l] = ws;
        ws += al(16 * nodes[l]);
        pos_off[l] = ws;
        ws += al(4 * nodes[l]);
    }
    const uint64_t cmax = n > 0 ? n : 1;
    const uint64_t he = radix_hist_elems(cmax);
    const uint64_t keys_off = ws;
    ws += al(8 * cmax);
    const uint64_t tmp_off = ws;
    ws += al(8 * cmax);
    const uint64_t xrank_off = ws;
    ws += al(4 * cmax);
    const uint64_t hist_off = ws;
    ws += al(4 * he);
    const uint64_t hscan_off = ws;
    ws += al(8 * (he + 1));
    const uint64_t stmp_off = ws;
    ws += al(8 * scan_tmp_elems(he + 1));
    const uint64_t flag_off = ws;
    ws += 256;
    const uint64_t partial_off = ws;
    ws += 256;

    void *mem = obj_alloc(KIND_TREE, sizeof(rt_tree));
    if (!mem) return fail(RT_ENOMEM, "host allocation failed");
    rt_tree *t = new (mem) rt_tree();
    (void)hipGetDevice(&t->device);
    t->fanout = F;
    t->layout = layout;
    t->sorted_lx = sort_lx ? 1u : 0u;
    t->height = H;
    t->n_nodes = (uint32_t)total;
    t->first_leaf = (uint32_t)first[0];
    t->node_bytes = 20u * F;
    t->n_objects = n;
    for (uint32_t l = 0; l < H; ++l) t->n_entries += items[l];
    for (uint32_t l = 0; l < H; ++l) t->level_start[l] = (uint32_t)first[l];
    auto bail = [&](int rc) {
        tree_release(t);
        std::free(reinterpret_cast<ObjHdr *>(t) - 1);
        return rc;
    };

    DevBuf work;
    hipError_t e = work.alloc(ws);
    if (e == hipSuccess) e = hipMalloc(&t->d_nodes, total * t->node_bytes);
    if (e == hipSuccess) e = hipMalloc(&t->d_meta, total * 4);
    if (e == hipSuccess) e = hipMalloc(&t->d_range, total * 8);
    if (e == hipSuccess) e = hipMalloc(&t->d_leaf_ids, n ? n * 4 : 16);
    if (e != hipSuccess) return bail(hip_fail(e, "device build allocation"));
    uint8_t *wb = static_cast<uint8_t *>(work.p);
    auto ord = [&](uint32_t l) {
        return (items[l] > F || sort_lx) ? reinterpret_cast<uint64_t *>(wb + ord_off[l]) : (uint64_t *)nullptr;
    };
    auto mbr = [&](uint32_t l) { return reinterpret_cast<float4 *>(wb + mbr_off[l]); };
    auto pos = [&](uint32_t l) { return reinterpret_cast<uint32_t *>(wb + pos_off[l]); };
    uint64_t *keys = reinterpret_cast<uint64_t *>(wb + keys_off);
    uint64_t *tmp = reinterpret_cast<uint64_t *>(wb + tmp_off);
    uint32_t *xrank = reinterpret_cast<uint32_t *>(wb + xrank_off);
    uint32_t *hist = reinterpret_cast<uint32_t *>(wb + hist_off);
    uint64_t *hscan = reinterpret_cast<uint64_t *>(wb + hscan_off);
    uint64_t *stmp = reinterpret_cast<uint64_t *>(wb + stmp_off);
    uint32_t *flag = reinterpret_cast<uint32_t *>(wb + flag_off);
    uint32_t *partial = reinterpret_cast<uint32_t *>(wb + partial_off);

    e = launch_zero(flag, 4, s);
    if (e == hipSuccess && n) {
        hipLaunchKernelGGL(str_validate, dim3(grid_for(n)), dim3(256), 0, s, d_rects, n, flag);
        e = hipGetLastError();
    }
    // bottom up: packing order and node MBRs of every level
    const int top32[4] = {32, 40, 48, 56};
    for (uint32_t l = 0; l < H && e == hipSuccess; ++l) {
        const uint32_t cl = (uint32_t)items[l];
        const float4 *it = l == 0 ? d_rects : mbr(l - 1);
        uint64_t *order = ord(l);
        if (cl > F) {
            const uint64_t P = nodes[l];
            uint64_t S = (uint64_t)std::sqrt((double)P);
            while (S * S < P) ++S;
            while (S > 1 && (S - 1) * (S - 1) >= P) --S;
            const uint64_t slice = S * F;
            const uint64_t nsl = (cl + slice - 1) / slice;
            int sb = 0;
            while ((1ull << sb) < nsl) ++sb;
            bool in_tmp = false;
            const uint32_t g = grid_for(cl);
            // x order -> x-rank of every item
            hipLaunchKernelGGL(str_center_keys, dim3(g), dim3(256), 0, s, it, cl, 0, keys);
            e = launch_radix_sort_u64(keys, tmp, cl, top32, 4, hist, hscan, stmp, &in_tmp, s);
            if (e != hipSuccess) break;
            hipLaunchKernelGGL(str_xrank, dim3(g), dim3(256), 0, s, in_tmp ? tmp : keys, cl, xrank);
            // (y key, index) order
            hipLaunchKernelGGL(str_center_keys, dim3(g), dim3(256), 0, s, it, cl, 1, keys);
            e = launch_radix_sort_u64(keys, tmp, cl, top32, 4, hist, hscan, stmp, &in_tmp, s);
            if (e != hipSuccess) break;
            const uint64_t *ys = in_tmp ? tmp : keys;
            // stable by slice; the passes end in `order`
            const int npass = (sb + 7) / 8;
            const int sshift[4] = {32, 40, 48, 56};
            uint64_t *a = (npass & 1) ? (ys == tmp ? keys : tmp) : order;
            uint64_t *b = (npass & 1) ? order : (ys == tmp ? keys : tmp);
            hipLaunchKernelGGL(str_slice_keys, dim3(g), dim3(256), 0, s, ys, xrank, cl, slice, a);
            e = launch_radix_sort_u64(a, b, cl, sshift, npass, hist, hscan, stmp, &in_tmp, s);
            if (e != hipSuccess) break;
            if ((in_tmp ? b : a) != order) {
                e = hipErrorUnknown;
                break;
            }
        }
        if (sort_lx) {   // the top level's packing order is the identity
            hipLaunchKernelGGL(str_sort_runs, dim3((uint32_t)((nodes[l] + 3) / 4)), dim3(256), 0, s,
                               cl > F ? order : (const uint64_t *)nullptr, order, it, cl, F, (uint32_t)nodes[l]);
        }
        hipLaunchKernelGGL(str_mbrs, dim3(grid_for(nodes[l])), dim3(256), 0, s, it, order, cl, F,
                           (uint32_t)nodes[l], mbr(l));
        e = hipGetLastError();
    }
    // top down: places of the nodes inside their level
    if (e == hipSuccess) e = launch_zero(pos(H - 1), 4, s);
    for (uint32_t l = H - 1; l >= 1 && e == hipSuccess; --l) {
        hipLaunchKernelGGL(str_child_pos, dim3(grid_for(items[l])), dim3(256), 0, s, ord(l), pos(l),
                           (uint32_t)items[l], F, (uint32_t)nodes[l], pos(l - 1));
        e = hipGetLastError();
    }
    for (uint32_t l = 0; l < H && e == hipSuccess; ++l) {
        const float4 *it = l == 0 ? d_rects : mbr(l - 1);
        hipLaunchKernelGGL(str_write_level, dim3(grid_for(nodes[l] * F)), dim3(256), 0, s, ord(l), it, pos(l),
                           l > 0 ? pos(l - 1) : (uint32_t *)nullptr, (uint32_t)items[l], (uint32_t)nodes[l], F,
                           layout, l, (uint32_t)first[l], l > 0 ? (uint32_t)first[l - 1] : 0u,
                           static_cast<uint8_t *>(t->d_nodes), static_cast<uint32_t *>(t->d_meta));
        e = hipGetLastError();
    }
    // leaf ranges, bottom up, and the leaf that is not full
    const uint32_t no_partial[3] = {0xFFFFFFFFu, F, 0u};
    if (e == hipSuccess) e = hipMemcpyAsync(partial, no_partial, 12, hipMemcpyHostToDevice, s);
    if (e == hipSuccess) {
        hipLaunchKernelGGL(str_range_leaves, dim3(grid_for(nodes[0])), dim3(256), 0, s, (uint32_t)first[0],
                           (uint32_t)nodes[0], F, static_cast<const uint32_t *>(t->d_meta),
                           static_cast<uint2 *>(t->d_range), partial);
        e = hipGetLastError();
    }
    if (e == hipSuccess && n) {
        hipLaunchKernelGGL(str_leaf_ids, dim3(grid_for(nodes[0] * F)), dim3(256), 0, s, (uint32_t)first[0],
                           (uint32_t)nodes[0], F, layout, static_cast<const uint8_t *>(t->d_nodes),
                           static_cast<const uint32_t *>(t->d_meta), partial, n,
                           static_cast<uint32_t *>(t->d_leaf_ids));
        e = hipGetLastError();
    }
    for (uint32_t l = 1; l < H && e == hipSuccess; ++l) {
        hipLaunchKernelGGL(str_range_up, dim3(grid_for(nodes[l])), dim3(256), 0, s, (uint32_t)first[l],
                           (uint32_t)nodes[l], F, layout, static_cast<const uint8_t *>(t->d_nodes),
                           static_cast<const uint32_t *>(t->d_meta), static_cast<uint2 *>(t->d_range));
        e = hipGetLastError();
    }
    uint32_t hpartial[3] = {0xFFFFFFFFu, F, 0u};
    if (e == hipSuccess) e = hipMemcpyAsync(hpartial, partial, 12, hipMemcpyDeviceToHost, s);
    float4 root = make_float4(NAN, NAN, NAN, NAN);
    uint32_t hflag = 0;
    if (e == hipSuccess) e = hipMemcpyAsync(&root, mbr(H - 1), 16, hipMemcpyDeviceToHost, s);
    if (e == hipSuccess) e = hipMemcpyAsync(&hflag, flag, 4, hipMemcpyDeviceToHost, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    if (e != hipSuccess) return bail(hip_fail(e, "device build"));
    if (hflag) return bail(fail(RT_EINVAL, "rects contain a NaN coordinate or low > high"));
    if (hpartial[2] > 1) return bail(fail(RT_EDEVICE, "packing left %u leaves short of %u entries", hpartial[2], F));
    t->partial_leaf = hpartial[0];
    t->partial_cnt = hpartial[1];
    t->mbr[0] = root.x;
    t->mbr[1] = root.y;
    t->mbr[2] = root.z;
    t->mbr[3] = root.w;
    *out = t;
    return RT_OK;
}

}  // namespace rtk

using namespace rtk;

extern "C" int rt_build_str_device(const float *d_rects, uint64_t n, uint32_t fanout, uint32_t layout, void *stream,
                                   rt_tree **out) {
    if (!out) return fail(RT_EINVAL, "out is NULL");
    *out = nullptr;
    try {
        if (fanout != 0 && (fanout < 2 || fanout > 64)) return fail(RT_EINVAL, "fanout %u not in 2..64", fanout);
        const bool sort_lx = (layout & RT_BUILD_SORT_LX) != 0;
        layout &= ~RT_BUILD_SORT_LX;
        if (layout != RT_LAYOUT_AOS && layout != RT_LAYOUT_SOA && layout != RT_LAYOUT_D2 && layout != RT_LAYOUT_AUTO)
            return fail(RT_EINVAL, "unknown layout %u", layout);
        if (n >= 0xFFFFFFFFull) return fail(RT_EINVAL, "n = %llu does not fit 32-bit ids", (unsigned long long)n);
        if (n && !d_rects) return fail(RT_EINVAL, "rects is NULL with n = %llu", (unsigned long long)n);
        if ((reinterpret_cast<uintptr_t>(d_rects) & 15) != 0) return fail(RT_EINVAL, "rects not 16-byte aligned");
        if (fanout == 0 || layout == RT_LAYOUT_AUTO)
            return build_tuned(reinterpret_cast<const float4 *>(d_rects), n, fanout, layout, sort_lx,
                               static_cast<hipStream_t>(stream), out);
        return build_str_on_device(reinterpret_cast<const float4 *>(d_rects), n, fanout, layout, sort_lx,
                                   static_cast<hipStream_t>(stream), out);
    } catch (const std::bad_alloc &) {
        return fail(RT_ENOMEM, "host allocation failed");
    } catch (...) {
        return fail(RT_EDEVICE, "unexpected failure");
    }
}
