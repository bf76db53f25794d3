// Sort-Tile-Recursive packing of rectangles into the device node layouts.
//
// The paper does not say how its R-trees are built; this library bulk-loads
// them with STR (Leutenegger, Lopez, Edgington 1997).  Per level with c
// items: P = ceil(c / F) nodes, S = ceil(sqrt(P)) vertical slices of S*F
// items ordered by x-center, each slice ordered by y-center, consecutive runs
// of F items become one node.  Because every slice holds a multiple of F
// items, all nodes of a level are full except possibly the last one, and the
// next level's items are the node MBRs.  The tree shape never changes a
// query result.
//
// Centers are compared as order-preserving 32-bit integers made from the
// float32 value 0.5*lo + 0.5*hi (a non-number center, from an infinite
// rectangle, is ordered as 0).
#include "str_pack.h"
#include "rt_internal.h"

#include <algorithm>
#include <cmath>
#include <cstring>
#include <thread>
#include <vector>

namespace rtk {

static inline uint32_t order_key(float c) {
    if (c != c) c = 0.0f;
    uint32_t u;
    std::memcpy(&u, &c, 4);
    return (u & 0x80000000u) ? ~u : (u | 0x80000000u);
}

static unsigned workers() {
    unsigned h = std::thread::hardware_concurrency();
    if (h == 0) h = 4;
    return h > 16 ? 16 : h;
}

template <class Fn>
static void parallel_for(size_t n, Fn fn) {
    const unsigned w = workers();
    if (n < 2 || w < 2) {
        for (size_t i = 0; i < n; ++i) fn(i);
        return;
    }
    std::vector<std::thread> th;
    std::atomic<size_t> next{0};
    for (unsigned k = 0; k < w; ++k)
        th.emplace_back([&]() {
            for (size_t i = next.fetch_add(1); i < n; i = next.fetch_add(1)) fn(i);
        });
    for (auto &t : th) t.join();
}

// Sort 64-bit words ascending using sorted chunks and pairwise merges.
static void par_sort(std::vector<uint64_t> &v) {
    const size_t n = v.size();
    const unsigned w = workers();
    if (n < (1u << 16) || w < 2) {
        std::sort(v.begin(), v.end());
        return;
    }
    size_t chunks = 1;
    while (chunks < w) chunks <<= 1;
    const size_t per = (n + chunks - 1) / chunks;
    parallel_for(chunks, [&](size_t c) {
        size_t a = std::min(n, c * per), b = std::min(n, (c + 1) * per);
        std::sort(v.begin() + a, v.begin() + b);
    });
    std::vector<uint64_t> tmp(n);
    std::vector<uint64_t> *src = &v, *dst = &tmp;
    for (size_t width = per; width < n; width *= 2) {
        const size_t pairs = (n + 2 * width - 1) / (2 * width);
        parallel_for(pairs, [&](size_t p) {
            size_t a = p * 2 * width, m = std::min(n, a + width), b = std::min(n, a + 2 * width);
            std::merge(src->begin() + a, src->begin() + m, src->begin() + m, src->begin() + b,
                       dst->begin() + a);
        });
        std::swap(src, dst);
    }
    if (src != &v) v.swap(tmp);
}

// Order of the items of one level after STR: out[r] = item packed at rank r.
static void str_order(const float *lx, const float *ly, const float *hx, const float *hy, uint64_t c,
                      uint32_t F, std::vector<uint32_t> &out) {
    std::vector<uint64_t> k(c);
    parallel_for((c + 65535) / 65536, [&](size_t b) {
        const uint64_t i0 = b * 65536, i1 = std::min<uint64_t>(c, i0 + 65536);
        for (uint64_t i = i0; i < i1; ++i)
            k[i] = ((uint64_t)order_key(0.5f * lx[i] + 0.5f * hx[i]) << 32) | (uint32_t)i;
    });
    par_sort(k);
    const uint64_t P = (c + F - 1) / F;
    uint64_t S = (uint64_t)std::sqrt((double)P);
    while (S * S < P) ++S;
    while (S > 1 && (S - 1) * (S - 1) >= P) --S;
    const uint64_t slice = S * F;
    const uint64_t nslices = (c + slice - 1) / slice;
    parallel_for(nslices, [&](size_t s) {
        const uint64_t a = s * slice, b = std::min(c, a + slice);
        for (uint64_t r = a; r < b; ++r) {
            const uint32_t i = (uint32_t)k[r];
            k[r] = ((uint64_t)order_key(0.5f * ly[i] + 0.5f * hy[i]) << 32) | i;
        }
        std::sort(k.begin() + a, k.begin() + b);
    });
    out.resize(c);
    for (uint64_t r = 0; r < c; ++r) out[r] = (uint32_t)k[r];
}

int str_pack(const float *rects, uint64_t n, uint32_t F, uint32_t layout, PackedTree &pt) {
    // Items of the current level (structure of arrays).
    std::vector<float> lx(n), ly(n), hx(n), hy(n);
    for (uint64_t i = 0; i < n; ++i) {
        lx[i] = rects[4 * i + 0];
        ly[i] = rects[4 * i + 1];
        hx[i] = rects[4 * i + 2];
        hy[i] = rects[4 * i + 3];
    }
    // Per level (leaf level first): packed item order and node count.
    std::vector<std::vector<uint32_t>> orders;
    std::vector<uint64_t> items;   // item count per level
    std::vector<std::vector<float>> L_lx, L_ly, L_hx, L_hy;
    uint64_t c = n;
    while (true) {
        items.push_back(c);
        L_lx.push_back(lx);
        L_ly.push_back(ly);
        L_hx.push_back(hx);
        L_hy.push_back(hy);
        std::vector<uint32_t> ord;
        if (c > F) {
            str_order(lx.data(), ly.data(), hx.data(), hy.data(), c, F, ord);
        } else {
            ord.resize(c);
            for (uint64_t i = 0; i < c; ++i) ord[i] = (uint32_t)i;
        }
        const uint64_t P = c > F ? (c + F - 1) / F : 1;
        // node MBRs become the next level's items
        std::vector<float> nlx(P), nly(P), nhx(P), nhy(P);
        parallel_for((P + 4095) / 4096, [&](size_t b) {
            const uint64_t k0 = b * 4096, k1 = std::min<uint64_t>(P, k0 + 4096);
            for (uint64_t k = k0; k < k1; ++k) {
                float a = INFINITY, bb = INFINITY, cc = -INFINITY, d = -INFINITY;
                const uint64_t r0 = k * F, r1 = std::min<uint64_t>(c, r0 + F);
                for (uint64_t r = r0; r < r1; ++r) {
                    const uint32_t i = ord[r];
                    a = std::min(a, lx[i]);
                    bb = std::min(bb, ly[i]);
                    cc = std::max(cc, hx[i]);
                    d = std::max(d, hy[i]);
                }
                if (r1 == r0) a = bb = cc = d = NAN;   // empty tree: no MBR
                nlx[k] = a;
                nly[k] = bb;
                nhx[k] = cc;
                nhy[k] = d;
            }
        });
        orders.push_back(std::move(ord));
        if (c <= F) {
            pt.mbr[0] = nlx[0];
            pt.mbr[1] = nly[0];
            pt.mbr[2] = nhx[0];
            pt.mbr[3] = nhy[0];
            break;
        }
        lx.swap(nlx);
        ly.swap(nly);
        hx.swap(nhx);
        hy.swap(nhy);
        c = P;
    }
    const uint32_t H = (uint32_t)orders.size();
    std::vector<uint64_t> nodes_at(H), first_at(H);
    for (uint32_t l = 0; l < H; ++l) nodes_at[l] = items[l] > F ? (items[l] + F - 1) / F : 1;
    uint64_t total = 0;
    for (int l = (int)H - 1; l >= 0; --l) {
        first_at[l] = total;
        total += nodes_at[l];
    }
    if (total >= 0xFFFFFFFFull) return -1;
    pt.fanout = F;
    pt.layout = layout;
    pt.height = H;
    pt.n_nodes = (uint32_t)total;
    pt.first_leaf = (uint32_t)first_at[0];
    for (uint32_t l = 0; l < H && l < 33; ++l) pt.level_start[l] = (uint32_t)first_at[l];
    pt.node_bytes = 20u * F;
    pt.n_objects = n;
    pt.bytes.assign((size_t)total * pt.node_bytes, 0);
    pt.meta.assign(total, 0);
    uint64_t n_entries = 0;
    for (uint32_t l = 0; l < H; ++l) n_entries += items[l];
    pt.n_entries = n_entries;

    // Final numbering: breadth first from the root, each node's children in
    // its entry order, so the children of every node are contiguous and a
    // child is found as (first child) + (entry slot).  newidx[l][k] is the
    // global index of node k of level l (k in creation order).
    std::vector<std::vector<uint32_t>> newidx(H);
    for (uint32_t l = 0; l < H; ++l) newidx[l].assign(nodes_at[l], 0);
    newidx[H - 1][0] = 0;
    for (uint32_t l = H - 1; l >= 1; --l) {
        // visit level-l nodes in their final order
        std::vector<uint32_t> inv(nodes_at[l]);
        for (uint64_t k = 0; k < nodes_at[l]; ++k) inv[newidx[l][k] - first_at[l]] = (uint32_t)k;
        uint64_t next = first_at[l - 1];
        const std::vector<uint32_t> &ord = orders[l];
        for (uint64_t g = 0; g < nodes_at[l]; ++g) {
            const uint64_t k = inv[g];
            const uint64_t r0 = k * F, r1 = std::min<uint64_t>(items[l], r0 + F);
            for (uint64_t r = r0; r < r1; ++r) newidx[l - 1][ord[r]] = (uint32_t)next++;
        }
    }

    for (uint32_t l = 0; l < H; ++l) {
        const std::vector<uint32_t> &ord = orders[l];
        const uint64_t c_l = items[l];
        const std::vector<float> &a = L_lx[l], &b = L_ly[l], &cc = L_hx[l], &d = L_hy[l];
        parallel_for((nodes_at[l] + 4095) / 4096, [&](size_t blk) {
            const uint64_t k0 = blk * 4096, k1 = std::min<uint64_t>(nodes_at[l], k0 + 4096);
            for (uint64_t k = k0; k < k1; ++k) {
                const uint64_t g = newidx[l][k];
                uint8_t *node = pt.bytes.data() + g * pt.node_bytes;
                float *f = reinterpret_cast<float *>(node);
                uint32_t *u = reinterpret_cast<uint32_t *>(node);
                const uint64_t r0 = k * F, r1 = std::min<uint64_t>(c_l, r0 + F);
                const uint32_t cnt = (uint32_t)(r1 - r0);
                pt.meta[g] = cnt | (l << 8);
                for (uint32_t e = 0; e < F; ++e) {
                    float vlx = NAN, vly = NAN, vhx = NAN, vhy = NAN;
                    uint32_t p = 0xFFFFFFFFu;
                    if (e < cnt) {
                        const uint32_t i = ord[r0 + e];
                        vlx = a[i];
                        vly = b[i];
                        vhx = cc[i];
                        vhy = d[i];
                        p = l == 0 ? i : newidx[l - 1][i];
                    }
                    if (layout == LAYOUT_SOA) {
                        f[e] = vlx;
                        f[F + e] = vly;
                        f[2 * F + e] = vhx;
                        f[3 * F + e] = vhy;
                        u[4 * F + e] = p;
                    } else if (layout == LAYOUT_AOS) {
                        f[5 * e + 0] = vlx;
                        f[5 * e + 1] = vly;
                        f[5 * e + 2] = vhx;
                        f[5 * e + 3] = vhy;
                        u[5 * e + 4] = p;
                    } else {
                        f[2 * e] = vlx;
                        f[2 * e + 1] = vly;
                        f[2 * F + 2 * e] = vhx;
                        f[2 * F + 2 * e + 1] = vhy;
                        u[4 * F + e] = p;
                    }
                }
            }
        });
    }
    return 0;
}

}  // namespace rtk
