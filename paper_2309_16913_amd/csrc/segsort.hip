// Segmented sort of the CSR id lists (each query's ids ascending).
//
// Object ids are spread over [0, n), so a segment splits evenly when it is
// bucketed by the top bits of its ids.  The sort is therefore one MSD
// bucketing pass followed by independent sorts of small buckets:
//
//   classify   every segment with >= 2 ids goes to a size-class list
//              (appends aggregated per block);
//   class S    (<= 256 ids)     one wave per segment: the ids sit in
//              registers (up to 4 per lane) and a bitonic network runs over
//              them with __shfl_xor for cross-lane partners;
//   class M    (257 .. 32768, in four block shapes: 128 x 8, 256 x 16,
//              512 x 32 and 1024 x 32 threads x ids)  one block per segment:
//              ids to registers, a counting sort on the top b id bits
//              (2^b ~ length/4 buckets, LDS counters), scatter into LDS,
//              then every bucket sorted in place by a register network (or,
//              for the shortest, each id counts the smaller ids of its own
//              bucket and is stored at bucket start + that count);
//   class L    (> 32768)        one block per segment: an MSD pass on the top
//              8 id bits into global scratch (chunks digit-sorted in LDS and
//              written as runs), then groups of consecutive sub-buckets
//              (<= 4096 ids each, or <= 32768 when a sub-bucket holds more)
//              sorted back by one block each;
//   fallback   a segment with a bucket too long for the in-bucket ranking
//              (ids far from uniform) is sorted by a block bitonic network in
//              LDS (class M) or, for class L with a sub-bucket over 32768 ids,
//              by sorting 16384-id tiles that way and merging runs pairwise
//              through LDS-staged merge-path windows.
#include "rt_internal.h"

namespace rtk {

constexpr uint32_t kKeyPad = 0xFFFFFFFFu;   // never an object id (ids < 2^32 - 1)
constexpr uint32_t kMidMax = 32768;         // longest class-M segment
constexpr uint32_t kTileMax = 16384;        // tile of the class-L fallback
constexpr uint32_t kNumCls = 6;             // S, M1, M2, M3, M4, L (by length)
constexpr uint32_t kLong = 5;
constexpr uint32_t kFallback = 6;           // fallback-L list
constexpr uint32_t kListCls = 7;

// Significant bits of the largest id below range (0 for range <= 1).
__device__ __forceinline__ int range_bits(uint32_t range) {
    return range > 1 ? 32 - __clz((int)(range - 1)) : 0;
}

// The id range of segment q: its own (seg_range, when given per segment) or
// the common one.
__device__ __forceinline__ uint32_t seg_id_range(const uint32_t *seg_range, uint32_t q, uint32_t id_range) {
    return seg_range ? seg_range[q] : id_range;
}

__device__ __forceinline__ uint32_t ceil_log2(uint32_t v) {
    uint32_t b = 0;
    while (b < 31 && (1u << b) < v) ++b;
    return b;
}

// The key of lane (lane ^ j), for the constant distances of a bitonic
// network: a DPP quad permutation for 1 and 2 (an ordinary vector move), the
// bit-mask swizzle for 4, 8 and 16 (within each 32-lane half, no address
// register), a lane permute for 32.  All 64 lanes must be active: DPP and
// swizzle reads of a lane outside the execution mask do not return its key.
__device__ __forceinline__ uint32_t xor_lane(uint32_t v, uint32_t j) {
    if (j == 1) return (uint32_t)__builtin_amdgcn_mov_dpp((int)v, 0xB1, 0xF, 0xF, true);   // quad [1,0,3,2]
    if (j == 2) return (uint32_t)__builtin_amdgcn_mov_dpp((int)v, 0x4E, 0xF, 0xF, true);   // quad [2,3,0,1]
    if (j == 4) return (uint32_t)__builtin_amdgcn_ds_swizzle((int)v, 0x1F | (4 << 10));
    if (j == 8) return (uint32_t)__builtin_amdgcn_ds_swizzle((int)v, 0x1F | (8 << 10));
    if (j == 16) return (uint32_t)__builtin_amdgcn_ds_swizzle((int)v, 0x1F | (16 << 10));
    return (uint32_t)__shfl_xor((int)v, (int)j);
}

// Bitonic sort of the 64*R keys v[r] (element index r*64 + lane) ascending.
template <int R>
__device__ __forceinline__ void wave_bitonic(uint32_t (&v)[R]) {
    const uint32_t lane = threadIdx.x & 63u;
#pragma unroll
    for (uint32_t k = 2; k <= 64u * R; k <<= 1) {
#pragma unroll
        for (uint32_t j = k >> 1; j > 0; j >>= 1) {
            if (j >= 64) {
#pragma unroll
                for (int r = 0; r < R; ++r) {
                    const int p = r ^ (int)(j / 64);
                    if (p > r) {
                        const bool up = (((uint32_t)r * 64 + lane) & k) == 0;
                        const uint32_t a = v[r], b = v[p];
                        const bool sw = up ? (a > b) : (a < b);
                        v[r] = sw ? b : a;
                        v[p] = sw ? a : b;
                    }
                }
            } else {
#pragma unroll
                for (int r = 0; r < R; ++r) {
                    const uint32_t o = xor_lane(v[r], j);
                    const bool up = (((uint32_t)r * 64 + lane) & k) == 0;
                    const bool lower = (lane & j) == 0;
                    v[r] = (lower == up) ? min(v[r], o) : max(v[r], o);
                }
            }
        }
    }
}

// Block bitonic sort of the first P (power of two) keys of an LDS array.
__device__ void block_bitonic(uint32_t *a, uint32_t P) {
    for (uint32_t k = 2; k <= P; k <<= 1) {
        for (uint32_t j = k >> 1; j > 0; j >>= 1) {
            for (uint32_t t = threadIdx.x; t < P / 2; t += blockDim.x) {
                const uint32_t i = ((t & ~(j - 1)) << 1) | (t & (j - 1));
                const uint32_t l = i | j;
                const uint32_t x = a[i], y = a[l];
                const bool up = (i & k) == 0;
                if ((x > y) == up) {
                    a[i] = y;
                    a[l] = x;
                }
            }
            __syncthreads();
        }
    }
}

// ---------------------------------------------------------------------------
// classify
// ---------------------------------------------------------------------------
constexpr uint32_t kClsPer = 16;                   // queries per thread
constexpr uint32_t kClsTile = 256 * kClsPer;       // queries per block

__global__ void __launch_bounds__(256)
seg_classify(const uint64_t *__restrict__ offsets, uint64_t nq, uint64_t cap, uint32_t *__restrict__ lists,
             uint32_t *__restrict__ counts) {
    __shared__ uint32_t bcnt[kNumCls], gbase[kNumCls];
    if (offsets[nq] > cap) return;
    const uint32_t lane = threadIdx.x & 63u;
    const uint64_t lt = lane ? (~0ull >> (64 - lane)) : 0ull;
    if (threadIdx.x < kNumCls) bcnt[threadIdx.x] = 0;
    __syncthreads();
    const uint64_t q0 = (uint64_t)blockIdx.x * kClsTile;
    int cls[kClsPer];
    uint32_t pos[kClsPer];
#pragma unroll
    for (uint32_t k = 0; k < kClsPer; ++k) {
        const uint64_t q = q0 + (uint64_t)k * 256 + threadIdx.x;
        int c = -1;
        if (q < nq) {
            const uint64_t len = offsets[q + 1] - offsets[q];
            if (len >= 2)
                c = len <= 256 ? 0 : len <= 1024 ? 1 : len <= 4096 ? 2 : len <= 16384 ? 3 : len <= kMidMax ? 4 : 5;
        }
        cls[k] = c;
        pos[k] = 0;
#pragma unroll
        for (int j = 0; j < (int)kNumCls; ++j) {
            const uint64_t m = __ballot(c == j);
            if (m == 0) continue;
            const uint32_t leader = (uint32_t)__builtin_ctzll(m);
            uint32_t at = 0;
            if (lane == leader) at = atomicAdd(&bcnt[j], (uint32_t)__popcll(m));
            at = __shfl(at, (int)leader);
            if (c == j) pos[k] = at + (uint32_t)__popcll(m & lt);
        }
    }
    __syncthreads();
    if (threadIdx.x < kNumCls)
        gbase[threadIdx.x] = bcnt[threadIdx.x] ? atomicAdd(&counts[threadIdx.x], bcnt[threadIdx.x]) : 0u;
    __syncthreads();
#pragma unroll
    for (uint32_t k = 0; k < kClsPer; ++k) {
        const int c = cls[k];
        if (c >= 0) lists[(uint64_t)c * nq + gbase[c] + pos[k]] = (uint32_t)(q0 + (uint64_t)k * 256 + threadIdx.x);
    }
}

// ---------------------------------------------------------------------------
// class S: one wave per segment
// ---------------------------------------------------------------------------
// Sort the s <= 256 keys a wave holds (v[r] = key r*64 + lane, pad beyond
// s) into dst[0..s).
__device__ __forceinline__ void wave_sort_regs4(uint32_t (&v)[4], uint32_t *dst, uint32_t s) {
    const uint32_t lane = threadIdx.x & 63u;
    if (s < 2) {
        if (s == 1 && lane == 0) dst[0] = v[0];
        return;
    }
    if (s <= 16) {   // ranks by broadcasting each key
        uint32_t rk = 0;
        for (uint32_t j = 0; j < s; ++j) {
            const uint32_t x = (uint32_t)__builtin_amdgcn_readlane((int)v[0], (int)j);
            rk += (x < v[0] || (x == v[0] && j < lane)) ? 1u : 0u;
        }
        if (lane < s) dst[rk] = v[0];
        return;
    }
    if (s <= 64) {
        uint32_t a[1] = {v[0]};
        wave_bitonic<1>(a);
        if (lane < s) dst[lane] = a[0];
    } else if (s <= 128) {
        uint32_t a[2] = {v[0], v[1]};
        wave_bitonic<2>(a);
#pragma unroll
        for (int r = 0; r < 2; ++r)
            if ((uint32_t)r * 64 + lane < s) dst[r * 64 + lane] = a[r];
    } else {
        wave_bitonic<4>(v);
#pragma unroll
        for (int r = 0; r < 4; ++r)
            if ((uint32_t)r * 64 + lane < s) dst[r * 64 + lane] = v[r];
    }
}

// One wave per segment; the wave's next segment is loaded into registers
// before the current one is sorted, so its load overlaps the sort.
__global__ void __launch_bounds__(256)
segsort_small(const uint64_t *__restrict__ offsets, uint32_t *__restrict__ ids, const uint32_t *__restrict__ list,
              const uint32_t *__restrict__ list_count) {
    const uint32_t m = *list_count;
    const uint32_t wpb = blockDim.x / 64;
    const uint32_t lane = threadIdx.x & 63u;
    const uint32_t step = gridDim.x * wpb;
    uint32_t nv[4];
    uint64_t no = 0;
    uint32_t nc = 0;
    auto load = [&](uint32_t i) {
        const uint32_t q = list[i];
        no = offsets[q];
        nc = (uint32_t)(offsets[q + 1] - no);
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            const uint32_t k = (uint32_t)r * 64 + lane;
            nv[r] = k < nc ? ids[no + k] : kKeyPad;
        }
    };
    uint32_t i = blockIdx.x * wpb + (threadIdx.x >> 6);
    if (i < m) load(i);
    for (; i < m; i += step) {
        uint32_t v[4];
#pragma unroll
        for (int r = 0; r < 4; ++r) v[r] = nv[r];
        const uint64_t o = no;
        const uint32_t c = nc;
        if (i + step < m) load(i + step);   // segments are disjoint: never the ids written below
        wave_sort_regs4(v, ids + o, c);
    }
}

// ---------------------------------------------------------------------------
// classes M and L: counting sort on the top id bits, then in-bucket sorts
// ---------------------------------------------------------------------------
// With 2^b ~ length/4 buckets on the top b bits of the ids, a bucket holds a
// handful of ids.  One LDS counter per bucket first counts, is then turned
// into the bucket's start by an exclusive scan, and serves as the scatter
// cursor; after the scatter counter b holds the end of bucket b, so bucket b
// spans [end(b-1), end(b)).  Every bucket is then sorted in place (one lane
// per bucket, a register network).  A bucket of more than kRankMax ids (ids
// far from uniform) sends the segment to a fallback.
constexpr uint32_t kRankMax = 64;

// Exclusive scan in place of cnt[0 .. nbk) by T threads (nbk <= 4*T or a
// multiple of 4*T handled in rounds); returns the largest count.
template <int T>
__device__ uint32_t block_scan_counters(uint32_t *cnt, uint32_t nbk, uint32_t *wsum, uint32_t *scal) {
    constexpr uint32_t W = T / 64;
    const uint32_t t = threadIdx.x, lane = t & 63u, w = t >> 6;
    uint32_t carry = 0, mxall = 0;
    for (uint32_t b0 = 0; b0 < nbk; b0 += 4 * T) {
        uint32_t v[4], sum = 0, mx = 0;
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            const uint32_t i = b0 + 4 * t + r;
            v[r] = i < nbk ? cnt[i] : 0u;
            sum += v[r];
            mx = max(mx, v[r]);
        }
        uint32_t inc = sum;
#pragma unroll
        for (int d = 1; d < 64; d <<= 1) {
            const uint32_t x = __shfl_up(inc, d);
            if ((int)lane >= d) inc += x;
            mx = max(mx, __shfl_xor(mx, d));
        }
        if (lane == 63) wsum[w] = inc;
        if (lane == 0) wsum[W + w] = mx;
        __syncthreads();
        uint32_t base = carry, tot = 0;
        for (uint32_t i = 0; i < W; ++i) {
            if (i < w) base += wsum[i];
            tot += wsum[i];
            mxall = max(mxall, wsum[W + i]);
        }
        uint32_t ex = base + inc - sum;
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            const uint32_t i = b0 + 4 * t + r;
            if (i < nbk) cnt[i] = ex;
            ex += v[r];
        }
        carry += tot;
        __syncthreads();
    }
    (void)scal;
    return mxall;
}

// Batcher's odd-even merge sort of N = 2^k inputs, restricted to its first M
// (all indices fixed at compile time).  With inputs M.. taken as +inf, every
// comparator touching them is a no-op (a +inf never leaves the top M..N-1
// positions), so dropping those comparators sorts any M values: 12, 19, 32,
// 42 and 63 comparators for M = 6, 8, 10, 12, 16 (bitonic over 8 and 16
// inputs: 24 and 80).
template <int N, int M>
__device__ __forceinline__ void reg_oem(uint32_t (&v)[M]) {
#pragma unroll
    for (int p = 1; p < N; p <<= 1) {
#pragma unroll
        for (int k = p; k >= 1; k >>= 1) {
#pragma unroll
            for (int j = k % p; j + k < N; j += 2 * k) {
#pragma unroll
                for (int i = 0; i < k; ++i) {
                    if (i + j + k < M && (i + j) / (2 * p) == (i + j + k) / (2 * p)) {
                        const uint32_t x = v[i + j], y = v[i + j + k];
                        v[i + j] = x < y ? x : y;
                        v[i + j + k] = x < y ? y : x;
                    }
                }
            }
        }
    }
}

// Sort the k <= M ids a[s0 .. s0 + k) in place through M registers.
template <int M>
__device__ __forceinline__ void sort_run_regs(uint32_t *a, uint32_t s0, uint32_t k) {
    uint32_t v[M];
#pragma unroll
    for (int j = 0; j < M; ++j) v[j] = (uint32_t)j < k ? a[s0 + j] : kKeyPad;
    reg_oem<(M <= 8 ? 8 : (M <= 16 ? 16 : 32)), M>(v);
#pragma unroll
    for (int j = 0; j < M; ++j)
        if ((uint32_t)j < k) a[s0 + j] = v[j];
}

// Sort every bucket [end(b-1), end(b)) of a in place, one lane per bucket:
// the ids of a bucket go through a register network sized by the longest
// bucket in the wave (6, 8, 10, 12 or 16 inputs, and 20 or 24 with WIDE),
// longer buckets (rare) are insertion-sorted.
template <int T, bool WIDE>
__device__ __forceinline__ void sort_buckets(uint32_t *a, const uint32_t *end, uint32_t nbk) {
    for (uint32_t b0 = 0; b0 < nbk; b0 += T) {
        const uint32_t b = b0 + threadIdx.x;
        uint32_t s0 = 0, k = 0;
        if (b < nbk) {
            s0 = b ? end[b - 1] : 0u;
            k = end[b] - s0;
        }
        uint32_t kmax = k;
        for (int d = 32; d >= 1; d >>= 1) kmax = max(kmax, (uint32_t)__shfl_xor((int)kmax, d));
        if (kmax <= 6) {
            sort_run_regs<6>(a, s0, k);
        } else if (kmax <= 8) {
            sort_run_regs<8>(a, s0, k);
        } else if (kmax <= 10) {
            sort_run_regs<10>(a, s0, k);
        } else if (kmax <= 12) {
            sort_run_regs<12>(a, s0, k);
        } else if (kmax <= 16) {
            sort_run_regs<16>(a, s0, k);
        } else {
            bool done = false;
            if constexpr (WIDE) {
                if (kmax <= 20) {
                    sort_run_regs<20>(a, s0, k);
                    done = true;
                } else if (kmax <= 24) {
                    sort_run_regs<24>(a, s0, k);
                    done = true;
                }
            }
            for (uint32_t i = 1; !done && i < k; ++i) {
                const uint32_t x = a[s0 + i];
                uint32_t j = i;
                while (j > 0 && a[s0 + j - 1] > x) {
                    a[s0 + j] = a[s0 + j - 1];
                    --j;
                }
                a[s0 + j] = x;
            }
        }
    }
}

// Sort c <= T*K ids, given in registers (key[k] holds id k*T + thread, pad
// beyond c), into dst with one block: counting sort into nbk = 2^b ~ c/4
// buckets of equal width over the id range (bucket of id x: (x - base) *
// nbk / range, as a 32-bit multiply-high; LDS counters), scatter into LDS,
// sort every bucket in place, copy out.  The caller guarantees base <= id <
// base + range for every id.  A: target ids per bucket (nbk ~ c/A, at most
// T*K/A; with A = 8 the bucket networks go up to 24 inputs).  A bucket longer than kRankMax (ids far from uniform) switches the
// segment to a block bitonic network.  PLACE: instead of sorting the buckets in place and copying
// out, every key is stored straight at its final place (faster for short
// segments, where the bucket networks are mostly padding); cnt must then
// follow buf in LDS.  buf: T*K words, cnt: T*K/A words, wsum: 2*T/64 words
// of LDS.
template <int T, int K, bool PLACE = false, int A = 4>
__device__ __forceinline__ void block_sort_keys(uint32_t (&key)[K], uint32_t *dst, uint32_t c, uint32_t range,
                                                uint32_t *buf, uint32_t *cnt, uint32_t *wsum, uint32_t base = 0) {
    constexpr uint32_t N = T * K;
    constexpr uint32_t NB = N / A;   // most buckets
    const uint32_t t = threadIdx.x;
    uint32_t nb = ceil_log2((c + A - 1) / A);
    const uint32_t nbmax = ceil_log2(NB);
    nb = nb < 1 ? 1 : (nb > nbmax ? nbmax : nb);
    const uint32_t nbk = 1u << nb;
    // floor(y * mul / 2^32) < nbk for every y < range, and it never decreases
    // with y; the min() only guards against ids outside the promised range
    const uint32_t mul = range > nbk ? (uint32_t)(((uint64_t)nbk << 32) / range) : 0xFFFFFFFFu;
    auto bucket = [&](uint32_t x) { return min(__umulhi(x - base, mul), nbk - 1); };
    for (uint32_t b = t; b < nbk; b += T) cnt[b] = 0;
    __syncthreads();
    // rows k with k*T >= c hold nothing: the (block-uniform) row loops stop
    // there, so the work follows c rather than the tile size
#pragma unroll
    for (int k = 0; k < K; ++k) {
        if ((uint32_t)k * T >= c) break;
        if ((uint32_t)k * T + t < c) atomicAdd(&cnt[bucket(key[k])], 1u);
    }
    __syncthreads();
    const uint32_t big = block_scan_counters<T>(cnt, nbk, wsum, nullptr);
#pragma unroll
    for (int k = 0; k < K; ++k) {
        if ((uint32_t)k * T >= c) break;
        if ((uint32_t)k * T + t < c) buf[atomicAdd(&cnt[bucket(key[k])], 1u)] = key[k];
    }
    __syncthreads();
    if (big <= kRankMax && PLACE) {
        // buckets are contiguous in buf: the key at position i goes to its
        // bucket's start plus the number of keys of the bucket that precede
        // it (smaller, or equal and earlier).  A wave's 64 positions land on
        // a permutation of about the same 64 outputs, so the stores stay
        // coalesced.  The 4-wide reads run up to 3 words past the keys: buf
        // must be followed by at least 3 words of LDS (the counters are).
        for (uint32_t i = t; i < c; i += T) {
            const uint32_t x = buf[i];
            const uint32_t b = bucket(x);
            const uint32_t s0 = b ? cnt[b - 1] : 0u;
            const uint32_t e0 = cnt[b];
            uint32_t r = s0;
            for (uint32_t j = s0; j < e0; j += 4) {
                const uint32_t y0 = buf[j], y1 = buf[j + 1], y2 = buf[j + 2], y3 = buf[j + 3];
                r += (y0 < x || (y0 == x && j < i)) ? 1u : 0u;
                r += (j + 1 < e0 && (y1 < x || (y1 == x && j + 1 < i))) ? 1u : 0u;
                r += (j + 2 < e0 && (y2 < x || (y2 == x && j + 2 < i))) ? 1u : 0u;
                r += (j + 3 < e0 && (y3 < x || (y3 == x && j + 3 < i))) ? 1u : 0u;
            }
            dst[r] = x;
        }
    } else if (big <= kRankMax) {
        // buckets are contiguous in buf: sort each in place, then one
        // coalesced copy out
        sort_buckets<T, (A >= 8)>(buf, cnt, nbk);
        __syncthreads();
        for (uint32_t i = t; i < c; i += T) dst[i] = buf[i];
    } else {   // ids far from uniform: block bitonic over the whole segment
        uint32_t P = 1;
        while (P < c) P <<= 1;
        for (uint32_t i = c + t; i < P; i += T) buf[i] = kKeyPad;
        __syncthreads();
        block_bitonic(buf, P);
        for (uint32_t i = t; i < c; i += T) dst[i] = buf[i];
    }
    __syncthreads();
}

template <int T, int K>
__device__ __forceinline__ void load_keys(const uint32_t *src, uint32_t c, uint32_t (&key)[K]) {
#pragma unroll
    for (int k = 0; k < K; ++k) {
        const uint32_t i = (uint32_t)k * T + threadIdx.x;
        key[k] = i < c ? src[i] : kKeyPad;
    }
}

// One block per segment of the class list.  With PF the next segment's ids
// are loaded into registers before the current one is sorted, so their load
// overlaps the sort (it costs K registers, which the widest shape cannot
// spare: a 1024-thread block has 128 per lane).  Register budgets: shapes of
// 16384 ids and up are held to 4 waves per SIMD, so that two 512-thread
// blocks share a CU; 256-thread blocks to 6 (six blocks of 20 KB LDS each).
template <int T, int K>
constexpr int mid_waves_per_simd() {
    return T * K >= 16384 ? 4 : (T == 256 ? 6 : 1);
}

template <int T, int K, bool PLACE, bool PF, int A>
__global__ void __launch_bounds__(T, (mid_waves_per_simd<T, K>()))
segsort_mid(const uint64_t *__restrict__ offsets, uint32_t *__restrict__ ids, const uint32_t *__restrict__ list,
            const uint32_t *__restrict__ list_count, uint32_t id_range, const uint32_t *__restrict__ seg_range) {
    constexpr uint32_t N = T * K;
    // keys, then the bucket counters; the scan's per-wave sums use the head
    // of buf, which holds nothing while the counters are scanned
    __shared__ uint32_t lds[N + N / A];
    uint32_t *buf = lds, *cnt = lds + N, *wsum = lds;
    const uint32_t m = *list_count;
    if constexpr (PF) {
        uint32_t nkey[K];
        uint64_t no = 0;
        uint32_t nc = 0, nr = id_range;
        if (blockIdx.x < m) {
            const uint32_t q = list[blockIdx.x];
            no = offsets[q];
            nc = (uint32_t)(offsets[q + 1] - no);
            nr = seg_id_range(seg_range, q, id_range);
            load_keys<T, K>(ids + no, nc, nkey);
        }
        for (uint32_t li = blockIdx.x; li < m; li += gridDim.x) {
            uint32_t key[K];
#pragma unroll
            for (int k = 0; k < K; ++k) key[k] = nkey[k];
            const uint64_t o = no;
            const uint32_t c = nc, rng = nr;
            const uint32_t ln = li + gridDim.x;
            if (ln < m) {   // segments are disjoint: this read never meets the writes below
                const uint32_t q = list[ln];
                no = offsets[q];
                nc = (uint32_t)(offsets[q + 1] - no);
                nr = seg_id_range(seg_range, q, id_range);
                load_keys<T, K>(ids + no, nc, nkey);
            }
            block_sort_keys<T, K, PLACE, A>(key, ids + o, c, rng, buf, cnt, wsum);
        }
    } else {
        for (uint32_t li = blockIdx.x; li < m; li += gridDim.x) {
            const uint32_t q = list[li];
            const uint64_t o = offsets[q];
            const uint32_t c = (uint32_t)(offsets[q + 1] - o);
            uint32_t key[K];
            load_keys<T, K>(ids + o, c, key);
            block_sort_keys<T, K, PLACE, A>(key, ids + o, c, seg_id_range(seg_range, q, id_range), buf, cnt, wsum);
        }
    }
}

// Class L: two levels.  First (segsort_long, one block per segment) the
// segment is split by its top 8 id bits into 256 sub-buckets in global
// scratch: a histogram (per-wave LDS counters, eight loads in flight per
// thread), a scan, then chunks of 8192
// ids are counting-sorted by that digit in LDS and written out as contiguous
// runs, one run per digit and chunk; the 257 sub-bucket starts go to the
// segment's descriptor.  Then groups of G consecutive sub-buckets are sorted
// from scratch back into place by the whole grid, one block per group
// (segsort_sub): G is chosen so that a group holds at most 4096 ids, or at
// most 32768 (a 1024-thread block) when a sub-bucket holds more than 4096
// (segments of about a million ids).  A segment with a sub-bucket over 32768
// ids (ids far from uniform) is left as it is and goes to the fallback list.
constexpr uint32_t kLongDigits = 256;
constexpr uint32_t kLongChunk = 8192;   // ids per chunk: 1024 threads x 8
constexpr uint32_t kSubMax = 4096;      // longest group sorted by a 256-thread block
constexpr uint32_t kSubBigMax = 32768;  // longest group sorted by a 1024-thread block
constexpr uint32_t kDesc = kLongDigits + 2;   // 257 sub-bucket starts, group width
constexpr uint32_t kSubCounts = 8;      // counters of the two group work lists (in the class counter block)

// 1024 threads held to 64 registers (two blocks, 32 waves per CU; one 4-byte
// spill, reloaded once per segment): the pass waits on LDS and memory, and
// at 16 waves per CU (512 threads, 122 registers) the 50M-rectangle loop's
// sort took 16.1 instead of 15.5 ms.
template <int T>
__global__ void __launch_bounds__(T, 8)
segsort_long(const uint64_t *__restrict__ offsets, uint32_t *__restrict__ ids, uint32_t *__restrict__ scratch,
             uint32_t *__restrict__ desc, uint32_t *__restrict__ sub_lists, uint32_t *__restrict__ sub_lists_wide,
             uint32_t *__restrict__ sub_counts,
             const uint32_t *__restrict__ list, const uint32_t *__restrict__ list_count,
             uint32_t *__restrict__ fb_list, uint32_t *__restrict__ fb_count, uint32_t id_range,
             const uint32_t *__restrict__ seg_range) {
    constexpr uint32_t W = T / 64, R = kLongChunk / T;
    static_assert(T >= kLongDigits, "one thread per digit");
    __shared__ uint32_t whist[W * kLongDigits];   // per-wave digit counts
    __shared__ uint32_t stage[kLongChunk];        // digit-sorted chunk
    __shared__ uint32_t start[kLongDigits + 1];   // sub-bucket starts (start[256] = c)
    __shared__ uint32_t cur[kLongDigits];         // write cursor per digit
    __shared__ uint32_t lh[kLongDigits], loff[kLongDigits], lcur[kLongDigits];
    __shared__ uint32_t big, subbase[1];
    const uint32_t m = *list_count;
    const uint32_t t = threadIdx.x, lane = t & 63u, w = t >> 6;
    for (uint32_t li = blockIdx.x; li < m; li += gridDim.x) {
        const uint32_t q = list[li];
        const int id_bits = range_bits(seg_id_range(seg_range, q, id_range));
        const int db = id_bits < 8 ? id_bits : 8;
        const int sh = id_bits - db;
        const uint32_t dmask = (1u << db) - 1u;
        const uint64_t o = offsets[q];
        const uint32_t c = (uint32_t)(offsets[q + 1] - o);
        const uint32_t *seg = ids + o;
        uint32_t *tmp = scratch + o;
        uint32_t *dsc = desc + (uint64_t)li * kDesc;
        // digit histogram
        for (uint32_t i = t; i < W * kLongDigits; i += T) whist[i] = 0;
        if (t == 0) big = 0;
        __syncthreads();
        constexpr uint32_t U = 8192 / T;   // loads in flight per thread
        for (uint32_t i0 = t; i0 < c; i0 += T * U) {
            uint32_t kk[U];
#pragma unroll
            for (uint32_t u = 0; u < U; ++u) {
                const uint32_t i = i0 + u * T;
                kk[u] = i < c ? seg[i] : 0u;
            }
#pragma unroll
            for (uint32_t u = 0; u < U; ++u)
                if (i0 + u * T < c) atomicAdd(&whist[w * kLongDigits + ((kk[u] >> sh) & dmask)], 1u);
        }
        __syncthreads();
        if (w == 0) {   // one wave: totals and exclusive scan over the 256 digits
            uint32_t v[4], sum = 0, mx = 0;
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const uint32_t d = lane * 4 + r;
                uint32_t x = 0;
                for (uint32_t ww = 0; ww < W; ++ww) x += whist[ww * kLongDigits + d];
                v[r] = x;
                sum += x;
                mx = max(mx, x);
            }
            uint32_t inc = sum;
#pragma unroll
            for (int d = 1; d < 64; d <<= 1) {
                const uint32_t x = __shfl_up(inc, d);
                if ((int)lane >= d) inc += x;
                mx = max(mx, (uint32_t)__shfl_xor((int)mx, d));
            }
            uint32_t ex = inc - sum;
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                start[lane * 4 + r] = ex;
                cur[lane * 4 + r] = ex;
                ex += v[r];
            }
            if (lane == 63) start[kLongDigits] = inc;
            if (lane == 0) big = mx;
        }
        __syncthreads();
        if (big > kSubBigMax) {   // leave the segment to the fallback
            if (t == 0) fb_list[atomicAdd(fb_count, 1u)] = q;
            __syncthreads();
            continue;
        }
        // sub-bucket groups for the block sorts: G consecutive digits each,
        // G = (group limit) / (largest digit count), so a group never exceeds
        // the limit: kSubMax ids for the 256-thread sort, or, when a digit
        // holds more (segments of about a million ids), kSubBigMax for the
        // 1024-thread sort (its own list); work items are li << 8 | group
        const bool wide = big > kSubMax;
        const uint32_t G = (wide ? kSubBigMax : kSubMax) / (big ? big : 1u);
        const uint32_t ngroups = (kLongDigits + G - 1) / G;
        for (uint32_t d = t; d <= kLongDigits; d += T) dsc[d] = start[d];
        if (t == 0) {
            dsc[kLongDigits + 1] = G;
            subbase[0] = atomicAdd(&sub_counts[wide ? 1 : 0], ngroups);
        }
        __syncthreads();
        if (t < ngroups) (wide ? sub_lists_wide : sub_lists)[subbase[0] + t] = (li << 8) | t;
        // chunks, digit-sorted in LDS, written out as runs; the next chunk's
        // ids are loaded while this one is sorted and written
        uint32_t nkey[R];
#pragma unroll
        for (uint32_t r = 0; r < R; ++r) {
            const uint32_t i = r * T + t;
            nkey[r] = i < c ? seg[i] : 0u;
        }
        for (uint32_t base = 0; base < c; base += kLongChunk) {
            const uint32_t len = (c - base) < kLongChunk ? (c - base) : kLongChunk;
            if (t < kLongDigits) lh[t] = 0;
            __syncthreads();
            uint32_t key[R];
#pragma unroll
            for (uint32_t r = 0; r < R; ++r) {
                key[r] = nkey[r];
                if (r * T + t < len) atomicAdd(&lh[(key[r] >> sh) & dmask], 1u);
            }
            const uint32_t nb = base + kLongChunk;
#pragma unroll
            for (uint32_t r = 0; r < R; ++r) {
                const uint32_t i = r * T + t;
                nkey[r] = nb + i < c ? seg[nb + i] : 0u;
            }
            __syncthreads();
            if (w == 0) {
                uint32_t v[4], sum = 0;
#pragma unroll
                for (int r = 0; r < 4; ++r) {
                    v[r] = lh[lane * 4 + r];
                    sum += v[r];
                }
                uint32_t inc = sum;
#pragma unroll
                for (int d = 1; d < 64; d <<= 1) {
                    const uint32_t x = __shfl_up(inc, d);
                    if ((int)lane >= d) inc += x;
                }
                uint32_t ex = inc - sum;
#pragma unroll
                for (int r = 0; r < 4; ++r) {
                    loff[lane * 4 + r] = ex;
                    lcur[lane * 4 + r] = ex;
                    ex += v[r];
                }
            }
            __syncthreads();
#pragma unroll
            for (uint32_t r = 0; r < R; ++r) {
                const uint32_t i = r * T + t;
                if (i < len) stage[atomicAdd(&lcur[(key[r] >> sh) & dmask], 1u)] = key[r];
            }
            __syncthreads();
            for (uint32_t j = t; j < len; j += T) {
                const uint32_t x = stage[j];
                const uint32_t d = (x >> sh) & dmask;
                tmp[cur[d] + (j - loff[d])] = x;
            }
            __syncthreads();
            if (t < kLongDigits) cur[t] += lh[t];
            __syncthreads();
        }
    }
}

// Groups of sub-buckets (digits [gG, gG + G)): one block each, sorted from
// scratch into place; the ids of a group lie in [gG << sh, (gG + G) << sh).
// Two shapes: 256 x 16 for groups of at most kSubMax ids, 1024 x 32 for the
// groups of segments whose digits hold more.  With PF the next group's ids
// are loaded before the current one is sorted.
template <int T, int K>
constexpr int sub_waves_per_simd() {
    return T == 256 ? 6 : 4;
}

template <int T, int K, int A, bool PF>
__global__ void __launch_bounds__(T, (sub_waves_per_simd<T, K>()))
segsort_sub(const uint64_t *__restrict__ offsets, uint32_t *__restrict__ ids, const uint32_t *__restrict__ scratch,
            const uint32_t *__restrict__ desc, const uint32_t *__restrict__ items,
            const uint32_t *__restrict__ item_count, const uint32_t *__restrict__ list, uint32_t id_range,
            const uint32_t *__restrict__ seg_range) {
    constexpr uint32_t N = T * K;
    __shared__ uint32_t buf[N];
    __shared__ uint32_t cnt[N / A];
    __shared__ uint32_t wsum[2 * (T / 64)];
    const uint32_t m = *item_count;
    struct Grp {
        uint64_t o;
        uint32_t n, base, range;
    };
    auto group = [&](uint32_t k) {
        const uint32_t it = items[k], li = it >> 8, g = it & 255u;
        const uint32_t *dsc = desc + (uint64_t)li * kDesc;
        const uint32_t G = dsc[kLongDigits + 1];
        const uint32_t d0 = g * G, d1 = (d0 + G) < kLongDigits ? (d0 + G) : kLongDigits;
        const uint32_t s0 = dsc[d0];
        const uint32_t q = list[li];
        const uint32_t rng = seg_id_range(seg_range, q, id_range);
        const int id_bits = range_bits(rng);
        const int sh = id_bits - (id_bits < 8 ? id_bits : 8);
        Grp r;
        r.o = offsets[q] + s0;
        r.n = dsc[d1] - s0;
        r.base = d0 << sh;   // ids of digits [d0, d1): [d0 << sh, d1 << sh) within [0, rng)
        const uint64_t hi = (uint64_t)d1 << sh;
        r.range = (uint32_t)((hi < rng ? hi : (uint64_t)rng) - r.base);
        return r;
    };
    if constexpr (PF) {
        uint32_t nkey[K];
        Grp nx{0, 0, 0, 1};
        if (blockIdx.x < m) {
            nx = group(blockIdx.x);
            load_keys<T, K>(scratch + nx.o, nx.n, nkey);
        }
        for (uint32_t k = blockIdx.x; k < m; k += gridDim.x) {
            uint32_t key[K];
#pragma unroll
            for (int r = 0; r < (int)K; ++r) key[r] = nkey[r];
            const Grp cu = nx;
            if (k + gridDim.x < m) {
                nx = group(k + gridDim.x);
                load_keys<T, K>(scratch + nx.o, nx.n, nkey);
            }
            block_sort_keys<T, K, false, A>(key, ids + cu.o, cu.n, cu.range, buf, cnt, wsum, cu.base);
        }
    } else {
        for (uint32_t k = blockIdx.x; k < m; k += gridDim.x) {
            const Grp cu = group(k);
            uint32_t key[K];
            load_keys<T, K>(scratch + cu.o, cu.n, key);
            block_sort_keys<T, K, false, A>(key, ids + cu.o, cu.n, cu.range, buf, cnt, wsum, cu.base);
        }
    }
}

// ---------------------------------------------------------------------------
// fallback for long segments with skewed ids: sorted tiles + pairwise merges
// ---------------------------------------------------------------------------
__global__ void __launch_bounds__(1024)
segsort_tiles(const uint64_t *__restrict__ offsets, uint32_t *__restrict__ ids, const uint32_t *__restrict__ list,
              const uint32_t *__restrict__ list_count) {
    __shared__ uint32_t buf[kTileMax];
    const uint32_t m = *list_count;
    for (uint32_t li = blockIdx.x; li < m; li += gridDim.x) {
        const uint32_t q = list[li];
        const uint64_t o = offsets[q];
        const uint64_t c = offsets[q + 1] - o;
        for (uint64_t t0 = 0; t0 < c; t0 += kTileMax) {
            const uint32_t tc = (uint32_t)((c - t0) < kTileMax ? (c - t0) : kTileMax);
            uint32_t P = 1;
            while (P < tc) P <<= 1;
            for (uint32_t i = threadIdx.x; i < P; i += 1024) buf[i] = i < tc ? ids[o + t0 + i] : kKeyPad;
            __syncthreads();
            block_bitonic(buf, P);
            for (uint32_t i = threadIdx.x; i < tc; i += 1024) ids[o + t0 + i] = buf[i];
            __syncthreads();
        }
    }
}

__device__ __forceinline__ uint32_t pidx(uint32_t i) { return i + (i >> 5); }

__device__ __forceinline__ uint32_t lds_merge_path(const uint32_t *lds, uint32_t a0, uint32_t la, uint32_t b0,
                                                   uint32_t lb, uint32_t d) {
    uint32_t lo = d > lb ? d - lb : 0;
    uint32_t hi = d < la ? d : la;
    while (lo < hi) {
        const uint32_t mid = (lo + hi) >> 1;
        if (lds[pidx(a0 + mid)] <= lds[pidx(b0 + d - mid - 1)])
            lo = mid + 1;
        else
            hi = mid;
    }
    return lo;
}

__device__ __forceinline__ uint64_t glb_merge_path(const uint32_t *a, uint64_t la, const uint32_t *b, uint64_t lb,
                                                   uint64_t d) {
    uint64_t lo = d > lb ? d - lb : 0;
    uint64_t hi = d < la ? d : la;
    while (lo < hi) {
        const uint64_t mid = (lo + hi) >> 1;
        if (a[mid] <= b[d - mid - 1])
            lo = mid + 1;
        else
            hi = mid;
    }
    return lo;
}

// Merge the sorted 16384-id runs of each listed segment pairwise until one
// run is left; every merge proceeds in windows of 16384 outputs whose inputs
// are staged in LDS.
__global__ void __launch_bounds__(1024)
segmerge_long(const uint64_t *__restrict__ offsets, uint32_t *__restrict__ ids, uint32_t *__restrict__ scratch,
              const uint32_t *__restrict__ list, const uint32_t *__restrict__ list_count) {
    constexpr uint32_t T = 1024, K = 16, N = T * K;
    __shared__ uint32_t lds[N + N / 32];
    __shared__ uint64_t split[2];
    const uint32_t m = *list_count;
    for (uint32_t li = blockIdx.x; li < m; li += gridDim.x) {
        const uint64_t q = list[li];
        const uint64_t o = offsets[q];
        const uint64_t c = offsets[q + 1] - o;
        uint32_t *src = ids + o, *dst = scratch + o;
        for (uint64_t w = kTileMax; w < c; w <<= 1) {
            for (uint64_t r0 = 0; r0 < c; r0 += 2 * w) {
                const uint64_t la = (c - r0) < w ? (c - r0) : w;
                const uint64_t rest = c - r0 - la;
                const uint64_t lb = rest < w ? rest : w;
                const uint32_t *A = src + r0, *B = src + r0 + la;
                uint32_t *out = dst + r0;
                for (uint64_t d0 = 0; d0 < la + lb; d0 += N) {
                    const uint64_t d1 = (d0 + N) < (la + lb) ? (d0 + N) : (la + lb);
                    if (threadIdx.x == 0) split[0] = glb_merge_path(A, la, B, lb, d0);
                    if (threadIdx.x == 1) split[1] = glb_merge_path(A, la, B, lb, d1);
                    __syncthreads();
                    const uint64_t ia0 = split[0], ia1 = split[1];
                    const uint32_t na = (uint32_t)(ia1 - ia0);
                    const uint32_t nb = (uint32_t)((d1 - d0) - na);
                    const uint64_t ib0 = d0 - ia0;
                    for (uint32_t i = threadIdx.x; i < na; i += T) lds[pidx(i)] = A[ia0 + i];
                    for (uint32_t i = threadIdx.x; i < nb; i += T) lds[pidx(na + i)] = B[ib0 + i];
                    __syncthreads();
                    uint32_t r[K];
                    const uint32_t dd = threadIdx.x * K;
                    const uint32_t tot = na + nb;
                    if (dd < tot) {
                        uint32_t ia = lds_merge_path(lds, 0, na, na, nb, dd);
                        uint32_t ib = dd - ia;
                        uint32_t a = ia < na ? lds[pidx(ia)] : kKeyPad;
                        uint32_t b = ib < nb ? lds[pidx(na + ib)] : kKeyPad;
#pragma unroll
                        for (uint32_t k = 0; k < K; ++k) {
                            const bool ta = ib >= nb || (ia < na && a <= b);
                            r[k] = ta ? a : b;
                            if (ta) {
                                ++ia;
                                a = ia < na ? lds[pidx(ia)] : kKeyPad;
                            } else {
                                ++ib;
                                b = ib < nb ? lds[pidx(na + ib)] : kKeyPad;
                            }
                        }
                    }
                    __syncthreads();
                    if (dd < tot) {
#pragma unroll
                        for (uint32_t k = 0; k < K; ++k)
                            if (dd + k < tot) lds[pidx(dd + k)] = r[k];
                    }
                    __syncthreads();
                    for (uint32_t i = threadIdx.x; i < tot; i += T) out[d0 + i] = lds[pidx(i)];
                    __syncthreads();
                }
            }
            uint32_t *t2 = src;
            src = dst;
            dst = t2;
        }
        if (src != ids + o) {
            for (uint64_t i = threadIdx.x; i < c; i += T) ids[o + i] = src[i];
        }
        __syncthreads();
    }
}

uint64_t segsort_ws_elems(uint64_t nq) { return (uint64_t)kListCls * nq + 64; }

// cap ids, then for each possible class-L segment (> kMidMax ids) its
// descriptor, then two lists with room for 256 work items per segment
uint64_t segsort_scratch_elems(uint64_t cap) {
    return cap + (cap / (kMidMax + 1) + 1) * (kDesc + 2 * kLongDigits);
}

template <typename Kern>
static uint32_t resident_per_cu(Kern kern, int threads) {
    int n = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, kern, threads, 0) != hipSuccess || n < 1) n = 1;
    return (uint32_t)n;
}

hipError_t launch_segsort(const uint64_t *offsets, uint64_t nq, uint32_t *ids, uint32_t *scratch, uint64_t cap,
                          uint32_t *ws, uint64_t id_range, const uint32_t *seg_range, hipStream_t s) {
    if (nq == 0) return hipSuccess;
    const uint32_t range = (uint32_t)(id_range < 0xFFFFFFFFull ? id_range : 0xFFFFFFFFull);
    uint32_t *counts = ws;            // class counters
    uint32_t *lists = ws + 64;        // kListCls lists of up to nq query indices
    const uint32_t cus = (uint32_t)num_cus();
    // blocks per CU that fit at once (registers and LDS): each persistent
    // grid holds that many, so no block waits for another to finish its share
    static const uint32_t g_small = resident_per_cu(segsort_small, 256);
    static const uint32_t g_m1 = resident_per_cu(segsort_mid<128, 8, true, true, 4>, 128);
    static const uint32_t g_m2 = resident_per_cu(segsort_mid<256, 16, false, true, 4>, 256);
    static const uint32_t g_m3 = resident_per_cu(segsort_mid<512, 32, false, true, 8>, 512);
    static const uint32_t g_m4 = resident_per_cu(segsort_mid<1024, 32, false, false, 8>, 1024);
    static const uint32_t g_long = resident_per_cu(segsort_long<1024>, 1024);
    static const uint32_t g_sub = resident_per_cu(segsort_sub<256, 16, 4, true>, 256);
    static const uint32_t g_subw = resident_per_cu(segsort_sub<1024, 32, 8, false>, 1024);
    hipError_t e = launch_zero(counts, 64 * 4, s);
    if (e != hipSuccess) return e;
    const uint64_t cg = (nq + kClsTile - 1) / kClsTile;
    hipLaunchKernelGGL(seg_classify, dim3((uint32_t)cg), dim3(256), 0, s, offsets, nq, cap, lists, counts);
    e = hipGetLastError();
    if (e != hipSuccess) return e;
    // every class on the caller's stream, shortest first (an extra stream
    // per call site would take one of the device's few hardware queues from
    // whatever else the process runs concurrently)
    // after the cap ids of scratch: kDesc words per class-L segment (257
    // sub-bucket starts and the group width), then its work items (at most
    // 256 groups per segment)
    const uint64_t nlong = cap / (kMidMax + 1) + 1;
    uint32_t *desc = scratch + cap;
    uint32_t *sub_list = desc + nlong * kDesc;
    uint32_t *sub_list_wide = sub_list + nlong * kLongDigits;
    hipLaunchKernelGGL(segsort_small, dim3(cus * g_small), dim3(256), 0, s, offsets, ids, lists, counts + 0);
    hipLaunchKernelGGL((segsort_mid<128, 8, true, true, 4>), dim3(cus * g_m1), dim3(128), 0, s, offsets, ids,
                       lists + nq, counts + 1, range, seg_range);
    hipLaunchKernelGGL((segsort_mid<256, 16, false, true, 4>), dim3(cus * g_m2), dim3(256), 0, s, offsets, ids,
                       lists + 2 * nq, counts + 2, range, seg_range);
    hipLaunchKernelGGL((segsort_mid<512, 32, false, true, 8>), dim3(cus * g_m3), dim3(512), 0, s, offsets, ids,
                       lists + 3 * nq, counts + 3, range, seg_range);
    hipLaunchKernelGGL((segsort_mid<1024, 32, false, false, 8>), dim3(cus * g_m4), dim3(1024), 0, s, offsets, ids,
                       lists + 4 * nq, counts + 4, range, seg_range);
    hipLaunchKernelGGL(segsort_long<1024>, dim3(cus * g_long), dim3(1024), 0, s, offsets, ids, scratch, desc, sub_list,
                       sub_list_wide, counts + kSubCounts, lists + kLong * nq, counts + kLong, lists + kFallback * nq,
                       counts + kFallback, range, seg_range);
    hipLaunchKernelGGL((segsort_sub<256, 16, 4, true>), dim3(cus * g_sub), dim3(256), 0, s, offsets, ids, scratch,
                       desc, sub_list, counts + kSubCounts, lists + kLong * nq, range, seg_range);
    hipLaunchKernelGGL((segsort_sub<1024, 32, 8, false>), dim3(cus * g_subw), dim3(1024), 0, s, offsets, ids,
                       scratch, desc, sub_list_wide, counts + kSubCounts + 1, lists + kLong * nq, range, seg_range);
    // the fallback kernels: almost always empty
    hipLaunchKernelGGL(segsort_tiles, dim3(cus * 2), dim3(1024), 0, s, offsets, ids, lists + kFallback * nq,
                       counts + kFallback);
    hipLaunchKernelGGL(segmerge_long, dim3(cus * 2), dim3(1024), 0, s, offsets, ids, scratch, lists + kFallback * nq,
                       counts + kFallback);
    e = hipGetLastError();
    return e;
}

}  // namespace rtk
