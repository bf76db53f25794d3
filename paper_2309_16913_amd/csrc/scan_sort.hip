// Prefix sums and sorts used to compact and canonicalize results.
//
//  * exclusive scan uint32 -> uint64 (counts -> CSR offsets), three kernels:
//    per-tile sums, a scan of the tile sums, and the per-tile scan with the
//    tile's base added;
//  * LSD radix sort of uint64 keys with 8-bit digits (join pairs), stable
//    per-tile ranking with wave ballots.
#include "rt_internal.h"

namespace rtk {

// ---------------------------------------------------------------------------
// wave / block scans
// ---------------------------------------------------------------------------
__device__ __forceinline__ uint64_t wave_incl_scan(uint64_t v) {
    const int lane = threadIdx.x & 63;
#pragma unroll
    for (int d = 1; d < 64; d <<= 1) {
        uint32_t lo = __shfl_up((uint32_t)v, d);
        uint32_t hi = __shfl_up((uint32_t)(v >> 32), d);
        uint64_t o = ((uint64_t)hi << 32) | lo;
        if (lane >= d) v += o;
    }
    return v;
}

// Exclusive scan over the 256 threads of a block; returns the exclusive
// prefix and writes the block total to *total.
__device__ __forceinline__ uint64_t block_excl_scan(uint64_t v, uint64_t *total) {
    __shared__ uint64_t wsum[4];
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    uint64_t inc = wave_incl_scan(v);
    if (lane == 63) wsum[w] = inc;
    __syncthreads();
    uint64_t base = 0, tot = 0;
    for (int i = 0; i < 4; ++i) {
        if (i < w) base += wsum[i];
        tot += wsum[i];
    }
    __syncthreads();
    *total = tot;
    return base + inc - v;
}

constexpr uint32_t kScanPer = 8;                 // elements per thread
constexpr uint32_t kScanTile = 256 * kScanPer;   // elements per block

// n_dev (if not NULL) holds the element count on the device, at most the n
// the grid was sized for.
__global__ void __launch_bounds__(256) scan_tile_sums(const uint32_t *__restrict__ in, uint64_t n,
                                                      const uint64_t *__restrict__ n_dev,
                                                      uint64_t *__restrict__ sums) {
    if (n_dev) n = min(n, *n_dev);
    const uint64_t base = (uint64_t)blockIdx.x * kScanTile + (uint64_t)threadIdx.x * kScanPer;
    uint64_t s = 0;
#pragma unroll
    for (uint32_t k = 0; k < kScanPer; ++k)
        if (base + k < n) s += in[base + k];
    uint64_t tot;
    block_excl_scan(s, &tot);
    if (threadIdx.x == 0) sums[blockIdx.x] = tot;
}

// single block: exclusive scan of the tile sums in place
__global__ void __launch_bounds__(256) scan_sums(uint64_t *__restrict__ sums, uint64_t nt) {
    uint64_t carry = 0;
    for (uint64_t b0 = 0; b0 < nt; b0 += 256) {
        const uint64_t i = b0 + threadIdx.x;
        uint64_t v = i < nt ? sums[i] : 0;
        uint64_t tot;
        uint64_t ex = block_excl_scan(v, &tot);
        if (i < nt) sums[i] = carry + ex;
        carry += tot;
        __syncthreads();
    }
}

// With n_dev, the block holding element n - 1 (block 0 for n = 0) writes
// out[n]; with next (not NULL) it also stores min(total, next_cap) there and
// sets *over when the total exceeds next_cap.
__global__ void __launch_bounds__(256) scan_tiles(const uint32_t *__restrict__ in, uint64_t n,
                                                  const uint64_t *__restrict__ n_dev,
                                                  const uint64_t *__restrict__ sums,
                                                  uint64_t *__restrict__ out, uint64_t *__restrict__ next,
                                                  uint64_t next_cap, uint32_t *__restrict__ over) {
    const bool dev = n_dev != nullptr;
    if (dev) n = min(n, *n_dev);
    const uint64_t base = (uint64_t)blockIdx.x * kScanTile + (uint64_t)threadIdx.x * kScanPer;
    uint32_t v[kScanPer];
    uint64_t s = 0;
#pragma unroll
    for (uint32_t k = 0; k < kScanPer; ++k) {
        v[k] = base + k < n ? in[base + k] : 0u;
        s += v[k];
    }
    uint64_t tot;
    uint64_t run = block_excl_scan(s, &tot) + sums[blockIdx.x];
#pragma unroll
    for (uint32_t k = 0; k < kScanPer; ++k) {
        if (base + k < n) out[base + k] = run;
        run += v[k];
    }
    const uint64_t last = dev ? (n ? (n - 1) / kScanTile : 0) : gridDim.x - 1;
    if (blockIdx.x == last && threadIdx.x == 255) {
        const uint64_t total = sums[blockIdx.x] + tot;
        out[n] = total;
        if (next) {
            next[0] = total < next_cap ? total : next_cap;
            if (total > next_cap) atomicOr(over, 1u);
        }
    }
}

__global__ void write_zero_total(uint64_t *out) { out[0] = 0; }

uint64_t scan_tmp_elems(uint64_t n) { return (n + kScanTile - 1) / kScanTile + 1; }
uint64_t scan_tile_elems() { return kScanTile; }

hipError_t launch_scan_u32(const uint32_t *in, uint64_t n, uint64_t *out, uint64_t *tmp, hipStream_t s) {
    if (n == 0) {
        hipLaunchKernelGGL(write_zero_total, dim3(1), dim3(1), 0, s, out);
        return hipGetLastError();
    }
    const uint64_t nt = (n + kScanTile - 1) / kScanTile;
    hipLaunchKernelGGL(scan_tile_sums, dim3((uint32_t)nt), dim3(256), 0, s, in, n, (const uint64_t *)nullptr, tmp);
    hipLaunchKernelGGL(scan_sums, dim3(1), dim3(256), 0, s, tmp, nt);
    hipLaunchKernelGGL(scan_tiles, dim3((uint32_t)nt), dim3(256), 0, s, in, n, (const uint64_t *)nullptr, tmp, out,
                       (uint64_t *)nullptr, (uint64_t)0, (uint32_t *)nullptr);
    return hipGetLastError();
}

hipError_t launch_scan_u32_dev(const uint32_t *in, const uint64_t *n_dev, uint64_t n_max, uint64_t *out,
                               uint64_t *tmp, uint64_t *next, uint64_t next_cap, uint32_t *over, hipStream_t s) {
    const uint64_t nt = n_max ? (n_max + kScanTile - 1) / kScanTile : 1;
    hipLaunchKernelGGL(scan_tile_sums, dim3((uint32_t)nt), dim3(256), 0, s, in, n_max, n_dev, tmp);
    hipLaunchKernelGGL(scan_sums, dim3(1), dim3(256), 0, s, tmp, nt);
    hipLaunchKernelGGL(scan_tiles, dim3((uint32_t)nt), dim3(256), 0, s, in, n_max, n_dev, tmp, out, next, next_cap,
                       over);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// zero fill (used instead of a memset node so the launches can be captured)
// ---------------------------------------------------------------------------
__global__ void zero_kernel(uint32_t *p, uint64_t n) {
    for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
         i += (uint64_t)gridDim.x * blockDim.x)
        p[i] = 0u;
}

hipError_t launch_zero(void *p, uint64_t bytes, hipStream_t s) {
    const uint64_t n = bytes / 4;
    if (n == 0) return hipSuccess;
    uint64_t blocks = (n + 255) / 256;
    if (blocks > 4096) blocks = 4096;
    hipLaunchKernelGGL(zero_kernel, dim3((uint32_t)blocks), dim3(256), 0, s, (uint32_t *)p, n);
    return hipGetLastError();
}

__global__ void finalize_kernel(const uint64_t *offsets, uint64_t nq, uint64_t cap, const Ctrl *ctrl,
                                uint64_t *status) {
    const uint64_t tot = offsets[nq];
    uint64_t flags = 0;
    if (tot > cap) flags |= 1;
    if (ctrl->err) flags |= 2;
    status[0] = tot;
    status[1] = flags;
}

hipError_t launch_finalize(const uint64_t *offsets, uint64_t nq, uint64_t cap, const Ctrl *ctrl,
                           uint64_t *status, hipStream_t s) {
    hipLaunchKernelGGL(finalize_kernel, dim3(1), dim3(1), 0, s, offsets, nq, cap, ctrl, status);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// LSD radix sort of uint64 keys (8- or 11-bit digits)
// ---------------------------------------------------------------------------
constexpr uint32_t kRadixPer = 16;                    // keys per lane
constexpr uint32_t kRadixWaveKeys = 64 * kRadixPer;   // 1024
constexpr uint32_t kRadixTile = 4 * kRadixWaveKeys;   // 4096 per block

uint64_t radix_hist_elems(uint64_t n, int digit_bits) {
    const uint64_t nb = (n + kRadixTile - 1) / kRadixTile;
    return nb << digit_bits;
}

// hist[digit * nblocks + block]
template <int DB>
__global__ void __launch_bounds__(256) radix_hist(const uint64_t *__restrict__ keys, uint64_t n, int shift,
                                                  uint32_t *__restrict__ hist) {
    constexpr uint32_t D = 1u << DB;
    __shared__ uint32_t h[D];
    for (uint32_t d = threadIdx.x; d < D; d += 256) h[d] = 0;
    __syncthreads();
    const uint64_t base = (uint64_t)blockIdx.x * kRadixTile;
    for (uint32_t k = threadIdx.x; k < kRadixTile; k += 256) {
        const uint64_t i = base + k;
        if (i < n) atomicAdd(&h[(uint32_t)(keys[i] >> shift) & (D - 1)], 1u);
    }
    __syncthreads();
    for (uint32_t d = threadIdx.x; d < D; d += 256) hist[(uint64_t)d * gridDim.x + blockIdx.x] = h[d];
}

// Stable within a block: a key's rank among the equal digits of its wave
// comes from DB ballots (one per digit bit), the waves' counts are added in
// wave order.
template <int DB>
__global__ void __launch_bounds__(256) radix_scatter(const uint64_t *__restrict__ in, uint64_t n, int shift,
                                                     const uint64_t *__restrict__ hscan,
                                                     uint64_t *__restrict__ out) {
    constexpr uint32_t D = 1u << DB;
    __shared__ uint32_t wcnt[4][D];
    __shared__ uint64_t dbase[D];
    const uint32_t lane = threadIdx.x & 63u, w = threadIdx.x >> 6;
    for (uint32_t d = threadIdx.x; d < D; d += 256) {
        for (int i = 0; i < 4; ++i) wcnt[i][d] = 0;
        dbase[d] = hscan[(uint64_t)d * gridDim.x + blockIdx.x];
    }
    __syncthreads();
    const uint64_t base = (uint64_t)blockIdx.x * kRadixTile + (uint64_t)w * kRadixWaveKeys;
    const uint64_t lt = lane ? (~0ull >> (64 - lane)) : 0ull;
    uint64_t key[kRadixPer];
    uint32_t pos[kRadixPer];
#pragma unroll
    for (uint32_t k = 0; k < kRadixPer; ++k) {
        const uint64_t i = base + (uint64_t)k * 64 + lane;
        const bool ok = i < n;
        key[k] = ok ? in[i] : 0ull;
        const uint32_t dg = (uint32_t)(key[k] >> shift) & (D - 1);
        uint64_t peers = __ballot(ok);
#pragma unroll
        for (int b = 0; b < DB; ++b) {
            const uint64_t bb = __ballot((dg >> b) & 1u);
            peers &= ((dg >> b) & 1u) ? bb : ~bb;
        }
        const uint32_t r = (uint32_t)__popcll(peers & lt);
        uint32_t p = 0;
        if (ok) p = wcnt[w][dg] + r;
        __builtin_amdgcn_wave_barrier();
        // highest lane of each digit group advances the wave's counter
        if (ok && (peers >> lane) == 1ull) wcnt[w][dg] += (uint32_t)__popcll(peers);
        __builtin_amdgcn_wave_barrier();
        pos[k] = p;
    }
    __syncthreads();
#pragma unroll
    for (uint32_t k = 0; k < kRadixPer; ++k) {
        const uint64_t i = base + (uint64_t)k * 64 + lane;
        if (i < n) {
            const uint32_t dg = (uint32_t)(key[k] >> shift) & (D - 1);
            uint64_t o = dbase[dg];
            for (uint32_t ww = 0; ww < w; ++ww) o += wcnt[ww][dg];
            out[o + pos[k]] = key[k];
        }
    }
}

template <int DB>
static hipError_t radix_passes(uint64_t *keys, uint64_t *tmp, uint64_t n, const int *shifts, int npasses,
                               uint32_t *hist, uint64_t *hscan, uint64_t *stmp, bool *in_tmp, hipStream_t s) {
    const uint64_t nb = (n + kRadixTile - 1) / kRadixTile;
    uint64_t *src = keys, *dst = tmp;
    for (int p = 0; p < npasses; ++p) {
        hipLaunchKernelGGL(radix_hist<DB>, dim3((uint32_t)nb), dim3(256), 0, s, src, n, shifts[p], hist);
        hipError_t e = launch_scan_u32(hist, nb << DB, hscan, stmp, s);
        if (e != hipSuccess) return e;
        hipLaunchKernelGGL(radix_scatter<DB>, dim3((uint32_t)nb), dim3(256), 0, s, src, n, shifts[p], hscan, dst);
        uint64_t *t = src;
        src = dst;
        dst = t;
    }
    *in_tmp = (src == tmp);
    return hipGetLastError();
}

hipError_t launch_radix_sort_u64(uint64_t *keys, uint64_t *tmp, uint64_t n, const int *shifts, int npasses,
                                 uint32_t *hist, uint64_t *hscan, uint64_t *stmp, bool *in_tmp, hipStream_t s,
                                 int digit_bits) {
    *in_tmp = false;
    if (n < 2 || npasses == 0) return hipSuccess;
    if (digit_bits == 11) return radix_passes<11>(keys, tmp, n, shifts, npasses, hist, hscan, stmp, in_tmp, s);
    if (digit_bits != 8) return hipErrorInvalidValue;
    return radix_passes<8>(keys, tmp, n, shifts, npasses, hist, hscan, stmp, in_tmp, s);
}

}  // namespace rtk
