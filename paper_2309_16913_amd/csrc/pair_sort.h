// Sort of the join's pair keys ((idA << 32) | idB, all distinct) by their top
// digit: the keys are split into kPairBuckets buckets by key >> shift (the
// bucket order is the key order), and every bucket is then sorted on its own
// in LDS (a bucket over the LDS cap in runs, merged through global memory).
// Four launches where an LSD radix sort of two 21-bit ids needs four passes
// of five.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

namespace rtk {

constexpr uint32_t kPairBuckets = 2048;      // 11-bit top digit
constexpr uint32_t kPairBucketCap = 4096;    // keys a bucket may hold to be sorted in LDS

// Workspace (uint32 words) of launch_pair_bucket_sort: counts, starts and
// cursors.
constexpr uint64_t kPairSortWords = 3 * kPairBuckets + 8;

// keys (n) -> out (n), sorted; keys is overwritten (merge space for buckets
// over the LDS cap).  shift: every key is below 2^(shift + 11).  ws:
// kPairSortWords uint32.  n_dev (if not NULL): the key count on the device,
// at most n (n then only sizes the grids).
hipError_t launch_pair_bucket_sort(uint64_t *keys, uint64_t n, int shift, uint64_t *out, uint32_t *ws,
                                   hipStream_t s, const uint64_t *n_dev = nullptr);

// Keys to (a, b) words with the count on the device (at most n_max): writes
// nothing when the count exceeds capacity or bit 0 of *skip is set.
hipError_t launch_keys_to_pairs_dev(const uint64_t *keys, const uint64_t *n_dev, uint64_t n_max, uint64_t capacity,
                                    const uint32_t *skip, uint32_t *pairs, hipStream_t s);

// Join status for a single read: *dst = ctrl->err (one thread).
struct Ctrl;
hipError_t launch_copy_err(const Ctrl *ctrl, uint32_t *dst, hipStream_t s);

}  // namespace rtk
