// Host-side STR packer producing the device node image of a tree.
#pragma once

#include <atomic>
#include <cstdint>
#include <vector>

namespace rtk {

enum : uint32_t { PACK_AOS = 0, PACK_SOA = 1, PACK_D2 = 3 };

struct PackedTree {
    uint32_t fanout = 0, layout = 0, height = 0, n_nodes = 0, first_leaf = 0, node_bytes = 0;
    uint64_t n_objects = 0, n_entries = 0;
    float mbr[4] = {0, 0, 0, 0};
    uint32_t level_start[33] = {0};   // first node index of each level (0 = leaves)
    std::vector<uint8_t> bytes;    // n_nodes * node_bytes, root first
    std::vector<uint32_t> meta;    // per node: entry count | level << 8
};

// rects: n*4 floats, already validated.  Returns 0 or -1 (too many nodes).
int str_pack(const float *rects, uint64_t n, uint32_t fanout, uint32_t layout, PackedTree &out);

}  // namespace rtk
