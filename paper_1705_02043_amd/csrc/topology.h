// Host topology of the periodic KIFMM library: the octree and the U/V/W/X lists (tree_host.cpp).
// Plain C++ with no HIP dependency, so that the host code builds with any host compiler (the
// sanitizer tests build it with g++).
#pragma once

#include <cstdint>
#include <vector>

namespace pk {

constexpr int kMaxLevel = 21;
constexpr int kNumM2L = 316;   // offsets in [-3,3]^3 with |delta|_inf >= 2

// ---------------------------------------------------------------- tree (host topology)

struct HostTree {
    std::vector<int> level, ix, iy, iz, begin, end, parent;
    std::vector<int> child;       // [nbox][8], -1 absent
    std::vector<int> leaf_id;     // box -> leaf index or -1
    std::vector<int> leaves;      // leaf index -> box
    std::vector<int> level_start; // boxes of level l are [level_start[l], level_start[l+1])
    int depth = 0;
    int nbox() const { return (int)level.size(); }
    bool is_leaf(int b) const {
        for (int o = 0; o < 8; ++o)
            if (child[8 * b + o] >= 0) return false;
        return true;
    }
};

struct Entry {
    int src;      // source box
    int8_t sx, sy, sz;   // image shift, each in {-1, 0, 1}
    bool operator<(const Entry& o) const {
        if (src != o.src) return src < o.src;
        if (sx != o.sx) return sx < o.sx;
        if (sy != o.sy) return sy < o.sy;
        return sz < o.sz;
    }
    bool operator==(const Entry& o) const { return src == o.src && sx == o.sx && sy == o.sy && sz == o.sz; }
};

struct HostLists {
    // CSR over boxes
    std::vector<int64_t> u_off, v_off, w_off, x_off;
    std::vector<Entry> u, v, w, x;
};

void build_tree_host(const uint64_t* sorted_keys, int64_t n, int s, HostTree& t);
void build_lists_host(const HostTree& t, unsigned periodic_mask, HostLists& l);
void add_root_ring(const HostTree& t, unsigned periodic_mask, int near_layers, HostLists& l);
// The trees and lists of independent problems (problem q owns sorted_keys[poff[q], poff[q+1])),
// several problems at a time on host threads, each as build_tree_host, build_lists_host and
// add_root_ring make it alone.
void build_forest_host(const uint64_t* sorted_keys, const std::vector<int64_t>& poff, int s, unsigned periodic_mask,
                       int near_layers, std::vector<HostTree>& trees, std::vector<HostLists>& lists);
void merge_forest(const std::vector<HostTree>& trees, const std::vector<HostLists>& lists,
                  const std::vector<int64_t>& poff, HostTree& t, HostLists& l, std::vector<int>& box_prob);
int m2l_offset_index(int dx, int dy, int dz);   // -> 0..315
void m2l_offset_vector(int idx, int& dx, int& dy, int& dz);

}  // namespace pk
