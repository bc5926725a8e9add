// Host-side cluster tree (geometric bisection) and block partition.
// Pure C++, no device code; compiled with FP contraction disabled so the
// box arithmetic is reproducible bit for bit.
#pragma once

#include <cstdint>
#include <vector>

namespace hm {

struct ClusterTree {
    int64_t n = 0;
    std::vector<int32_t> perm;                 // cluster position -> original index
    std::vector<int32_t> begin, end, left, right, depth;
    std::vector<double> lo, hi;                // 3 per node
    int32_t nodes() const { return (int32_t)begin.size(); }
    bool is_leaf(int32_t t) const { return left[t] < 0; }
    int32_t size(int32_t t) const { return end[t] - begin[t]; }
};

enum BlockKind : int32_t { BLOCK_DENSE = 0, BLOCK_LOWRANK = 1 };

struct Block {
    int32_t row, col, kind;
};

// Geometric bisection of an (n, 3) row-major point array.
ClusterTree build_cluster_tree(const double *pts, int64_t n, int32_t leaf);

// Box admissibility min(diam2 X, diam2 Y) < eta^2 dist2(X, Y) (strict).
bool box_admissible(const ClusterTree &tx, int32_t t, const ClusterTree &ty, int32_t s,
                    double eta);

// Leaves of the block cluster tree in depth-first order.
std::vector<Block> build_block_tree(const ClusterTree &tx, const ClusterTree &ty, double eta);

// Box diameter and distance (not squared) for rank-model features.
double box_diam(const ClusterTree &t, int32_t v);
double box_dist(const ClusterTree &tx, int32_t t, const ClusterTree &ty, int32_t s);

}  // namespace hm
