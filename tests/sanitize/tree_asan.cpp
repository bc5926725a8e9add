// Host build of the library's cluster tree and block partition
// (paper_1706_09384_amd/csrc/tree.cpp) under AddressSanitizer and UBSan:
// a Fibonacci sphere, a cloud with duplicated points (zero-extent boxes) and
// a two-point cloud, each checked for a permutation and for blocks that
// cover the matrix exactly once.
#include <cmath>
#include <cstdio>
#include <vector>

#include "tree.hpp"

using namespace hm;

static int check(const std::vector<double> &P, int32_t leaf, double eta, const char *name) {
    const int64_t n = (int64_t)P.size() / 3;
    const ClusterTree t = build_cluster_tree(P.data(), n, leaf);
    std::vector<int> seen(n, 0);
    for (int32_t v : t.perm) {
        if (v < 0 || v >= n || seen[v]++) {
            std::printf("%s: perm is not a permutation\n", name);
            return 1;
        }
    }
    const std::vector<Block> b = build_block_tree(t, t, eta);
    // every (row point, column point) pair lies in exactly one block
    std::vector<int> cover((size_t)(n * n), 0);
    for (const Block &k : b)
        for (int32_t i = t.begin[k.row]; i < t.end[k.row]; ++i)
            for (int32_t j = t.begin[k.col]; j < t.end[k.col]; ++j) ++cover[(size_t)i * n + j];
    for (int c : cover)
        if (c != 1) {
            std::printf("%s: blocks do not partition the matrix\n", name);
            return 1;
        }
    int64_t lr = 0;
    for (const Block &k : b) lr += k.kind == BLOCK_LOWRANK;
    std::printf("%s: n %lld nodes %d blocks %zu low-rank %lld\n", name, (long long)n, t.nodes(), b.size(),
                (long long)lr);
    return 0;
}

int main() {
    int rc = 0;
    {
        const int n = 1500;
        std::vector<double> P(3 * n);
        const double ga = M_PI * (3.0 - std::sqrt(5.0));
        for (int i = 0; i < n; ++i) {
            const double z = 1.0 - 2.0 * (i + 0.5) / n, r = std::sqrt(1.0 - z * z);
            P[3 * i] = r * std::cos(ga * i);
            P[3 * i + 1] = r * std::sin(ga * i);
            P[3 * i + 2] = z;
        }
        rc |= check(P, 16, 3.0, "sphere");
    }
    {
        std::vector<double> P;
        for (int i = 0; i < 300; ++i) {
            const double x = (i % 10) * 0.1;   // ten copies of each of 30 points
            P.push_back(x);
            P.push_back((i / 10 % 3) * 0.5);
            P.push_back((i / 30) * 0.25);
        }
        rc |= check(P, 4, 2.0, "duplicates");
    }
    {
        std::vector<double> P = {0, 0, 0, 1, 0, 0};
        rc |= check(P, 1, 3.0, "two points");
    }
    return rc;
}
