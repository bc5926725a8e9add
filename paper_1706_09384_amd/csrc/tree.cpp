// Cluster tree and block partition (Section 2.1; admissibility Section 6.1).
//
// Splitting rule (the paper fixes "bisect the enclosing box along its largest
// dimension until a minimum size"; the remaining choices are this library's):
//   * tight float64 bounding box per node;
//   * at most `leaf` points -> leaf;
//   * axis of largest extent, lowest axis on ties; zero extent -> leaf;
//   * split value (lo + hi) * 0.5; points with coordinate < split go left,
//     the rest right, each side keeping its incoming order;
//   * an empty side -> leaf;
//   * nodes numbered in pre-order, left child first.
// Block recursion: admissible -> low-rank leaf; two leaves -> dense leaf;
// one leaf -> split the other side only; else the four child pairs with the
// row child outermost.  Both are iterative (explicit stacks).
#include "tree.hpp"

#include <algorithm>
#include <cmath>

namespace hm {

namespace {
struct Pending {
    int32_t b, e, depth, parent;
    bool is_left;
};
}  // namespace

ClusterTree build_cluster_tree(const double *P, int64_t n, int32_t leaf) {
    ClusterTree t;
    t.n = n;
    t.perm.resize(n);
    for (int64_t i = 0; i < n; ++i) t.perm[i] = (int32_t)i;
    std::vector<int32_t> tmp(n);
    std::vector<Pending> stack;
    stack.push_back({0, (int32_t)n, 0, -1, false});
    while (!stack.empty()) {
        Pending p = stack.back();
        stack.pop_back();
        const int32_t id = (int32_t)t.begin.size();
        t.begin.push_back(p.b);
        t.end.push_back(p.e);
        t.left.push_back(-1);
        t.right.push_back(-1);
        t.depth.push_back(p.depth);
        if (p.parent >= 0) (p.is_left ? t.left : t.right)[p.parent] = id;
        double lo[3], hi[3];
        for (int a = 0; a < 3; ++a) {
            lo[a] = INFINITY;
            hi[a] = -INFINITY;
        }
        for (int32_t k = p.b; k < p.e; ++k) {
            const double *q = P + 3 * (int64_t)t.perm[k];
            for (int a = 0; a < 3; ++a) {
                lo[a] = std::min(lo[a], q[a]);
                hi[a] = std::max(hi[a], q[a]);
            }
        }
        for (int a = 0; a < 3; ++a) {
            t.lo.push_back(lo[a]);
            t.hi.push_back(hi[a]);
        }
        if (p.e - p.b <= leaf) continue;
        int ax = 0;
        double ext = hi[0] - lo[0];
        for (int a = 1; a < 3; ++a) {
            const double e = hi[a] - lo[a];
            if (e > ext) {
                ext = e;
                ax = a;
            }
        }
        if (ext == 0.0) continue;
        const double mid = (lo[ax] + hi[ax]) * 0.5;
        int32_t nl = 0, nr = 0;
        const int32_t cnt = p.e - p.b;
        for (int32_t k = p.b; k < p.e; ++k)
            if (P[3 * (int64_t)t.perm[k] + ax] < mid) ++nl;
        if (nl == 0 || nl == cnt) continue;
        int32_t wl = 0;
        nr = nl;
        for (int32_t k = p.b; k < p.e; ++k) {
            const int32_t v = t.perm[k];
            if (P[3 * (int64_t)v + ax] < mid)
                tmp[wl++] = v;
            else
                tmp[nr++] = v;
        }
        std::copy(tmp.begin(), tmp.begin() + cnt, t.perm.begin() + p.b);
        // Right pushed first so that the left subtree is numbered next.
        stack.push_back({p.b + nl, p.e, p.depth + 1, id, false});
        stack.push_back({p.b, p.b + nl, p.depth + 1, id, true});
    }
    return t;
}

static inline double sq(double v) { return v * v; }

bool box_admissible(const ClusterTree &tx, int32_t t, const ClusterTree &ty, int32_t s,
                    double eta) {
    const double *lx = &tx.lo[3 * t], *hx = &tx.hi[3 * t];
    const double *ly = &ty.lo[3 * s], *hy = &ty.hi[3 * s];
    const double dx0 = hx[0] - lx[0], dx1 = hx[1] - lx[1], dx2 = hx[2] - lx[2];
    const double dy0 = hy[0] - ly[0], dy1 = hy[1] - ly[1], dy2 = hy[2] - ly[2];
    const double diam2x = dx0 * dx0 + dx1 * dx1 + dx2 * dx2;
    const double diam2y = dy0 * dy0 + dy1 * dy1 + dy2 * dy2;
    double g[3];
    for (int a = 0; a < 3; ++a) {
        const double u = std::max(0.0, ly[a] - hx[a]);
        const double v = std::max(0.0, lx[a] - hy[a]);
        g[a] = u * u + v * v;
    }
    const double dist2 = g[0] + g[1] + g[2];
    return std::min(diam2x, diam2y) < (eta * eta) * dist2;
}

std::vector<Block> build_block_tree(const ClusterTree &tx, const ClusterTree &ty, double eta) {
    std::vector<Block> out;
    std::vector<std::pair<int32_t, int32_t>> stack;
    stack.push_back({0, 0});
    while (!stack.empty()) {
        auto [t, s] = stack.back();
        stack.pop_back();
        if (box_admissible(tx, t, ty, s, eta)) {
            out.push_back({t, s, BLOCK_LOWRANK});
            continue;
        }
        const bool tl = tx.is_leaf(t), sl = ty.is_leaf(s);
        if (tl && sl) {
            out.push_back({t, s, BLOCK_DENSE});
            continue;
        }
        // Push in reverse visiting order.
        if (tl) {
            stack.push_back({t, ty.right[s]});
            stack.push_back({t, ty.left[s]});
        } else if (sl) {
            stack.push_back({tx.right[t], s});
            stack.push_back({tx.left[t], s});
        } else {
            stack.push_back({tx.right[t], ty.right[s]});
            stack.push_back({tx.right[t], ty.left[s]});
            stack.push_back({tx.left[t], ty.right[s]});
            stack.push_back({tx.left[t], ty.left[s]});
        }
    }
    return out;
}

double box_diam(const ClusterTree &t, int32_t v) {
    double s = 0;
    for (int a = 0; a < 3; ++a) s += sq(t.hi[3 * v + a] - t.lo[3 * v + a]);
    return std::sqrt(s);
}

double box_dist(const ClusterTree &tx, int32_t t, const ClusterTree &ty, int32_t s) {
    double d = 0;
    for (int a = 0; a < 3; ++a) {
        d += sq(std::max(0.0, ty.lo[3 * s + a] - tx.hi[3 * t + a]));
        d += sq(std::max(0.0, tx.lo[3 * t + a] - ty.hi[3 * s + a]));
    }
    return std::sqrt(d);
}

}  // namespace hm
