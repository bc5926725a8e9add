// CPU build of the H-LU host logic (paper_1706_09384_amd/csrc/lu_core.hpp)
// for the tests: the same recursion, formats and batching as the device
// library, with a backend that does the arithmetic in plain loops and checks
// every matrix view against the allocation it points into (a view that
// leaves its allocation, or touches released stack memory, is an error).
// Truncation keeps every column (exact; eps_LU must be 0), so the packed
// factors can be checked against A_H.
//
// Usage: lu_cpu <input> <output>.  Input (little endian):
//   int32 nodes, nblk; int64 dofs; double eps
//   int32 begin[nodes], end[nodes], left[nodes], right[nodes]
//   int32 blocks[3 nblk] (row node, col node, kind), int32 rank[nblk]
//   complex128 data: per block, dense 3m x 3n column-major, or U (3m x r)
//     then W = V^* (r x 3n), column-major
//   complex128 b[dofs] (cluster order)
// Output: int32 status (0 ok), int32 message length, message bytes, then on
//   success: complex128 packed L \ U (dofs x dofs, column-major), complex128
//   x[dofs], int64 stats[4] (n_recompressed, n_batches, n_gemm, n_diag).
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <fstream>
#include <iostream>
#include <memory>
#include <string>

#include "lu_core.hpp"

using namespace hm;
using namespace hm::lu;

namespace {

struct Alloc {
    const Z *lo;
    int64_t n;
    bool live;
};

struct CpuBackend {
    std::vector<std::unique_ptr<Z[]>> mem;   // never freed before exit: stale views stay detectable
    std::vector<Alloc> reg;
    std::vector<size_t> tmp_stack;           // indices into reg of live stack allocations
    hm_lu_stats st{};
    using Mark = size_t;

    Z *make(int64_t n) {
        const int64_t nn = std::max<int64_t>(n, 1);
        mem.emplace_back(new Z[nn]);
        Z *p = mem.back().get();
        for (int64_t i = 0; i < nn; ++i) p[i] = Z{std::nan(""), std::nan("")};   // poison
        reg.push_back({p, n, true});
        return p;
    }
    Z *keep_alloc(int64_t n) { return make(n); }
    // freed keep memory is poisoned and marked dead, never reused: a later view
    // into it is reported
    void keep_free(Z *p, int64_t n) {
        for (Alloc &a : reg)
            if (a.lo == p) {
                if (!a.live) throw std::runtime_error("keep memory freed twice");
                if (a.n != n) throw std::runtime_error("keep memory freed with another size");
                a.live = false;
                for (int64_t i = 0; i < n; ++i) p[i] = Z{std::nan(""), std::nan("")};
                return;
            }
        throw std::runtime_error("keep_free of memory that was never allocated");
    }
    Z *tmp_alloc(int64_t n) {
        Z *p = make(n);
        tmp_stack.push_back(reg.size() - 1);
        return p;
    }
    Mark tmp_mark() { return tmp_stack.size(); }
    void tmp_release(Mark m) {
        if (m > tmp_stack.size()) throw std::runtime_error("stack release above the top");
        while (tmp_stack.size() > m) {
            reg[tmp_stack.back()].live = false;
            tmp_stack.pop_back();
        }
    }
    hm_lu_stats &stats() { return st; }
    // one host thread runs every branch in order: nothing to order
    struct Fork {};
    Fork fork() { return {}; }
    void branch(Fork &, int) {}
    void join(Fork &) {}

    void check(const DMat &v, const char *what) const {
        if (v.m == 0 || v.n == 0) return;
        if (v.m < 0 || v.n < 0 || v.rs < 0 || v.cs < 0) throw std::runtime_error(std::string(what) + ": negative shape or stride");
        if (!v.p) throw std::runtime_error(std::string(what) + ": null view");
        const Z *lo = v.p, *hi = v.p + (v.m - 1) * v.rs + (v.n - 1) * v.cs;
        for (const Alloc &a : reg)
            if (lo >= a.lo && hi < a.lo + a.n) {
                if (!a.live) throw std::runtime_error(std::string(what) + ": view into released memory");
                return;
            }
        throw std::runtime_error(std::string(what) + ": view outside every allocation");
    }
    static Z &at(const DMat &v, int64_t i, int64_t j) { return v.p[i * v.rs + j * v.cs]; }

    void gemm(DMat C, DMat A, DMat B, Z alpha, bool beta) {
        check(C, "gemm C");
        check(A, "gemm A");
        check(B, "gemm B");
        std::vector<Z> out((size_t)C.m * C.n);
        for (int64_t j = 0; j < C.n; ++j)
            for (int64_t i = 0; i < C.m; ++i) {
                Z s{0, 0};
                for (int64_t k = 0; k < A.n; ++k) s = s + at(A, i, k) * at(B, k, j);
                out[i + j * C.m] = alpha * s;
            }
        for (int64_t j = 0; j < C.n; ++j)
            for (int64_t i = 0; i < C.m; ++i) {
                Z &c = at(C, i, j);
                c = beta ? c + out[i + j * C.m] : out[i + j * C.m];
            }
    }
    void copy(DMat dst, DMat src, Z alpha, bool cj, bool acc) {
        check(dst, "copy dst");
        check(src, "copy src");
        for (int64_t j = 0; j < dst.n; ++j)
            for (int64_t i = 0; i < dst.m; ++i) {
                Z v = at(src, i, j);
                if (cj) v = conj(v);
                v = alpha * v;
                Z &d = at(dst, i, j);
                d = acc ? d + v : v;
            }
    }
    void fill(DMat dst, Z diag) {
        check(dst, "fill");
        for (int64_t j = 0; j < dst.n; ++j)
            for (int64_t i = 0; i < dst.m; ++i) at(dst, i, j) = i == j ? diag : Z{0, 0};
    }
    void getrf_inv(Z *D, Z *Linv, Z *Uinv, int32_t n) {
        check(cm(D, n, n, n), "getrf D");
        check(cm(Linv, n, n, n), "getrf Linv");
        check(cm(Uinv, n, n, n), "getrf Uinv");
        auto A = [&](int i, int j) -> Z & { return D[i + (int64_t)j * n]; };
        for (int k = 0; k < n; ++k) {
            const Z piv = A(k, k);
            const double d = piv.re * piv.re + piv.im * piv.im;
            if (d == 0.0) throw std::runtime_error("zero pivot");
            const Z inv{piv.re / d, -piv.im / d};
            for (int i = k + 1; i < n; ++i) A(i, k) = A(i, k) * inv;
            for (int j = k + 1; j < n; ++j)
                for (int i = k + 1; i < n; ++i) A(i, j) = A(i, j) - A(i, k) * A(k, j);
        }
        for (int j = 0; j < n; ++j) {
            Z *x = Linv + (int64_t)j * n;
            for (int i = 0; i < n; ++i) x[i] = Z{i == j ? 1.0 : 0.0, 0};
            for (int i = j + 1; i < n; ++i) {
                Z s{0, 0};
                for (int k = j; k < i; ++k) s = s + A(i, k) * x[k];
                x[i] = Z{-s.re, -s.im};
            }
            Z *y = Uinv + (int64_t)j * n;
            for (int i = 0; i < n; ++i) y[i] = Z{0, 0};
            for (int i = j; i >= 0; --i) {
                Z s = i == j ? Z{1, 0} : Z{0, 0};
                for (int k = i + 1; k <= j; ++k) s = s - A(i, k) * y[k];
                const Z p = A(i, i);
                const double dd = p.re * p.re + p.im * p.im;
                y[i] = Z{(s.re * p.re + s.im * p.im) / dd, (s.im * p.re - s.re * p.im) / dd};
            }
        }
    }
    void truncate(std::vector<RcItem> &items, double eps) {
        if (eps != 0.0) throw std::runtime_error("the CPU backend truncates only at eps_LU = 0");
        for (RcItem &it : items) {
            if (it.m % 3 || it.n % 3 || it.K < 1) throw std::runtime_error("truncate: bad item");
            check(cm(it.U, it.m, it.K, it.m), "truncate U");
            check(cm(it.V, it.n, it.K, it.n), "truncate V");
            it.keep = it.K;
            it.Uout = keep_alloc((int64_t)it.m * it.K);
            const int32_t ldv = even(it.K);
            it.Vrow = tmp_alloc((int64_t)it.n * ldv);
            for (int64_t c = 0; c < it.K; ++c) {
                for (int64_t i = 0; i < it.m; ++i) it.Uout[i + c * it.m] = it.U[i + c * it.m];
                for (int64_t j = 0; j < it.n; ++j) it.Vrow[j * ldv + c] = it.V[j + c * it.n];
            }
        }
    }
};

template <typename T>
void rd(std::ifstream &f, T *p, size_t n) {
    f.read(reinterpret_cast<char *>(p), n * sizeof(T));
    if (!f) throw std::runtime_error("short input");
}

}  // namespace

int main(int argc, char **argv) {
    if (argc != 3) {
        std::fprintf(stderr, "usage: lu_cpu <input> <output>\n");
        return 2;
    }
    std::ofstream out(argv[2], std::ios::binary);
    auto fail = [&](const std::string &m) {
        const int32_t s = 1, l = (int32_t)m.size();
        out.write(reinterpret_cast<const char *>(&s), 4);
        out.write(reinterpret_cast<const char *>(&l), 4);
        out.write(m.data(), l);
        return 0;
    };
    try {
        std::ifstream f(argv[1], std::ios::binary);
        int32_t nodes, nblk;
        int64_t dofs;
        double eps;
        rd(f, &nodes, 1);
        rd(f, &nblk, 1);
        rd(f, &dofs, 1);
        rd(f, &eps, 1);
        std::vector<int32_t> begin(nodes), end(nodes), left(nodes), right(nodes), blk(3 * (size_t)nblk), rank(nblk);
        rd(f, begin.data(), nodes);
        rd(f, end.data(), nodes);
        rd(f, left.data(), nodes);
        rd(f, right.data(), nodes);
        rd(f, blk.data(), blk.size());
        rd(f, rank.data(), rank.size());
        const TreeView tv{begin.data(), end.data(), left.data(), right.data(), nodes};
        std::vector<std::pair<int64_t, int32_t>> key;
        for (int32_t b = 0; b < nblk; ++b) key.push_back({(int64_t)blk[3 * b] * nodes + blk[3 * b + 1], b});
        std::sort(key.begin(), key.end());
        std::vector<int64_t> leaf_of;
        std::vector<int32_t> leaf_block;
        for (auto &kv : key) {
            leaf_of.push_back(kv.first);
            leaf_block.push_back(kv.second);
        }
        std::vector<LuNode> N;
        std::vector<std::pair<int, int64_t>> leaves;
        build_node(N, tv, leaf_of, 0, 0, leaves);
        if ((int32_t)leaves.size() != nblk) return fail("block list and tree disagree");
        CpuBackend be;
        // block data in block order
        std::vector<int> node_of_block(nblk, -1);
        for (auto &pr : leaves) node_of_block[leaf_block[pr.second]] = pr.first;
        for (int32_t b = 0; b < nblk; ++b) {
            LuNode &X = N[node_of_block[b]];
            if (blk[3 * b + 2] == 0) {
                X.kind = FMT_F;
                X.D = be.keep_alloc((int64_t)X.m * X.n);
                rd(f, X.D, (size_t)X.m * X.n);
            } else {
                X.kind = FMT_R;
                X.k = rank[b];
                X.U = X.k ? be.keep_alloc((int64_t)X.m * X.k) : nullptr;
                X.W = X.k ? be.keep_alloc((int64_t)X.k * X.n) : nullptr;
                if (X.k) {
                    rd(f, X.U, (size_t)X.m * X.k);
                    rd(f, X.W, (size_t)X.k * X.n);
                }
            }
        }
        std::vector<Z> b(dofs);
        rd(f, b.data(), dofs);
        Core<CpuBackend> core(be, N, eps);
        // one block per recompression batch: the split of a batch is exercised
        if (std::getenv("LU_CPU_SMALL_BATCHES")) core.batch_bytes = 1;
        core.hlu(0);
        DMat P = cm(be.keep_alloc(dofs * dofs), (int32_t)dofs, (int32_t)dofs, dofs);
        core.densify(0, P);
        DMat x = cm(be.keep_alloc(dofs), (int32_t)dofs, 1, dofs);
        std::memcpy(x.p, b.data(), dofs * sizeof(Z));
        core.lower_solve(0, x);
        core.upper_solve_left(0, x);
        const int32_t s = 0, l = 0;
        out.write(reinterpret_cast<const char *>(&s), 4);
        out.write(reinterpret_cast<const char *>(&l), 4);
        out.write(reinterpret_cast<const char *>(P.p), dofs * dofs * sizeof(Z));
        out.write(reinterpret_cast<const char *>(x.p), dofs * sizeof(Z));
        const int64_t stats[4] = {be.st.n_recompressed, be.st.n_batches, be.st.n_gemm, be.st.n_diag};
        out.write(reinterpret_cast<const char *>(stats), sizeof(stats));
        return 0;
    } catch (const StatusError &e) {
        return fail(e.msg);
    } catch (const std::exception &e) {
        return fail(e.what());
    }
}
