// Host logic of the H-LU factorisation and solve (Section 3.2): the block
// structure of the factors, the recursive 2 x 2 block LU, the formatted
// update A <- A + A' A'' over the dense (F), low-rank (R) and subdivided (H)
// formats, the block substitutions, and the batching of the eps_LU
// recompressions.  Every arithmetic step is delegated to a backend B:
//
//   Z *keep_alloc(int64_t n)            memory that lives as long as the factors
//   void keep_free(Z *p, int64_t n)     keep memory no kernel will touch again
//                                       (called after a truncate, which ends
//                                       with its stream drained)
//   Z *tmp_alloc(int64_t n)             stack memory, released by tmp_release
//   Mark tmp_mark(); void tmp_release(Mark)
//   void gemm(DMat C, DMat A, DMat B, Z alpha, bool beta)   C = alpha A B (+ C)
//   void copy(DMat dst, DMat src, Z alpha, bool cj, bool acc)
//                                       dst = alpha op(src) (+ dst), op = conj if cj
//   void fill(DMat dst, Z diag)         dst = diag I
//   void getrf_inv(Z *D, Z *Linv, Z *Uinv, int32_t n)
//                                       D = L \ U without pivoting, both inverses
//   void truncate(std::vector<RcItem> &items, double eps)
//                                       QR + truncated SVD of every U V^*:
//                                       fills keep, Uout (keep_alloc, m x keep
//                                       column-major) and Vrow (tmp_alloc,
//                                       n x even(keep) row-major)
//   hm_lu_stats &stats()
//   Fork fork(); void branch(Fork &, int b); void join(Fork &)
//                                       independent branches of the recursion:
//                                       branch b's work may run beside the others',
//                                       join orders everything after them
//
// The device library runs it with HIP kernels; the tests also compile it for
// the CPU with a backend that checks every access against its allocation.
#pragma once

#include <algorithm>
#include <cstdint>
#include <stdexcept>
#include <utility>
#include <vector>

#include "common.hpp"

namespace hm {
namespace lu {

using Z = cplx<double>;

inline void need(bool ok, const char *msg) {
    if (!ok) throw StatusError(HM_ERR_ARG, msg);
}

inline int32_t even(int32_t v) { return v + (v & 1); }

// Dense view: element (i, j) at p[i rs + j cs].
struct DMat {
    Z *p;
    int64_t rs, cs;
    int32_t m, n;
    DMat sub(int32_t r0, int32_t c0, int32_t mm, int32_t nn) const {
        return {p + r0 * rs + c0 * cs, rs, cs, mm, nn};
    }
};
inline DMat cm(Z *p, int32_t m, int32_t n, int64_t ld) { return {p, 1, ld, m, n}; }

// A sum waiting in a low-rank block: U (mp x k, column stride ldu) W (k x np,
// column stride k), at rows ro.., columns co.. of the block.  A factor of a
// finished block (never written again) is referenced rather than copied:
// own_u / own_w say which parts the piece owns.
struct Piece {
    Z *U, *W;
    int32_t k, ro, co, mp, np;
    int64_t ldu;
    bool own_u, own_w;
};

enum : int32_t { FMT_F = 0, FMT_R = 1, FMT_H = 2 };

struct LuNode {
    int32_t t = 0, s = 0, m = 0, n = 0, kind = FMT_F;   // m, n: rows and columns (3 per point)
    Z *D = nullptr, *Linv = nullptr, *Uinv = nullptr;   // F: m x n, ld m; inverses of a diagonal leaf
    Z *U = nullptr, *W = nullptr;                       // R: U (m x k), W = V^* (k x n)
    int32_t k = 0;
    std::vector<Piece> pend;
    int32_t nr = 1, nc = 1;                             // H: children grid
    int32_t rofs[2] = {0, 0}, rsz[2] = {0, 0}, cofs[2] = {0, 0}, csz[2] = {0, 0};
    int32_t ch[2][2] = {{-1, -1}, {-1, -1}};
};

struct RcItem {
    Z *U, *V;          // m x K and n x K, column-major: block U V^*
    int32_t m, n, K;   // m, n: rows (multiples of 3)
    int32_t keep = 0;
    Z *Uout = nullptr, *Vrow = nullptr;
};

// Cluster tree arrays (pre-order nodes, children -1 at leaves).
struct TreeView {
    const int32_t *begin, *end, *left, *right;
    int32_t nodes;
    int32_t size(int32_t t) const { return end[t] - begin[t]; }
    bool leaf(int32_t t) const { return left[t] < 0; }
};

// Block structure of the factors from the block cluster tree: an H block
// (t, s) splits the rows iff t is not a leaf and the columns iff s is not;
// the leaves are the blocks of the partition (leaf_of: sorted keys
// t * nodes + s), recorded in `leaves` as (node id, index into leaf_of).
inline int build_node(std::vector<LuNode> &N, const TreeView &tr, const std::vector<int64_t> &leaf_of,
                      int32_t t, int32_t s, std::vector<std::pair<int, int64_t>> &leaves) {
    const int id = (int)N.size();
    N.emplace_back();
    N[id].t = t;
    N[id].s = s;
    N[id].m = 3 * tr.size(t);
    N[id].n = 3 * tr.size(s);
    const int64_t key = (int64_t)t * tr.nodes + s;
    const auto it = std::lower_bound(leaf_of.begin(), leaf_of.end(), key);
    if (it != leaf_of.end() && *it == key) {
        leaves.push_back({id, (int64_t)(it - leaf_of.begin())});
        return id;
    }
    need(!(tr.leaf(t) && tr.leaf(s)), "leaf pair missing from the block list");
    int32_t rows[2] = {t, -1}, cols[2] = {s, -1};
    int nr = 1, nc = 1;
    if (!tr.leaf(t)) {
        rows[0] = tr.left[t];
        rows[1] = tr.right[t];
        nr = 2;
    }
    if (!tr.leaf(s)) {
        cols[0] = tr.left[s];
        cols[1] = tr.right[s];
        nc = 2;
    }
    int chid[2][2] = {{-1, -1}, {-1, -1}};
    for (int i = 0; i < nr; ++i)
        for (int j = 0; j < nc; ++j) chid[i][j] = build_node(N, tr, leaf_of, rows[i], cols[j], leaves);
    LuNode &X = N[id];
    X.kind = FMT_H;
    X.nr = nr;
    X.nc = nc;
    int32_t off = 0;
    for (int i = 0; i < nr; ++i) {
        X.rofs[i] = off;
        X.rsz[i] = 3 * tr.size(rows[i]);
        off += X.rsz[i];
    }
    off = 0;
    for (int j = 0; j < nc; ++j) {
        X.cofs[j] = off;
        X.csz[j] = 3 * tr.size(cols[j]);
        off += X.csz[j];
    }
    for (int i = 0; i < 2; ++i)
        for (int j = 0; j < 2; ++j) X.ch[i][j] = chid[i][j];
    return id;
}

template <typename B>
struct Core {
    B &be;
    std::vector<LuNode> &N;
    double eps;

    Core(B &b, std::vector<LuNode> &nodes, double e) : be(b), N(nodes), eps(e) {}

    // ---------------------------------------------------------- helpers
    void gemm(DMat C, DMat A, DMat Bm, Z alpha, bool beta) {
        need(A.m == C.m && Bm.n == C.n && A.n == Bm.m, "H-LU: product shapes");
        if (C.m == 0 || C.n == 0) return;
        if (A.n == 0) {
            if (!beta) be.fill(C, Z{0, 0});
            return;
        }
        be.gemm(C, A, Bm, alpha, beta);
        ++be.stats().n_gemm;
        be.stats().gemm_flops += 8.0 * C.m * C.n * A.n;
    }
    void copy(DMat dst, DMat src, Z alpha, bool cj, bool acc) {
        need(dst.m == src.m && dst.n == src.n, "H-LU: copy shapes");
        if (dst.m == 0 || dst.n == 0) return;
        be.copy(dst, src, alpha, cj, acc);
    }
    void fill(DMat dst, Z diag) {
        if (dst.m == 0 || dst.n == 0) return;
        be.fill(dst, diag);
    }
    DMat tmpmat(int32_t m, int32_t n, bool zero) {
        DMat d = cm(be.tmp_alloc((int64_t)m * n), m, n, std::max(m, 1));
        if (zero) fill(d, Z{0, 0});
        return d;
    }
    DMat keepmat(int32_t m, int32_t n) { return cm(be.keep_alloc((int64_t)m * n), m, n, std::max(m, 1)); }
    static DMat dview(const LuNode &X) { return cm(X.D, X.m, X.n, X.m); }
    static DMat uview(const LuNode &X) { return cm(X.U, X.m, X.k, X.m); }
    static DMat wview(const LuNode &X) { return cm(X.W, X.k, X.n, std::max(X.k, 1)); }

    // ---------------------------------------------- block times dense
    // Y += alpha A X
    void matmat(int a, DMat X, DMat Y, Z alpha) {
        const LuNode &A = N[a];
        if (A.kind == FMT_F) {
            gemm(Y, dview(A), X, alpha, true);
        } else if (A.kind == FMT_R) {
            need(A.pend.empty(), "H-LU: product with a pending low-rank block");
            if (A.k == 0) return;
            const auto mk = be.tmp_mark();
            DMat T = tmpmat(A.k, X.n, false);
            gemm(T, wview(A), X, Z{1, 0}, false);
            gemm(Y, uview(A), T, alpha, true);
            be.tmp_release(mk);
        } else {
            for (int i = 0; i < A.nr; ++i)
                for (int j = 0; j < A.nc; ++j)
                    matmat(A.ch[i][j], X.sub(A.cofs[j], 0, A.csz[j], X.n),
                           Y.sub(A.rofs[i], 0, A.rsz[i], Y.n), alpha);
        }
    }
    // Y += alpha X A
    void matmat_right(DMat X, int a, DMat Y, Z alpha) {
        const LuNode &A = N[a];
        if (A.kind == FMT_F) {
            gemm(Y, X, dview(A), alpha, true);
        } else if (A.kind == FMT_R) {
            need(A.pend.empty(), "H-LU: product with a pending low-rank block");
            if (A.k == 0) return;
            const auto mk = be.tmp_mark();
            DMat T = tmpmat(X.m, A.k, false);
            gemm(T, X, uview(A), Z{1, 0}, false);
            gemm(Y, T, wview(A), alpha, true);
            be.tmp_release(mk);
        } else {
            for (int i = 0; i < A.nr; ++i)
                for (int j = 0; j < A.nc; ++j)
                    matmat_right(X.sub(0, A.rofs[i], X.m, A.rsz[i]), A.ch[i][j],
                                 Y.sub(0, A.cofs[j], Y.m, A.csz[j]), alpha);
        }
    }

    // --------------------------------------------------- formatted sums
    // C[ro:, co:] += alpha U W (C an F or R block, or a whole H block).  share:
    // 'U' when U is a finished factor's U (column-major view, kept by
    // reference), 'W' when W is a finished factor's W (column stride W.m, kept
    // by reference), 0 when both are temporaries (copied).
    void add_lowrank(int c, int32_t ro, int32_t co, DMat U, DMat W, Z alpha, char share = 0) {
        LuNode &C = N[c];
        need(ro >= 0 && co >= 0 && ro + U.m <= C.m && co + W.n <= C.n && U.n == W.m,
             "H-LU: low-rank sum outside its block");
        if (U.n == 0) return;
        if (C.kind == FMT_F) {
            gemm(dview(C).sub(ro, co, U.m, W.n), U, W, alpha, true);
        } else if (C.kind == FMT_R) {
            Piece p{nullptr, nullptr, U.n, ro, co, U.m, W.n, U.m, true, true};
            if (share == 'U') {
                need(U.rs == 1, "H-LU: shared U not column-major");
                p.U = U.p;
                p.ldu = U.cs;
                p.own_u = false;
                DMat Wp = keepmat(W.m, W.n);
                copy(Wp, W, alpha, false, false);
                p.W = Wp.p;
            } else if (share == 'W') {
                need(W.rs == 1 && W.cs == W.m, "H-LU: shared W not packed column-major");
                p.W = W.p;
                p.own_w = false;
                DMat Up = keepmat(U.m, U.n);
                copy(Up, U, alpha, false, false);
                p.U = Up.p;
            } else {
                DMat Up = keepmat(U.m, U.n), Wp = keepmat(W.m, W.n);
                copy(Up, U, alpha, false, false);
                copy(Wp, W, Z{1, 0}, false, false);
                p.U = Up.p;
                p.W = Wp.p;
            }
            C.pend.push_back(p);
        } else {
            need(ro == 0 && co == 0 && U.m == C.m && W.n == C.n, "H-LU: partial sum into H");
            for (int i = 0; i < C.nr; ++i)
                for (int j = 0; j < C.nc; ++j)
                    add_lowrank(C.ch[i][j], 0, 0, U.sub(C.rofs[i], 0, C.rsz[i], U.n),
                                W.sub(0, C.cofs[j], W.m, C.csz[j]), alpha, share);
        }
    }
    // C[ro:, co:] += alpha D
    void add_dense(int c, int32_t ro, int32_t co, DMat D, Z alpha) {
        LuNode &C = N[c];
        need(ro >= 0 && co >= 0 && ro + D.m <= C.m && co + D.n <= C.n,
             "H-LU: dense sum outside its block");
        if (C.kind == FMT_F) {
            copy(dview(C).sub(ro, co, D.m, D.n), D, alpha, false, true);
        } else if (C.kind == FMT_R) {
            DMat Up = keepmat(D.m, D.n), Wp = keepmat(D.n, D.n);
            copy(Up, D, alpha, false, false);
            fill(Wp, Z{1, 0});
            C.pend.push_back({Up.p, Wp.p, D.n, ro, co, D.m, D.n, D.m, true, true});
        } else {
            need(ro == 0 && co == 0 && D.m == C.m && D.n == C.n, "H-LU: partial sum into H");
            for (int i = 0; i < C.nr; ++i)
                for (int j = 0; j < C.nc; ++j)
                    add_dense(C.ch[i][j], 0, 0, D.sub(C.rofs[i], C.cofs[j], C.rsz[i], C.csz[j]), alpha);
        }
    }
    // C[ro:, co:] += alpha A B: step 4's formatted update
    void muladd(int c, int32_t ro, int32_t co, int a, int b, Z alpha) {
        const LuNode &A = N[a], &Bn = N[b];
        need(A.n == Bn.m, "H-LU: update shapes");
        if (A.kind == FMT_R) {
            if (A.k == 0) return;
            const auto mk = be.tmp_mark();
            DMat Wn = tmpmat(A.k, Bn.n, true);
            matmat_right(wview(A), b, Wn, Z{1, 0});
            add_lowrank(c, ro, co, uview(A), Wn, alpha, 'U');   // A is a finished factor
            be.tmp_release(mk);
        } else if (Bn.kind == FMT_R) {
            if (Bn.k == 0) return;
            const auto mk = be.tmp_mark();
            DMat Un = tmpmat(A.m, Bn.k, true);
            matmat(a, uview(Bn), Un, Z{1, 0});
            add_lowrank(c, ro, co, Un, wview(Bn), alpha, 'W');   // so is B
            be.tmp_release(mk);
        } else if (A.kind == FMT_F && Bn.kind == FMT_F) {
            if (N[c].kind == FMT_F) {
                need(ro + A.m <= N[c].m && co + Bn.n <= N[c].n, "H-LU: dense update outside its block");
                gemm(dview(N[c]).sub(ro, co, A.m, Bn.n), dview(A), dview(Bn), alpha, true);
            } else {
                const auto mk = be.tmp_mark();
                DMat T = tmpmat(A.m, Bn.n, false);
                gemm(T, dview(A), dview(Bn), Z{1, 0}, false);
                add_dense(c, ro, co, T, alpha);
                be.tmp_release(mk);
            }
        } else {
            const bool ah = A.kind == FMT_H, bh = Bn.kind == FMT_H;
            const int nri = ah ? A.nr : 1, ncj = bh ? Bn.nc : 1, nk = ah ? A.nc : Bn.nr;
            need(!ah || !bh || A.nc == Bn.nr, "H-LU: inner block structure");
            if (N[c].kind == FMT_H) {
                need(N[c].nr == nri && N[c].nc == ncj && ro == 0 && co == 0, "H-LU: update structure");
                // distinct target blocks are independent; the k terms of one
                // target stay in order
                auto f = be.fork();
                for (int i = 0; i < nri; ++i)
                    for (int j = 0; j < ncj; ++j) {
                        be.branch(f, i * ncj + j);
                        for (int k = 0; k < nk; ++k)
                            muladd(N[c].ch[i][j], 0, 0, ah ? A.ch[i][k] : a, bh ? Bn.ch[k][j] : b, alpha);
                    }
                be.join(f);
            } else {
                for (int i = 0; i < nri; ++i)
                    for (int j = 0; j < ncj; ++j)
                        for (int k = 0; k < nk; ++k)
                            muladd(c, ro + (ah ? A.rofs[i] : 0), co + (bh ? Bn.cofs[j] : 0),
                                   ah ? A.ch[i][k] : a, bh ? Bn.ch[k][j] : b, alpha);
            }
        }
    }

    // ------------------------------------------------- substitutions
    // X <- L^-1 X (unit lower factor held by the diagonal block l)
    void lower_solve(int l, DMat X) {
        const LuNode &L = N[l];
        need(X.m == L.m, "H-LU: forward substitution shapes");
        if (L.kind == FMT_F) {
            const auto mk = be.tmp_mark();
            DMat T = tmpmat(X.m, X.n, false);
            gemm(T, cm(L.Linv, L.m, L.m, L.m), X, Z{1, 0}, false);
            copy(X, T, Z{1, 0}, false, false);
            be.tmp_release(mk);
            return;
        }
        DMat X1 = X.sub(L.rofs[0], 0, L.rsz[0], X.n), X2 = X.sub(L.rofs[1], 0, L.rsz[1], X.n);
        lower_solve(L.ch[0][0], X1);
        matmat(L.ch[1][0], X1, X2, Z{-1, 0});
        lower_solve(L.ch[1][1], X2);
    }
    // X <- X U^-1
    void upper_solve_right(int u, DMat X) {
        const LuNode &U = N[u];
        need(X.n == U.n, "H-LU: backward substitution shapes");
        if (U.kind == FMT_F) {
            const auto mk = be.tmp_mark();
            DMat T = tmpmat(X.m, X.n, false);
            gemm(T, X, cm(U.Uinv, U.n, U.n, U.n), Z{1, 0}, false);
            copy(X, T, Z{1, 0}, false, false);
            be.tmp_release(mk);
            return;
        }
        DMat X1 = X.sub(0, U.cofs[0], X.m, U.csz[0]), X2 = X.sub(0, U.cofs[1], X.m, U.csz[1]);
        upper_solve_right(U.ch[0][0], X1);
        matmat_right(X1, U.ch[0][1], X2, Z{-1, 0});
        upper_solve_right(U.ch[1][1], X2);
    }
    // X <- U^-1 X
    void upper_solve_left(int u, DMat X) {
        const LuNode &U = N[u];
        need(X.m == U.m, "H-LU: backward substitution shapes");
        if (U.kind == FMT_F) {
            const auto mk = be.tmp_mark();
            DMat T = tmpmat(X.m, X.n, false);
            gemm(T, cm(U.Uinv, U.m, U.m, U.m), X, Z{1, 0}, false);
            copy(X, T, Z{1, 0}, false, false);
            be.tmp_release(mk);
            return;
        }
        DMat X1 = X.sub(U.rofs[0], 0, U.rsz[0], X.n), X2 = X.sub(U.rofs[1], 0, U.rsz[1], X.n);
        upper_solve_left(U.ch[1][1], X2);
        matmat(U.ch[0][1], X2, X1, Z{-1, 0});
        upper_solve_left(U.ch[0][0], X1);
    }

    // Steps 2 and 3 for lists of blocks against the factors held by the
    // diagonal block d: every block of `lo` (a block row to the right of d)
    // becomes L^-1 B, every block of `up` (a block column below d) B U^-1.
    // All blocks of both lists go down d's tree together, so that each level
    // recompresses the pending sums of all of them in one batch (the blocks
    // are independent: a sum into one of them reads only blocks of its own
    // block row or column, and factors).
    void trsm_multi(int d, const std::vector<int> &lo, const std::vector<int> &up) {
        {
            std::vector<int> q;
            for (int b : lo) collect(b, q);
            for (int b : up) collect(b, q);
            if (!q.empty()) recompress(q);
        }
        std::vector<int> hlo, hup;
        auto f = be.fork();
        int br = 0;
        for (int b : lo) {
            LuNode &Bn = N[b];
            if (Bn.kind == FMT_H) {
                hlo.push_back(b);
            } else if (Bn.kind == FMT_F || Bn.k) {
                be.branch(f, br++);
                lower_solve(d, Bn.kind == FMT_F ? dview(Bn) : uview(Bn));
            }
        }
        for (int b : up) {
            LuNode &Bn = N[b];
            if (Bn.kind == FMT_H) {
                hup.push_back(b);
            } else if (Bn.kind == FMT_F || Bn.k) {
                be.branch(f, br++);
                upper_solve_right(d, Bn.kind == FMT_F ? dview(Bn) : wview(Bn));
            }
        }
        be.join(f);
        if (hlo.empty() && hup.empty()) return;
        if (N[d].kind == FMT_F) {
            // a dense diagonal leaf: the subdivided blocks' children in turn
            std::vector<int> klo, kup;
            for (int b : hlo) {
                need(N[b].nr == 1, "H-LU: block row split against a dense diagonal leaf");
                for (int j = 0; j < N[b].nc; ++j) klo.push_back(N[b].ch[0][j]);
            }
            for (int b : hup) {
                need(N[b].nc == 1, "H-LU: block column split against a dense diagonal leaf");
                for (int i = 0; i < N[b].nr; ++i) kup.push_back(N[b].ch[i][0]);
            }
            trsm_multi(d, klo, kup);
            return;
        }
        // d = [D00 D01; D10 D11] holds L00, L10, L11 and U00, U01, U11:
        // B0j <- L00^-1 B0j, B1j -= L10 B0j, B1j <- L11^-1 B1j for the rows,
        // Bi0 <- Bi0 U00^-1, Bi1 -= Bi0 U01, Bi1 <- Bi1 U11^-1 for the columns
        const LuNode &D = N[d];
        std::vector<int> lo0, lo1, up0, up1;
        for (int b : hlo) {
            need(N[b].nr == 2, "H-LU: block row not split like its diagonal block");
            for (int j = 0; j < N[b].nc; ++j) {
                lo0.push_back(N[b].ch[0][j]);
                lo1.push_back(N[b].ch[1][j]);
            }
        }
        for (int b : hup) {
            need(N[b].nc == 2, "H-LU: block column not split like its diagonal block");
            for (int i = 0; i < N[b].nr; ++i) {
                up0.push_back(N[b].ch[i][0]);
                up1.push_back(N[b].ch[i][1]);
            }
        }
        trsm_multi(D.ch[0][0], lo0, up0);
        auto g = be.fork();
        br = 0;
        for (size_t k = 0; k < lo0.size(); ++k) {
            be.branch(g, br++);
            muladd(lo1[k], 0, 0, D.ch[1][0], lo0[k], Z{-1, 0});
        }
        for (size_t k = 0; k < up0.size(); ++k) {
            be.branch(g, br++);
            muladd(up1[k], 0, 0, up0[k], D.ch[0][1], Z{-1, 0});
        }
        be.join(g);
        trsm_multi(D.ch[1][1], lo1, up1);
    }
    void hlu(int x) {
        LuNode &X = N[x];
        if (X.kind == FMT_F) {
            need(X.m == X.n, "H-LU: non-square diagonal leaf");
            X.Linv = be.keep_alloc((int64_t)X.m * X.m);
            X.Uinv = be.keep_alloc((int64_t)X.m * X.m);
            be.getrf_inv(X.D, X.Linv, X.Uinv, X.m);
            ++be.stats().n_diag;
            return;
        }
        need(X.kind == FMT_H && X.nr == 2 && X.nc == 2, "H-LU: diagonal block not 2 x 2");
        const int a11 = X.ch[0][0], a12 = X.ch[0][1], a21 = X.ch[1][0], a22 = X.ch[1][1];
        hlu(a11);                                   // 1
        trsm_multi(a11, {a12}, {a21});              // 2 and 3, level by level together
        muladd(a22, 0, 0, a21, a12, Z{-1, 0});      // 4
        hlu(a22);
    }

    // --------------------------------------------------- recompression
    void collect(int x, std::vector<int> &out) const {
        const LuNode &X = N[x];
        if (X.kind == FMT_R && !X.pend.empty()) out.push_back(x);
        if (X.kind == FMT_H)
            for (int i = 0; i < X.nr; ++i)
                for (int j = 0; j < X.nc; ++j) collect(X.ch[i][j], out);
    }
    void finalize(int x) {
        std::vector<int> q;
        collect(x, q);
        if (!q.empty()) recompress(q);
    }
    // [U, pieces] [W; pieces] -> U' W' at eps_LU.  A block whose stacked
    // factors hold more columns than its rank can be is first summed densely.
    // Stack memory one recompression batch may take (stacked factors, or the
    // dense sum, and the core workspace); larger lists run as several batches.
    int64_t batch_bytes = int64_t(8) << 30;
    void recompress(const std::vector<int> &q) {
        size_t i0 = 0;
        int64_t acc = 0;
        for (size_t i = 0; i < q.size(); ++i) {
            const LuNode &X = N[q[i]];
            int64_t K = X.k;
            for (const Piece &p : X.pend) K += p.k;
            const int64_t Ke = std::min<int64_t>(K, std::min(X.m, X.n));
            const int64_t b = (int64_t)sizeof(Z) * (K > Ke ? (int64_t)X.m * X.n + (X.m + X.n) * Ke
                                                           : (X.m + X.n) * K) +
                              (int64_t)sizeof(double) * (8 * Ke * Ke + 2 * Ke);
            if (i > i0 && acc + b > batch_bytes) {
                recompress_batch(std::vector<int>(q.begin() + i0, q.begin() + i));
                i0 = i;
                acc = 0;
            }
            acc += b;
        }
        recompress_batch(std::vector<int>(q.begin() + i0, q.end()));
    }
    void recompress_batch(const std::vector<int> &q) {
        const auto mk = be.tmp_mark();
        std::vector<RcItem> items;
        for (int x : q) {
            LuNode &X = N[x];
            int32_t K = X.k;
            for (const Piece &p : X.pend) K += p.k;
            const int32_t mn = std::min(X.m, X.n);
            DMat Uc, Vc;   // Uc: m x K, Vc = W^*: n x K
            if (K > mn) {
                DMat D = tmpmat(X.m, X.n, true);
                if (X.k) gemm(D, uview(X), wview(X), Z{1, 0}, true);
                for (const Piece &p : X.pend)
                    gemm(D.sub(p.ro, p.co, p.mp, p.np), cm(p.U, p.mp, p.k, p.ldu),
                         cm(p.W, p.k, p.np, p.k), Z{1, 0}, true);
                if (X.n <= X.m) {
                    Uc = D;
                    Vc = tmpmat(X.n, X.n, false);
                    fill(Vc, Z{1, 0});
                } else {
                    Uc = tmpmat(X.m, X.m, false);
                    fill(Uc, Z{1, 0});
                    Vc = tmpmat(X.n, X.m, false);
                    copy(Vc, DMat{D.p, D.cs, D.rs, X.n, X.m}, Z{1, 0}, true, false);
                }
                K = mn;
            } else {
                Uc = tmpmat(X.m, K, true);
                Vc = tmpmat(X.n, K, true);
                int32_t k0 = 0;
                if (X.k) {
                    copy(Uc.sub(0, 0, X.m, X.k), uview(X), Z{1, 0}, false, false);
                    copy(Vc.sub(0, 0, X.n, X.k), DMat{X.W, X.k, 1, X.n, X.k}, Z{1, 0}, true, false);
                    k0 = X.k;
                }
                for (const Piece &p : X.pend) {
                    copy(Uc.sub(p.ro, k0, p.mp, p.k), cm(p.U, p.mp, p.k, p.ldu), Z{1, 0}, false, false);
                    copy(Vc.sub(p.co, k0, p.np, p.k), DMat{p.W, p.k, 1, p.np, p.k}, Z{1, 0}, true,
                         false);
                    k0 += p.k;
                }
            }
            RcItem it;
            it.U = Uc.p;
            it.V = Vc.p;
            it.m = X.m;
            it.n = X.n;
            it.K = K;
            items.push_back(it);
        }
        be.truncate(items, eps);
        // the superseded factors and the pieces were last read by the copies and
        // products queued before the truncate: their memory goes back to the backend
        for (int x : q) {
            LuNode &X = N[x];
            if (X.k) {
                be.keep_free(X.U, (int64_t)X.m * X.k);
                be.keep_free(X.W, (int64_t)X.k * X.n);
            }
            for (const Piece &p : X.pend) {
                if (p.own_u) be.keep_free(p.U, (int64_t)p.mp * p.k);
                if (p.own_w) be.keep_free(p.W, (int64_t)p.k * p.np);
            }
        }
        for (size_t i = 0; i < q.size(); ++i) {
            LuNode &X = N[q[i]];
            const RcItem &it = items[i];
            need(it.keep >= 0 && it.keep <= it.K, "H-LU: recompressed rank out of range");
            X.k = it.keep;
            X.pend.clear();
            X.U = it.keep ? it.Uout : nullptr;
            X.W = nullptr;
            if (!it.keep) continue;
            // V' is row-major (n x keep, even row stride): W = V'^*
            X.W = be.keep_alloc((int64_t)X.k * X.n);
            copy(cm(X.W, X.k, X.n, X.k), DMat{it.Vrow, 1, even(X.k), X.k, X.n}, Z{1, 0}, true, false);
        }
        be.stats().n_recompressed += (int32_t)q.size();
        ++be.stats().n_batches;
        be.tmp_release(mk);
    }

    // -------------------------------------------------------- exports
    void tally(int x) {
        const LuNode &X = N[x];
        if (X.kind == FMT_F) {
            be.stats().storage_entries += (int64_t)X.m * X.n;
        } else if (X.kind == FMT_R) {
            be.stats().storage_entries += (int64_t)(X.m + X.n) * X.k;
            be.stats().max_rank = std::max(be.stats().max_rank, X.k);
        } else {
            for (int i = 0; i < X.nr; ++i)
                for (int j = 0; j < X.nc; ++j) tally(X.ch[i][j]);
        }
    }
    // the factors (or any block) as one dense matrix
    void densify(int x, DMat out) {
        const LuNode &X = N[x];
        if (X.kind == FMT_F) {
            copy(out, dview(X), Z{1, 0}, false, false);
        } else if (X.kind == FMT_R) {
            gemm(out, uview(X), wview(X), Z{1, 0}, false);
        } else {
            for (int i = 0; i < X.nr; ++i)
                for (int j = 0; j < X.nc; ++j)
                    densify(X.ch[i][j], out.sub(X.rofs[i], X.cofs[j], X.rsz[i], X.csz[j]));
        }
    }
};

}  // namespace lu
}  // namespace hm
