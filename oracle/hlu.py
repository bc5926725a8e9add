"""H-LU factorisation, H-LU solve and the certification estimator (oracle).

TEST INFRASTRUCTURE.  Only the tests, ``__graft_entry__.smoke()`` and the CPU
baseline leg of ``bench.py`` may use this module.  It shares no code with the
library and never imports it.

The method is the one of Section 3.2 of arXiv 1706.09384: the LU factors of
an H-matrix are computed recursively on the 2 x 2 block structure of the
block cluster tree,

    1. A11 = L11 U11                      (recursion)
    2. U12 = L11^-1 A12                   (block forward substitution)
    3. L21 = A21 U11^-1                   (block backward substitution)
    4. A22 - L21 U12 = L22 U22            (update, then recursion),

where every block is dense (F), low-rank (R, stored as U W with W = V^*) or
subdivided (H), so that step 4 is the formatted update A <- A + A' A'' over
the 27 combinations of formats.  Low-rank results are recompressed with the
QR + truncated SVD of the same section at the tolerance eps_LU.  Section 3.3
(eq. est_direct) bounds the residual of the solution x0 of L_H U_H x0 = b:
    |b - A x0| / |b| <= (delta + delta_H |x0|) / |b|,
with delta = |b - A_H x0| and delta_H = |A_H - A| (Frobenius norm).

Readings where the paper is silent (it defers the 27 cases to a reference):

* The LU is unpivoted: the factors are L_H with unit diagonal and U_H, and
  a dense diagonal leaf is factorised by Gaussian elimination without
  pivoting (Section 3.2 writes A = L U block by block, which leaves no room
  for row exchanges across blocks).
* Sums into a low-rank block are kept exactly, as extra columns of the
  factors (a piece may cover only part of the block, with zeros elsewhere),
  and the block is recompressed once, with eps_LU, when every update of the
  elimination has reached it: right before its block substitution (steps 2
  and 3).  Recompression keeps the singular values whose Frobenius tail
  exceeds eps_LU times the total, the rule of the assembly.
* The product of two blocks goes through a low-rank factor whenever one of
  them is low-rank (A' = U W: the product is U (W A''); A'' = U W: it is
  (A' U) W); two dense leaves multiply densely; otherwise the product
  recurses on the children, with a dense or low-rank target split along the
  children's clusters.  A dense product added into a low-rank block becomes
  the piece (D, I).
* Block substitutions recurse over the subdivided blocks; at a dense diagonal
  leaf they use triangular substitution.
* delta_H in eq. est_direct is the absolute Frobenius norm of A_H - A (the
  equation's definition); the tables print it next to |x0|/|b| and
  delta/|b|, and their products reproduce the printed estimator.
"""
from __future__ import annotations

import collections

import numpy as np
import scipy.linalg as sla
from threadpoolctl import threadpool_limits

F, R, H = 0, 1, 2

# (target, left, right) formats met by the formatted update, for the tests
CASES = collections.Counter()


class HBlock:
    """One block (t, s) of the block cluster tree in format F, R or H."""

    def __init__(self, t, s, m, n):
        self.t, self.s, self.m, self.n = int(t), int(s), int(m), int(n)
        self.kind = F
        self.D = None            # F: m x n
        self.U = None            # R: m x k
        self.W = None            # R: k x n (block = U W)
        self.pend = []           # R: pieces (U, W, row offset, col offset) not yet recompressed
        self.rparts = [(0, m)]   # H: (offset, size) of the row children
        self.cparts = [(0, n)]
        self.ch = None           # H: ch[i][j]

    def child(self, i, j):
        return self.ch[i][j] if self.kind == H else self

    def rank(self):
        return self.U.shape[1] if self.kind == R else 0


def _dofs(tr, t):
    return 3 * int(tr.end[t] - tr.begin[t])


def build(tree, leaves):
    """H-matrix in block form from its leaves.

    ``leaves`` is a list of (row node, col node, kind, data) with kind 0 =
    dense (data: 3m x 3n in cluster-local order) or 1 = low-rank (data:
    (U, V) with block U V^*), e.g. the oracle's own assembly.  The
    subdivision follows the block tree's rule: an H block (t, s) splits the
    rows iff t is not a leaf and the columns iff s is not a leaf.
    """
    by = {(int(a), int(b)): (int(k), d) for a, b, k, d in leaves}

    def rec(t, s):
        X = HBlock(t, s, _dofs(tree, t), _dofs(tree, s))
        if (t, s) in by:
            kind, d = by[(t, s)]
            if kind == 0:
                X.kind, X.D = F, np.array(d, dtype=np.complex128)
            else:
                U, V = d
                X.kind = R
                X.U = np.array(U, dtype=np.complex128)
                X.W = np.array(V, dtype=np.complex128).conj().T.copy()
            return X
        X.kind = H
        rows = [t] if tree.left[t] < 0 else [int(tree.left[t]), int(tree.right[t])]
        cols = [s] if tree.left[s] < 0 else [int(tree.left[s]), int(tree.right[s])]
        X.ch = [[rec(a, b) for b in cols] for a in rows]
        off, X.rparts = 0, []
        for a in rows:
            X.rparts.append((off, _dofs(tree, a)))
            off += _dofs(tree, a)
        off, X.cparts = 0, []
        for b in cols:
            X.cparts.append((off, _dofs(tree, b)))
            off += _dofs(tree, b)
        return X

    return rec(0, 0)


def to_dense(X):
    """Explicit matrix of a block (pending low-rank pieces included)."""
    if X.kind == F:
        return X.D.copy()
    if X.kind == R:
        D = X.U @ X.W
        for U, W, ro, co in X.pend:
            D[ro:ro + U.shape[0], co:co + W.shape[1]] += U @ W
        return D
    D = np.zeros((X.m, X.n), dtype=np.complex128)
    for i, (ro, rm) in enumerate(X.rparts):
        for j, (co, cn) in enumerate(X.cparts):
            D[ro:ro + rm, co:co + cn] = to_dense(X.ch[i][j])
    return D


def _recompress(U, W, eps):
    """QR of both factors, truncated SVD of R_U R_W^T (Section 3.2), rank by
    the Frobenius tail."""
    if U.shape[1] == 0:
        return U, W
    Qu, Ru = np.linalg.qr(U)
    Qv, Rv = np.linalg.qr(W.conj().T)
    P, S, Lh = np.linalg.svd(Ru @ Rv.conj().T)
    tot = float(np.sum(S * S))
    r = S.size
    if tot == 0.0:
        r = 0
    else:
        tail = 0.0
        for k in range(S.size, -1, -1):      # smallest r with tail <= eps^2 total
            if tail <= eps * eps * tot:
                r = k
            else:
                break
            if k > 0:
                tail += float(S[k - 1] ** 2)
    sq = np.sqrt(S[:r])
    Un = (Qu @ P[:, :r]) * sq
    Vn = (Qv @ Lh.conj().T[:, :r]) * sq
    return Un, Vn.conj().T.copy()


def finalize(X, eps):
    """Recompress every low-rank block below X that holds pending sums."""
    if X.kind == R and X.pend:
        K = X.U.shape[1] + sum(p[0].shape[1] for p in X.pend)
        U = np.zeros((X.m, K), dtype=np.complex128)
        W = np.zeros((K, X.n), dtype=np.complex128)
        k = X.U.shape[1]
        U[:, :k], W[:k] = X.U, X.W
        for Up, Wp, ro, co in X.pend:
            kp = Up.shape[1]
            U[ro:ro + Up.shape[0], k:k + kp] = Up
            W[k:k + kp, co:co + Wp.shape[1]] = Wp
            k += kp
        X.U, X.W = _recompress(U, W, eps)
        X.pend = []
    elif X.kind == H:
        for row in X.ch:
            for c in row:
                finalize(c, eps)


# ------------------------------------------------------------------ products

def matmat(A, Xd):
    """A Xd for a block A (m x n) and a dense Xd (n x p)."""
    if A.kind == F:
        return A.D @ Xd
    if A.kind == R:
        assert not A.pend
        return A.U @ (A.W @ Xd)
    Y = np.zeros((A.m, Xd.shape[1]), dtype=np.complex128)
    for i, (ro, rm) in enumerate(A.rparts):
        for j, (co, cn) in enumerate(A.cparts):
            Y[ro:ro + rm] += matmat(A.ch[i][j], Xd[co:co + cn])
    return Y


def matmat_right(Xd, A):
    """Xd A for a dense Xd (p x m) and a block A (m x n)."""
    if A.kind == F:
        return Xd @ A.D
    if A.kind == R:
        assert not A.pend
        return (Xd @ A.U) @ A.W
    Y = np.zeros((Xd.shape[0], A.n), dtype=np.complex128)
    for i, (ro, rm) in enumerate(A.rparts):
        for j, (co, cn) in enumerate(A.cparts):
            Y[:, co:co + cn] += matmat_right(Xd[:, ro:ro + rm], A.ch[i][j])
    return Y


def add_lowrank(C, ro, co, U, W):
    """C[ro:ro+m, co:co+n] += U W into the block C (a view of it when C is
    F or R; the whole block when C is H)."""
    if C.kind == F:
        C.D[ro:ro + U.shape[0], co:co + W.shape[1]] += U @ W
    elif C.kind == R:
        if U.shape[1]:
            C.pend.append((U, W, ro, co))
    else:
        assert ro == 0 and co == 0 and U.shape[0] == C.m and W.shape[1] == C.n
        for i, (r0, rm) in enumerate(C.rparts):
            for j, (c0, cn) in enumerate(C.cparts):
                add_lowrank(C.ch[i][j], 0, 0, U[r0:r0 + rm], W[:, c0:c0 + cn])


def add_dense(C, ro, co, D):
    if C.kind == F:
        C.D[ro:ro + D.shape[0], co:co + D.shape[1]] += D
    elif C.kind == R:
        C.pend.append((D, np.eye(D.shape[1], dtype=np.complex128), ro, co))
    else:
        assert ro == 0 and co == 0 and D.shape == (C.m, C.n)
        for i, (r0, rm) in enumerate(C.rparts):
            for j, (c0, cn) in enumerate(C.cparts):
                add_dense(C.ch[i][j], 0, 0, D[r0:r0 + rm, c0:c0 + cn])


def muladd(C, ro, co, A, B, alpha):
    """C[ro:, co:] += alpha A B: the formatted update of step 4."""
    CASES[(C.kind, A.kind, B.kind)] += 1
    if A.kind == R:
        add_lowrank(C, ro, co, alpha * A.U, matmat_right(A.W, B))
    elif B.kind == R:
        add_lowrank(C, ro, co, alpha * matmat(A, B.U), B.W)
    elif A.kind == F and B.kind == F:
        add_dense(C, ro, co, alpha * (A.D @ B.D))
    else:
        kparts = A.cparts if A.kind == H else B.rparts
        for i, (r0, _) in enumerate(A.rparts if A.kind == H else [(0, A.m)]):
            for j, (c0, _) in enumerate(B.cparts if B.kind == H else [(0, B.n)]):
                for k in range(len(kparts)):
                    if C.kind == H:
                        muladd(C.ch[i][j], 0, 0, A.child(i, k), B.child(k, j), alpha)
                    else:
                        muladd(C, ro + r0, co + c0, A.child(i, k), B.child(k, j), alpha)


# ------------------------------------------------------------ substitutions

def lower_solve(L, Xd):
    """L^-1 Xd with L the unit lower factor held by the diagonal block L."""
    if L.kind == F:
        return sla.solve_triangular(L.D, Xd, lower=True, unit_diagonal=True)
    (o1, m1), (o2, m2) = L.rparts
    X1 = lower_solve(L.ch[0][0], Xd[o1:o1 + m1])
    X2 = lower_solve(L.ch[1][1], Xd[o2:o2 + m2] - matmat(L.ch[1][0], X1))
    return np.vstack([X1, X2])


def upper_solve_left(Ud, Xd):
    """U^-1 Xd with U the upper factor held by the diagonal block Ud."""
    if Ud.kind == F:
        return sla.solve_triangular(Ud.D, Xd, lower=False)
    (o1, m1), (o2, m2) = Ud.rparts
    X2 = upper_solve_left(Ud.ch[1][1], Xd[o2:o2 + m2])
    X1 = upper_solve_left(Ud.ch[0][0], Xd[o1:o1 + m1] - matmat(Ud.ch[0][1], X2))
    return np.vstack([X1, X2])


def upper_solve_right(Ud, Xd):
    """Xd U^-1 with U the upper factor held by the diagonal block Ud."""
    if Ud.kind == F:
        return sla.solve_triangular(Ud.D, Xd.T, trans="T", lower=False).T
    (o1, n1), (o2, n2) = Ud.cparts
    X1 = upper_solve_right(Ud.ch[0][0], Xd[:, o1:o1 + n1])
    X2 = upper_solve_right(Ud.ch[1][1], Xd[:, o2:o2 + n2] - matmat_right(X1, Ud.ch[0][1]))
    return np.hstack([X1, X2])


def trsm_lower(L, B, eps):
    """Step 2: B <- L^-1 B for the block B in the block row of L."""
    finalize(B, eps)
    if B.kind == R:
        B.U = lower_solve(L, B.U)
    elif B.kind == F:
        B.D = lower_solve(L, B.D)
    elif L.kind == F:
        for j in range(len(B.cparts)):
            trsm_lower(L, B.ch[0][j], eps)
    else:
        for j in range(len(B.cparts)):
            trsm_lower(L.ch[0][0], B.ch[0][j], eps)
            muladd(B.ch[1][j], 0, 0, L.ch[1][0], B.ch[0][j], -1.0)
            trsm_lower(L.ch[1][1], B.ch[1][j], eps)


def trsm_upper(Ud, B, eps):
    """Step 3: B <- B U^-1 for the block B in the block column of U."""
    finalize(B, eps)
    if B.kind == R:
        B.W = upper_solve_right(Ud, B.W)
    elif B.kind == F:
        B.D = upper_solve_right(Ud, B.D)
    elif Ud.kind == F:
        for i in range(len(B.rparts)):
            trsm_upper(Ud, B.ch[i][0], eps)
    else:
        for i in range(len(B.rparts)):
            trsm_upper(Ud.ch[0][0], B.ch[i][0], eps)
            muladd(B.ch[i][1], 0, 0, B.ch[i][0], Ud.ch[0][1], -1.0)
            trsm_upper(Ud.ch[1][1], B.ch[i][1], eps)


def lu_nopivot(D):
    """Gaussian elimination without pivoting: returns L \\ U packed in one array."""
    A = np.array(D, dtype=np.complex128)
    n = A.shape[0]
    for k in range(n - 1):
        A[k + 1:, k] /= A[k, k]
        A[k + 1:, k + 1:] -= np.outer(A[k + 1:, k], A[k, k + 1:])
    return A


def _hlu(X, eps):
    if X.kind == F:
        X.D = lu_nopivot(X.D)
        return
    assert X.kind == H and len(X.rparts) == 2 and len(X.cparts) == 2
    _hlu(X.ch[0][0], eps)                                       # 1
    trsm_lower(X.ch[0][0], X.ch[0][1], eps)                     # 2
    trsm_upper(X.ch[0][0], X.ch[1][0], eps)                     # 3
    muladd(X.ch[1][1], 0, 0, X.ch[1][0], X.ch[0][1], -1.0)      # 4
    _hlu(X.ch[1][1], eps)


def hlu(X, eps):
    """In-place H-LU of the diagonal block X (the four steps of Section 3.2).

    The many small products run on one BLAS thread (threads only add
    overhead at these sizes)."""
    with threadpool_limits(1):
        _hlu(X, eps)
    return X


def hlu_solve(LU, b):
    """x0 with L_H U_H x0 = b (b in cluster order, shape (N,) or (N, p))."""
    vec = b.ndim == 1
    B = np.asarray(b, dtype=np.complex128).reshape(b.shape[0], -1)
    with threadpool_limits(1):
        x = upper_solve_left(LU, lower_solve(LU, B))
    return x[:, 0] if vec else x


def factors_dense(LU):
    """Explicit (L_H, U_H) of a factorised diagonal block."""
    D = to_dense(LU)
    return np.tril(D, -1) + np.eye(D.shape[0]), np.triu(D)


def storage(X):
    """Complex entries held by the block: m n (F) or (m + n) k (R)."""
    if X.kind == F:
        return X.m * X.n
    if X.kind == R:
        return (X.m + X.n) * X.rank()
    return sum(storage(c) for row in X.ch for c in row)


def max_rank(X):
    if X.kind == R:
        return X.rank()
    if X.kind == H:
        return max(max_rank(c) for row in X.ch for c in row)
    return 0


def estimator(delta, delta_h, x0_norm, b_norm):
    """I(delta_H, delta) = (delta + delta_H |x0|) / |b| (eq. est_direct)."""
    return (delta + delta_h * x0_norm) / b_norm
