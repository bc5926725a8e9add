"""Pins of the oracle's trees, dense solve, ACA, recompression, H-matvec and MLP.

Each test checks the oracle against an independent fact: invariants that the
paper states (Sections 2.1, 5.1, 6.1), textbook linear algebra (LU residual,
Eckart-Young optimality of the truncated SVD, exact-rank reconstruction),
brute force on tiny inputs, and finite differences for gradients.
"""
import json
import math
import os

import numpy as np
import pytest

from paper_1706_09384_amd import workloads as W

GOLD = os.path.join(os.path.dirname(__file__), "golden")


@pytest.fixture(scope="module")
def sphere1k(orc):
    w = W.plain_sphere_1k()
    X, _ = w.points()
    pb = orc.Problem.from_workload(w, X)
    t = orc.cluster_tree(X, w.leaf)
    blocks = orc.block_tree(t, t, w.eta)
    A = orc.dense(pb)
    return w, X, pb, t, blocks, A


# ----------------------------------------------------------------- trees

def check_tree(orc, P, t, leaf):
    n = P.shape[0]
    assert np.array_equal(np.sort(t.perm), np.arange(n))
    assert t.begin[0] == 0 and t.end[0] == n
    for v in range(t.n_nodes):
        b, e = t.begin[v], t.end[v]
        pts = P[t.perm[b:e]]
        assert np.array_equal(t.lo[v], pts.min(0)) and np.array_equal(t.hi[v], pts.max(0))
        if t.left[v] < 0:
            ext = pts.max(0) - pts.min(0)
            assert e - b <= leaf or ext.max() == 0.0
        else:
            l, r = t.left[v], t.right[v]
            assert t.begin[l] == b and t.end[l] == t.begin[r] and t.end[r] == e
            assert t.depth[l] == t.depth[v] + 1 == t.depth[r]
            assert l == v + 1                       # pre-order, left first
            # The split is at the midpoint of the parent box's longest side
            # (lowest axis on ties): left < (lo + hi) * 0.5 <= right.
            ax = int(np.argmax(t.hi[v] - t.lo[v]))
            mid = (t.lo[v][ax] + t.hi[v][ax]) * 0.5
            assert t.hi[l][ax] < mid <= t.lo[r][ax]


@pytest.mark.parametrize("n,leaf", [(1000, 32), (4000, 16), (777, 5)])
def test_cluster_tree_invariants(orc, n, leaf):
    P = W.fibonacci_sphere(n)
    t = orc.cluster_tree(P, leaf)
    check_tree(orc, P, t, leaf)
    # Balanced for a uniform cloud: L(I) = ceil(log2(N / N_leaf)) (Section 2.1), +-2.
    L = t.levels() - 1
    assert abs(L - math.ceil(math.log2(n / leaf))) <= 2


def test_cluster_tree_cube_and_duplicates(orc):
    P, _ = W.cube_surface(3000, seed=0)
    check_tree(orc, P, orc.cluster_tree(P, 32), 32)
    Q = np.repeat(W.fibonacci_sphere(10), 7, axis=0)   # coincident points end as leaves
    t = orc.cluster_tree(Q, 3)
    check_tree(orc, Q, t, 3)


def test_block_tree_partitions_matrix(orc):
    P = W.fibonacci_sphere(600)
    t = orc.cluster_tree(P, 16)
    B = orc.block_tree(t, t, 3.0)
    cover = np.zeros((600, 600), np.int32)
    for tt, s, kind in B:
        ri = t.perm[t.begin[tt]:t.end[tt]]
        ci = t.perm[t.begin[s]:t.end[s]]
        cover[np.ix_(ri, ci)] += 1
        if kind == orc.DENSE:
            assert t.left[tt] < 0 and t.left[s] < 0     # dense blocks only at leaf level
        else:
            assert orc.admissible(t, tt, t, s, 3.0)
            # brute-force separation: the true distance exceeds the box distance > 0
            d = np.linalg.norm(P[ri][:, None, :] - P[ci][None, :, :], axis=2).min()
            assert d > 0
    assert np.all(cover == 1)


def test_admissibility_brute_force(orc):
    """Box quantities bound the true diameter from above and distance from below (Section 6.1)."""
    rng = np.random.default_rng(0)
    P = W.uniform_ball(400, seed=1)
    t = orc.cluster_tree(P, 8)
    for _ in range(200):
        a, b = rng.integers(0, t.n_nodes, 2)
        X = P[t.perm[t.begin[a]:t.end[a]]]
        Y = P[t.perm[t.begin[b]:t.end[b]]]
        dist = np.linalg.norm(X[:, None] - Y[None], axis=2).min()
        diamx = np.linalg.norm(X[:, None] - X[None], axis=2).max()
        diamy = np.linalg.norm(Y[:, None] - Y[None], axis=2).max()
        if orc.admissible(t, a, t, b, 3.0):
            assert min(diamx, diamy) < 3.0 * dist + 1e-12


def test_block_tree_two_clouds(orc):
    X = W.fibonacci_sphere(500)
    Y = W.fibonacci_sphere(300) * 0.5 + np.array([2.5, 0, 0])
    tx, ty = orc.cluster_tree(X, 16), orc.cluster_tree(Y, 16)
    B = orc.block_tree(tx, ty, 3.0)
    tot = sum((tx.end[a] - tx.begin[a]) * (ty.end[b] - ty.begin[b]) for a, b, _ in B)
    assert tot == 500 * 300


# ----------------------------------------------------------- dense / LU

def test_dense_matches_blocks_and_streamed_rows(orc, sphere1k):
    w, X, pb, t, blocks, A = sphere1k
    rng = np.random.default_rng(0)
    for i, j in rng.integers(0, 1000, (30, 2)):
        if i == j:
            continue
        assert np.array_equal(A[3 * i:3 * i + 3, 3 * j:3 * j + 3],
                              orc.green_block(0, X[i], X[j], None, w.omega, w.lam, w.mu, w.rho))
    assert np.array_equal(A[0:3, 0:3], w.self_re * np.eye(3))
    b = w.rhs()
    y = orc.matvec_rows(pb, b)
    ref = A @ b
    assert np.linalg.norm(y - ref) <= 1e-13 * np.linalg.norm(ref)
    rows = np.array([5, 17, 999])
    ys = orc.matvec_rows(pb, b, rows)
    idx = (3 * rows[:, None] + np.arange(3)).ravel()
    assert np.linalg.norm(ys - ref[idx]) <= 1e-13 * np.linalg.norm(ref[idx])


def test_lu_solve_residual(orc, sphere1k):
    w, X, pb, t, blocks, A = sphere1k
    b = w.rhs()[:, 0]
    x, rcond = orc.lu_solve(A, b)
    assert np.linalg.norm(A @ x - b) <= 1e-12 * np.linalg.norm(b)
    assert 0 < rcond < 1


# ------------------------------------------------------------------ ACA

def small_admissible(orc, t, blocks, maxpts=32, count=12):
    out = []
    for a, b, kind in blocks:
        if kind != orc.LOWRANK:
            continue
        m, n = t.end[a] - t.begin[a], t.end[b] - t.begin[b]
        if m <= maxpts and n <= maxpts:
            out.append((a, b))
    step = max(1, len(out) // count)
    return out[::step][:count]


def sub(t, A, a, b):
    ri = t.perm[t.begin[a]:t.end[a]]
    ci = t.perm[t.begin[b]:t.end[b]]
    rd = (3 * ri[:, None] + np.arange(3)).ravel()
    cd = (3 * ci[:, None] + np.arange(3)).ravel()
    return A[np.ix_(rd, cd)]


@pytest.mark.parametrize("eps", [1e-4, 1e-6])
def test_aca_vs_truncated_svd_tiny_blocks(orc, sphere1k, eps):
    """ACA error ~ eps, rank never below the optimal (Eckart-Young) rank, multiple of 3."""
    w, X, pb, t, blocks, A = sphere1k
    for a, b in small_admissible(orc, t, blocks):
        Ab = sub(t, A, a, b)
        res = orc.vector_aca(Ab, eps)
        err = np.linalg.norm(Ab - res.U @ res.V.conj().T) / np.linalg.norm(Ab)
        assert err <= 3 * eps
        assert res.rank >= orc.numerical_rank(Ab, eps)
        assert res.rank % 3 == 0 and res.fallbacks == 0
        # the recursive Frobenius norm equals the explicit one
        Bk = np.linalg.norm(res.U @ res.V.conj().T) ** 2
        assert abs(res.norm2 - Bk) <= 1e-10 * Bk


def test_aca_exact_rank_block(orc):
    """A block of exact rank 3k is reproduced to rounding; recompression finds 3k."""
    rng = np.random.default_rng(3)
    for k, m, n in [(2, 20, 25), (4, 30, 18), (1, 6, 9)]:
        Xf = rng.standard_normal((3 * m, 3 * k)) + 1j * rng.standard_normal((3 * m, 3 * k))
        Yf = rng.standard_normal((3 * n, 3 * k)) + 1j * rng.standard_normal((3 * n, 3 * k))
        A = Xf @ Yf.conj().T
        res = orc.vector_aca(A, 1e-8)
        assert res.rank in (3 * k, 3 * k + 3)
        assert np.linalg.norm(A - res.U @ res.V.conj().T) <= 1e-12 * np.linalg.norm(A)
        U2, V2, S = orc.recompress(res.U, res.V, 1e-8)
        assert U2.shape[1] == 3 * k


def test_aca_full_rank_reaches_min_dim(orc):
    """A random full-rank block needs min(m, n) steps and is then exact."""
    rng = np.random.default_rng(4)
    A = rng.standard_normal((12, 18)) + 1j * rng.standard_normal((12, 18))
    res = orc.vector_aca(A, 1e-14)
    assert res.steps == 4 and res.rank == 12
    assert np.linalg.norm(A - res.U @ res.V.conj().T) <= 1e-12 * np.linalg.norm(A)


def test_aca_singular_pivots_use_fallback(orc):
    """Coplanar T blocks: every 3x3 subblock is singular, the pivot fallback fires."""
    n_side = 8
    g = np.linspace(0, 0.3, n_side)
    Xp = np.array([[u, v, 0.0] for u in g for v in g])
    Yp = Xp + np.array([2.0, 0.3, 0.0])
    nrm = np.array([0.0, 0.0, 1.0])
    m = Xp.shape[0]
    A = np.zeros((3 * m, 3 * m), np.complex128)
    for i in range(m):
        for j in range(m):
            A[3 * i:3 * i + 3, 3 * j:3 * j + 3] = orc.green_block(1, Xp[i], Yp[j], nrm, 3.0)
    res = orc.vector_aca(A, 1e-6)
    assert res.fallbacks > 0
    assert np.linalg.norm(A - res.U @ res.V.conj().T) <= 1e-5 * np.linalg.norm(A)


# --------------------------------------------------------- recompression

def test_recompression_is_truncated_svd_of_product(orc, sphere1k):
    w, X, pb, t, blocks, A = sphere1k
    for a, b in small_admissible(orc, t, blocks, maxpts=40, count=6):
        Ab = sub(t, A, a, b)
        res = orc.vector_aca(Ab, 1e-5)
        U2, V2, S = orc.recompress(res.U, res.V, 1e-4)
        B = res.U @ res.V.conj().T
        Sb = np.linalg.svd(B, compute_uv=False)
        assert np.allclose(S, Sb[:S.size], rtol=0, atol=1e-12 * Sb[0])
        r = U2.shape[1]
        assert orc.numerical_rank(Ab, 1e-4) - 3 <= r <= res.rank
        # Eckart-Young: the recompressed block is the best rank-r approximation of B.
        P, Sv, Qh = np.linalg.svd(B)
        Br = (P[:, :r] * Sv[:r]) @ Qh[:r]
        assert np.linalg.norm(U2 @ V2.conj().T - Br) <= 1e-10 * np.linalg.norm(B)
        assert np.linalg.norm(Ab - U2 @ V2.conj().T) <= (1e-4 + 3e-5) * np.linalg.norm(Ab) * 1.5


def test_truncation_rank_rule(orc):
    S = np.array([1.0, 0.5, 1e-3, 1e-5, 0.0])
    assert orc.truncation_rank(S, 1e-2) == 2
    assert orc.truncation_rank(S, 1e-4) == 3
    assert orc.truncation_rank(S, 1e-7) == 4
    assert orc.truncation_rank(np.zeros(3), 1e-4) == 0


# ------------------------------------------------------------ H-matvec

def build_oracle_hmatrix(orc, t, blocks, A, eps):
    out = []
    for a, b, kind in blocks:
        Ab = sub(t, A, a, b)
        if kind == orc.DENSE:
            out.append((a, b, kind, Ab))
        else:
            res = orc.vector_aca(Ab, eps)
            U2, V2, _ = orc.recompress(res.U, res.V, eps)
            out.append((a, b, kind, (U2, V2)))
    return out


def test_hmatvec_eta_zero_is_dense(orc, sphere1k):
    w, X, pb, t, _, A = sphere1k
    B0 = orc.block_tree(t, t, 0.0)
    assert np.all(B0[:, 2] == orc.DENSE)
    blocks = [(a, b, k, sub(t, A, a, b)) for a, b, k in B0]
    x = w.rhs()
    y = orc.hmatvec(blocks, t, t, x)
    assert np.linalg.norm(y - A @ x) <= 1e-13 * np.linalg.norm(A @ x)


@pytest.mark.slow
def test_hmatrix_error_close_to_eps(orc, sphere1k):
    """Representation error delta_H,F ~ eps as in the paper's tables (Section 7.3)."""
    w, X, pb, t, blocks, A = sphere1k
    H = build_oracle_hmatrix(orc, t, blocks, A, 1e-4)
    Ad = orc.densify(H, t, t)
    dHF = np.linalg.norm(Ad - A) / np.linalg.norm(A)
    assert dHF <= 5e-4
    x = w.rhs()
    e = np.linalg.norm(orc.hmatvec(H, t, t, x) - A @ x) / np.linalg.norm(A @ x)
    assert e <= 5e-4


def test_storage_bound(orc, sphere1k):
    """N_st <= 2 C_sp max(r_max, N_leaf) N L (Section 5.1), in DOF units."""
    w, X, pb, t, blocks, A = sphere1k
    sizes, rmax = [], 0
    for a, b, kind in blocks:
        m, n = int(t.end[a] - t.begin[a]), int(t.end[b] - t.begin[b])
        r = 0
        if kind == orc.LOWRANK and m * n <= 2500:
            r = orc.vector_aca(sub(t, A, a, b), 1e-4).rank
        elif kind == orc.LOWRANK:
            r = 3 * min(m, n)      # crude upper bound for the big blocks
        rmax = max(rmax, r)
        sizes.append((kind, m, n, r))
    nst = orc.storage_entries(sizes)
    csp = orc.sparsity_constant(blocks, t.n_nodes, t.n_nodes)
    bound = 2 * csp * max(rmax, 3 * w.leaf) * 3 * 1000 * t.levels()
    assert nst <= bound


# --------------------------------------------------------------- GMRES

def test_gmres_matches_lu(orc, sphere1k):
    w, X, pb, t, blocks, A = sphere1k
    b = w.rhs()[:, 0]
    x, it, rr = orc.gmres(lambda v: A @ v, b, 1e-10, restart=100, maxit=3000)
    xl, _ = orc.lu_solve(A, b)
    assert rr <= 1e-10
    assert np.linalg.norm(x - xl) <= 1e-7 * np.linalg.norm(xl)


# ----------------------------------------------------------------- MLP

def test_mlp_gradient_finite_difference(orc):
    rng = np.random.default_rng(0)
    params = orc.mlp_init(1)
    X = rng.standard_normal((17, 6))
    tgt = rng.standard_normal(17)
    loss, grads = orc.mlp_loss_grad(params, X, tgt)
    for pi, (p, g) in enumerate(zip(params, grads)):
        flat = p.reshape(-1)
        for k in rng.choice(flat.size, size=min(6, flat.size), replace=False):
            old = flat[k]
            h = 1e-6
            flat[k] = old + h
            lp, _ = orc.mlp_loss_grad(params, X, tgt)
            flat[k] = old - h
            lm, _ = orc.mlp_loss_grad(params, X, tgt)
            flat[k] = old
            fd = (lp - lm) / (2 * h)
            assert abs(fd - g.reshape(-1)[k]) <= 1e-6 * (1 + abs(fd))


def test_adam_first_step_is_signed_lr(orc):
    """First bias-corrected Adam step moves each weight by lr * g/(|g| + eps)."""
    p = [np.array([1.0, -2.0, 3.0])]
    g = [np.array([0.5, -1e-3, 0.0])]
    z = [np.zeros(3)]
    newp, m, v = orc.adam_step(p, g, z, [np.zeros(3)], 1, lr=0.1)
    assert np.allclose(newp[0], [1.0 - 0.1 * 0.5 / (0.5 + 1e-8), -2.0 + 0.1 * 1e-3 / (1e-3 + 1e-8), 3.0])


def test_paper_rank_tables_properties():
    """Printed max ranks (Section 7.2 tables): ACA ranks are multiples of 3 and
    recompression lowers them -- the two invariants the oracle's ACA obeys."""
    g = json.load(open(os.path.join(GOLD, "paper_max_ranks.json")))
    for table in ("single_layer", "double_layer"):
        for omega, pairs in g[table].items():
            for before, after in pairs:
                assert before % 3 == 0 and after < before
