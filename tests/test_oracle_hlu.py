"""Pins of the oracle's H-LU (Section 3.2) and certification estimator (Section 3.3).

* With eps_LU = 0 no truncation happens, so the H-LU is exact: its factors are
  unit lower / upper triangular with L U = A_H, which by uniqueness of the
  unpivoted LU is the textbook dense factorisation of A_H.
* With eps_LU > 0 the factorisation error tracks eps_LU, and the storage of
  the factors drops as eps_LU grows.
* The estimator reproduces every row the paper prints (three tables), and on
  a real solve it bounds the true residual (triangle inequality).
"""
import json
import os

import numpy as np
import pytest

from paper_1706_09384_amd import workloads as W

GOLD = os.path.join(os.path.dirname(__file__), "golden")


def _sub(t, A, a, b):
    ri = t.perm[t.begin[a]:t.end[a]]
    ci = t.perm[t.begin[b]:t.end[b]]
    rd = (3 * ri[:, None] + np.arange(3)).ravel()
    cd = (3 * ci[:, None] + np.arange(3)).ravel()
    return A[np.ix_(rd, cd)]


def svd_leaves(orc, t, blocks, A, eps):
    """A_H with every admissible block replaced by its truncated SVD."""
    out = []
    for a, b, kind in blocks:
        Ab = _sub(t, A, a, b)
        if kind == orc.DENSE:
            out.append((a, b, 0, Ab))
        else:
            U, S, Vh = np.linalg.svd(Ab, full_matrices=False)
            r = orc.truncation_rank(S, eps)
            sq = np.sqrt(S[:r])
            out.append((a, b, 1, (U[:, :r] * sq, Vh[:r].conj().T * sq)))
    return out


@pytest.fixture(scope="module")
def sphere400(orc):
    w = W.small_sphere(400, leaf=16)
    X, _ = w.points()
    pb = orc.Problem.from_workload(w, X)
    t = orc.cluster_tree(X, w.leaf)
    blocks = orc.block_tree(t, t, w.eta)
    A = orc.dense(pb)
    dof = (3 * t.perm[:, None] + np.arange(3)).ravel()
    Ac = A[np.ix_(dof, dof)]            # cluster order
    b = w.rhs()[:, 0][dof]
    return w, t, blocks, A, Ac, b


def factorise(orc, t, blocks, A, eps_aca, eps_lu):
    leaves = svd_leaves(orc, t, blocks, A, eps_aca)
    root = orc.hlu.build(t, leaves)
    AH = orc.hlu.to_dense(root)
    orc.hlu.hlu(root, eps_lu)
    return root, AH


def test_exact_hlu_is_the_unpivoted_lu(orc, sphere400):
    w, t, blocks, A, Ac, b = sphere400
    assert (blocks[:, 2] == orc.LOWRANK).sum() > 100
    root, AH = factorise(orc, t, blocks, A, 1e-4, 0.0)
    L, U = orc.hlu.factors_dense(root)
    assert np.allclose(np.diag(L), 1.0) and not np.triu(L, 1).any() and not np.tril(U, -1).any()
    assert np.linalg.norm(L @ U - AH) <= 1e-13 * np.linalg.norm(AH)
    x0 = orc.hlu.hlu_solve(root, b)
    xd = np.linalg.solve(AH, b)
    assert np.linalg.norm(x0 - xd) <= 1e-12 * np.linalg.norm(xd)
    # the formatted update visited the low-rank, dense and subdivided formats
    cases = orc.hlu.CASES
    assert any(k[1] == orc.hlu.R for k in cases) and any(k[2] == orc.hlu.R for k in cases)
    assert any(k[0] == orc.hlu.R for k in cases) and any(k[0] == orc.hlu.F for k in cases)
    assert any(k[0] == orc.hlu.H for k in cases)


def test_eta_zero_reduces_to_dense_block_lu(orc, sphere400):
    """Without admissible blocks the recursion is a plain block LU."""
    w, t, _, A, Ac, b = sphere400
    B0 = orc.block_tree(t, t, 0.0)
    root, AH = factorise(orc, t, B0, A, 1e-4, 1e-4)
    assert np.array_equal(AH, Ac)
    L, U = orc.hlu.factors_dense(root)
    assert np.linalg.norm(L @ U - Ac) <= 1e-13 * np.linalg.norm(Ac)
    # the same factors as elimination without pivoting on the whole matrix
    LU = orc.hlu.lu_nopivot(Ac)
    assert np.linalg.norm(np.triu(LU) - U) <= 1e-11 * np.linalg.norm(U)


@pytest.mark.parametrize("eps_lu", [1e-4, 1e-6, 1e-8])
def test_truncated_hlu_error_tracks_eps(orc, sphere400, eps_lu):
    w, t, blocks, A, Ac, b = sphere400
    root, AH = factorise(orc, t, blocks, A, 1e-8, eps_lu)
    L, U = orc.hlu.factors_dense(root)
    e = np.linalg.norm(L @ U - AH) / np.linalg.norm(AH)
    assert 1e-3 * eps_lu <= e <= 2 * eps_lu
    x0 = orc.hlu.hlu_solve(root, b)
    delta = np.linalg.norm(b - AH @ x0) / np.linalg.norm(b)
    assert delta <= 10 * eps_lu


def test_storage_drops_with_eps(orc, sphere400):
    """Blocks that receive updates are recompressed at eps_LU (blocks that
    receive none keep their assembly rank, so the maximum need not move)."""
    w, t, blocks, A, Ac, b = sphere400
    r = []
    for eps_lu in (1e-8, 1e-4):
        root, _ = factorise(orc, t, blocks, A, 1e-8, eps_lu)
        r.append((orc.hlu.max_rank(root), orc.hlu.storage(root)))
    assert r[1][0] <= r[0][0] and r[1][1] < 0.9 * r[0][1]


def test_estimator_reproduces_paper_rows(orc):
    d = json.load(open(os.path.join(GOLD, "paper_estimator_rows.json")))
    n = 0
    for table in ("error_freq_single", "error_freq_double", "error_dens_single"):
        for dofs, omega, eps, I, res, dh, xb, db in d[table]:
            est = orc.hlu.estimator(db, dh, xb, 1.0)
            assert abs(est - I) <= 0.01 * I, (table, dofs, omega, eps)
            if eps >= 1e-6 and dofs > 1926:   # rows at rounding level carry no bound
                assert res <= I
            n += 1
    assert n == 30


@pytest.mark.parametrize("eps", [1e-4, 1e-6])
def test_estimator_bounds_true_residual(orc, sphere400, eps):
    w, t, blocks, A, Ac, b = sphere400
    root, AH = factorise(orc, t, blocks, A, eps, eps)
    x0 = orc.hlu.hlu_solve(root, b)
    res = np.linalg.norm(b - Ac @ x0) / np.linalg.norm(b)
    delta = np.linalg.norm(b - AH @ x0)
    dh = np.linalg.norm(AH - Ac)
    I = orc.hlu.estimator(delta, dh, np.linalg.norm(x0), np.linalg.norm(b))
    assert res <= I
    assert I <= 1e3 * eps
