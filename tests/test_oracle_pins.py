"""Pins of the oracle's splitting rule, pivot rule and block bookkeeping.

Each fixture is built by hand so that the rule the oracle follows gives a
different answer from the plausible alternatives.  A docstring names the
mutation of the oracle that the test catches:

* cluster split at the midpoint of the box's longest side (Section 2.1,
  bisection of the enclosing box) -- a median split, or the split axis
  chosen some other way, fails;
* vector-ACA pivot with the largest smallest singular value sigma_3
  (Section 2.3, the third pivoting strategy) -- pivoting on the largest entry
  or on the largest 3x3 Frobenius norm (the first two strategies), fails;
* rank-model features, sparsity constant and storage count computed by hand.
"""
import math
import os

import numpy as np
import pytest

from paper_1706_09384_amd import workloads as W


def _line(xs):
    return np.array([[x, 0.0, 0.0] for x in xs], dtype=np.float64)


# ------------------------------------------------------------- splitting

def test_split_hand_example_midpoint_not_median(orc):
    """Mutation caught: a median split, or an unstable partition.

    Points x = 10, 1, 0, 10.5, 2 (input order) with leaf 2.  The root box is
    [0, 10.5], so the midpoint 5.25 sends {1, 0, 2} left and {10, 10.5} right
    (a median split would send 2 right).  The left box [0, 2] splits at 1:
    {0} left, {1, 2} right.  Stable partitions keep the incoming order.
    """
    t = orc.cluster_tree(_line([10.0, 1.0, 0.0, 10.5, 2.0]), 2)
    assert t.perm.tolist() == [2, 1, 4, 0, 3]
    assert t.begin.tolist() == [0, 0, 0, 1, 3]
    assert t.end.tolist() == [5, 3, 1, 3, 5]
    assert t.left.tolist() == [1, 2, -1, -1, -1]
    assert t.right.tolist() == [4, 3, -1, -1, -1]
    assert t.depth.tolist() == [0, 1, 2, 2, 1]

    # The fixture discriminates: the median of the root's five points is the
    # third smallest (x = 2), and a median split puts two points on the left.
    xs = np.sort([10.0, 1.0, 0.0, 10.5, 2.0])
    assert int(np.sum(xs < np.median(xs))) == 2 != t.end[1] - t.begin[1]


def test_split_axis_is_longest_side_ties_to_lowest(orc):
    """Mutation caught: ties resolved to the last maximal axis, or a fixed axis
    (x first) instead of the box's longest side.

    Five points in the plane z = 0 with a 2 x 2 box: x and y tie, so the split
    is along x at 0 (splitting along y would send points 1, 2 and 4 left).
    The second fixture's box is longest along y, where only two of its six
    points lie off the axis."""
    P = np.array([[1.0, 1.0, 0.0], [-1.0, -1.0, 0.0], [1.0, -1.0, 0.0], [-1.0, 1.0, 0.0],
                  [0.5, -0.9, 0.0]])
    t = orc.cluster_tree(P, 2)
    left = set(t.perm[t.begin[1]:t.end[1]].tolist())
    assert left == {1, 3}                      # x < 0

    Q = np.array([[-1.0, 0.0, 0.0], [-0.9, 0.0, 0.0], [0.9, 0.0, 0.0], [1.0, 0.0, 0.0],
                  [0.0, -1.5, 0.0], [0.0, 1.5, 0.0]])
    tq = orc.cluster_tree(Q, 3)
    # box extents: x 2.0, y 3.0 -> split along y at 0: y < 0 goes left
    assert set(tq.perm[tq.begin[1]:tq.end[1]].tolist()) == {4}
    assert set(tq.perm[tq.begin[2]:tq.end[2]].tolist()) == {0, 1, 2, 3, 5}


@pytest.mark.parametrize("which", ["sphere", "cube", "spheroid"])
def test_every_split_is_at_the_box_midpoint(orc, which):
    """Mutation caught: any split value other than (lo + hi) * 0.5 on the
    longest side (lowest axis on ties), e.g. the median of the coordinates.

    On every internal node: left coordinates < (lo + hi) * 0.5 <= right
    coordinates along argmax(hi - lo), and each child keeps its points in
    the parent's order."""
    if which == "sphere":
        P, leaf = W.fibonacci_sphere(3000), 32
    elif which == "cube":
        P, _ = W.cube_surface(3000, seed=0)
        leaf = 16
    else:
        P, _ = W.prolate_spheroid(2000, seed=0)
        leaf = 8
    t = orc.cluster_tree(P, leaf)
    n_internal = 0
    for v in range(t.n_nodes):
        if t.left[v] < 0:
            continue
        n_internal += 1
        ext = t.hi[v] - t.lo[v]
        ax = int(np.flatnonzero(ext == ext.max())[0])
        mid = (t.lo[v][ax] + t.hi[v][ax]) * 0.5
        l, r = t.left[v], t.right[v]
        lc = P[t.perm[t.begin[l]:t.end[l]], ax]
        rc = P[t.perm[t.begin[r]:t.end[r]], ax]
        assert lc.max() < mid <= rc.min()
    assert n_internal > 10
    # stable partitions: every leaf keeps its points in input order
    for v in range(t.n_nodes):
        if t.left[v] < 0:
            assert np.all(np.diff(t.perm[t.begin[v]:t.end[v]]) > 0)


# ------------------------------------------------------------------ pivots

def _pivot_fixture():
    """A 4 x 4-point block (12 x 12) whose first row's candidates are:
    j = 0: 10 e1 e1^T (largest entry, largest Frobenius norm, sigma_3 ~ 0),
    j = 1: 2 I (sigma_3 = 2), j = 2, 3: noise;
    and whose column j = 1 has, below row 0: i = 1: 8 e2 e2^T (largest entry
    and norm, singular), i = 2: 1.5 I (sigma_3 = 1.5), i = 3: noise."""
    rng = np.random.default_rng(11)
    A = 1e-3 * (rng.standard_normal((12, 12)) + 1j * rng.standard_normal((12, 12)))
    A[0:3, 0:3] += np.diag([10.0, 0.0, 0.0])
    A[0:3, 3:6] += 2.0 * np.eye(3)
    A[3:6, 3:6] += np.diag([0.0, 8.0, 0.0])
    A[6:9, 3:6] += 1.5 * np.eye(3)
    return A


def test_aca_column_pivot_is_largest_sigma3(orc):
    """Mutation caught: column pivot by the largest entry or the largest 3x3
    Frobenius norm of the residual row (both pick j = 0 here)."""
    A = _pivot_fixture()
    blk = A[0:3].reshape(3, 4, 3).transpose(1, 0, 2)
    fro = np.sqrt((np.abs(blk) ** 2).sum(axis=(1, 2)))
    big = np.abs(blk).reshape(4, -1).max(axis=1)
    s3 = np.linalg.svd(blk, compute_uv=False)[:, 2]
    assert int(np.argmax(fro)) == 0 and int(np.argmax(big)) == 0 and int(np.argmax(s3)) == 1
    res = orc.vector_aca(A, 1e-12)
    assert res.row_pivots[0] == 0
    assert res.col_pivots[0] == 1


def test_aca_row_pivot_is_largest_sigma3_of_residual_column(orc):
    """Mutation caught: next row pivot by the largest entry or Frobenius norm of
    the residual column (both pick i = 1), or a pivot search that does not
    exclude the used row 0 (whose block 2 I has the largest sigma_3)."""
    A = _pivot_fixture()
    cb = A[:, 3:6].reshape(4, 3, 3)
    s3 = np.linalg.svd(cb, compute_uv=False)[:, 2]
    fro = np.sqrt((np.abs(cb) ** 2).sum(axis=(1, 2)))
    assert int(np.argmax(s3)) == 0                      # row 0 is used: excluded
    assert int(np.argmax(fro[1:])) + 1 == 1 and int(np.argmax(s3[1:])) + 1 == 2
    res = orc.vector_aca(A, 1e-12)
    assert res.row_pivots[:2] == [0, 2]


def test_aca_first_update_is_rank3_through_pivot_inverse(orc):
    """Mutation caught: a transposed or conjugated pivot in U_new = R_col M^-1,
    V_new = R_row^*: the first term must reproduce row 0 and column j = 1
    exactly (the interpolation property of cross approximation)."""
    A = _pivot_fixture()
    res = orc.vector_aca(A, 1e-12, max_rank=3)     # one rank-3 term
    assert res.rank == 3
    B = res.U @ res.V.conj().T
    assert np.allclose(B[0:3], A[0:3], rtol=0, atol=1e-12)
    assert np.allclose(B[:, 3:6], A[:, 3:6], rtol=0, atol=1e-12)


# ------------------------------------------------- features and bookkeeping

def test_rank_features_hand_values(orc):
    """Mutation caught: point-based instead of box-based diameter, a distance
    without positive parts, swapped X/Y, or log2 instead of ln sizes.

    X = {(0,0,0), (1,0,0), (0,2,0)}: box [0,1]x[0,2]x[0,0], diameter sqrt 5
    (the points' own diameter is sqrt 5 as well, so a third point set below
    separates box and point diameters).  Y = {(4,0,0), (5,1,0)}: box
    [4,5]x[0,1]x[0,0], diameter sqrt 2.  Box gap: 3 along x, the y ranges
    overlap, so dist = 3."""
    X = np.array([[0.0, 0.0, 0.0], [1.0, 0.0, 0.0], [0.0, 2.0, 0.0]])
    Y = np.array([[4.0, 0.0, 0.0], [5.0, 1.0, 0.0]])
    tx, ty = orc.cluster_tree(X, 8), orc.cluster_tree(Y, 8)
    kappa, eps = 2.5, 1e-4
    f = orc.rank_features(tx, ty, [(0, 0, orc.LOWRANK), (0, 0, orc.DENSE)], kappa, eps)
    ref = [math.log(3), math.log(2), kappa * math.sqrt(5), kappa * math.sqrt(2), kappa * 3.0, -4.0]
    assert f.shape == (1, 6)
    assert np.allclose(f[0], ref, rtol=1e-15, atol=1e-15)

    # Box diameter differs from the point diameter for an L-shaped set:
    # {(0,0,0), (2,0,0), (0,2,0)} has box diagonal sqrt 8 = point diameter;
    # {(0,0,0), (2,1,0), (1,2,0)} has box diagonal sqrt 8 but point diameter sqrt 5.
    Z = np.array([[0.0, 0.0, 0.0], [2.0, 1.0, 0.0], [1.0, 2.0, 0.0]])
    tz = orc.cluster_tree(Z, 8)
    g = orc.rank_features(tz, ty, [(0, 0, orc.LOWRANK)], 1.0, 1e-3)
    assert g[0, 2] == pytest.approx(math.sqrt(8.0), rel=1e-15)
    # gap along x: 4 - 2 = 2; y ranges [0,2] and [0,1] overlap
    assert g[0, 4] == pytest.approx(2.0, rel=1e-15)
    assert g[0, 5] == pytest.approx(-3.0, rel=1e-15)


def test_sparsity_constant_and_storage_by_hand(orc):
    """C_sp counts blocks per row and per column cluster and takes the larger
    (Section 2.1); N_st = 9mn per dense block + 3r(m + n) per low-rank block
    (Section 5.1), in entries of the 3N x 3N matrix."""
    blocks = np.array([[0, 1, 1], [0, 2, 0], [0, 3, 1], [1, 1, 0], [2, 1, 1], [3, 1, 0]])
    # row counts: node 0: 3, others 1; column counts: node 1: 4
    assert orc.sparsity_constant(blocks, 4, 4) == 4
    assert orc.sparsity_constant(blocks[:3], 4, 4) == 3
    sizes = [(orc.DENSE, 2, 3, 0), (orc.LOWRANK, 4, 5, 6), (orc.LOWRANK, 7, 1, 0)]
    assert orc.storage_entries(sizes) == 9 * 2 * 3 + 3 * 6 * (4 + 5)


def test_sweep_recipe_matches_table_corr():
    """The fixed-density sweep uses the paper's (N, omega) pairs (Section 8, Table
    table_corr), and its reading of n_lambda_s holds: the unit sphere's diameter 2
    spans D omega / (2 pi) S-wavelengths (kappa_s = omega with mu = rho = 1)."""
    import json
    import math
    from paper_1706_09384_amd import workloads as W
    g = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "paper_table_corr.json")))
    assert [n for n, _ in W.TABLE_CORR] == g["N"]
    assert [w for _, w in W.TABLE_CORR] == [float(x) for x in g["omega"]]
    for (n, w), nl in zip(W.TABLE_CORR, g["n_lambda_s"]):
        assert n % 3 == 0
        assert abs(2.0 * w / (2.0 * math.pi) - nl) <= 0.06 * nl
    # about ten mesh points per S-wavelength at every row: h = sqrt(4 pi / N_c)
    for n_c, w in W.fixed_density_series():
        ppw = (2.0 * math.pi / w) / math.sqrt(4.0 * math.pi / n_c)
        assert 10.0 <= ppw <= 11.5
