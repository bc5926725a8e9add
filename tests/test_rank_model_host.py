"""Rank-model features (host side of the library, no GPU): the library's
features of every admissible block equal the oracle's, computed from the
oracle's own trees."""
import numpy as np
import pytest

import oracle as orc
from paper_1706_09384_amd import workloads as W


@pytest.fixture(scope="module")
def hm():
    from paper_1706_09384_amd import hmat
    return hmat


@pytest.mark.parametrize("wl", ["sphere1k", "spheroid3k", "cube2k_T"])
def test_features_match_oracle(hm, wl):
    if wl == "sphere1k":
        w = W.plain_sphere_1k()
        X, N = w.points()
    elif wl == "spheroid3k":
        X, _ = W.prolate_spheroid(3000, seed=0)
        N = None
        w = W.Workload("spheroid3k", 3000, 0, omega=20.0, eps=1e-5, leaf=32)
    else:
        X, N = W.cube_surface(2000, seed=1)
        w = W.Workload("cube2k", 2000, 1, omega=1.1547, eps=1e-3, leaf=16)
    H = hm.build(X, normals=N, kernel=w.kernel, omega=w.omega, eta=w.eta, eps=w.eps, leaf=w.leaf,
                 plan_only=True)
    f, r = H.rank_samples()
    assert np.all(r == -1)
    tx = orc.cluster_tree(X, w.leaf)
    blocks = orc.block_tree(tx, tx, w.eta)
    ref = orc.rank_features(tx, tx, blocks, w.omega, w.eps)
    assert f.shape == ref.shape and f.shape[0] == H.info()["n_lowrank"]
    assert np.allclose(f, ref, rtol=2e-7, atol=1e-6)


def test_rank_target_is_log2():
    assert np.allclose(orc.rank_target([0, 3, 9, 21]), [0.0, 1.0, 2.0, 3.0])
