"""Host side of the collocation operator (Section 4) through the C ABI, no GPU:
the clusters and blocks on the mesh vertices equal the oracle's, and bad
meshes are rejected before any device work."""
import numpy as np
import pytest

from paper_1706_09384_amd import workloads as W


@pytest.fixture(scope="module")
def hm():
    from paper_1706_09384_amd import hmat
    return hmat


@pytest.mark.parametrize("level,leaf", [(3, 32), (4, 100)])
def test_blocks_on_vertices_equal_oracle(hm, orc, level, leaf):
    P, T = W.icosphere(level)
    H = hm.build_colloc(P, T, plan_only=True, leaf=leaf, eta=3.0)
    b, _, _ = H.export_blocklist()
    t = orc.cluster_tree(P, leaf)
    assert np.array_equal(H.export_tree(0)[0], t.perm)
    assert np.array_equal(b, orc.block_tree(t, t, 3.0))


def test_bad_meshes_are_rejected(hm):
    P, T = W.icosphere(2)
    cases = [
        (dict(kernel=1), P, T, "single-layer"),
        ({}, P, np.where(np.arange(T.size).reshape(T.shape) == 0, T[0, 1], T), "repeated vertex"),
        ({}, P, np.where(np.arange(T.size).reshape(T.shape) == 7, len(P), T), "out of range"),
        ({}, np.vstack([P, [[2.0, 2.0, 2.0]]]), T, "no element"),
        (dict(q_reg=0), P, T, "quadrature"),
        (dict(q_sing=33), P, T, "quadrature"),
    ]
    for kw, PP, TT, msg in cases:
        q = {k: kw.pop(k) for k in ("q_reg", "q_sing") if k in kw}
        with pytest.raises(RuntimeError, match=msg):
            hm.build_colloc(PP, TT, plan_only=True, **q, **kw)
