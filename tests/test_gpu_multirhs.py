"""Multi-RHS panels (complex64 operators, FP32 matrix-core products) against the
oracle and against the one-column path, through the C ABI.

Gates, per right-hand side column c (relative 2-norm):
* panel product vs the one-column product of the same operator: <= 2e-6
  (both FP32 accumulations of the same stored factors, different order);
* panel product vs the oracle's re-application of the exported operator to
  the complex64-rounded input: <= 1e-5;
* panel product vs the dense oracle product: <= 5 eps + C64_FLOOR.

C64_FLOOR is the complex64 allowance: the all-dense (eta = 0) product of a
complex64 operator, which has no approximation error at all, already differs
from the FP64 oracle by up to 2e-6 (float32 kernel evaluation, storage and
accumulation); the gate adds 1.5 times that floor to 5 eps.
"""
C64_FLOOR = 3e-6
import sys

import numpy as np
import pytest

from paper_1706_09384_amd import workloads as W

pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def hm():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    from paper_1706_09384_amd import hmat
    return hmat


def to_dev(a, dtype=None):
    import torch
    t = torch.from_numpy(np.ascontiguousarray(a)).cuda()
    return t if dtype is None else t.to(dtype)


def colrel(a, b):
    return np.linalg.norm(a - b, axis=0) / np.linalg.norm(b, axis=0)


def export_all(A):
    blocks, rank, _ = A.export_blocklist()
    _, nx, _ = A.export_tree(0)
    _, ny, _ = A.export_tree(1)
    out = []
    for b in range(blocks.shape[0]):
        t, s, k = blocks[b]
        data = A.export_block(b, blocks, rank, nx, ny)
        if k == 0:
            data = data.astype(np.complex128)
        else:
            data = (data[0].astype(np.complex128), data[1].astype(np.complex128))
        out.append((int(t), int(s), int(k), data))
    return out


class _T:
    def __init__(self, perm, nodes):
        self.perm = perm.astype(np.int64)
        self.begin = nodes[:, 0]
        self.end = nodes[:, 1]


def check_panels(hm, orc, H, A, B, eps, tol_dense):
    import torch
    Y = H.matvec(to_dev(B, torch.complex64)).cpu().numpy().astype(np.complex128)
    cols = np.stack([H.matvec(to_dev(np.ascontiguousarray(B[:, c]), torch.complex64)).cpu().numpy()
                     for c in range(B.shape[1])], axis=1).astype(np.complex128)
    d1 = colrel(Y, cols).max()
    p0, n0, _ = H.export_tree(0)
    p1, n1, _ = H.export_tree(1)
    Bq = B.astype(np.complex64).astype(np.complex128)
    Yo = orc.hmatvec(export_all(H), _T(p0, n0), _T(p1, n1), Bq)
    d2 = colrel(Y, Yo).max()
    d3 = colrel(Y, A @ B).max()
    say(f"panel vs columns {d1:.2e}, vs oracle re-apply {d2:.2e}, vs dense {d3:.2e}")
    assert d1 <= 2e-6
    assert d2 <= 1e-5
    assert d3 <= tol_dense
    return Y


@pytest.fixture(scope="module")
def sphere1k(orc):
    w = W.plain_sphere_1k()
    X, _ = w.points()
    pb = orc.Problem.from_workload(w, X)
    return w, X, orc.dense(pb)


@pytest.mark.parametrize("nrhs", [8, 64, 70, 130])
def test_panels_sphere1k(hm, orc, sphere1k, nrhs):
    """One full panel, a panel plus a ragged one, three panels."""
    w, X, A = sphere1k
    say(f"case multirhs sphere1k nrhs={nrhs}")
    H = hm.build_workload(w, X=X, prec=1)
    B = W.complex_normal(3 * w.n_points, nrhs, seed=7)
    check_panels(hm, orc, H, A, B, w.eps, 5 * w.eps + C64_FLOOR)


@pytest.mark.parametrize("kernel,n,leaf,omega", [(1, 513, 5, 9.0), (0, 97, 7, 0.5), (1, 300, 40, 3.0)])
def test_panels_small_ragged(hm, orc, kernel, n, leaf, omega):
    """Tiles of 15..120 rows (partial 16-row groups), both kernels."""
    say(f"case multirhs small kernel={kernel} n={n} leaf={leaf}")
    w = W.small_sphere(n, kernel=kernel, omega=omega, leaf=leaf, eps=1e-5)
    X, N = w.points()
    pb = orc.Problem.from_workload(w, X, N)
    A = orc.dense(pb)
    H = hm.build_workload(w, X=X, N=N, prec=1)
    B = W.complex_normal(3 * n, 24, seed=8)
    check_panels(hm, orc, H, A, B, w.eps, 5 * w.eps + C64_FLOOR)


def test_panels_two_clouds(hm, orc):
    say("case multirhs two clouds")
    X = W.fibonacci_sphere(400)
    Y = W.uniform_ball(300, seed=2) * 0.6 + np.array([2.2, 0.0, 0.1])
    pb = orc.Problem(0, X, Y, None, 4.0, same=False)
    A = orc.dense(pb)
    H = hm.build(to_dev(X), to_dev(Y), kernel=0, omega=4.0, leaf=16, eps=1e-5, prec=1)
    B = W.complex_normal(900, 16, seed=9)
    check_panels(hm, orc, H, A, B, 1e-5, 5e-5 + C64_FLOOR)


def test_panels_single_point(hm, orc):
    say("case multirhs n=1")
    w = W.small_sphere(1, leaf=3)
    X, _ = w.points()
    pb = orc.Problem.from_workload(w, X)
    A = orc.dense(pb)
    H = hm.build_workload(w, X=X, prec=1)
    B = W.complex_normal(3, 9, seed=10)
    check_panels(hm, orc, H, A, B, 1e-4, C64_FLOOR)


@pytest.mark.parametrize("nrhs", [4, 12])
def test_lockstep_gmres_on_panels(hm, orc, sphere1k, nrhs):
    """Several right-hand sides share each panel product of the inner complex64 GMRES.
    With 4 columns the Gram-Schmidt dots reduce per column inside a wave (4 divides 64);
    with 12 they take the per-block fallback."""
    w, X, A = sphere1k
    say(f"case multirhs gmres {nrhs} rhs")
    H = hm.build_workload(w, X=X, prec=1)
    B = W.complex_normal(3 * w.n_points, nrhs, seed=11)
    x, info = H.gmres(to_dev(B), tol=1e-8, restart=50, maxit=6000)
    say("gmres", info)
    assert info["converged"] == nrhs
    x = x.cpu().numpy()
    p0, n0, _ = H.export_tree(0)
    p1, n1, _ = H.export_tree(1)
    R = B - orc.hmatvec(export_all(H), _T(p0, n0), _T(p1, n1), x)
    assert (np.linalg.norm(R, axis=0) / np.linalg.norm(B, axis=0)).max() <= 1.5e-8


def test_sphere200k_T_64rhs_sampled_rows(hm, orc):
    """The full multi-RHS workload: 200,000 points, T kernel, 64 right-hand sides,
    checked on 64 sampled rows for every right-hand side."""
    import torch
    w = W.multirhs_sphere_200k()
    say(f"case {w.name}")
    X, N = w.points()
    H = hm.build_workload(w, X=X, N=N, prec=1)
    s = H.info()
    say({k: s[k] for k in ("n_lowrank", "max_rank", "n_overflow", "n_fallback", "storage_bytes",
                           "t_total")})
    assert s["n_capped"] == 0   # every block met its stopping test below the rank cap
    B = w.rhs()
    assert B.shape == (3 * w.n_points, 64)
    Y = H.matvec(to_dev(B, torch.complex64)).cpu().numpy().astype(np.complex128)
    rows = np.random.default_rng(0).choice(w.n_points, 64, replace=False)
    pb = orc.Problem.from_workload(w, X, N)
    ref = orc.matvec_rows(pb, B, rows)
    idx = (3 * rows[:, None] + np.arange(3)).ravel()
    e = colrel(Y[idx], ref)
    say("sampled e max", e.max())
    assert e.max() <= 5 * w.eps


def test_lockstep_gmres_T_sphere_64rhs(hm, orc):
    """The 200k T sphere's recipe (T kernel, n = x, leaf 64, eps 1e-4, 64 right-hand
    sides, FP64 refinement to 1e-8) scaled to the largest size whose unpreconditioned
    GMRES converges in a test's time: 20,000 points with kappa_s = 56 sqrt(20000 / 200000)
    = 17.7.  Every column reaches 1e-8 in FP64 against A_H, and the sampled rows of the
    oracle's exact operator give a backward error of order eps."""
    import math
    import torch
    n = 20000
    ks = 56.0 * math.sqrt(n / 200000)
    w = W.small_sphere(n, kernel=1, omega=ks, leaf=64, eps=1e-4)
    say(f"case lockstep GMRES T sphere n={n} kappa_s={ks:.2f} 64 RHS")
    X, N = w.points()
    H = hm.build_workload(w, X=X, N=N, prec=1)
    B = W.complex_normal(3 * n, 64, seed=0)
    x, info = H.gmres(to_dev(B), tol=1e-8, restart=30, maxit=4000)
    say("gmres", info)
    assert info["converged"] == 64 and info["relres"] <= 1e-8
    rows = np.random.default_rng(4).choice(n, 24, replace=False)
    Ax = orc.matvec_rows(orc.Problem.from_workload(w, X, N), x.cpu().numpy(), rows)
    idx = (3 * rows[:, None] + np.arange(3)).ravel()
    be = np.linalg.norm(B[idx] - Ax, axis=0) / np.linalg.norm(B[idx], axis=0)
    say(f"backward error vs the exact operator on sampled rows: max {be.max():.2e}")
    assert be.max() <= 10 * w.eps
