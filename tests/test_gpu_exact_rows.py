"""hm_exact_rows (sampled rows of the exact operator, FP64) against the oracle's
rows: point U with self blocks, point T with normals, two distinct clouds,
complex64 operators (the reference stays FP64), the collocation operator, and
argument errors.  Gate: 1e-12 relative (both sides evaluate the same entries in
FP64, summed in different orders)."""
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


def rel(a, b):
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


def check(H, ref_fn, n_cols_pts, nrhs, seed=0):
    import torch
    x = W.complex_normal(3 * n_cols_pts, nrhs, seed=seed)
    rows = np.random.default_rng(seed).choice(H.nx, 40, replace=False)
    y = H.exact_rows(rows, torch.from_numpy(x).cuda()).cpu().numpy()
    ref = ref_fn(x, rows)
    e = rel(y, ref.reshape(y.shape))
    say("exact rows vs oracle", e)
    assert e <= 1e-12


@pytest.mark.parametrize("prec", [0, 1])
@pytest.mark.parametrize("nrhs", [1, 5])
def test_point_u_with_self_blocks(hm, orc, prec, nrhs):
    w = W.small_sphere(5000, leaf=32)
    say(f"case exact rows U sphere5000 prec {prec} nrhs {nrhs}")
    X, _ = w.points()
    H = hm.build_workload(w, X=X, prec=prec)
    pb = orc.Problem.from_workload(w, X)
    check(H, lambda x, rows: orc.matvec_rows(pb, x, rows), w.n_points, nrhs)


def test_point_t_with_normals_and_many_rhs(hm, orc):
    w = W.small_sphere(3000, kernel=W.KERNEL_T, leaf=32)
    say("case exact rows T sphere3000 nrhs 64")
    X, N = w.points()
    H = hm.build_workload(w, X=X, N=N)
    pb = orc.Problem.from_workload(w, X, N)
    check(H, lambda x, rows: orc.matvec_rows(pb, x, rows), w.n_points, 64, seed=2)


def test_two_clouds(hm, orc):
    import torch
    say("case exact rows two clouds")
    X = W.uniform_ball(700, seed=1)
    Y = W.uniform_ball(9000, seed=2) + np.array([3.0, 0.0, 0.0])
    H = hm.build(torch.from_numpy(X).cuda(), torch.from_numpy(Y).cuda(), omega=2.0, leaf=16)
    pb = orc.Problem(0, X, Y, None, 2.0, same=False)
    check(H, lambda x, rows: orc.matvec_rows(pb, x, rows), 9000, 3, seed=3)


def test_collocation_operator(hm):
    from oracle import bem
    P, T = W.icosphere(3)
    say("case exact rows collocation level 3")
    H = hm.build_colloc(P, T, omega=3.0, leaf=32)
    check(H, lambda x, rows: bem.apply_rows(P, T, x[:, 0], rows, 3.0), P.shape[0], 1, seed=4)


def test_argument_errors(hm):
    import torch
    w = W.small_sphere(500, leaf=32)
    X, _ = w.points()
    H = hm.build_workload(w, X=X)
    x = torch.zeros(3 * 500, dtype=torch.complex128, device="cuda")
    with pytest.raises(RuntimeError, match="out of range"):
        H.exact_rows([0, 500], x)
    with pytest.raises(RuntimeError, match="nrhs"):
        H.exact_rows([0], torch.zeros((3 * 500, 257), dtype=torch.complex128, device="cuda"))
