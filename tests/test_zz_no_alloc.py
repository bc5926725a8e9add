"""The allocation-free product hm_matvec_noalloc against hm_matvec (C ABI).

For callers that cannot allocate: the product with its work vectors in the
library's fixed device array.  Two calls in a row on one GPU, the second on a
smaller matrix, each compared with hm_matvec on the same matrix and input
(the same kernels in the same order: equal bit for bit) and with the FP64
dense oracle product (5 eps).  Complex64 and complex128 operators, one and
three right-hand-side columns.
"""
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


@pytest.mark.parametrize("prec", [1, 0], ids=["c64", "c128"])
def test_noalloc_matches_matvec_two_calls(hm, orc, prec):
    import torch
    dt = torch.complex64 if prec == 1 else torch.complex128
    for n, nrhs in ((3000, 1), (1200, 3)):
        say(f"case noalloc prec={prec} N={n} nrhs={nrhs}")
        w = W.small_sphere(n, omega=8.0, leaf=32, eps=1e-4)
        X, _ = w.points()
        H = hm.build_workload(w, X=X, prec=prec)
        b = w.rhs(nrhs)
        xb = torch.from_numpy(np.ascontiguousarray(b)).cuda().to(dt)
        y_ref = H.matvec(xb) if nrhs == 1 else torch.stack(
            [H.matvec(xb[:, c].contiguous()) for c in range(nrhs)], dim=1)
        y = torch.full((3 * n, nrhs), float("nan"), dtype=dt, device="cuda")
        H.matvec_noalloc(xb, y)
        torch.cuda.synchronize()
        got = y.cpu().numpy()
        ref = y_ref.reshape(3 * n, nrhs).cpu().numpy()
        assert np.array_equal(got, ref), float(np.max(np.abs(got - ref)))
        A = orc.dense(orc.Problem.from_workload(w, X))
        exact = A @ b
        for c in range(nrhs):
            e = np.linalg.norm(got[:, c] - exact[:, c]) / np.linalg.norm(exact[:, c])
            say(f"  column {c}: rel err vs oracle {e:.3e}")
            assert e <= 5 * w.eps
        H.close()


def test_noalloc_rejects_bad_arguments(hm):
    import torch
    w = W.small_sphere(400, omega=5.6, leaf=16)
    X, _ = w.points()
    H = hm.build_workload(w, X=X, prec=1)
    x = torch.zeros(3 * 400, 1, dtype=torch.complex64, device="cuda")
    y = torch.zeros(3 * 400, 1, dtype=torch.complex64, device="cuda")
    rc = hm.LIB.hm_matvec_noalloc(H._h, hm._ptr(x), hm._ptr(y), 0, hm._stream(None))
    assert rc == hm.HM_ERR_ARG
    rc = hm.LIB.hm_matvec_noalloc(H._h, None, hm._ptr(y), 1, hm._stream(None))
    assert rc == hm.HM_ERR_ARG
    P = hm.build_workload(w, device=None, X=X, plan_only=True)
    rc = hm.LIB.hm_matvec_noalloc(P._h, hm._ptr(x), hm._ptr(y), 1, hm._stream(None))
    assert rc == hm.HM_ERR_STATE
