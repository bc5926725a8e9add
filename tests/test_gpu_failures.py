"""Failure paths of the C ABI on the GPU, forced from the host.

* HM_FAULT_ALLOC=k makes the k-th device allocation of the calling thread
  fail: every such build and GMRES call returns HM_ERR_ALLOC, leaves no
  handle, and after hm_release_cache the device holds no more memory than
  before the failed calls (nothing leaks on the error path);
* GMRES with a tiny iteration limit returns HM_ERR_NOCONV with its info
  filled in (iterations, residual) and the last iterate in x.
No kernel is made to fault: each failure is raised by host code.
"""
import os
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


def free_bytes(hm):
    import torch
    torch.cuda.synchronize()
    hm.release_cache()
    torch.cuda.empty_cache()
    return torch.cuda.mem_get_info()[0]


@pytest.mark.parametrize("prec", [1, 0], ids=["c64", "c128"])
def test_injected_allocation_failures_leak_nothing(hm, prec):
    import torch
    w = W.small_sphere(4000, omega=8.0, leaf=32, eps=1e-4)
    X, _ = w.points()
    Xt = torch.from_numpy(X).cuda()
    # one successful build first, so that lazily created runtime state exists
    H = hm.build_workload(w, X=X, prec=prec)
    b = torch.from_numpy(w.rhs()[:, 0]).cuda()
    x, info = H.gmres(b, tol=1e-6, restart=30, maxit=400, check=False)
    del x
    H.close()
    base = free_bytes(hm)
    failed = 0
    try:
        for k in range(1, 400):
            os.environ["HM_FAULT_ALLOC"] = str(k)
            try:
                hm.build(Xt, kernel=w.kernel, prec=prec, omega=w.omega, eps=w.eps, leaf=w.leaf,
                         self_re=w.self_re)
            except hm.HMError as e:
                assert e.status == hm.HM_ERR_ALLOC, str(e)
                assert "injected" in str(e)
                failed += 1
                continue
            say(f"prec={prec}: builds fail at allocations 1..{k - 1}, allocation {k} is past the last")
            break
        else:
            raise AssertionError("a build made 400 allocations")
    finally:
        os.environ.pop("HM_FAULT_ALLOC", None)
    assert failed >= 10
    after = free_bytes(hm)
    say(f"free before {base / 2**20:.1f} MiB, after {failed} failed builds {after / 2**20:.1f} MiB")
    assert after >= base - (8 << 20)
    # GMRES: allocations inside the solver fail cleanly too
    H = hm.build_workload(w, X=X, prec=prec)
    base = free_bytes(hm)
    gm_failed = 0
    try:
        for k in range(1, 40):
            os.environ["HM_FAULT_ALLOC"] = str(k)
            x, info = H.gmres(b, tol=1e-6, restart=30, maxit=60, check=False)
            if info["status"] == hm.HM_ERR_ALLOC:
                gm_failed += 1
                continue
            assert info["status"] in (hm.HM_OK, hm.HM_ERR_NOCONV), info
            break
    finally:
        os.environ.pop("HM_FAULT_ALLOC", None)
    del x
    assert gm_failed >= 1
    after = free_bytes(hm)
    say(f"gmres: {gm_failed} failed calls, free before {base / 2**20:.1f} MiB after "
        f"{after / 2**20:.1f} MiB")
    assert after >= base - (8 << 20)
    H.close()


def test_gmres_iteration_limit_reports_noconv(hm, orc):
    import torch
    w = W.plain_sphere_1k()
    X, _ = w.points()
    H = hm.build_workload(w, X=X, prec=0)
    b = w.rhs()[:, 0]
    x, info = H.gmres(torch.from_numpy(b).cuda(), tol=1e-10, restart=20, maxit=5, check=False)
    say("info", info)
    assert info["status"] == hm.HM_ERR_NOCONV
    assert 0 < info["iters"] <= 5 and info["converged"] == 0
    assert 1e-10 < info["relres"] < 1.0
    # x holds the last iterate: its residual is the one reported
    xh = x.cpu().numpy()
    r = H.residual(torch.from_numpy(b).cuda(), x).cpu().numpy()
    assert abs(np.linalg.norm(r) / np.linalg.norm(b) - info["relres"]) <= 1e-6 * info["relres"]
    assert np.all(np.isfinite(xh))
