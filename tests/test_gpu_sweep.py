"""Frequency sweeps of the paper's Section 8 on Fibonacci spheres (C ABI, complex64).

* Fixed density (the (N, omega) pairs of Table table_corr, N_c = N / 3): the
  maximum recompressed rank grows like a power of omega near 1 (the paper's
  pre-asymptotic regime: linear in omega, O(N^(1/2)) in the DOFs), for the
  single-layer (U) and double-layer (T) kernels; every point meets 5 eps on
  sampled rows of the oracle's dense product.
* Fixed frequency (omega = 14, as in Section 7.2): the maximum recompressed
  rank stays flat as N grows.
The full table (to 985,818 DOFs) runs in bench.py --sweep-only.
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


def run_point(hm, orc, n, omega, kernel):
    import torch
    w = W.sweep_sphere(n, omega, kernel=kernel)
    X, N = w.points()
    H = hm.build_workload(w, X=X, N=N, prec=1)
    s = H.info()
    b = w.rhs()
    y = H.matvec(torch.from_numpy(b[:, 0]).cuda().to(torch.complex64)).cpu().numpy()
    rows = np.random.default_rng(7).choice(n, 32, replace=False)
    ref = orc.matvec_rows(orc.Problem.from_workload(w, X, N), b, rows)[:, 0]
    idx = (3 * rows[:, None] + np.arange(3)).ravel()
    e = float(np.linalg.norm(y.astype(np.complex128)[idx] - ref) / np.linalg.norm(ref))
    H.close()
    say(f"  {w.name}: max rank ACA {s['max_rank_aca']} recompressed {s['max_rank']}, "
        f"sampled e {e:.2e}")
    assert e <= 5 * w.eps
    assert s["n_capped"] == 0
    return s["max_rank"]


@pytest.mark.parametrize("kernel", [0, 1], ids=["U", "T"])
def test_fixed_density_rank_grows_with_frequency(hm, orc, kernel):
    pts = W.fixed_density_series()[:4]     # N_c = 2,562 .. 61,033, omega = 8.25 .. 40
    say(f"case fixed density kernel={kernel}")
    ranks = [run_point(hm, orc, n, om, kernel) for n, om in pts]
    assert all(b > a for a, b in zip(ranks, ranks[1:]))
    lw = np.log([om for _, om in pts])
    ln_ = np.log([3 * n for n, _ in pts])
    lr = np.log(ranks)
    p_w = float(np.polyfit(lw, lr, 1)[0])
    p_n = float(np.polyfit(ln_, lr, 1)[0])
    say(f"  exponents: rank ~ omega^{p_w:.2f}, rank ~ N^{p_n:.2f}")
    assert 0.5 <= p_w <= 1.2
    assert 0.25 <= p_n <= 0.6


@pytest.mark.parametrize("kernel", [0, 1], ids=["U", "T"])
def test_fixed_frequency_rank_is_flat(hm, orc, kernel):
    pts = [(n, 14.0) for n, _ in W.fixed_density_series()[:4]]
    say(f"case fixed frequency omega=14 kernel={kernel}")
    ranks = np.array([run_point(hm, orc, n, om, kernel) for n, om in pts], dtype=float)
    assert ranks.max() <= 1.25 * ranks.min()
