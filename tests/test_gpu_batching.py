"""Batching pattern: graph-captured matvec, per-block (unbatched) assembly as the
baseline of the batched default, the matvec autotuner, and the 100k cube workload."""
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


def same_blocks(H0, H1):
    b0, r0, a0 = H0.export_blocklist()
    b1, r1, a1 = H1.export_blocklist()
    assert np.array_equal(b0, b1) and np.array_equal(r0, r1) and np.array_equal(a0, a1)
    n0, n1 = H0.export_tree(0)[1], H1.export_tree(0)[1]
    for k in range(b0.shape[0]):
        d0, d1 = H0.export_block(k, b0, r0, n0, n0), H1.export_block(k, b1, r1, n1, n1)
        if isinstance(d0, tuple):
            assert all(np.array_equal(u, v) for u, v in zip(d0, d1)), k
        else:
            assert np.array_equal(d0, d1), k


@pytest.mark.parametrize("prec,nrhs", [(0, 1), (1, 1), (1, 64), (1, 3)])
def test_graph_replays_match_eager(hm, prec, nrhs):
    """Every replay of the captured matvec equals the eager product on the same input,
    with eager work (new inputs written into the captured buffer) between replays."""
    import torch
    say(f"case graph prec={prec} nrhs={nrhs}")
    w = W.plain_sphere_1k()
    X, _ = w.points()
    He = hm.build_workload(w, X=X, prec=prec)
    Hg = hm.build_workload(w, X=X, prec=prec, matvec_graph=True)
    dt = He.complex_dtype
    xg = torch.zeros((3 * w.n_points, nrhs), dtype=dt, device="cuda")
    yg = torch.empty_like(xg)
    for k in range(4):
        xn = torch.from_numpy(W.complex_normal(3 * w.n_points, nrhs, seed=20 + k)).cuda().to(dt)
        xg.copy_(xn)                       # eager work between replays
        Hg.matvec(xg, yg)                  # first call captures, the rest replay
        ye = He.matvec(xn)
        torch.cuda.synchronize()
        assert torch.equal(yg, ye), k
    # a new output buffer re-captures
    y2 = torch.empty_like(yg)
    Hg.matvec(xg, y2)
    torch.cuda.synchronize()
    assert torch.equal(y2, yg)


@pytest.mark.parametrize("which", ["sphere_c64", "cube_T_c64", "sphere_c128", "bigrank_c64",
                                   "bigrank_c128"])
def test_unbatched_assembly_is_bit_identical(hm, which):
    """Per-block launches run the same kernels on the same blocks: identical factors.
    The bigrank cases have ACA ranks above 100, whose cores the batched build
    factorises with one launch per Jacobi round over many workgroups, and the
    per-block build inside one workgroup."""
    say(f"case unbatched {which}")
    if which == "cube_T_c64":
        P, Nrm = W.cube_surface(2000, seed=3)
        w = W.Workload("cube2k", 2000, 1, omega=1.1547, eps=1e-4, leaf=32,
                       self_re=W._t_self(W.CUBE_AREA, 2000), geometry="cube")
        X, N, prec = P, Nrm, 1
    elif which.startswith("bigrank"):
        w = W.small_sphere(4000, omega=25.0, leaf=32, eps=1e-4)
        X, _ = w.points()
        N, prec = None, (1 if which.endswith("c64") else 0)
    else:
        w = W.small_sphere(1500, omega=7.0, leaf=24, eps=1e-5)
        X, _ = w.points()
        N, prec = None, (1 if which == "sphere_c64" else 0)
    H0 = hm.build_workload(w, X=X, N=N, prec=prec)
    if which.startswith("bigrank"):
        say("max ACA rank", H0.info()["max_rank_aca"])
        assert H0.info()["max_rank_aca"] > 100
    H1 = hm.build_workload(w, X=X, N=N, prec=prec, unbatched=True)
    same_blocks(H0, H1)


@pytest.mark.skip(reason="the persistent form of the one-workgroup ACA stopped making progress on its "
                         "first GPU run (complex128, 6,000-point sphere) and was taken out of the "
                         "library: no cause was found by reading it, so it stays off the GPU")
@pytest.mark.parametrize("prec", [0, 1])
def test_persistent_aca_is_bit_identical(hm, monkeypatch, prec):
    """The persistent form of the one-workgroup ACA (a grid of one workgroup per CU
    taking blocks from an atomic counter, selected by HM_ACA_PERSISTENT=1) would run
    the same steps on every block as the dispatcher-fed launch: identical factors.
    Also the collocation operator."""
    say(f"case persistent ACA prec {prec}")
    w = W.small_sphere(6000, omega=12.0, leaf=32, eps=1e-5)
    X, _ = w.points()
    H0 = hm.build_workload(w, X=X, prec=prec)
    monkeypatch.setenv("HM_ACA_PERSISTENT", "1")
    H1 = hm.build_workload(w, X=X, prec=prec)
    same_blocks(H0, H1)
    P, T = W.icosphere(3)
    monkeypatch.delenv("HM_ACA_PERSISTENT")
    C0 = hm.build_colloc(P, T, omega=3.0, leaf=16, prec=prec)
    monkeypatch.setenv("HM_ACA_PERSISTENT", "1")
    C1 = hm.build_colloc(P, T, omega=3.0, leaf=16, prec=prec)
    same_blocks(C0, C1)


def test_autotune_changes_shape_not_result(hm, orc):
    import torch
    say("case autotune sphere20k")
    w = W.precision_sphere_20k(1e-4)
    X, _ = w.points()
    H = hm.build_workload(w, X=X, prec=1)
    b = torch.from_numpy(w.rhs()[:, 0]).cuda().to(torch.complex64)
    y0 = H.matvec(b).cpu().numpy()
    table = H.autotune(reps=5)
    s = H.info()
    say("table ms\n", table, "chosen", s["acc_waves"], s["proj_rows"])
    assert np.all(table > 0)
    assert s["acc_waves"] in (4, 8, 16) and s["proj_rows"] in (256, 512, 1024)
    y1 = H.matvec(b).cpu().numpy()
    assert rel(y1, y0) <= 2e-6


@pytest.mark.parametrize("leaf", [32, 64])
def test_cube100k_T_sampled_rows(hm, orc, leaf):
    """The batching workload: 100,000 points on the cube surface, T kernel, complex64,
    autotuned graph matvec, checked on sampled rows."""
    import torch
    w = W.batching_cube_100k(leaf)
    say(f"case {w.name}")
    X, N = w.points()
    H = hm.build_workload(w, X=X, N=N, prec=1, matvec_graph=True)
    H.autotune(reps=3)
    s = H.info()
    say({k: s[k] for k in ("n_lowrank", "max_rank_aca", "max_rank", "n_fallback", "n_overflow",
                           "t_total", "acc_waves", "proj_rows")})
    assert s["n_capped"] == 0   # every block met its stopping test below the rank cap
    b = w.rhs()
    y = H.matvec(torch.from_numpy(b[:, 0]).cuda().to(torch.complex64)).cpu().numpy()
    rows = np.random.default_rng(0).choice(w.n_points, 256, replace=False)
    ref = orc.matvec_rows(orc.Problem.from_workload(w, X, N), b[:, :1], rows)[:, 0]
    idx = (3 * rows[:, None] + np.arange(3)).ravel()
    e = rel(y.astype(np.complex128)[idx], ref)
    say("sampled e", e)
    assert e <= 5 * w.eps


@pytest.mark.parametrize("prec", [0, 1])
def test_chunked_assembly_is_bit_identical(hm, prec):
    """A tiny scratch cap splits the admissible blocks into many chunks; every factor is
    the same as in the single-chunk build."""
    say(f"case chunked prec={prec}")
    w = W.small_sphere(4000, omega=11.0, leaf=32, eps=1e-4)
    X, _ = w.points()
    H0 = hm.build_workload(w, X=X, prec=prec)
    H1 = hm.build_workload(w, X=X, prec=prec, aca_scratch_mb=2)
    s0, s1 = H0.info(), H1.info()
    say("chunks", s0["aca_chunks"], s1["aca_chunks"])
    assert s0["aca_chunks"] == 1 and s1["aca_chunks"] > 4
    same_blocks(H0, H1)


@pytest.mark.parametrize("which,prec", [("sphere12k", 0), ("sphere12k", 1), ("sphere20k", 1),
                                        ("cube12k_T", 1)])
def test_overflow_resume_is_bit_identical(hm, which, prec):
    """A block that outgrows its first column budget continues from where it
    stopped with a larger one: with a first budget of 12 (many blocks resume
    several times, on the split and the one-workgroup path) the factors equal
    those of a build whose first budget is never exceeded.  On the 20k sphere
    the split blocks hold enough points for their ACA to run beside the other
    blocks' recompression; on the planar faces of the cube many steps take
    the pseudo-inverse fallback, whose V update can still be open when a
    block reaches its budget."""
    import torch
    say(f"case overflow resume {which} prec={prec}")
    N = None
    if which == "cube12k_T":
        X, N = W.cube_surface(12000, seed=5)
        w = W.Workload("cube12k", 12000, 1, omega=2.0, eps=1e-4, leaf=32,
                       self_re=W._t_self(W.CUBE_AREA, 12000), geometry="cube")
    else:
        w = (W.small_sphere(12000, omega=19.4, leaf=32, eps=1e-4) if which == "sphere12k"
             else W.precision_sphere_20k(1e-4))
        X, _ = w.points()
    H0 = hm.build_workload(w, X=X, N=N, prec=prec, rank_budget=600)
    H1 = hm.build_workload(w, X=X, N=N, prec=prec, rank_budget=12)
    s0, s1 = H0.info(), H1.info()
    say("overflow", s0["n_overflow"], s1["n_overflow"], "max ACA rank", s0["max_rank_aca"],
        "fallbacks", s0["n_fallback"])
    assert s0["n_overflow"] == 0 and s1["n_overflow"] > 100
    if which == "cube12k_T":
        assert s0["n_fallback"] > 0 and s1["n_fallback"] == s0["n_fallback"]
    b0, r0, a0 = H0.export_blocklist()
    b1, r1, a1 = H1.export_blocklist()
    assert np.array_equal(b0, b1) and np.array_equal(r0, r1) and np.array_equal(a0, a1)
    nx, ny = H0.export_tree(0)[1], H0.export_tree(1)[1]
    pts = (nx[b0[:, 0], 1] - nx[b0[:, 0], 0]) + (ny[b0[:, 1], 1] - ny[b0[:, 1], 0])
    lowrank = np.flatnonzero(b0[:, 2] == 1)
    big = lowrank[pts[lowrank] >= 1500]
    resumed = lowrank[a0[lowrank] > 12]
    say("split blocks", big.size, "resumed blocks", resumed.size)
    assert big.size > 0
    if which == "cube12k_T":
        # coplanar cube faces: some split blocks converge within the first 12 columns
        assert np.any(a0[big] > 12)
    else:
        assert np.all(a0[big] > 12)
    rng = np.random.default_rng(5)
    pick = np.concatenate([big, rng.choice(resumed, min(200, resumed.size), replace=False)])
    for k in pick:
        d0 = H0.export_block(int(k), b0, r0, nx, ny)
        d1 = H1.export_block(int(k), b1, r1, nx, ny)
        assert all(np.array_equal(u, v) for u, v in zip(d0, d1)), int(k)
    dt = H0.complex_dtype
    x = torch.from_numpy(W.complex_normal(3 * w.n_points, 1, seed=9)[:, 0]).cuda().to(dt)
    assert torch.equal(H0.matvec(x), H1.matvec(x))
