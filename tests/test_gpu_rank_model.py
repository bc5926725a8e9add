"""Rank model on the GPU: the library's FP32 forward, backward and Adam kernels
against the oracle's FP64 MLP, training on samples of real builds, and the
rule that a prediction changes budgets and scheduling but never the factors."""
import sys

import numpy as np
import pytest

import oracle as orc
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


def unpack(w):
    """Packed float32 weights -> oracle parameter list (float64)."""
    w = np.asarray(w, np.float64)
    sizes = [(64, 6), (64,), (64, 64), (64,), (1, 64), (1,)]
    out, k = [], 0
    for sh in sizes:
        n = int(np.prod(sh))
        out.append(w[k:k + n].reshape(sh))
        k += n
    assert k == w.size
    return out


def pack(params):
    return np.concatenate([p.ravel() for p in params])


def synthetic_samples(n, seed):
    """Feature ranges of real blocks: log sizes, kappa*diam, kappa*dist, log10 eps."""
    rng = np.random.default_rng(seed)
    f = np.stack([rng.uniform(2.5, 7.5, n), rng.uniform(2.5, 7.5, n), rng.uniform(0.5, 40, n),
                  rng.uniform(0.5, 40, n), rng.uniform(1.0, 120, n),
                  rng.choice([-3.0, -4.0, -5.0], n)], axis=1)
    t = rng.uniform(0.0, 7.0, n)
    return f.astype(np.float32), t.astype(np.float32)


@pytest.mark.parametrize("n", [1, 200, 1000])
def test_grad_matches_oracle(hm, n):
    import torch
    say(f"case mlp grad n={n}")
    w = hm.rank_model_init(seed=3)
    f, t = synthetic_samples(n, seed=4)
    loss, g = hm.rank_model_grad(w, torch.from_numpy(f).cuda(), torch.from_numpy(t).cuda())
    P = unpack(w)
    lref, gref = orc.mlp_loss_grad(P, f.astype(np.float64), t.astype(np.float64))
    gref = pack(gref)
    say("loss", loss, lref, "grad rel", np.linalg.norm(g - gref) / np.linalg.norm(gref))
    assert abs(loss - lref) <= 1e-5 * abs(lref)
    assert np.linalg.norm(g - gref) <= 1e-4 * np.linalg.norm(gref)
    # every parameter group, not just the dominant one
    k = 0
    for p in gref_split(gref):
        seg = g[k:k + p.size]
        if np.linalg.norm(p) > 0:
            assert np.linalg.norm(seg - p) <= 1e-4 * np.linalg.norm(p) + 1e-7
        k += p.size


def gref_split(gvec):
    sizes = [384, 64, 4096, 64, 64, 1]
    out, k = [], 0
    for s in sizes:
        out.append(gvec[k:k + s])
        k += s
    return out


def test_forward_matches_oracle(hm):
    import torch
    say("case mlp forward")
    w = hm.rank_model_init(seed=5)
    f, _ = synthetic_samples(777, seed=6)
    y = hm.rank_model_predict(w, torch.from_numpy(f).cuda()).cpu().numpy()
    ref, _ = orc.mlp_forward(unpack(w), f.astype(np.float64))
    assert np.abs(y - ref).max() <= 1e-5 * max(1.0, np.abs(ref).max())


def test_one_adam_step_matches_oracle(hm):
    say("case mlp adam step")
    w = hm.rank_model_init(seed=7)
    f, _ = synthetic_samples(200, seed=8)
    ranks = np.random.default_rng(9).integers(0, 300, 200).astype(np.int32)
    lr = 1e-3
    w1, loss = hm.rank_model_train(f, ranks, w, epochs=1, batch=256, lr=lr, seed=1)
    P = unpack(w)
    t = orc.rank_target(ranks)
    _, G = orc.mlp_loss_grad(P, f.astype(np.float64), t)
    zeros = [np.zeros_like(p) for p in P]
    P1, _, _ = orc.adam_step(P, G, zeros, zeros, 1, lr=lr)
    d = pack(P1) - pack(P)
    dg = w1.astype(np.float64) - w.astype(np.float64)
    g = np.abs(pack(G))
    big = g >= 1e-3 * g.max()
    # first Adam step moves each weight by about lr * sign(g)
    assert np.abs(dg[big] - d[big]).max() <= 1e-2 * lr
    assert np.abs(dg - d).max() <= 2 * lr


@pytest.fixture(scope="module")
def samples(hm):
    """(features, ACA ranks) of the 1k sphere (complex128) and a 6k sphere at three tolerances."""
    fs, rs = [], []
    w = W.plain_sphere_1k()
    X, _ = w.points()
    H = hm.build_workload(w, X=X, prec=0)
    f, r = H.rank_samples()
    fs.append(f); rs.append(r)
    for eps in (1e-3, 1e-4, 1e-5):
        w = W.small_sphere(6000, omega=14.0, leaf=32, eps=eps)
        X, _ = w.points()
        H = hm.build_workload(w, X=X, prec=1)
        f, r = H.rank_samples()
        fs.append(f); rs.append(r)
    return np.concatenate(fs), np.concatenate(rs)


def test_training_learns_ranks(hm, samples):
    f, r = samples
    say(f"case mlp training on {r.size} samples")
    assert np.all(r >= 0)
    w0 = hm.rank_model_init(seed=0)
    w, loss = hm.rank_model_train(f, r, w0, epochs=150, batch=256, lr=1e-3, seed=0)
    say("loss first/last", loss[0], loss[-1])
    assert np.all(np.isfinite(loss))
    assert loss[-1] < 0.2 * loss[0]
    pred, _ = orc.mlp_forward(unpack(w), f.astype(np.float64))
    err = np.abs(pred - orc.rank_target(r))
    say("median |log2 error| of (1 + r/3)", np.median(err))
    assert np.median(err) < 0.5


def test_model_changes_budgets_not_factors(hm, samples):
    """A prediction sizes first budgets and orders the work; every factor stays bit-identical."""
    f, r = samples
    say("case model invariance")
    w, _ = hm.rank_model_train(f, r, hm.rank_model_init(seed=0), epochs=60, batch=256, seed=0)
    wl = W.small_sphere(4000, omega=11.0, leaf=32, eps=1e-4)
    X, _ = wl.points()
    H0 = hm.build_workload(wl, X=X, prec=1)
    H1 = hm.build_workload(wl, X=X, prec=1, rank_model=w)
    s0, s1 = H0.info(), H1.info()
    say("hits", s1["n_model_hits"], "of", s1["n_lowrank"], "overflow", s0["n_overflow"], s1["n_overflow"],
        "scratch", s0["aca_scratch_bytes"], s1["aca_scratch_bytes"])
    assert s1["n_model_hits"] > 0 and s0["n_model_hits"] == 0
    # what the model gains over the size rule: no more re-runs, less first-pass scratch
    assert s1["n_overflow"] <= s0["n_overflow"]
    assert s1["aca_scratch_bytes"] < 0.8 * s0["aca_scratch_bytes"]
    b0, r0, a0 = H0.export_blocklist()
    b1, r1, a1 = H1.export_blocklist()
    assert np.array_equal(b0, b1) and np.array_equal(r0, r1) and np.array_equal(a0, a1)
    n0 = H0.export_tree(0)[1]
    n1 = H1.export_tree(0)[1]
    assert np.array_equal(n0, n1)
    for k in range(b0.shape[0]):
        d0, d1 = H0.export_block(k, b0, r0, n0, n0), H1.export_block(k, b1, r1, n1, n1)
        if isinstance(d0, tuple):
            assert all(np.array_equal(u, v) for u, v in zip(d0, d1)), k
        else:
            assert np.array_equal(d0, d1), k


def test_spheroid50k_with_model_sampled_rows(hm, samples):
    """The rank model's evaluation workload (50,000-point prolate spheroid) built with
    predicted budgets stays within 5 eps of the oracle on sampled rows."""
    import torch
    f, r = samples
    w = W.learned_spheroid_50k()
    say(f"case {w.name} with rank model")
    wts, _ = hm.rank_model_train(f, r, hm.rank_model_init(seed=0), epochs=100, batch=256, seed=0)
    X, _ = w.points()
    H = hm.build_workload(w, X=X, prec=1, rank_model=wts)
    s = H.info()
    say({k: s[k] for k in ("n_lowrank", "n_model_hits", "n_overflow", "aca_scratch_bytes", "t_aca",
                           "t_total")})
    assert s["n_capped"] == 0   # every block met its stopping test below the rank cap
    assert s["n_model_hits"] > 0.9 * s["n_lowrank"]
    b = w.rhs()
    y = H.matvec(torch.from_numpy(b).cuda().to(torch.complex64)).cpu().numpy().astype(np.complex128)
    rows = np.random.default_rng(0).choice(w.n_points, 256, replace=False)
    pb = orc.Problem.from_workload(w, X)
    ref = orc.matvec_rows(pb, b, rows)
    idx = (3 * rows[:, None] + np.arange(3)).ravel()
    e = float(np.linalg.norm(y[idx] - ref) / np.linalg.norm(ref))
    say("sampled e", e)
    assert e <= 5 * w.eps
