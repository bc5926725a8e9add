"""Benchmark of the H-matrix hot path on one MI355X.

Workload: 20,000 Fibonacci points on the unit sphere, U kernel, kappa_s = 25,
lambda = 2, mu = rho = 1, leaf 32, eta = 3, eps = 1e-4, complex64 storage and
compute with FP64 ACA norms / recompression / refinement (the precision form).
Inputs are synthetic (seeded); points are resident in HBM before timing.

A step is one pass of the hot path: hm_build (cluster tree, block tree,
near-field tiles, vector ACA, recompression, matvec plan) followed by one
hm_matvec.  The reported value is the H-matvec throughput in GB/s of
algorithmic bytes (stored factors + one read of x + one write of y), median
of 50 timed matvecs after 5 warm-ups, in the launch shape hm_autotune picks;
assembly seconds, GMRES, the plain
complex128 form and the CPU oracle baseline are reported beside it.

Usage: python bench.py [--gpus 1] [--steps K] [--warmup W] [--no-cpu] [--no-fp64]
"""
import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "H-assembly s + H-matvec GB/s (3N_c unknowns) vs plain FP64 GPU at 5eps rel err"
HBM_PEAK_GBPS = 8000.0
FP32_MFMA_PEAK_TFLOPS = 157.3


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def timed_matvecs(H, x, reps=50, warm=5):
    import torch
    y = torch.empty_like(x)
    for _ in range(warm):
        H.matvec(x, y)
    torch.cuda.synchronize()
    ts = []
    for _ in range(reps):
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        H.matvec(x, y)
        e1.record()
        e1.synchronize()
        ts.append(e0.elapsed_time(e1))
    return float(np.median(ts)), y


TRAFFIC_FILE = os.path.join(ROOT, "profiles", "hbm_traffic_matvec_sphere20k_c64.md")
TRAFFIC_SOURCES = ["paper_1706_09384_amd/csrc/matvec.hip", "paper_1706_09384_amd/csrc/internal.hpp",
                   "paper_1706_09384_amd/csrc/api.hip"]


def measured_traffic(kernel):
    """HBM bytes per launch of `kernel` from the committed FETCH_SIZE/WRITE_SIZE summary
    (copy-calibrated), or None when that summary was taken on other sources."""
    import hashlib
    try:
        lines = open(TRAFFIC_FILE).read().splitlines()
    except OSError:
        return None
    h = hashlib.sha256()
    for f in TRAFFIC_SOURCES:
        h.update(open(os.path.join(ROOT, f), "rb").read())
    for ln in lines:
        if ln.startswith("traffic-per-launch "):
            kv = dict(t.split("=", 1) for t in ln.split()[1:])
            if kv.get("kernel") == kernel and kv.get("sources-sha256") == h.hexdigest():
                return int(kv["bytes"])
    return None


def sampled_error(orc, w, X, y, b, rows):
    pb = orc.Problem.from_workload(w, X)
    ref = orc.matvec_rows(pb, b, rows)
    idx = (3 * rows[:, None] + np.arange(3)).ravel()
    yy = y.cpu().numpy().astype(np.complex128).reshape(-1, b.shape[1])[idx]
    return float(np.linalg.norm(yy - ref) / np.linalg.norm(ref)), ref


def multirhs_leg(hmat, W, orc):
    """Multi-RHS panels on the 200k-point T workload: 64 right-hand sides on FP32 matrix cores."""
    import torch
    w = W.multirhs_sphere_200k()
    X, N = w.points()
    tb = time.perf_counter()
    H = hmat.build_workload(w, X=X, N=N, prec=hmat.C64)
    torch.cuda.synchronize()
    t_build = time.perf_counter() - tb
    s = H.info()
    B = w.rhs()
    Bd = torch.from_numpy(B).cuda().to(torch.complex64)
    Y = torch.empty_like(Bd)
    for _ in range(2):
        H.matvec(Bd, Y)
    torch.cuda.synchronize()
    ts = []
    for _ in range(10):
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        H.matvec(Bd, Y)
        e1.record()
        e1.synchronize()
        ts.append(e0.elapsed_time(e1))
    ms = float(np.median(ts))
    kms, kfl, _ = H.profile_matvec_multi(Bd, reps=5)
    flops = sum(kfl)
    dom = int(np.argmax(kms))
    names = ["gather", "project", "accum"]
    roof = {"bound": "mfma", "kernel": names[dom], "achieved": kfl[dom] / (kms[dom] * 1e-3) / 1e12,
            "peak": FP32_MFMA_PEAK_TFLOPS, "unit": "TFLOP/s", "traffic": None}
    roof["frac"] = roof["achieved"] / roof["peak"]
    rows = np.random.default_rng(0).choice(w.n_points, 64, replace=False)
    pb = orc.Problem.from_workload(w, X, N)
    ref = orc.matvec_rows(pb, B, rows)
    idx = (3 * rows[:, None] + np.arange(3)).ravel()
    y = Y.cpu().numpy().astype(np.complex128)[idx]
    err = float((np.linalg.norm(y - ref, axis=0) / np.linalg.norm(ref, axis=0)).max())
    out = {"workload": w.name, "N_c": w.n_points, "nrhs": 64, "kernel": "T", "kappa_s": w.omega,
           "leaf": w.leaf, "eps": w.eps, "assembly_s": round(t_build, 3),
           "storage_bytes": s["storage_bytes"], "max_rank": s["max_rank"],
           "panel_ms": round(ms, 3), "TFLOPs": round(flops / (ms * 1e-3) / 1e12, 2),
           "kernel_ms": [round(k, 4) for k in kms], "roofline": roof,
           "err_vs_oracle_sampled_max_over_rhs": err}
    log(f"[bench] multirhs {out}")
    H.close()
    return out


def batching_leg(hmat, W, orc):
    """Batched assembly on the 100k cube (leaf 32 and 64) with autotuned and graph-captured
    matvecs; the per-block (unbatched) baseline on a 10k cube of the same recipe."""
    import torch

    def mv_time(H, x, reps=50):
        y = torch.empty_like(x)
        for _ in range(5):
            H.matvec(x, y)
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        for _ in range(reps):
            H.matvec(x, y)
        e1.record()
        e1.synchronize()
        return e0.elapsed_time(e1) / reps, y

    out = {}
    for leaf in (32, 64):
        w = W.batching_cube_100k(leaf)
        X, N = w.points()
        Xd, Nd = torch.from_numpy(X).cuda(), torch.from_numpy(N).cuda()
        times = []
        for k in range(3):
            tb = time.perf_counter()
            H = hmat.build(Xd, normals=Nd, kernel=w.kernel, prec=hmat.C64, omega=w.omega,
                           lam=w.lam, mu=w.mu, rho=w.rho, eta=w.eta, eps=w.eps, leaf=w.leaf,
                           self_re=w.self_re, self_im=w.self_im)
            torch.cuda.synchronize()
            times.append(time.perf_counter() - tb)
            if k < 2:
                H.close()
        s = H.info()
        b = w.rhs()
        x = torch.from_numpy(b[:, 0]).cuda().to(torch.complex64)
        ms0, _ = mv_time(H, x)
        H.autotune(reps=5)
        ms1, y = mv_time(H, x)
        s1 = H.info()
        rows = np.random.default_rng(0).choice(w.n_points, 256, replace=False)
        ref = orc.matvec_rows(orc.Problem.from_workload(w, X, N), b[:, :1], rows)[:, 0]
        idx = (3 * rows[:, None] + np.arange(3)).ravel()
        yy = y.cpu().numpy().astype(np.complex128)[idx]
        H.close()
        Hg = hmat.build(Xd, normals=Nd, kernel=w.kernel, prec=hmat.C64, omega=w.omega, lam=w.lam,
                        mu=w.mu, rho=w.rho, eta=w.eta, eps=w.eps, leaf=w.leaf, self_re=w.self_re,
                        self_im=w.self_im, matvec_graph=True)
        msg, _ = mv_time(Hg, x)
        Hg.close()
        out[f"leaf{leaf}"] = {
            "assembly_s": round(float(np.median(times[1:])), 4),
            "phases_s": {k: round(s[k], 4) for k in ("t_tree", "t_nearfield", "t_aca",
                                                     "t_recompress", "t_plan")},
            "n_dense": s["n_dense"], "n_lowrank": s["n_lowrank"], "max_rank": s["max_rank"],
            "n_fallback": s["n_fallback"], "storage_bytes": s["storage_bytes"],
            "matvec_ms_default": round(ms0, 4), "matvec_ms_autotuned": round(ms1, 4),
            "matvec_ms_graph_default_shape": round(msg, 4),
            "autotuned": {"acc_waves": s1["acc_waves"], "proj_rows": s1["proj_rows"]},
            "matvec_GBps_autotuned": round(s["matvec_bytes"] / (ms1 * 1e-3) / 1e9, 1),
            "err_vs_oracle_sampled": float(np.linalg.norm(yy - ref) / np.linalg.norm(ref))}
        log(f"[bench] batching leaf {leaf}: {out[f'leaf{leaf}']}")
    n = 10000
    P, Nrm = W.cube_surface(n, seed=0)
    Pd, Nd = torch.from_numpy(P).cuda(), torch.from_numpy(Nrm).cuda()
    kw = dict(normals=Nd, kernel=1, prec=hmat.C64, omega=4.0 / (2.0 * np.sqrt(3.0)), eps=1e-4,
              leaf=32, self_re=W._t_self(W.CUBE_AREA, n))
    hmat.build(Pd, **kw).close()
    tb = time.perf_counter()
    hmat.build(Pd, **kw).close()
    torch.cuda.synchronize()
    t_b = time.perf_counter() - tb
    tb = time.perf_counter()
    hmat.build(Pd, unbatched=True, **kw).close()
    torch.cuda.synchronize()
    t_u = time.perf_counter() - tb
    out["unbatched_baseline"] = {"workload": "cube10k_T_leaf32 (same recipe as the 100k cube)",
                                 "batched_s": round(t_b, 4), "unbatched_s": round(t_u, 3),
                                 "speedup": round(t_u / t_b, 1)}
    log(f"[bench] batching baseline {out['unbatched_baseline']}")
    return out


def collect_rank_samples(hmat, W):
    """(features, ACA ranks) from the 1k complex128 sphere and the 20k sphere at three eps."""
    fs, rs = [], []
    w = W.plain_sphere_1k()
    H = hmat.build_workload(w, prec=hmat.C128)
    f, r = H.rank_samples()
    fs.append(f); rs.append(r)
    H.close()
    for eps in (1e-3, 1e-4, 1e-5):
        w = W.precision_sphere_20k(eps)
        H = hmat.build_workload(w, prec=hmat.C64)
        f, r = H.rank_samples()
        fs.append(f); rs.append(r)
        H.close()
    return np.concatenate(fs), np.concatenate(rs)


def learned_leg(hmat, W, orc):
    """Rank model trained on the 1k and 20k spheres, used on the 50k prolate spheroid."""
    import torch
    t0 = time.perf_counter()
    f, r = collect_rank_samples(hmat, W)
    t1 = time.perf_counter()
    wts, loss = hmat.rank_model_train(f, r, hmat.rank_model_init(0), epochs=150, batch=256,
                                      lr=1e-3, seed=0)
    t_train = time.perf_counter() - t1
    w = W.learned_spheroid_50k()
    X, _ = w.points()
    Xd = torch.from_numpy(X).cuda()
    res = {}
    for tag, model in (("size_rule", None), ("model", wts)):
        times, st = [], None
        for k in range(3):
            tb = time.perf_counter()
            H = hmat.build(Xd, kernel=w.kernel, prec=hmat.C64, omega=w.omega, lam=w.lam, mu=w.mu,
                           rho=w.rho, eta=w.eta, eps=w.eps, leaf=w.leaf, self_re=w.self_re,
                           self_im=w.self_im, rank_model=model)
            torch.cuda.synchronize()
            times.append(time.perf_counter() - tb)
            st = H.info()
            if k < 2:
                H.close()
        res[tag] = {"assembly_s": round(float(np.median(times)), 4), "t_aca": round(st["t_aca"], 4),
                    "n_overflow": st["n_overflow"], "n_model_hits": st["n_model_hits"],
                    "aca_scratch_bytes": st["aca_scratch_bytes"]}
        if tag == "model":
            fe, ra = H.rank_samples()
            pred = hmat.rank_model_predict(wts, torch.from_numpy(fe).cuda()).cpu().numpy()
            tgt = np.log2(1.0 + ra / 3.0)
            res[tag]["pred_err_median_log2"] = round(float(np.median(np.abs(pred - tgt))), 4)
            res[tag]["underpredicted_frac"] = round(float(np.mean(pred < tgt)), 4)
            b = w.rhs()
            y = H.matvec(torch.from_numpy(b).cuda().to(torch.complex64)).cpu().numpy()
            rows = np.random.default_rng(0).choice(w.n_points, 128, replace=False)
            pb = orc.Problem.from_workload(w, X)
            ref = orc.matvec_rows(pb, b, rows)
            idx = (3 * rows[:, None] + np.arange(3)).ravel()
            res[tag]["err_vs_oracle_sampled"] = float(
                np.linalg.norm(y.astype(np.complex128)[idx] - ref) / np.linalg.norm(ref))
        H.close()
    out = {"workload": w.name, "N_c": w.n_points, "train_samples": int(r.size),
           "sampling_s": round(t1 - t0, 3), "train_s": round(t_train, 3),
           "train_loss_first_last": [float(loss[0]), float(loss[-1])], **res,
           "speedup_assembly": round(res["size_rule"]["assembly_s"] / res["model"]["assembly_s"], 3)}
    log(f"[bench] learned {out}")
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--eps", type=float, default=1e-4)
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--no-fp64", action="store_true")
    ap.add_argument("--no-gmres", action="store_true")
    ap.add_argument("--cpu-rows", type=int, default=20000,
                    help="row points of the oracle's dense product in the CPU baseline")
    ap.add_argument("--no-multirhs", action="store_true")
    ap.add_argument("--no-learned", action="store_true")
    ap.add_argument("--no-batching", action="store_true")
    ap.add_argument("--counters", action="store_true",
                    help="profiling mode: one build, the autotuner, 10 matvecs, then a 256 MiB "
                         "device copy (x3) whose known byte count calibrates FETCH_SIZE / WRITE_SIZE")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for --gpus {args.gpus}); the multi-GPU "
              "sharding of this path is a design note, not an implemented mode.", file=sys.stderr)
        sys.exit(2)

    import torch
    from paper_1706_09384_amd import hmat, workloads as W

    w = W.precision_sphere_20k(args.eps)
    X, _ = w.points()
    Xd = torch.from_numpy(X).cuda()
    b = w.rhs()
    bd = torch.from_numpy(b[:, 0]).cuda()
    b64 = bd.to(torch.complex64)

    def step(prec):
        H = hmat.build_workload(w, X=X, prec=prec) if False else hmat.build(
            Xd, kernel=w.kernel, prec=prec, omega=w.omega, lam=w.lam, mu=w.mu, rho=w.rho,
            eta=w.eta, eps=w.eps, leaf=w.leaf, self_re=w.self_re, self_im=w.self_im)
        y = H.matvec(b64 if prec == hmat.C64 else bd)
        return H, y

    if args.counters:
        H, _ = step(hmat.C64)
        H.autotune(reps=2)
        log(f"[counters] autotuned shape {H.info()['acc_waves']} waves, {H.info()['proj_rows']} rows")
        for k in range(10):
            H.matvec(b64)
        torch.cuda.synchronize()
        log(f"[counters] 10 matvecs done; matvec_bytes {H.info()['matvec_bytes']}")
        src = torch.empty(64 * 1024 * 1024, dtype=torch.float32, device="cuda").fill_(1.0)
        dst = torch.empty_like(src)
        for k in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
        log("[counters] calibration copy: 3 x (268435456 B read + 268435456 B written)")
        H.close()
        return

    log(f"[bench] workload {w.name}: N_c={w.n_points}, warmup {args.warmup}, steps {args.steps}")
    for _ in range(args.warmup):
        H, _ = step(hmat.C64)
        H.close()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    builds = []
    for k in range(args.steps):
        tb = time.perf_counter()
        H, y = step(hmat.C64)
        torch.cuda.synchronize()
        builds.append(time.perf_counter() - tb)
        log(f"[bench] step {k}: {builds[-1]:.3f} s")
        if k < args.steps - 1:
            H.close()
    torch.cuda.synchronize()
    t_steps = time.perf_counter() - t0
    # launch shape of the 1-RHS matvec picked by the library's autotuner
    H.autotune(reps=5)
    s = H.info()
    mv_ms, y = timed_matvecs(H, b64)
    gbps = s["matvec_bytes"] / (mv_ms * 1e-3) / 1e9
    kms, kbytes = H.profile_matvec(b64, reps=20)
    dom = int(np.argmax(kms))
    names = ["gather", "project", "accum"]
    roof = {"bound": "hbm", "kernel": names[dom], "achieved": kbytes[dom] / (kms[dom] * 1e-3) / 1e9,
            "peak": HBM_PEAK_GBPS, "unit": "GB/s"}
    roof["frac"] = roof["achieved"] / roof["peak"]
    roof["traffic"] = measured_traffic(names[dom])
    roof["traffic_unit"] = "B/launch (rocprofv3 FETCH_SIZE + WRITE_SIZE, copy-calibrated)"
    log(f"[bench] matvec {mv_ms:.3f} ms, {gbps:.1f} GB/s; kernels ms {kms} bytes {kbytes}")

    import oracle as orc
    rows = np.random.default_rng(1).choice(w.n_points, 256, replace=False)
    err, _ = sampled_error(orc, w, X, y, b, rows)
    log(f"[bench] sampled-row error {err:.3e} (gate {5 * w.eps:.1e})")

    out = {
        "metric": METRIC, "value": round(gbps, 3), "unit": "GB/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": round(1e3 * t_steps / args.steps, 3),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "c64",
        "data": "synthetic",
        "config": {"workload": w.name, "N_c": w.n_points, "unknowns": 3 * w.n_points,
                   "kernel": "U", "kappa_s": w.omega, "eps": w.eps, "leaf": w.leaf, "eta": w.eta,
                   "precision_form": "c64 + FP64 norms/recompression/refinement"},
        "assembly_s": round(float(np.median(builds)), 4),
        "matvec_ms": round(mv_ms, 4),
        "matvec_bytes": s["matvec_bytes"],
        "matvec_shape": {"acc_waves": s["acc_waves"], "proj_rows": s["proj_rows"]},
        "err_vs_oracle_sampled": err,
        "stats": {k: s[k] for k in ("n_dense", "n_lowrank", "max_rank_aca", "max_rank",
                                    "sum_rank", "storage_bytes", "n_overflow", "n_fallback",
                                    "t_tree", "t_nearfield", "t_aca", "t_recompress", "t_plan")},
        "roofline": roof,
    }
    if not args.no_gmres:
        tg = time.perf_counter()
        x, inf = H.gmres(bd, tol=1e-8, restart=400, maxit=12000, check=False)
        torch.cuda.synchronize()
        out["gmres"] = {"tol": 1e-8, "restart": 400, "s": round(time.perf_counter() - tg, 3), **inf}
        log(f"[bench] gmres {out['gmres']}")
    H.close()
    if not args.no_fp64:
        tb = time.perf_counter()
        H2, y2 = step(hmat.C128)
        torch.cuda.synchronize()
        asm2 = time.perf_counter() - tb
        tb = time.perf_counter()
        H2.close()
        H2, y2 = step(hmat.C128)
        torch.cuda.synchronize()
        asm2 = min(asm2, time.perf_counter() - tb)
        s2 = H2.info()
        mv2, y2 = timed_matvecs(H2, bd)
        err2, _ = sampled_error(orc, w, X, y2, b, rows)
        out["plain_fp64_form"] = {"assembly_s": round(asm2, 4), "matvec_ms": round(mv2, 4),
                                  "matvec_GBps": round(s2["matvec_bytes"] / (mv2 * 1e-3) / 1e9, 3),
                                  "err_vs_oracle_sampled": err2,
                                  "speedup_assembly": round(asm2 / out["assembly_s"], 3),
                                  "speedup_matvec": round(mv2 / mv_ms, 3)}
        log(f"[bench] fp64 form {out['plain_fp64_form']}")
        H2.close()
    if not args.no_cpu:
        # The oracle's streamed FP64 dense product y = A b over a row sample (the
        # whole matrix by default), repeated until about 10 s of CPU work, scaled to
        # one full product and expressed in the metric's unit.
        nrows = min(args.cpu_rows, w.n_points)
        rows_c = (np.arange(w.n_points) if nrows == w.n_points else
                  np.random.default_rng(2).choice(w.n_points, nrows, replace=False))
        pb = orc.Problem.from_workload(w, X)
        ts = []
        while sum(ts) < 10.0 and len(ts) < 50:
            tc = time.perf_counter()
            orc.matvec_rows(pb, b, rows_c)
            ts.append(time.perf_counter() - tc)
        dt = float(np.median(ts))
        t_full = dt * w.n_points / nrows
        out["cpu_baseline"] = {"value": round(s["matvec_bytes"] / t_full / 1e9, 6), "unit": "GB/s",
                               "cores": orc.num_threads(), "kind": "oracle",
                               "sample": f"{nrows} of {w.n_points} row points of the streamed FP64 "
                                         f"dense product, {len(ts)} runs ({sum(ts):.1f} s of CPU "
                                         f"work), median {dt:.2f} s; {t_full:.2f} s per full product"}
    if not args.no_multirhs:
        out["multirhs"] = multirhs_leg(hmat, W, orc)
    if not args.no_learned:
        out["learned"] = learned_leg(hmat, W, orc)
    if not args.no_batching:
        out["batching"] = batching_leg(hmat, W, orc)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
