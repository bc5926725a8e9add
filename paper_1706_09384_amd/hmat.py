"""Thin ctypes binding of libhmat.so (argument marshalling only).

Every computational step runs inside the library's HIP kernels.  PyTorch is
used for device memory (tensor data pointers) and streams.  If the shared
library is missing the import of this module raises -- there is no fallback.

Names mirror the C ABI in ``include/hmat.h``: :func:`build` (hm_build),
:func:`build_colloc` (hm_build_colloc, the P1 collocation operator),
:meth:`HMatrix.matvec` (hm_matvec), :meth:`HMatrix.residual` (hm_residual),
:meth:`HMatrix.gmres` (hm_gmres), :meth:`HMatrix.info` (hm_info),
:meth:`HMatrix.exact_rows` (hm_exact_rows), :meth:`HMatrix.lu` (hm_lu_factor,
with :class:`HLU` for the solve), :meth:`HMatrix.frob_error`,
:meth:`HMatrix.lu_estimate`, exports and the rank-model calls.
"""
from __future__ import annotations

import ctypes
import os
from dataclasses import dataclass

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libhmat.so")

HM_OK, HM_ERR_ARG, HM_ERR_ALLOC, HM_ERR_HIP, HM_ERR_SINGULAR, HM_ERR_NOCONV, HM_ERR_STATE = range(7)
KERNEL_U, KERNEL_T = 0, 1
C128, C64 = 0, 1
RANK_MODEL_PARAMS = 64 * 6 + 64 + 64 * 64 + 64 + 64 + 1

_STATUS = {0: "HM_OK", 1: "HM_ERR_ARG", 2: "HM_ERR_ALLOC", 3: "HM_ERR_HIP", 4: "HM_ERR_SINGULAR",
           5: "HM_ERR_NOCONV", 6: "HM_ERR_STATE"}


class HMError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__(f"{_STATUS.get(status, status)}: {msg}")
        self.status = status


class Params(ctypes.Structure):
    _fields_ = [
        ("kernel", ctypes.c_int32), ("prec", ctypes.c_int32),
        ("omega", ctypes.c_double), ("lam", ctypes.c_double), ("mu", ctypes.c_double),
        ("rho", ctypes.c_double), ("eta", ctypes.c_double), ("eps", ctypes.c_double),
        ("leaf", ctypes.c_int32), ("same", ctypes.c_int32),
        ("self_re", ctypes.c_double), ("self_im", ctypes.c_double),
        ("points_on_host", ctypes.c_int32), ("plan_only", ctypes.c_int32),
        ("rank_budget", ctypes.c_int32), ("recompress", ctypes.c_int32),
        ("tau_piv", ctypes.c_double),
        ("rank_model", ctypes.c_void_p),
        ("matvec_graph", ctypes.c_int32), ("unbatched", ctypes.c_int32),
        ("aca_scratch_mb", ctypes.c_int32),
        ("rsvd", ctypes.c_int32),
        ("reserved", ctypes.c_int32 * 4),
    ]


class Stats(ctypes.Structure):
    _fields_ = [
        ("nx", ctypes.c_int64), ("ny", ctypes.c_int64),
        ("nodes_x", ctypes.c_int32), ("nodes_y", ctypes.c_int32),
        ("leaves_x", ctypes.c_int32), ("leaves_y", ctypes.c_int32),
        ("levels_x", ctypes.c_int32), ("levels_y", ctypes.c_int32),
        ("n_blocks", ctypes.c_int64), ("n_dense", ctypes.c_int64), ("n_lowrank", ctypes.c_int64),
        ("c_sp", ctypes.c_int32), ("prec", ctypes.c_int32),
        ("dense_entries", ctypes.c_int64), ("lowrank_entries", ctypes.c_int64),
        ("storage_bytes", ctypes.c_int64),
        ("max_rank_aca", ctypes.c_int32), ("max_rank", ctypes.c_int32),
        ("sum_rank_aca", ctypes.c_int64), ("sum_rank", ctypes.c_int64),
        ("n_overflow", ctypes.c_int32), ("n_fallback", ctypes.c_int32),
        ("n_model_hits", ctypes.c_int32),
        ("t_tree", ctypes.c_double), ("t_upload", ctypes.c_double),
        ("t_nearfield", ctypes.c_double), ("t_aca", ctypes.c_double),
        ("t_recompress", ctypes.c_double), ("t_plan", ctypes.c_double),
        ("t_total", ctypes.c_double),
        ("matvec_bytes", ctypes.c_int64),
        ("aca_scratch_bytes", ctypes.c_int64), ("aca_chunks", ctypes.c_int32),
        ("acc_waves", ctypes.c_int32), ("proj_rows", ctypes.c_int32),
        ("n_capped", ctypes.c_int32), ("n_rsvd", ctypes.c_int32),
    ]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


class LuStats(ctypes.Structure):
    _fields_ = [("t_import", ctypes.c_double), ("t_factor", ctypes.c_double),
                ("storage_entries", ctypes.c_int64), ("device_bytes", ctypes.c_int64),
                ("max_rank", ctypes.c_int32), ("n_nodes", ctypes.c_int32),
                ("n_diag", ctypes.c_int32), ("n_recompressed", ctypes.c_int32),
                ("n_batches", ctypes.c_int32), ("n_gemm", ctypes.c_int32),
                ("gemm_flops", ctypes.c_double), ("n_sampled", ctypes.c_int32),
                ("reserved", ctypes.c_int32)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


class LuEstimate(ctypes.Structure):
    _fields_ = [("delta", ctypes.c_double), ("delta_h", ctypes.c_double),
                ("b_norm", ctypes.c_double), ("x0_norm", ctypes.c_double),
                ("estimate", ctypes.c_double)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


class GmresInfo(ctypes.Structure):
    _fields_ = [("iters", ctypes.c_int32), ("restarts", ctypes.c_int32),
                ("refinements", ctypes.c_int32), ("converged", ctypes.c_int32),
                ("relres", ctypes.c_double), ("relres_inner", ctypes.c_double)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


def _load():
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is missing: build it with __graft_entry__.build() "
                          "(the HIP path has no fallback)")
    # torch carries its own HIP runtime library: it is loaded before this
    # library's, because with the opposite load order the library's HIP calls
    # have reported no device on the MI355X boxes
    import torch  # noqa: F401
    lib = ctypes.CDLL(LIB_PATH)
    P, i32, i64, d = ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64, ctypes.c_double
    sig = {
        "hm_params_default": ([P], i32),
        "hm_build": ([P, i64, P, i64, P, P, P, P], i32),
        "hm_build_colloc": ([P, i64, P, i64, i32, i32, P, P, P], i32),
        "hm_matvec": ([P, P, P, i32, P], i32),
        "hm_matvec_noalloc": ([P, P, P, i32, P], i32),
        "hm_residual": ([P, P, P, P, i32, P], i32),
        "hm_gmres": ([P, P, P, i32, d, i32, i32, P, P], i32),
        "hm_info": ([P, P], i32),
        "hm_profile_matvec": ([P, P, P, i32, P, P, P], i32),
        "hm_profile_matvec_multi": ([P, P, P, i32, P, P, P], i32),
        "hm_autotune": ([P, i32, P, P], i32),
        "hm_export_tree": ([P, i32, P, P, P], i32),
        "hm_export_blocklist": ([P, P, P, P], i32),
        "hm_export_block": ([P, i64, P], i32),
        "hm_destroy": ([P], None),
        "hm_release_cache": ([], None),
        "hm_last_error": ([], ctypes.c_char_p),
        "hm_rank_samples": ([P, P, P], i32),
        "hm_rank_model_train": ([P, P, i64, P, i32, i32, ctypes.c_float, ctypes.c_uint64, P, P], i32),
        "hm_rank_model_predict": ([P, P, P, i64, P], i32),
        "hm_rank_model_grad": ([P, P, P, i64, P, P, P], i32),
        "hm_lu_factor": ([P, d, P, P], i32),
        "hm_lu_solve": ([P, P, P, i32, P], i32),
        "hm_lu_get_stats": ([P, P], i32),
        "hm_lu_export_dense": ([P, P], i32),
        "hm_lu_destroy": ([P], None),
        "hm_frob_error": ([P, P, P, P], i32),
        "hm_exact_rows": ([P, P, i64, P, i32, P, P], i32),
        "hm_lu_estimate": ([P, P, P, d, P, P], i32),
    }
    for name, (args, res) in sig.items():
        f = getattr(lib, name)
        f.argtypes = args
        f.restype = res
    return lib


LIB = _load()
EXPORTED = ["hm_params_default", "hm_build", "hm_build_colloc", "hm_matvec", "hm_matvec_noalloc", "hm_residual", "hm_gmres", "hm_info",
            "hm_profile_matvec", "hm_profile_matvec_multi", "hm_autotune",
            "hm_export_tree", "hm_export_blocklist", "hm_export_block", "hm_destroy",
            "hm_release_cache",
            "hm_last_error", "hm_rank_samples", "hm_rank_model_train", "hm_rank_model_predict",
            "hm_rank_model_grad", "hm_lu_factor", "hm_lu_solve", "hm_lu_get_stats",
            "hm_lu_export_dense", "hm_lu_destroy", "hm_frob_error", "hm_lu_estimate", "hm_exact_rows"]


def _check(rc):
    if rc != HM_OK:
        raise HMError(rc, LIB.hm_last_error().decode())


def _stream(stream):
    if stream is not None:
        return ctypes.c_void_p(stream)
    import torch
    return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)


def _ptr(t):
    if t is None:
        return None
    if isinstance(t, np.ndarray):
        return ctypes.c_void_p(t.ctypes.data)
    return ctypes.c_void_p(t.data_ptr())


def make_params(kernel=KERNEL_U, prec=C128, omega=1.0, lam=2.0, mu=1.0, rho=1.0, eta=3.0,
                eps=1e-4, leaf=32, same=True, self_re=0.0, self_im=0.0, points_on_host=False,
                plan_only=False, rank_budget=0, recompress=True, tau_piv=0.0, rank_model=None,
                matvec_graph=False, unbatched=False, aca_scratch_mb=0, rsvd=True):
    p = Params()
    _check(LIB.hm_params_default(ctypes.byref(p)))
    p.kernel, p.prec = int(kernel), int(prec)
    p.omega, p.lam, p.mu, p.rho = float(omega), float(lam), float(mu), float(rho)
    p.eta, p.eps, p.leaf, p.same = float(eta), float(eps), int(leaf), int(bool(same))
    p.self_re, p.self_im = float(self_re), float(self_im)
    p.points_on_host, p.plan_only = int(bool(points_on_host)), int(bool(plan_only))
    p.rank_budget, p.recompress, p.tau_piv = int(rank_budget), int(bool(recompress)), float(tau_piv)
    p.matvec_graph, p.unbatched = int(bool(matvec_graph)), int(bool(unbatched))
    p.aca_scratch_mb = int(aca_scratch_mb)
    p.rsvd = int(bool(rsvd))
    p._model_keepalive = None
    if rank_model is not None:
        w = np.ascontiguousarray(rank_model, dtype=np.float32)
        assert w.size == RANK_MODEL_PARAMS
        p.rank_model = w.ctypes.data
        p._model_keepalive = w
    return p


class HLU:
    """Owning handle of H-LU factors (hm_lu*)."""

    def __init__(self, handle, dofs):
        self._h = handle
        self._destroy = LIB.hm_lu_destroy
        self.dofs = dofs

    def __del__(self):
        self.close()

    def close(self):
        h = getattr(self, "_h", None)
        if h:
            self._h = None
            self._destroy(h)

    def stats(self) -> dict:
        s = LuStats()
        _check(LIB.hm_lu_get_stats(self._h, ctypes.byref(s)))
        return s.as_dict()

    def solve(self, b, x=None, stream=None):
        """x0 = U_H^-1 L_H^-1 b; b a complex128 cuda tensor (3N,) or (3N, nrhs)."""
        import torch
        vec = b.dim() == 1
        B = b.reshape(b.shape[0], -1).contiguous()
        assert B.dtype == torch.complex128 and B.is_cuda and B.shape[0] == self.dofs
        if x is None:
            x = torch.empty_like(B)
        _check(LIB.hm_lu_solve(self._h, _ptr(B), _ptr(x), B.shape[1], _stream(stream)))
        return x.reshape(-1) if vec else x

    def export_dense(self) -> np.ndarray:
        """L_H (strictly lower, unit diagonal implied) and U_H packed, cluster order."""
        out = np.zeros((self.dofs, self.dofs), dtype=np.complex128, order="F")
        _check(LIB.hm_lu_export_dense(self._h, out.ctypes.data_as(ctypes.c_void_p)))
        return out


class HMatrix:
    """Owning handle of an assembled H-matrix (hm_matrix*)."""

    def __init__(self, handle, params):
        self._h = handle
        # kept on the instance: at interpreter exit the module globals may be gone
        self._destroy = LIB.hm_destroy
        self.params = params
        self.prec = params.prec
        s = self.info()
        self.nx, self.ny = s["nx"], s["ny"]

    def __del__(self):
        self.close()

    def close(self):
        h = getattr(self, "_h", None)
        if h:
            self._h = None
            self._destroy(h)

    @property
    def complex_dtype(self):
        import torch
        return torch.complex64 if self.prec == C64 else torch.complex128

    def info(self) -> dict:
        s = Stats()
        _check(LIB.hm_info(self._h, ctypes.byref(s)))
        return s.as_dict()

    def matvec(self, x, y=None, stream=None):
        """y = A_H x; x is a cuda tensor (3 ny,) or (3 ny, nrhs) of the operator's type."""
        import torch
        vec = x.dim() == 1
        X = x.reshape(x.shape[0], -1).contiguous()
        assert X.dtype == self.complex_dtype and X.is_cuda and X.shape[0] == 3 * self.ny
        if y is None:
            y = torch.empty((3 * self.nx, X.shape[1]), dtype=X.dtype, device=X.device)
        _check(LIB.hm_matvec(self._h, _ptr(X), _ptr(y), X.shape[1], _stream(stream)))
        return y.reshape(-1) if vec else y

    def matvec_noalloc(self, x, y, stream=None):
        """hm_matvec_noalloc: y = A_H x into the caller's y, with the library's fixed
        device scratch (no allocation inside the call)."""
        X = x.reshape(x.shape[0], -1)
        Y = y.reshape(y.shape[0], -1)
        assert X.is_contiguous() and Y.is_contiguous() and X.dtype == self.complex_dtype
        assert Y.dtype == X.dtype and X.shape[0] == 3 * self.ny and Y.shape == (3 * self.nx, X.shape[1])
        _check(LIB.hm_matvec_noalloc(self._h, _ptr(X), _ptr(Y), X.shape[1], _stream(stream)))
        return y

    def residual(self, b, x, r=None, stream=None):
        """r = b - A_H x in FP64 (complex128 tensors)."""
        import torch
        vec = b.dim() == 1
        B = b.reshape(b.shape[0], -1).contiguous()
        X = x.reshape(x.shape[0], -1).contiguous()
        assert B.dtype == torch.complex128 and X.dtype == torch.complex128
        if r is None:
            r = torch.empty_like(B)
        _check(LIB.hm_residual(self._h, _ptr(B), _ptr(X), _ptr(r), B.shape[1], _stream(stream)))
        return r.reshape(-1) if vec else r

    def lu(self, eps_lu, stream=None) -> "HLU":
        """H-LU factors of this operator at eps_LU (hm_lu_factor)."""
        h = ctypes.c_void_p()
        _check(LIB.hm_lu_factor(self._h, float(eps_lu), _stream(stream), ctypes.byref(h)))
        return HLU(h.value, 3 * self.nx)

    def frob_error(self, stream=None):
        """(|A_H - A|_F, |A|_F) (hm_frob_error)."""
        d, a = ctypes.c_double(), ctypes.c_double()
        _check(LIB.hm_frob_error(self._h, _stream(stream), ctypes.byref(d), ctypes.byref(a)))
        return d.value, a.value

    def exact_rows(self, rows, x, stream=None):
        """Rows of the exact operator times x (hm_exact_rows): x complex128 cuda tensor
        (3 ny,) or (3 ny, nrhs); returns (3 len(rows),) or (3 len(rows), nrhs)."""
        import torch
        r = np.ascontiguousarray(rows, np.int64)
        vec = x.dim() == 1
        X = x.reshape(x.shape[0], -1).contiguous()
        assert X.dtype == torch.complex128 and X.shape[0] == 3 * self.ny
        Y = torch.empty((3 * r.size, X.shape[1]), dtype=torch.complex128, device=X.device)
        _check(LIB.hm_exact_rows(self._h, _ptr(r), int(r.size), _ptr(X), X.shape[1], _ptr(Y),
                                 _stream(stream)))
        return Y.reshape(-1) if vec else Y

    def lu_estimate(self, b, x0, delta_h, stream=None) -> dict:
        """Estimator of eq. est_direct for one right-hand side (hm_lu_estimate)."""
        import torch
        assert b.dtype == torch.complex128 and x0.dtype == torch.complex128
        e = LuEstimate()
        _check(LIB.hm_lu_estimate(self._h, _ptr(b.contiguous()), _ptr(x0.contiguous()),
                                  float(delta_h), _stream(stream), ctypes.byref(e)))
        return e.as_dict()

    def gmres(self, b, tol=1e-6, restart=50, maxit=2000, stream=None, check=True):
        """Solve A_H x = b (complex128 cuda tensors); returns (x, info dict)."""
        import torch
        vec = b.dim() == 1
        B = b.reshape(b.shape[0], -1).contiguous()
        assert B.dtype == torch.complex128
        x = torch.empty_like(B)
        inf = GmresInfo()
        rc = LIB.hm_gmres(self._h, _ptr(B), _ptr(x), B.shape[1], float(tol), int(restart),
                          int(maxit), _stream(stream), ctypes.byref(inf))
        if check and rc not in (HM_OK,):
            raise HMError(rc, LIB.hm_last_error().decode())
        out = inf.as_dict()
        out["status"] = rc
        return (x.reshape(-1) if vec else x), out

    def profile_matvec_multi(self, x, reps=10, stream=None):
        """Mean duration (ms) and algorithmic flops of the gather/project/accum passes of one
        64-column multi-RHS panel (complex64 operators)."""
        import torch
        assert x.shape == (3 * self.ny, 64) and x.dtype == torch.complex64
        y = torch.empty(3 * self.nx, 64, dtype=x.dtype, device=x.device)
        ms = (ctypes.c_double * 3)()
        fl = (ctypes.c_double * 3)()
        _check(LIB.hm_profile_matvec_multi(self._h, _ptr(x.contiguous()), _ptr(y), int(reps),
                                           _stream(stream), ms, fl))
        return list(ms), list(fl), y

    def profile_matvec(self, x, reps=20, stream=None):
        """Mean duration (ms) and algorithmic bytes of the gather/project/accum kernels."""
        import torch
        y = torch.empty(3 * self.nx, dtype=x.dtype, device=x.device)
        ms = (ctypes.c_double * 3)()
        by = (ctypes.c_int64 * 3)()
        _check(LIB.hm_profile_matvec(self._h, _ptr(x.contiguous()), _ptr(y), int(reps),
                                     _stream(stream), ms, by))
        return list(ms), list(by)

    def autotune(self, reps=10, stream=None):
        """Pick the fastest 1-RHS matvec launch shape; returns the 3 x 3 table of mean ms
        (rows: projection chunk 256/512/1024, columns: waves 4/8/16)."""
        t = (ctypes.c_double * 9)()
        _check(LIB.hm_autotune(self._h, int(reps), _stream(stream), t))
        return np.array(list(t)).reshape(3, 3)

    def rank_samples(self):
        """(features float32 (n_lowrank, 6), ACA ranks int32 (n_lowrank,)) of every admissible
        block, in block-list order."""
        n = self.info()["n_lowrank"]
        f = np.zeros((n, 6), np.float32)
        r = np.zeros(n, np.int32)
        _check(LIB.hm_rank_samples(self._h, _ptr(f), _ptr(r)))
        return f, r

    def export_tree(self, which=0):
        s = self.info()
        n = s["nx"] if which == 0 else s["ny"]
        nodes = s["nodes_x"] if which == 0 else s["nodes_y"]
        perm = np.zeros(n, np.int32)
        nd = np.zeros((nodes, 5), np.int32)
        bx = np.zeros((nodes, 6), np.float64)
        _check(LIB.hm_export_tree(self._h, int(which), _ptr(perm), _ptr(nd), _ptr(bx)))
        return perm, nd, bx

    def export_blocklist(self):
        nb = self.info()["n_blocks"]
        blocks = np.zeros((nb, 3), np.int32)
        rank = np.zeros(nb, np.int32)
        rank_aca = np.zeros(nb, np.int32)
        _check(LIB.hm_export_blocklist(self._h, _ptr(blocks), _ptr(rank), _ptr(rank_aca)))
        return blocks, rank, rank_aca

    def export_block(self, b, blocks=None, rank=None, nodes_x=None, nodes_y=None):
        """Host copy of block b: dense tile (3m x 3n) or (U, V)."""
        if blocks is None:
            blocks, rank, _ = self.export_blocklist()
        if nodes_x is None:
            nodes_x = self.export_tree(0)[1]
            nodes_y = self.export_tree(1)[1]
        t, s, kind = blocks[b]
        m = int(nodes_x[t, 1] - nodes_x[t, 0])
        n = int(nodes_y[s, 1] - nodes_y[s, 0])
        dt = np.complex64 if self.prec == C64 else np.complex128
        if kind == 0:
            buf = np.zeros(9 * m * n, dt)
            _check(LIB.hm_export_block(self._h, int(b), _ptr(buf)))
            return buf.reshape(3 * n, 3 * m).T.copy()
        r = int(rank[b])
        buf = np.zeros(3 * (m + n) * max(r, 0), dt)
        _check(LIB.hm_export_block(self._h, int(b), _ptr(buf)))
        U = buf[:3 * m * r].reshape(r, 3 * m).T.copy()
        V = buf[3 * m * r:].reshape(r, 3 * n).T.copy()
        return U, V


def release_cache():
    """Return the library's cached device memory to the driver (hm_release_cache)."""
    LIB.hm_release_cache()


def rank_model_init(seed=0):
    """Initial rank-model weights: uniform(-sqrt(6/fan_in), +sqrt(6/fan_in)) weights and zero
    biases, packed W1 b1 W2 b2 W3 b3 (float32)."""
    rng = np.random.default_rng(seed)
    parts = []
    for fi, fo in ((6, 64), (64, 64), (64, 1)):
        lim = np.sqrt(6.0 / fi)
        parts.append(rng.uniform(-lim, lim, size=fo * fi))
        parts.append(np.zeros(fo))
    w = np.concatenate(parts).astype(np.float32)
    assert w.size == RANK_MODEL_PARAMS
    return w


def rank_model_train(feats, ranks, weights, epochs=100, batch=256, lr=1e-3, seed=0, stream=None):
    """Train with the library's FP32 kernels; returns (weights, mean loss per epoch)."""
    f = np.ascontiguousarray(feats, np.float32)
    r = np.ascontiguousarray(ranks, np.int32)
    w = np.array(weights, dtype=np.float32, copy=True)
    loss = np.zeros(int(epochs), np.float32)
    _check(LIB.hm_rank_model_train(_ptr(f), _ptr(r), int(r.size), _ptr(w), int(epochs), int(batch),
                                   float(lr), int(seed), _ptr(loss), _stream(stream)))
    return w, loss


def rank_model_predict(weights, feats, stream=None):
    """Forward pass on the device: feats float32 cuda tensor (n, 6) -> (n,)."""
    import torch
    w = np.ascontiguousarray(weights, np.float32)
    X = feats.contiguous()
    out = torch.empty(X.shape[0], dtype=torch.float32, device=X.device)
    _check(LIB.hm_rank_model_predict(_ptr(w), _ptr(X), _ptr(out), int(X.shape[0]), _stream(stream)))
    return out


def rank_model_grad(weights, feats, targets, stream=None):
    """(loss, gradient) of the mean squared error on the device (float32 cuda tensors)."""
    w = np.ascontiguousarray(weights, np.float32)
    g = np.zeros(RANK_MODEL_PARAMS, np.float32)
    loss = np.zeros(1, np.float32)
    X, t = feats.contiguous(), targets.contiguous()
    _check(LIB.hm_rank_model_grad(_ptr(w), _ptr(X), _ptr(t), int(X.shape[0]), _ptr(loss), _ptr(g),
                                  _stream(stream)))
    return float(loss[0]), g


def build(x, y=None, normals=None, stream=None, **kw) -> HMatrix:
    """hm_build.  x, y, normals: (n, 3) float64 cuda tensors (or numpy arrays with
    points_on_host=True / plan_only=True)."""
    same = y is None
    kw.setdefault("same", same)
    host = isinstance(x, np.ndarray)
    if host:
        kw["points_on_host"] = True
    p = make_params(**kw)
    X = x if not host else np.ascontiguousarray(x, np.float64)
    Y = None if same else (y if not host else np.ascontiguousarray(y, np.float64))
    Nn = None if normals is None else (normals if not host else np.ascontiguousarray(normals, np.float64))
    if not host:
        X = X.contiguous()
        Y = None if Y is None else Y.contiguous()
        Nn = None if Nn is None else Nn.contiguous()
    nx = X.shape[0]
    ny = nx if same else Y.shape[0]
    h = ctypes.c_void_p()
    st = ctypes.c_void_p(0) if (host or p.plan_only) and stream is None else _stream(stream)
    rc = LIB.hm_build(_ptr(X), nx, _ptr(Y), ny, _ptr(Nn), ctypes.byref(p), st, ctypes.byref(h))
    _check(rc)
    return HMatrix(h, p)


def build_colloc(nodes, tri, q_reg=3, q_sing=6, stream=None, **kw) -> HMatrix:
    """hm_build_colloc.  nodes (nc, 3) float64 and tri (ne, 3) int32, numpy arrays
    (host) or cuda tensors (device)."""
    host = isinstance(nodes, np.ndarray)
    if host:
        kw["points_on_host"] = True
        X = np.ascontiguousarray(nodes, np.float64)
        T = np.ascontiguousarray(tri, np.int32)
    else:
        X, T = nodes.contiguous(), tri.contiguous()
    kw["same"] = True
    p = make_params(**kw)
    h = ctypes.c_void_p()
    st = ctypes.c_void_p(0) if p.plan_only and stream is None else _stream(stream)
    _check(LIB.hm_build_colloc(_ptr(X), X.shape[0], _ptr(T), T.shape[0], int(q_reg), int(q_sing),
                               ctypes.byref(p), st, ctypes.byref(h)))
    return HMatrix(h, p)


def build_mesh(m, prec=C128, **kw) -> HMatrix:
    """Build the collocation operator of a :class:`workloads.Mesh`."""
    P, T = m.mesh()
    args = dict(kernel=0, prec=prec, omega=m.omega, lam=m.lam, mu=m.mu, rho=m.rho, eta=m.eta,
                eps=m.eps, leaf=m.leaf)
    args.update(kw)
    return build_colloc(P, T, m.q_reg, m.q_sing, **args)


def build_workload(w, device="cuda", prec=C128, X=None, N=None, **kw) -> HMatrix:
    """Build the H-matrix of a :class:`workloads.Workload`."""
    import torch
    if X is None:
        X, N = w.points()
    args = dict(kernel=w.kernel, prec=prec, omega=w.omega, lam=w.lam, mu=w.mu, rho=w.rho,
                eta=w.eta, eps=w.eps, leaf=w.leaf, self_re=w.self_re, self_im=w.self_im)
    args.update(kw)
    if device is None:
        return build(X, normals=N, **args)
    Xt = torch.from_numpy(np.ascontiguousarray(X)).to(device)
    Nt = None if N is None else torch.from_numpy(np.ascontiguousarray(N)).to(device)
    return build(Xt, normals=Nt, **args)
