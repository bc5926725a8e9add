"""The H-LU's host logic (recursion, formats, views, stack memory) on the CPU.

The library's recursion (paper_1706_09384_amd/csrc/lu_core.hpp) is compiled
with g++ against a backend that does the arithmetic in plain loops, poisons
fresh memory with NaN, and checks every matrix view against the allocation it
points into (released stack memory included).  With eps_LU = 0 that backend
truncates nothing, so the packed factors must reproduce A_H exactly (up to
rounding) and the solve must match a dense solve: the block structure, the
offsets of every partial sum and the order of the steps are all exercised.
The input A_H is the oracle's (cluster tree, block tree, truncated SVD of the
admissible blocks).
"""
import os
import struct
import subprocess

import numpy as np
import pytest

from paper_1706_09384_amd import workloads as W

HERE = os.path.dirname(os.path.abspath(__file__))
REPO = os.path.dirname(HERE)


@pytest.fixture(scope="module")
def lu_cpu(tmp_path_factory):
    exe = str(tmp_path_factory.mktemp("lu_cpu") / "lu_cpu")
    cmd = ["g++", "-std=c++17", "-O1", "-g", "-D__HIP_PLATFORM_AMD__", "-I/opt/rocm/include",
           "-I" + os.path.join(REPO, "paper_1706_09384_amd", "csrc"), "-I" + os.path.join(REPO, "include"),
           "-fsanitize=address,undefined", "-fno-sanitize-recover=all",
           os.path.join(HERE, "lu_cpu", "lu_cpu.cpp"), "-o", exe]
    r = subprocess.run(cmd, capture_output=True, text=True)
    assert r.returncode == 0, r.stderr[-4000:]
    return exe


def run_lu_cpu(exe, tmp, t, blocks, leaves, b, eps=0.0):
    nodes, dofs = t.n_nodes, 3 * t.perm.size
    by = {(int(a), int(c)): (k, d) for a, c, k, d in leaves}
    inp, out = str(tmp / "in.bin"), str(tmp / "out.bin")
    with open(inp, "wb") as f:
        f.write(struct.pack("<iiqd", nodes, len(blocks), dofs, eps))
        for arr in (t.begin, t.end, t.left, t.right):
            f.write(np.asarray(arr, np.int32).tobytes())
        f.write(np.asarray(blocks, np.int32).reshape(-1).tobytes())
        ranks = [-1 if k == 0 else by[(int(a), int(c))][1][0].shape[1] for a, c, k in blocks]
        f.write(np.asarray(ranks, np.int32).tobytes())
        for a, c, k in blocks:
            kind, d = by[(int(a), int(c))]
            if kind == 0:
                f.write(np.asarray(d, np.complex128).tobytes(order="F"))
            else:
                U, V = d
                f.write(np.asarray(U, np.complex128).tobytes(order="F"))
                f.write(np.asarray(V.conj().T, np.complex128).tobytes(order="F"))
        f.write(np.asarray(b, np.complex128).tobytes())
    r = subprocess.run([exe, inp, out], capture_output=True, text=True, timeout=900)
    assert r.returncode == 0, r.stderr[-4000:]
    data = open(out, "rb").read()
    status, ln = struct.unpack("<ii", data[:8])
    assert status == 0, data[8:8 + ln].decode()
    off = 8
    P = np.frombuffer(data[off:off + dofs * dofs * 16], np.complex128).reshape(dofs, dofs, order="F")
    off += dofs * dofs * 16
    x = np.frombuffer(data[off:off + dofs * 16], np.complex128)
    off += dofs * 16
    stats = np.frombuffer(data[off:off + 32], np.int64)
    return P, x, stats


@pytest.mark.parametrize("kernel,small", [(W.KERNEL_U, False), (W.KERNEL_T, False), (W.KERNEL_U, True)])
def test_host_logic_exact_lu_in_bounds(orc, lu_cpu, tmp_path, kernel, small, monkeypatch):
    """small: every recompression list split into batches of one block (the split a
    stack-memory budget makes on large problems)."""
    if small:
        monkeypatch.setenv("LU_CPU_SMALL_BATCHES", "1")
    import sys
    sys.path.insert(0, HERE)
    from test_oracle_hlu import svd_leaves
    w = W.small_sphere(400, kernel=kernel, leaf=16)
    X, N = w.points()
    A = orc.dense(orc.Problem.from_workload(w, X, N))
    t = orc.cluster_tree(X, w.leaf)
    blocks = orc.block_tree(t, t, w.eta)
    leaves = svd_leaves(orc, t, blocks, A, 1e-4)
    AH = orc.hlu.to_dense(orc.hlu.build(t, leaves))
    dof = (3 * t.perm[:, None] + np.arange(3)).ravel()
    b = w.rhs()[:, 0][dof]
    P, x, stats = run_lu_cpu(lu_cpu, tmp_path, t, blocks, leaves, b)
    n_rec, n_batch, n_gemm, n_diag = stats
    assert n_rec > 100 and n_batch > 10 and n_diag == sum(1 for a, c, k in blocks if a == c)
    if small:
        assert n_batch == n_rec
    L = np.tril(P, -1) + np.eye(P.shape[0])
    U = np.triu(P)
    assert np.linalg.norm(L @ U - AH) <= 1e-13 * np.linalg.norm(AH)
    xd = np.linalg.solve(AH, b)
    assert np.linalg.norm(x - xd) <= 1e-12 * np.linalg.norm(xd)
