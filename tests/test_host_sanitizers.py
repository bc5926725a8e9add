"""Host code under AddressSanitizer and UBSan (compiled here with g++/gcc, no GPU).

* the library's cluster tree and block partition (csrc/tree.cpp): permutation
  and exact block cover on a sphere, on a cloud of duplicated points (zero-
  extent boxes) and on two points (tests/sanitize/tree_asan.cpp);
* the oracle's C part (oracle/green.c): dense U and T matrices finite, and
  streamed rows equal to the dense product (tests/sanitize/green_asan.c).

The H-LU's host logic has its own sanitized CPU build (tests/test_lu_host.py).
"""
import os
import subprocess

HERE = os.path.dirname(os.path.abspath(__file__))
REPO = os.path.dirname(HERE)
SAN = ["-fsanitize=address,undefined", "-fno-sanitize-recover=all"]


def run(cmd, exe, env=None):
    r = subprocess.run(cmd, capture_output=True, text=True)
    assert r.returncode == 0, r.stderr[-4000:]
    r = subprocess.run([exe], capture_output=True, text=True, env=env, timeout=600)
    assert r.returncode == 0, (r.stdout[-2000:], r.stderr[-4000:])
    return r.stdout


def test_tree_under_sanitizers(tmp_path):
    exe = str(tmp_path / "tree_asan")
    out = run(["g++", "-std=c++17", "-O1", "-g", "-ffp-contract=off", *SAN,
               "-I" + os.path.join(REPO, "paper_1706_09384_amd", "csrc"),
               os.path.join(HERE, "sanitize", "tree_asan.cpp"),
               os.path.join(REPO, "paper_1706_09384_amd", "csrc", "tree.cpp"), "-o", exe], exe)
    assert "sphere:" in out and "duplicates:" in out and "two points:" in out


def test_oracle_green_under_sanitizers(tmp_path):
    exe = str(tmp_path / "green_asan")
    env = dict(os.environ, OMP_NUM_THREADS="2")
    out = run(["gcc", "-std=gnu11", "-O1", "-g", "-ffp-contract=off", "-fopenmp", *SAN,
               os.path.join(HERE, "sanitize", "green_asan.c"),
               os.path.join(REPO, "oracle", "green.c"), "-o", exe, "-lm"], exe, env)
    assert out.count("rows vs dense") == 2
