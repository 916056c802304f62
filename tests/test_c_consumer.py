"""The C ABI used from plain C99 (tests/c_consumer.c): the header compiles as C, the
library links from C, a tensor builds and reports its sizes, invalid arguments are
rejected with a message; on the GPU the right-hand side computed through the C ABI
matches the oracle."""
import os
import shutil
import subprocess

import numpy as np
import pytest

from paper_2607_13740_amd import gracedg as G

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
ROCM = os.environ.get("ROCM_PATH", "/opt/rocm")


def _build(tmp_path):
    if shutil.which("gcc") is None:
        pytest.skip("gcc not available")
    lib = os.path.dirname(G.lib()._name)
    exe = str(tmp_path / "c_consumer")
    cmd = ["gcc", "-std=c99", "-Wall", "-Wextra", "-Werror", "-D__HIP_PLATFORM_AMD__",
           "-I", os.path.join(ROOT, "include"), "-I", os.path.join(ROCM, "include"),
           os.path.join(HERE, "c_consumer.c"), "-o", exe,
           "-L", lib, "-lgracedg", "-Wl,-rpath," + lib,
           "-L", os.path.join(ROCM, "lib"), "-lamdhip64", "-Wl,-rpath," + os.path.join(ROCM, "lib")]
    subprocess.run(cmd, check=True, capture_output=True, text=True)
    return exe


def _run(exe, *args):
    r = subprocess.run([exe, *args], capture_output=True, text=True, timeout=120)
    assert r.returncode == 0, r.stderr
    return r.stdout.splitlines()


def test_c_consumer_builds_and_runs_on_the_host(tmp_path):
    exe = _build(tmp_path)
    out = _run(exe)
    P, n_out, nnz = (int(x) for x in out[0].split()[1:])
    t = G.Tensor(8, 2, 1e-4, 1e8, kernel="ballistic", frag="powerlaw", levels=(0.5,), conservative=True)
    inf = t.info()
    assert (P, n_out, nnz) == (inf["P"], inf["n_out"], inf["nnz_folded"])
    code, msg = out[1].split(maxsplit=2)[1:]
    assert int(code) == G.GD_EINVAL and "order" in msg


@pytest.mark.gpu
def test_c_consumer_right_hand_side_matches_oracle(tmp_path, oracle):
    O = oracle
    exe = _build(tmp_path)
    print("case c_consumer gpu", flush=True)
    rows = [ln for ln in _run(exe, "gpu") if ln.startswith("raw")]
    Yg = np.array([[float(x) for x in ln.split()[1:]] for ln in rows])
    N, k, C = 8, 2, 3
    cfg = O.Config(N=N, k=k, xmin=1e-4, xmax=1e8, kernel="ballistic", frag="powerlaw", conservative=True,
                   vfrag=0.5)
    g = np.zeros((C, N, k + 1))
    for c in range(C):
        for j in range(N):
            g[c, j, 0] = 1.0 / (1 + j + c)
            for i in range(1, k + 1):
                g[c, j, i] = 0.05 * i / (1 + j)
    Yo, _, _ = O.rhs(cfg, g.reshape(C, -1))
    assert Yg.shape == Yo.shape
    eps = np.abs(Yg - Yo).max(axis=1) / np.abs(Yo).max(axis=1)
    assert eps.max() <= 1e-12, eps
