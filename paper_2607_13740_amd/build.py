"""Build the gfx950 collision-operator library in-tree.

    python -m paper_2607_13740_amd.build

compiles ``csrc/tensor_build.cpp`` (host C++) and the HIP sources of ``csrc/``
(for gfx950) into ``paper_2607_13740_amd/libgracedg.so``; ``build(checks=True)``
(``python -m paper_2607_13740_amd.build checks``) compiles the same sources with the
device checks on (``-DGD_CHECKS``) into ``libgracedg_checks.so``.
"""
from __future__ import annotations

import os
import subprocess
import sys
from concurrent.futures import ThreadPoolExecutor

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
LIB = os.path.join(HERE, "libgracedg.so")
LIB_CHECKS = os.path.join(HERE, "libgracedg_checks.so")
ARCH = os.environ.get("GRACEDG_ARCH", "gfx950")

HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
HIP_FLAGS = [
    "-O3", "-std=c++17", "-fPIC", f"--offload-arch={ARCH}",
    # keep the compiler from emitting packed FP32 arithmetic
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-Wno-unused-result",
]


SOURCES_HIP = ["api.hip", "contract_mixed.hip", "contract_fp64.hip", "state.hip", "adjoint.hip", "noalloc.hip", "hydro.hip"]


def build(verbose: bool = False, checks: bool = False) -> str:
    lib = LIB_CHECKS if checks else LIB
    tag = "_checks" if checks else ""
    flags = HIP_FLAGS + (["-DGD_CHECKS"] if checks else [])
    objs = []
    cmds = []
    obj = os.path.join(CSRC, f"tensor_build{tag}.o")
    cmds.append(["g++", "-O2", "-std=c++17", "-fPIC", "-pthread", "-c", os.path.join(CSRC, "tensor_build.cpp"),
                 "-o", obj])
    objs.append(obj)
    for src in SOURCES_HIP:
        o = os.path.join(CSRC, src.replace(".hip", f"{tag}.o"))
        cmds.append([HIPCC, *flags, "-c", os.path.join(CSRC, src), "-o", o])
        objs.append(o)
    cmds.append([HIPCC, f"--offload-arch={ARCH}", "-shared", *objs, "-pthread", "-o", lib + ".tmp"])
    def run(c):
        if verbose:
            print(" ".join(c), flush=True)
        r = subprocess.run(c, capture_output=True, text=True)
        if r.returncode != 0:
            sys.stderr.write(r.stdout + r.stderr)
            raise RuntimeError("build failed: " + " ".join(c))
        if verbose and r.stderr.strip():
            # hipcc's host pass warns that it does not know the packed-FP32 feature
            msgs = [ln for ln in r.stderr.splitlines() if "packed-fp32-ops" not in ln]
            if msgs:
                sys.stderr.write("\n".join(msgs) + "\n")

    # objects in parallel (the contraction sources take the longest), then the link
    with ThreadPoolExecutor(max_workers=min(8, os.cpu_count() or 1)) as ex:
        for f in [ex.submit(run, c) for c in cmds[:-1]]:
            f.result()
    run(cmds[-1])
    os.replace(lib + ".tmp", lib)
    for o in objs:
        os.remove(o)
    return lib


if __name__ == "__main__":
    print(build(verbose=True, checks=len(sys.argv) > 1 and sys.argv[1] == "checks"))
