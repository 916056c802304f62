"""Writes c2_trajectory.json beside this script: the FP64 oracle's states of the
single-cell ballistic workload -- 32 bins of order 2 on [1e-4, 1e8], ballistic kernel
K = (x^1/3 + y^1/3)^2 dv with dv = x^-1/6 + y^-1/6, power-law fragments (alpha = -11/6)
for dv > v_frag = 0.5, conservative flux, LN(0,1) unit-mass initial profile projected
with 16 points per bin (Sec. 3.2, Eq. init) -- after 100, 300 and 1000 SSP-RK3 steps of
dt = 5e-7 with the limiter on the start state and after every stage (Eq. RK3,
Eq. gamma), run as consecutive calls of 100, 200 and 700 steps.  It calls only the
oracle (and the seeded input module for the profile); the GPU trajectory test reads
the file.

    python tests/golden/make_c2_trajectory.py        (about 6 minutes on one core)
"""
import json
import os
import sys
import time

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

from oracle import oracle as O  # noqa: E402
from paper_2607_13740_amd import workloads as W  # noqa: E402

CONFIG = dict(N=32, k=2, xmin=1e-4, xmax=1e8, kernel="ballistic", frag="powerlaw", conservative=True, vfrag=0.5)
DT = 5e-7
CHUNKS = (100, 200, 700)


def main():
    cfg = O.Config(**CONFIG)
    g0 = O.project(cfg, W.lognormal_density)
    out = {"config": CONFIG, "dt": DT, "g0": g0.tolist(), "states": {}, "violations": 0}
    g, n = g0.copy(), 0
    t0 = time.time()
    for m in CHUNKS:
        g, v = O.rk(cfg, g, DT, m)
        g = g.reshape(-1)
        n += m
        out["states"][str(n)] = g.tolist()
        out["violations"] += v
        print(f"{n} steps, {v} violations, {time.time() - t0:.0f} s", flush=True)
    with open(os.path.join(HERE, "c2_trajectory.json"), "w") as f:
        json.dump(out, f)


if __name__ == "__main__":
    main()
