"""Writes c5_fd.json beside this script: central finite differences of the FP64
oracle for the reverse-mode test of the adjoint workload.  Four cells of the adjoint
workload (32 bins of order 2 on [1e-4, 1e8], ballistic kernel with power-law
fragmentation, per-cell kernel scale and fragmentation threshold blended between the
levels 0.3 .. 1.0, conservative flux; the seeded per-cell lognormal profiles, seed 3),
200 SSP-RK3 steps of dt = 2e-8, loss
    L = sum_c sum_{p=0..3} ((M_p,c - M*_p,c) / M*_p,c)^2,
M_p = int x^(p-1) g dx (Sec. 4.1) of the final state, M* = the oracle's unperturbed
final moments times exp(0.1 eps), eps ~ N(0,1) from numpy's PCG64 with seed 3 (rows
of the workload's 4096 x 4 draw).  Stored: the inputs, the targets, and
  * along 8 seeded directions d = g0 * zeta (zeta ~ N(0,1), seed 20, per coefficient):
    (L(g0 + h d) - L(g0 - h d)) / (2h), h = 1e-6;
  * per cell: dL_c/ds_c from s_c (1 +- h) and dL_c/dv_c from v_c +- hv, hv = 1e-3
    (the threshold moves the loss by less than an ulp at h; hv keeps every cell
    inside its bracket of levels, where the flux is linear in the blend weight)
    (cells are independent, so all cells move at once and each cell's own loss term
    is read), with each cell's loss term at v_c +- hv for the resolution of the
    quotient;
  * whether the limiter changed the same bins in the perturbed and the unperturbed
    runs (a hash of every bin the limiter touched, per cell).
It calls only the oracle and the seeded input module.

    python tests/golden/make_c5_fd.py         (about 30-60 minutes on 4 cores)
"""
import json
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

from oracle import oracle as O  # noqa: E402
from paper_2607_13740_amd import workloads as W  # noqa: E402

CELLS = (0, 1, 2, 3)
DT, STEPS, H, HV = 2e-8, 200, 1e-6, 1e-3
N_DIRS, DIR_SEED = 8, 20


def main():
    w = W.WORKLOADS["c5_adjoint"]
    cfg = O.Config(N=w.bins, k=w.order, xmin=w.x_min, xmax=w.x_max, kernel=w.kernel, frag=w.frag,
                   conservative=w.conservative, levels=w.levels)
    p = W.lognormal_cells(w.cells, w.seed)
    ids = np.array(CELLS)
    g0 = np.stack([O.project(cfg, lambda x, c=c: W.lognormal_density(x, p["mu"][c], p["sigma"][c], p["mass"][c]))
                   for c in ids])
    ks, vf = p["kscale"][ids], p["vfrag"][ids]
    t0 = time.time()

    def run(g, k, v):
        gT, viol, tr = O.rk_traced(cfg, g, DT, STEPS, kscale=k, vfrag=v)
        M = np.stack([O.moments(cfg, gT, q) for q in range(4)], axis=1)
        print(f"  trajectory done, {time.time() - t0:.0f} s", flush=True)
        return M, viol, tr

    M0, viol0, tr0 = run(g0, ks, vf)
    eps = np.random.default_rng(w.seed).standard_normal((w.cells, 4))[ids]
    Mstar = M0 * np.exp(0.1 * eps)
    per_cell = lambda M: (((M - Mstar) / Mstar) ** 2).sum(axis=1)
    zeta = np.random.default_rng(DIR_SEED).standard_normal((N_DIRS,) + g0.shape)
    fd_dir, same_dir = [], []
    for i in range(N_DIRS):
        d = g0 * zeta[i]
        Mp, _, trp = run(g0 + H * d, ks, vf)
        Mm, _, trm = run(g0 - H * d, ks, vf)
        fd_dir.append(float((per_cell(Mp).sum() - per_cell(Mm).sum()) / (2 * H)))
        same_dir.append(bool(np.array_equal(trp, tr0) and np.array_equal(trm, tr0)))
    Mp, _, trp = run(g0, ks * (1 + H), vf)
    Mm, _, trm = run(g0, ks * (1 - H), vf)
    fd_ks = ((per_cell(Mp) - per_cell(Mm)) / (2 * H * ks)).tolist()
    same_ks = [bool(a == b == c) for a, b, c in zip(trp, trm, tr0)]
    Mp, _, trp = run(g0, ks, vf + HV)
    Mm, _, trm = run(g0, ks, vf - HV)
    fd_vf = ((per_cell(Mp) - per_cell(Mm)) / (2 * HV)).tolist()
    loss_vf = np.stack([per_cell(Mp), per_cell(Mm)], axis=1).tolist()
    same_vf = [bool(a == b == c) for a, b, c in zip(trp, trm, tr0)]
    out = {"cells": list(CELLS), "dt": DT, "steps": STEPS, "h": H, "g0": g0.tolist(), "kscale": ks.tolist(),
           "vfrag": vf.tolist(), "levels": list(w.levels), "Mstar": Mstar.tolist(), "loss": float(per_cell(M0).sum()),
           "violations": int(viol0), "n_dirs": N_DIRS, "dir_seed": DIR_SEED, "fd_dir": fd_dir,
           "same_active_set_dir": same_dir, "fd_kscale": fd_ks, "same_active_set_kscale": same_ks,
           "fd_vfrag": fd_vf, "same_active_set_vfrag": same_vf, "hv": HV, "loss_vfrag_pm": loss_vf}
    with open(os.path.join(HERE, "c5_fd.json"), "w") as f:
        json.dump(out, f)
    print("written", flush=True)


if __name__ == "__main__":
    main()
