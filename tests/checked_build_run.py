"""Runs a fixed sequence of library calls on seeded inputs and stores the results
(used by tests/test_gpu_checks.py, once with the regular build and once, in a child
process with GRACEDG_LIBRARY=checks, with the checked build):

    python tests/checked_build_run.py OUT.npz

Two groups (a 12-bin order-3 tensor with blended threshold levels and a 16-bin
order-2 tensor), both precisions, two lanes: the raw flux vector and L of one
evaluation, three SSP-RK3 steps, two per-cell sub-steps; then L of a state with one
non-finite coefficient.  Where the build has device checks, the check word after
the regular calls and after the non-finite one is stored too."""
import os
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(HERE))

import numpy as np  # noqa: E402
import torch  # noqa: E402

from paper_2607_13740_amd import gracedg as G  # noqa: E402
from paper_2607_13740_amd import workloads as W  # noqa: E402

DEV = "cuda:0"


def cells(t, n, seed):
    p = W.lognormal_cells(n, seed)
    x = t.projection_points()
    smp = np.stack([W.lognormal_density(x, p["mu"][c] + 3.0, p["sigma"][c], p["mass"][c]) for c in range(n)])
    return t.project(torch.tensor(smp, device=DEV)).reshape(-1), p


def main(out):
    lv = W.VFRAG_LEVELS
    t1 = G.Tensor(12, 3, 1e-4, 1e8, kernel="ballistic", frag="powerlaw", levels=lv, conservative=True)
    t2 = G.Tensor(16, 2, 1e-4, 1e8, kernel="ballistic", frag="powerlaw", levels=(0.5,), conservative=True)
    C1, C2 = 300, 200
    g1, p1 = cells(t1, C1, 5)
    g2, p2 = cells(t2, C2, 6)
    g0 = torch.cat([g1, g2])
    ks = torch.tensor(np.concatenate([p1["kscale"], p2["kscale"]]), device=DEV)
    vf = np.concatenate([p1["vfrag"], np.full(C2, 0.5)])
    res = {}
    for prec in ("fp64", "mixed"):
        plan = G.Plan([t1, t2], [C1, C2], precision=prec, vfrag=vf)
        plan.set_lanes(2)
        raw = torch.zeros(plan.n_raw, dtype=torch.float64, device=DEV)
        L = plan.collision_rhs(g0, kscale=ks, raw=raw)
        g = g0.clone()
        plan.rk_step(g, 1e-9, 3, kscale=ks)
        ga = g0.clone()
        td = torch.zeros(plan.n_cells, dtype=torch.float64, device=DEV)
        plan.rk_advance(ga, td, 1e-7, 0.1, 1e-8, 2, kscale=ks, flux_floor=1e-4)
        torch.cuda.synchronize()
        for name, v in (("raw", raw), ("L", L), ("step", g), ("advance", ga), ("clock", td)):
            res[f"{prec}_{name}"] = v.cpu().numpy()
        try:
            res[f"{prec}_checks"] = np.array(plan.checks())
            bad = g0.clone()
            bad[7] = float("nan")
            plan.collision_rhs(bad, kscale=ks)
            res[f"{prec}_checks_nonfinite"] = np.array(plan.checks())
            res[f"{prec}_checks_after_read"] = np.array(plan.checks())
        except G.GDError as e:
            res[f"{prec}_checks_error"] = np.array(e.code)
    np.savez(out, **res)


if __name__ == "__main__":
    main(sys.argv[1])
