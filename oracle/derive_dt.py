"""Half of the CFL bound (Eq. dt) over the seeded initial states of each workload,
evaluated with the oracle on a sample of cells.  Prints the values that the
workload table freezes as time steps.  Test infrastructure (uses the oracle)."""
import os
import sys

import numpy as np

sys.path.insert(0, os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
from oracle import oracle as O  # noqa: E402
from paper_2607_13740_amd import workloads as W  # noqa: E402


def cfg_for(w, bins, order):
    return O.Config(N=bins, k=order, xmin=w.x_min, xmax=w.x_max, kernel=w.kernel, frag=w.frag,
                    conservative=w.conservative, vfrag=w.levels[0] if len(w.levels) == 1 else 0.5,
                    levels=w.levels if len(w.levels) > 1 else ())


def initial(w, cfg, n, params=None):
    out = []
    for c in range(n):
        if w.profile == "xexp":
            f = W.xexp_density
        elif w.profile == "lognormal_unit":
            f = W.lognormal_density
        else:
            f = (lambda mu, s, m: (lambda x: W.lognormal_density(x, mu, s, m)))(
                params["mu"][c], params["sigma"][c], params["mass"][c])
        out.append(O.project(cfg, f))
    g, _ = O.limit(cfg, np.array(out))
    return g


def main(sample=128):
    for name, w in W.WORKLOADS.items():
        params = W.lognormal_cells(w.cells, w.seed) if w.profile == "lognormal_cells" else None
        shapes = w.groups if w.groups else ((w.bins, w.order),)
        best = np.inf
        for (n, k) in shapes:
            cfg = cfg_for(w, n, k)
            m = min(sample, w.cells)
            g = initial(w, cfg, m, params)
            ks = params["kscale"][:m] if (params is not None and w.per_cell) else None
            vf = params["vfrag"][:m] if (params is not None and w.per_cell) else None
            best = min(best, O.cfl_dt(cfg, g, kscale=ks, vfrag=vf))
        print(f"{name}: CFL bound {best:.3e}  -> dt {0.5 * best:.3e}  (table: {w.dt:.3e})", flush=True)


if __name__ == "__main__":
    main(int(sys.argv[1]) if len(sys.argv) > 1 else 128)
