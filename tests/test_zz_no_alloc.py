"""The no-allocation right-hand side (gd_collision_rhs_noalloc) against the plan-based
gd_collision_rhs, through the C ABI, on two calls in a row (the second with fewer
cells, so that stale workspace contents of the first would show), in both
precisions.  Same kernels and the same per-tile arithmetic: the results agree to the
parity bars (1e-12 FP64, 1e-6 split FP16, per cell normwise on the raw flux vector)
and are expected to be bit-identical."""
import numpy as np
import pytest

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

from paper_2607_13740_amd import gracedg as G  # noqa: E402
from paper_2607_13740_amd import workloads as W  # noqa: E402

DEV = "cuda:0"


def _states(t, C, seed):
    p = W.lognormal_cells(C, seed)
    x = t.projection_points()
    smp = np.stack([W.lognormal_density(x, p["mu"][c], p["sigma"][c], p["mass"][c]) for c in range(C)])
    g = t.project(torch.tensor(smp, device=DEV))
    return g.reshape(-1).contiguous(), torch.tensor(p["kscale"], device=DEV)


@pytest.mark.parametrize("prec", ["fp64", "mixed"])
def test_noalloc_rhs_matches_plan(prec):
    t = G.Tensor(24, 3, 1e-4, 1e8, kernel="ballistic", frag="powerlaw", levels=(0.5,), conservative=True)
    t.upload()
    for C, seed in ((200, 11), (70, 12)):
        print(f"noalloc {prec} C={C} P={t.P}", flush=True)
        g, ks = _states(t, C, seed)
        plan = G.Plan(t, C, precision=prec)
        raw_p = torch.zeros(C * t.n_out, dtype=torch.float64, device=DEV)
        L_p = plan.collision_rhs(g, kscale=ks, raw=raw_p)
        raw_n = torch.full((C * t.n_out,), float("nan"), dtype=torch.float64, device=DEV)
        L_n = t.collision_rhs_noalloc(g, precision=prec, kscale=ks, raw=raw_n)
        torch.cuda.synchronize()
        a, b = raw_n.view(C, -1).cpu().numpy(), raw_p.view(C, -1).cpu().numpy()
        eps = np.max(np.abs(a - b), axis=1) / np.max(np.abs(b), axis=1)
        tol = 1e-12 if prec == "fp64" else 1e-6
        assert np.isfinite(a).all() and eps.max() <= tol, (C, eps.max())
        Ln, Lp = L_n.view(C, -1).cpu().numpy(), L_p.view(C, -1).cpu().numpy()
        assert np.isfinite(Ln).all()
        h = np.repeat(np.diff(t.edges()), t.order + 1)
        scale = (h[None, :] * np.abs(Lp)).max(axis=1)
        assert (np.max(np.abs(Ln - Lp) * h[None, :], axis=1) / scale).max() <= 3 * tol
        print(f"  max eps {eps.max():.2e}, bit-identical raw: {np.array_equal(a, b)}", flush=True)


def test_noalloc_rejects_beyond_scratch_and_unuploaded():
    t = G.Tensor(24, 3, 1e-4, 1e8, kernel="ballistic", frag="powerlaw", levels=(0.5,), conservative=True)
    g = torch.zeros(t.P, dtype=torch.float64, device=DEV)
    with pytest.raises(G.GDError):
        t.collision_rhs_noalloc(g)                      # device layouts not uploaded yet
    t.upload()
    C = 20000                                           # beyond 16 MiB at P = 96
    big = torch.zeros(C * t.P, dtype=torch.float64, device=DEV)
    with pytest.raises(G.GDError):
        t.collision_rhs_noalloc(big, precision="mixed")
