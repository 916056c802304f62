"""GPU tests of the reverse mode: the FP64 adjoint of the collision step against
central finite differences of the oracle (FP64, CPU).

The right-hand side is quadratic in the state and linear in the kernel scale and
(inside a threshold bracket) in the blend weight, so central differences of the
oracle's L are exact up to rounding there; through RK steps and the limiter they
are accurate to O(h^2).  Bar: 1e-7 relative for the FP64 adjoint.  Directions are
seeded; the limiter is active in the start state (noisy higher coefficients), and
the step stays inside the region where the oracle reports no violation.
"""
import numpy as np
import pytest

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

from paper_2607_13740_amd import gracedg as G  # noqa: E402
from paper_2607_13740_amd import workloads as W  # noqa: E402

DEV = "cuda:0"
LV = W.VFRAG_LEVELS


def _case(O, N=8, k=2, C=12, seed=3, conservative=True, levels=LV, kernel="ballistic", noise=0.3):
    t = G.Tensor(N, k, 1e-4, 1e8, kernel=kernel, frag="powerlaw", levels=levels, conservative=conservative)
    cfg = O.Config(N=N, k=k, xmin=1e-4, xmax=1e8, kernel=kernel, frag="powerlaw", conservative=conservative,
                   levels=levels if len(levels) > 1 else (), vfrag=levels[0])
    rng = np.random.default_rng(seed)
    g = np.stack([O.project(cfg, lambda x, mu=mu: W.lognormal_density(x, mu, 1.0, 1.0))
                  for mu in rng.uniform(np.log(30.0), np.log(3000.0), C)])
    g = g.reshape(C, N, k + 1)
    g[:, :, 1:] += noise * rng.standard_normal((C, N, k)) * np.abs(g[:, :, :1])
    g = g.reshape(C, -1)
    ks = np.exp(0.5 * rng.standard_normal(C))
    vf = rng.uniform(0.32, 0.98, C) if len(levels) > 1 else None
    return t, cfg, g, ks, vf, rng


def _dev(a):
    return torch.tensor(np.ascontiguousarray(a), device=DEV)


@pytest.mark.parametrize("conservative,N,k,C", [(True, 8, 2, 12), (False, 8, 2, 12), (True, 52, 3, 4)])
def test_collision_vjp_matches_oracle_differences(oracle, conservative, N, k, C):
    """One right-hand-side product; the last case is the widest shape (P = 208, 13 K
    steps of the transposed tensor)."""
    O = oracle
    t, cfg, g, ks, vf, rng = _case(O, N=N, k=k, C=C, conservative=conservative)
    C, P = g.shape
    plan = G.Plan(t, C, precision="fp64", vfrag=vf)
    mu = rng.standard_normal((C, P))
    grad, dks, dvf = plan.collision_vjp(_dev(g).view(-1), _dev(mu).view(-1), kscale=_dev(ks))
    grad, dks, dvf = grad.cpu().numpy().reshape(C, P), dks.cpu().numpy(), dvf.cpu().numpy()

    def f(gg, kk=ks, vv=vf):
        return (O.rhs(cfg, gg, kscale=kk, vfrag=vv)[1] * mu).sum(axis=1)

    for _ in range(3):
        d = rng.standard_normal((C, P)) * np.abs(g).max(axis=1, keepdims=True)
        h = 1e-3
        fd = (f(g + h * d) - f(g - h * d)) / (2 * h)
        ad = (grad * d).sum(axis=1)
        assert np.max(np.abs(ad - fd) / np.maximum(np.abs(fd), 1e-300)) <= 1e-7, (ad, fd)
    # kernel scale: mu . L is linear in s
    fd = (f(g, ks * (1 + 1e-3)) - f(g, ks * (1 - 1e-3))) / (2e-3 * ks)
    assert np.max(np.abs(dks - fd) / np.abs(fd)) <= 1e-7
    # threshold: linear in the blend weight inside a bracket
    hv = 1e-4
    assert np.min(np.abs(vf[:, None] - np.array(LV)[None, :])) > 2 * hv
    fd = (f(g, ks, vf + hv) - f(g, ks, vf - hv)) / (2 * hv)
    scale = np.abs(fd).max()
    assert np.max(np.abs(dvf - fd)) <= 1e-7 * scale, (dvf, fd)


def _loss_oracle(O, cfg, g0, ks, vf, dt, n, w):
    gf, v = O.rk(cfg, g0, dt, n, kscale=ks, vfrag=vf)
    assert v == 0
    return (gf * w).sum(axis=1)


@pytest.mark.parametrize("prec", ["fp64", "mixed"])
def test_rk_adjoint_matches_oracle_differences(oracle, prec):
    """Loss = sum_c w_c . g_c(final) after 3 limited SSP-RK3 steps; gradients with
    respect to the initial state (directional), kernel scales and thresholds."""
    O = oracle
    t, cfg, g, ks, vf, rng = _case(O, C=10, seed=5)
    C, P = g.shape
    # a step well inside the oracle's violation-free range for these states (3e-5
    # already produces a negative bin average)
    dt, n = 1e-5, 3
    w = rng.standard_normal((C, P))
    plan = G.Plan(t, C, precision=prec, vfrag=vf)
    gd = _dev(g).view(-1)
    st, gm, v = plan.rk_forward(gd, dt, n, kscale=_dev(ks), count_violations=True)
    assert v == 0
    # the limiter was active on the start state (the adjoint passes through it)
    assert (gm[:plan.n_bins].cpu().numpy() < 1.0).sum() > 0
    lam = _dev(w).view(-1).clone()
    dks, dvf = plan.adjoint(st, gm, dt, n, lam, kscale=_dev(ks))
    lam, dks, dvf = lam.cpu().numpy().reshape(C, P), dks.cpu().numpy(), dvf.cpu().numpy()
    tol = 1e-7 if prec == "fp64" else 1e-5
    for _ in range(2):
        # relative perturbation of every coefficient (d_p = g_p zeta_p), so that bins
        # holding almost no mass stay where they are
        d = rng.standard_normal((C, P)) * g
        h = 1e-6
        fd = (_loss_oracle(O, cfg, g + h * d, ks, vf, dt, n, w) - _loss_oracle(O, cfg, g - h * d, ks, vf, dt, n, w)) / (2 * h)
        ad = (lam * d).sum(axis=1)
        assert np.max(np.abs(ad - fd) / np.abs(fd)) <= tol, (ad, fd)
    # steps small enough for O(h^2) to vanish at this bar (1e-3 is not), large enough
    # for rounding of the loss
    hk = 1e-5
    fd = (_loss_oracle(O, cfg, g, ks * (1 + hk), vf, dt, n, w) - _loss_oracle(O, cfg, g, ks * (1 - hk), vf, dt, n, w)) / (2 * hk * ks)
    assert np.max(np.abs(dks - fd)) <= tol * np.abs(fd).max(), (dks, fd)
    hv = 1e-5
    assert np.min(np.abs(vf[:, None] - np.array(LV)[None, :])) > 2 * hv
    fd = (_loss_oracle(O, cfg, g, ks, vf + hv, dt, n, w) - _loss_oracle(O, cfg, g, ks, vf - hv, dt, n, w)) / (2 * hv)
    assert np.max(np.abs(dvf - fd)) <= tol * np.abs(fd).max(), (dvf, fd)


@pytest.mark.parametrize("N,k,dt,n", [(12, 0, 1e-5, 2), (10, 1, 1e-5, 2), (28, 3, 5e-6, 1), (8, 4, 1e-5, 2)])
def test_rk_adjoint_orders_and_wide_state(oracle, N, k, dt, n):
    """Orders 0, 1, 3 and 4, order 3 with P = 112 (more than 96 coefficients: the wide
    reverse-stage and vector-Jacobian instantiations): FP64 adjoint against oracle
    differences for the initial state, kernel scales and thresholds."""
    O = oracle
    t, cfg, g, ks, vf, rng = _case(O, N=N, k=k, C=4, seed=17)
    C, P = g.shape
    w = rng.standard_normal((C, P))
    plan = G.Plan(t, C, precision="fp64", vfrag=vf)
    st, gm, v = plan.rk_forward(_dev(g).view(-1), dt, n, kscale=_dev(ks), count_violations=True)
    assert v == 0
    if k > 0:
        assert (gm[:plan.n_bins].cpu().numpy() < 1.0).sum() > 0
    lam = _dev(w).view(-1).clone()
    dks, dvf = plan.adjoint(st, gm, dt, n, lam, kscale=_dev(ks))
    lam, dks, dvf = lam.cpu().numpy().reshape(C, P), dks.cpu().numpy(), dvf.cpu().numpy()
    loss = lambda gg=g, kk=ks, vv=vf: _loss_oracle(O, cfg, gg, kk, vv, dt, n, w)
    d = rng.standard_normal((C, P)) * g
    h = 1e-6
    fd = (loss(gg=g + h * d) - loss(gg=g - h * d)) / (2 * h)
    assert np.max(np.abs((lam * d).sum(axis=1) - fd) / np.abs(fd)) <= 1e-7, ((lam * d).sum(axis=1), fd)
    hk = 1e-5
    fd = (loss(kk=ks * (1 + hk)) - loss(kk=ks * (1 - hk))) / (2 * hk * ks)
    assert np.max(np.abs(dks - fd)) <= 1e-7 * np.abs(fd).max(), (dks, fd)
    hv = 1e-5
    assert np.min(np.abs(vf[:, None] - np.array(LV)[None, :])) > 2 * hv
    fd = (loss(vv=vf + hv) - loss(vv=vf - hv)) / (2 * hv)
    assert np.max(np.abs(dvf - fd)) <= 1e-7 * np.abs(fd).max(), (dvf, fd)


def test_mass_gradient(oracle):
    """Total mass is conserved by every stage and untouched by the limiter, so for
    Loss = sum_j h_j g_j^0(final) the gradient is h_j on the averages, zero on the
    higher coefficients, and zero for the kernel scales and thresholds."""
    O = oracle
    t, cfg, g, ks, vf, rng = _case(O, C=16, seed=8)
    C, P = g.shape
    plan = G.Plan(t, C, precision="fp64", vfrag=vf)
    gd = _dev(g).view(-1)
    dt, n = 1e-5, 4
    st, gm = plan.rk_forward(gd, dt, n, kscale=_dev(ks))
    h = np.diff(O.edges(cfg))
    w = np.zeros((C, cfg.N, cfg.k + 1))
    w[:, :, 0] = h
    lam = _dev(w).view(-1).clone()
    dks, dvf = plan.adjoint(st, gm, dt, n, lam, kscale=_dev(ks))
    lam = lam.cpu().numpy().reshape(C, cfg.N, cfg.k + 1)
    assert np.max(np.abs(lam[:, :, 0] - h) / h) <= 1e-10
    assert np.max(np.abs(lam[:, :, 1:])) <= 1e-10 * h.max()
    # scale of the individual terms: |lam| times the size of one stage's mass flux
    ref = np.abs(O.rhs(cfg, g, kscale=ks, vfrag=vf)[1].reshape(C, cfg.N, -1)[:, :, 0] * h).sum(axis=1) * dt * n
    assert np.all(np.abs(dks.cpu().numpy()) <= 1e-10 * ref / ks)
    assert np.all(np.abs(dvf.cpu().numpy()) <= 1e-9 * ref * 10)


def test_autograd_function(oracle):
    """torch.autograd through RKSolve gives the adjoint's gradients."""
    O = oracle
    t, cfg, g, ks, vf, rng = _case(O, C=6, seed=11)
    C, P = g.shape
    plan = G.Plan(t, C, precision="fp64", vfrag=vf)
    g0 = _dev(g).view(-1).requires_grad_(True)
    kst = _dev(ks).requires_grad_(True)
    vft = _dev(vf).requires_grad_(True)
    w = _dev(rng.standard_normal((C, P))).view(-1)
    out = G.rk_solve(plan, g0, 2e-6, 2, kscale=kst, vfrag=vft)
    loss = (out * w).sum()
    gg, gk, gv = torch.autograd.grad(loss, (g0, kst, vft))
    st, gm = plan.rk_forward(_dev(g).view(-1), 2e-6, 2, kscale=_dev(ks))
    lam = w.clone()
    dks, dvf = plan.adjoint(st, gm, 2e-6, 2, lam, kscale=_dev(ks))
    assert torch.equal(gg, lam) and torch.equal(gk, dks) and torch.equal(gv, dvf)


def test_adjoint_of_uneven_batch_matches_single_groups(oracle):
    """Two groups of different shape (one with threshold levels, one without) in one
    plan: the reverse pass over the batch equals the reverse passes of the groups run
    alone."""
    O = oracle
    t1, cfg1, g1, ks1, vf1, rng = _case(O, N=8, k=2, C=9, seed=13)
    t2, cfg2, g2, ks2, _, _ = _case(O, N=6, k=1, C=5, seed=14, levels=(0.5,))
    dt, n = 5e-6, 2
    w1 = rng.standard_normal(g1.shape)
    w2 = rng.standard_normal(g2.shape)
    both = G.Plan([t1, t2], [9, 5], precision="fp64", vfrag=np.concatenate([vf1, np.full(5, 0.5)]))
    g = _dev(np.concatenate([g1.reshape(-1), g2.reshape(-1)]))
    ks = _dev(np.concatenate([ks1, ks2]))
    st, gm = both.rk_forward(g, dt, n, kscale=ks)
    lam = _dev(np.concatenate([w1.reshape(-1), w2.reshape(-1)]))
    dks, dvf = both.adjoint(st, gm, dt, n, lam, kscale=ks)
    outs = []
    for t, gg, kk, vv, ww in ((t1, g1, ks1, vf1, w1), (t2, g2, ks2, None, w2)):
        p = G.Plan(t, len(gg), precision="fp64", vfrag=vv)
        s1, m1 = p.rk_forward(_dev(gg).view(-1), dt, n, kscale=_dev(kk))
        l1 = _dev(ww).view(-1).clone()
        d1, v1 = p.adjoint(s1, m1, dt, n, l1, kscale=_dev(kk))
        outs.append((l1, d1, v1))
    n1 = g1.size
    assert torch.allclose(lam[:n1], outs[0][0], rtol=1e-13, atol=0)
    assert torch.allclose(lam[n1:], outs[1][0], rtol=1e-13, atol=0)
    assert torch.allclose(dks[:9], outs[0][1], rtol=1e-12, atol=1e-300)
    assert torch.allclose(dks[9:], outs[1][1], rtol=1e-12, atol=1e-300)
    assert torch.allclose(dvf[:9], outs[0][2], rtol=1e-12, atol=1e-300)
    assert float(dvf[9:].abs().max()) == 0.0      # single-level group: no threshold dependence


def _moment_weights(edges, k, R=32):
    """W[p][j(k+1)+i] = int_{I_j} x^(p-1) P_i(xi(x)) dx, p = 0..3 (R-point Gauss per bin), so
    that the moment M_p = W[p] . g (Sec. 4.1)."""
    s, w = np.polynomial.legendre.leggauss(R)
    N = len(edges) - 1
    W = np.zeros((4, N * (k + 1)))
    for j in range(N):
        a, b = edges[j], edges[j + 1]
        x = 0.5 * (a + b) + 0.5 * (b - a) * s
        for i in range(k + 1):
            Pi = np.polynomial.legendre.Legendre.basis(i)(s)
            for p in range(4):
                W[p, j * (k + 1) + i] = 0.5 * (b - a) * np.sum(w * x ** (p - 1) * Pi)
    return W


@pytest.mark.parametrize("prec", ["fp64", "mixed"])
def test_c5_moment_loss_gradient_matches_oracle_finite_differences(prec):
    """The adjoint workload's loss (Sec. 4.1 moments M_0..M_3 of the final state against
    seeded targets) over 200 steps of dt = 2e-8 on four of its cells, per-cell kernel
    scale and threshold blended between levels: the library's reverse pass against
    central differences of the FP64 oracle (h = 1e-6; tests/golden/c5_fd.json, written
    by the oracle alone) along 8 seeded directions d = g0 * zeta and per cell for the
    kernel scale, and per cell for the threshold with step 1e-3 inside its bracket (the
    threshold moves the loss by less than an ulp at 1e-6; its check allows the
    quotient's rounding resolution).  Cases where the oracle's limiter changed a
    different set of bins in the perturbed runs are reported and left out.  Bar
    (relative to the largest derivative of each kind): 1e-7 for the FP64 forward, 1e-4
    with the split-FP16 forward (its states carry ~1e-7 of rounding)."""
    import json
    import os
    gold = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "c5_fd.json")))
    w = W.WORKLOADS["c5_adjoint"]
    C = len(gold["cells"])
    t = G.Tensor(w.bins, w.order, w.x_min, w.x_max, kernel=w.kernel, frag=w.frag, levels=tuple(gold["levels"]),
                 conservative=w.conservative)
    g0 = np.asarray(gold["g0"])
    ks, vf = np.asarray(gold["kscale"]), np.asarray(gold["vfrag"])
    plan = G.Plan(t, C, precision=prec, vfrag=vf)
    Wm = _moment_weights(t.edges(), w.order)
    Mstar = np.asarray(gold["Mstar"])
    g = torch.tensor(g0, device=DEV).view(-1).clone()
    ksd = torch.tensor(ks, device=DEV)
    st, gm = plan.rk_forward(g, gold["dt"], gold["steps"], kscale=ksd)
    M = g.view(C, -1).cpu().numpy() @ Wm.T
    loss = float((((M - Mstar) / Mstar) ** 2).sum())
    print(f"c5 {prec}: loss {loss:.10e} (oracle {gold['loss']:.10e})", flush=True)
    assert abs(loss - gold["loss"]) <= (1e-10 if prec == "fp64" else 1e-5) * abs(gold["loss"])
    lam = torch.tensor(((2.0 * (M - Mstar) / Mstar ** 2) @ Wm).reshape(-1), device=DEV)
    dks, dvf = plan.adjoint(st, gm, gold["dt"], gold["steps"], lam, kscale=ksd)
    grad = lam.view(C, -1).cpu().numpy()
    tol = 1e-7 if prec == "fp64" else 1e-4
    zeta = np.random.default_rng(gold["dir_seed"]).standard_normal((gold["n_dirs"],) + g0.shape)
    fd = np.asarray(gold["fd_dir"])
    ad = np.array([np.sum(grad * g0 * zeta[i]) for i in range(len(fd))])
    keep = np.asarray(gold["same_active_set_dir"])
    rel = np.abs(ad - fd) / np.abs(fd).max()
    print(f"  directions: max rel error {rel[keep].max():.2e}, left out (active set changed): {int((~keep).sum())}",
          flush=True)
    assert keep.sum() >= 4 and rel[keep].max() <= tol, rel
    a, b = dks.cpu().numpy(), np.asarray(gold["fd_kscale"])
    keep = np.asarray(gold["same_active_set_kscale"])
    rel = np.abs(a - b) / np.abs(b).max()
    print(f"  kscale: max rel error {rel[keep].max():.2e}, left out: {int((~keep).sum())}", flush=True)
    assert keep.sum() >= 2 and rel[keep].max() <= tol, ("kscale", rel)
    # the threshold moves each cell's loss term by ~1e-12 per unit over this horizon:
    # the oracle's quotient (step hv) resolves it only to the rounding of the loss
    # terms, taken here as 256 ulp of the larger of L_c(v +- hv) over 2 hv
    a, b = dvf.cpu().numpy(), np.asarray(gold["fd_vfrag"])
    keep = np.asarray(gold["same_active_set_vfrag"])
    res = 256 * np.finfo(float).eps * np.abs(np.asarray(gold["loss_vfrag_pm"])).max(axis=1) / (2 * gold["hv"])
    err = np.abs(a - b)
    print(f"  vfrag: adjoint {a}, oracle quotient {b}, resolution {res}, left out: {int((~keep).sum())}", flush=True)
    assert keep.sum() >= 2 and np.all(err[keep] <= tol * np.abs(b).max() + res[keep]), ("vfrag", err, res)
