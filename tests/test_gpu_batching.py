"""GPU tests of the batching layer: uneven batches of several (bins, order) groups in
one contraction launch, the contraction variants, the autotuner and the captured
RK step.

 * every contraction variant (waves per workgroup, row blocks per work item)
   accumulates in the same order, so results must be bit-identical;
 * an uneven batch of the twelve (bins, order) shapes is checked group by group
   against the oracle (FP64: 1e-12, split FP16: 1e-6 per-cell normwise);
 * the captured RK step (a HIP graph replayed once per step) must reproduce the
   launch-by-launch step bit for bit, on every replay, with other work between.
"""
import numpy as np
import pytest

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

from paper_2607_13740_amd import gracedg as G  # noqa: E402
from paper_2607_13740_amd import workloads as W  # noqa: E402

DEV = "cuda:0"
# (waves, rows, xcd, tiles per wave)
VARIANTS = [(4, 1, 1, 1), (4, 2, 1, 1), (4, 0, 1, 1), (8, 1, 1, 1), (8, 2, 1, 1), (8, 0, 1, 1), (4, 1, 0, 1),
            (8, 2, 0, 1), (4, 1, 1, 2), (4, 0, 0, 2)]


def _eps(Yg, Yo):
    return np.max(np.abs(Yg - Yo), axis=1) / np.max(np.abs(Yo), axis=1)


def _cells(O, cfg, idx, p):
    if len(idx) == 0:
        return np.zeros((0, cfg.P))
    return np.stack([O.project(cfg, lambda x, c=c: W.lognormal_density(x, p["mu"][c], p["sigma"][c], p["mass"][c]))
                     for c in idx])


def _raw(plan, g, ks=None):
    raw = torch.zeros(plan.n_raw, dtype=torch.float64, device=DEV)
    plan.collision_rhs(g, kscale=ks, raw=raw)
    torch.cuda.synchronize()
    return raw


def _level_case(O):
    lv = W.VFRAG_LEVELS
    N, k, C = 12, 3, 600
    t = G.Tensor(N, k, 1e-4, 1e8, kernel="ballistic", frag="powerlaw", levels=lv, conservative=True)
    cfg = O.Config(N=N, k=k, xmin=1e-4, xmax=1e8, kernel="ballistic", frag="powerlaw", conservative=True, levels=lv)
    rng = np.random.default_rng(31)
    vf = rng.uniform(0.3, 1.0, C)
    g = np.stack([O.project(cfg, lambda x, mu=mu: W.lognormal_density(x, mu, 1.0, 1.0))
                  for mu in rng.uniform(np.log(30.0), np.log(3000.0), C)])
    ks = np.exp(0.5 * rng.standard_normal(C))
    return t, cfg, g, ks, vf


@pytest.mark.parametrize("prec", ["mixed", "fp64"])
def test_variants_are_bit_identical(oracle, prec):
    O = oracle
    t, cfg, g, ks, vf = _level_case(O)
    C = len(g)
    plan = G.Plan(t, C, precision=prec, vfrag=vf)
    gd = torch.tensor(g, device=DEV).view(-1)
    ksd = torch.tensor(ks, device=DEV)
    ref = None
    for w, r, x, tpw in VARIANTS:
        if tpw == 2 and prec == "fp64":
            continue
        print(f"variant {prec} waves={w} rows={r} xcd={x} tiles/wave={tpw}", flush=True)
        plan.set_variant(w, r, x, tpw)
        v = plan.variant()
        assert v["waves"] == w and v["rows"] == r and v["xcd"] == x and v["tiles_per_wave"] == tpw
        assert v["n_items"] > 0
        raw = _raw(plan, gd, ksd)
        if ref is None:
            ref = raw.clone()
            idx = np.arange(0, C, 37)
            Yo, _, _ = O.rhs(cfg, g[idx], kscale=ks[idx], vfrag=vf[idx])
            tol = 1e-12 if prec == "fp64" else 1e-6
            assert _eps(raw.view(C, -1)[idx].cpu().numpy(), Yo).max() <= tol
        else:
            assert torch.equal(raw, ref), (w, r, x, tpw)


def _uneven(O, counts, kernel="additive"):
    w = W.WORKLOADS["c4_uneven"]
    p = W.lognormal_cells(int(sum(counts)), 2)
    tensors, cfgs, states = [], [], []
    c0 = 0
    for (N, k), n in zip(w.groups, counts):
        tensors.append(G.Tensor(N, k, w.x_min, w.x_max, kernel=kernel, frag=w.frag, levels=w.levels,
                                conservative=w.conservative))
        cfg = O.Config(N=N, k=k, xmin=w.x_min, xmax=w.x_max, kernel=kernel, frag=w.frag,
                       conservative=w.conservative, vfrag=w.levels[0])
        cfgs.append(cfg)
        states.append(_cells(O, cfg, range(c0, c0 + n), p))
        c0 += n
    return tensors, cfgs, states


@pytest.mark.parametrize("prec", ["mixed", "fp64"])
def test_uneven_batch_matches_oracle(oracle, prec):
    """All twelve (bins, order) shapes, P = 32..192, in one plan with uneven cell
    counts (one group empty); each group's raw flux vectors against the oracle."""
    O = oracle
    counts = [7, 33, 0, 40, 5, 17, 1, 9, 3, 2, 31, 4]
    tensors, cfgs, states = _uneven(O, counts)
    plan = G.Plan(tensors, counts, precision=prec)
    g = np.concatenate([s.reshape(-1) for s in states if s.size])
    raw = _raw(plan, torch.tensor(g, device=DEV)).cpu().numpy()
    tol = 1e-12 if prec == "fp64" else 1e-6
    off = 0
    for cfg, s, n in zip(cfgs, states, counts):
        if n == 0:
            continue
        Yo, _, _ = O.rhs(cfg, s)
        Yg = raw[off:off + n * cfg.n_out].reshape(n, -1)
        off += n * cfg.n_out
        assert _eps(Yg, Yo).max() <= tol, (cfg.N, cfg.k, _eps(Yg, Yo).max())
    assert off == raw.size
    for w, r, x, tpw in VARIANTS[1:]:
        if tpw == 2:
            continue       # P up to 192 here: two tiles per wave serve P <= 96 only
        plan.set_variant(w, r, x, tpw)
        assert np.array_equal(_raw(plan, torch.tensor(g, device=DEV)).cpu().numpy(), raw), (w, r, x)


@pytest.mark.parametrize("prec", ["mixed", "fp64"])
def test_graph_replays_match_eager_steps(oracle, prec):
    """The captured step against the launch-by-launch step: several calls, every
    replay compared, with unrelated device work and host synchronisation between,
    and a change of dt (a new capture) in the middle."""
    O = oracle
    t, cfg, g, ks, vf = _level_case(O)
    C = len(g)
    g, _ = O.limit(cfg, g)
    # a step the oracle runs for 8 steps on these states without a limiter violation
    # (1/50 of the outflow bound of Eq. dt over all cells; 1/20 of it already diverges)
    dt = 2e-6
    ksd = torch.tensor(ks, device=DEV)
    pg = G.Plan(t, C, precision=prec, vfrag=vf)
    pe = G.Plan(t, C, precision=prec, vfrag=vf)
    pe.use_graph(False)
    a = torch.tensor(g, device=DEV).view(-1)
    b = a.clone()
    junk = torch.zeros(1 << 20, device=DEV)
    for n, d in ((1, dt), (2, dt), (1, 0.5 * dt), (3, 0.5 * dt)):
        va = pg.rk_step(a, d, n, kscale=ksd, count_violations=True)
        junk += 1.0
        torch.cuda.synchronize()
        vb = pe.rk_step(b, d, n, kscale=ksd, count_violations=True)
        assert bool(torch.isfinite(a).all())
        assert torch.equal(a, b), (n, d)
        assert va == vb
    assert float(junk[0]) == 4.0


def test_autotune_keeps_results_and_uses_cache(oracle, tmp_path):
    O = oracle
    t, cfg, g, ks, vf = _level_case(O)
    C = len(g)
    gd = torch.tensor(g, device=DEV).view(-1)
    ksd = torch.tensor(ks, device=DEV)
    plan = G.Plan(t, C, precision="mixed", vfrag=vf)
    ref = _raw(plan, gd, ksd)
    cache = str(tmp_path / "tune.txt")
    choice = plan.autotune(gd, kscale=ksd, cache_path=cache)
    assert (choice["waves"], choice["rows"]) in [(w, r) for w, r, _, _ in VARIANTS] and choice["xcd"] in (0, 1)
    assert choice["tiles_per_wave"] in (1, 2)
    assert torch.equal(_raw(plan, gd, ksd), ref)
    lines = open(cache).read().splitlines()
    assert len(lines) == 1 and lines[0].startswith("mixed;12x3r8c600")
    # a second plan of the same shape takes the stored choice (the file is not extended)
    p2 = G.Plan(t, C, precision="mixed", vfrag=vf)
    assert p2.autotune(gd, kscale=ksd, cache_path=cache) == choice
    assert open(cache).read().splitlines() == lines
    v = p2.variant()
    assert (v["waves"], v["rows"], v["xcd"], v["tiles_per_wave"]) == (choice["waves"], choice["rows"], choice["xcd"],
                                                                       choice["tiles_per_wave"])
    # a tensor of the same shape without fragmentation stores other fragments (the
    # contraction's cost follows the stored blocks, not their values): its plan does
    # not take the stored line, it is timed and appended; every key names the device
    t_nf = G.Tensor(12, 3, 1e-4, 1e8, kernel="const", frag="none", levels=W.VFRAG_LEVELS, conservative=True)
    p3 = G.Plan(t_nf, C, precision="mixed", vfrag=vf)
    assert p3.schedule_stats()["frags_mixed"] != plan.schedule_stats()["frags_mixed"]
    p3.autotune(gd, kscale=ksd, cache_path=cache)
    lines3 = open(cache).read().splitlines()
    assert len(lines3) == 2 and lines3[0] == lines[0], lines3
    assert lines3[1].split()[0] != lines[0].split()[0]
    assert all("@gfx" in ln.split()[0] for ln in lines3), lines3


def test_autotune_per_group_rows_keep_results_and_cache(tmp_path):
    """On an uneven batch the autotuner also picks the row blocks per item group by
    group; every choice accumulates in the same order (results bit for bit those of
    the default variant), the choice goes to the cache file, and a plan of the same
    shape takes it back from there."""
    w = W.WORKLOADS["c4_uneven"]
    shapes = ((16, 1), (24, 3), (32, 2), (48, 3))
    counts = [700, 500, 400, 300]
    tensors = [G.Tensor(N, k, w.x_min, w.x_max, kernel=w.kernel, frag=w.frag, levels=w.levels,
                        conservative=w.conservative) for N, k in shapes]
    parts = []
    for i, (t, n) in enumerate(zip(tensors, counts)):
        smp = torch.tensor(W.samples(w, t.projection_points(), cells=n, params=W.lognormal_cells(n, 40 + i)),
                           device=DEV)
        parts.append(t.project(smp).reshape(-1))
    g0 = torch.cat(parts)
    for prec in ("mixed", "fp64"):
        plan = G.Plan(tensors, counts, precision=prec)
        ref = _raw(plan, g0)
        cache = str(tmp_path / f"tune_{prec}.txt")
        plan.autotune(g0, cache_path=cache)
        rows = plan.group_rows()
        assert len(rows) == 4 and all(r in (0, 1, 2) for r in rows), rows
        assert torch.equal(_raw(plan, g0), ref)
        line = open(cache).read().splitlines()[-1]
        assert line.split()[-1].startswith("g:"), line
        p2 = G.Plan(tensors, counts, precision=prec)
        p2.autotune(g0, cache_path=cache)
        assert p2.group_rows() == rows
        assert torch.equal(_raw(p2, g0), ref)


@pytest.mark.parametrize("prec", ["mixed", "fp64"])
def test_full_size_uneven_workload_sampled(oracle, prec):
    """The uneven batch at full size (100000 cells over the twelve shapes) in the
    benchmark's launch configuration; sampled cells of every group against the oracle."""
    O = oracle
    w = W.WORKLOADS["c4_uneven"]
    counts, order = W.uneven_groups(w)
    p = W.lognormal_cells(w.cells, w.seed)
    tensors, parts, cfgs = [], [], []
    c0 = 0
    for (N, k), n in zip(w.groups, counts):
        t = G.Tensor(N, k, w.x_min, w.x_max, kernel=w.kernel, frag=w.frag, levels=w.levels,
                     conservative=w.conservative)
        ids = order[c0:c0 + n]
        c0 += n
        sub = {key: v[ids] for key, v in p.items()}
        smp = torch.tensor(W.samples(w, t.projection_points(), cells=n, params=sub), device=DEV)
        parts.append(t.project(smp).reshape(-1))
        tensors.append(t)
        cfgs.append(O.Config(N=N, k=k, xmin=w.x_min, xmax=w.x_max, kernel=w.kernel, frag=w.frag,
                             conservative=w.conservative, vfrag=w.levels[0]))
    g = torch.cat(parts)
    del parts
    plan = G.Plan(tensors, counts, precision=prec)
    raw = _raw(plan, g)
    tol = 1e-12 if prec == "fp64" else 1e-6
    rng = np.random.default_rng(11)
    voff = roff = 0
    for t, cfg, n in zip(tensors, cfgs, counts):
        P, no = cfg.P, cfg.n_out
        idx = rng.choice(n, 3, replace=False)
        idx[0] = n - 1
        gs = g[voff:voff + n * P].view(n, P)[idx].cpu().numpy()
        Yg = raw[roff:roff + n * no].view(n, no)[idx].cpu().numpy()
        Yo, _, _ = O.rhs(cfg, gs)
        assert _eps(Yg, Yo).max() <= tol, (cfg.N, cfg.k)
        voff += n * P
        roff += n * no


def test_algorithmic_flops_count_each_cells_level():
    """gd_plan_algorithmic_flops: per cell 2 nnz of the folded tensor of its bracket's
    level plus 2 nnz of the difference to the next level, counted here from the
    exported FP64 tensors; an uneven plan adds its single-level group."""
    lv = W.VFRAG_LEVELS
    N, k, C = 6, 2, 90
    t = G.Tensor(N, k, 1e-4, 1e8, kernel="ballistic", frag="powerlaw", levels=lv, conservative=True)
    t2 = G.Tensor(5, 1, 1e-4, 1e8, kernel="additive", frag="powerlaw", levels=(0.5,), conservative=True)
    P, NO, R = t.P, t.n_out, len(lv)
    iu = np.triu_indices(P)

    def fold(T, P=P, NO=NO, iu=iu):
        T = T.reshape(NO, P, P)
        F = T + T.transpose(0, 2, 1)
        d = np.arange(P)
        F[:, d, d] = T[:, d, d]
        return F[:, iu[0], iu[1]]

    Fs = [fold(t.export(r)) for r in range(R)]
    rng = np.random.default_rng(5)
    vf = rng.uniform(0.25, 1.05, C)
    r = np.clip(np.searchsorted(np.array(lv), vf, side="right") - 1, 0, R - 2)
    want = sum(2.0 * (np.count_nonzero(Fs[ri]) + np.count_nonzero(Fs[ri + 1] - Fs[ri])) for ri in r)
    plan = G.Plan(t, C, precision="mixed", vfrag=vf)
    assert plan.algorithmic_flops() == want
    P2, NO2 = t2.P, t2.n_out
    want2 = 2.0 * np.count_nonzero(fold(t2.export(0), P2, NO2, np.triu_indices(P2))) * 7
    both = G.Plan([t, t2], [C, 7], precision="fp64", vfrag=np.concatenate([vf, np.full(7, 0.5)]))
    assert both.algorithmic_flops() == want + want2


@pytest.mark.parametrize("prec", ["mixed", "fp64"])
def test_set_vfrag_rebrackets_in_place(oracle, prec):
    """New per-cell thresholds on an existing plan (gd_plan_set_vfrag): the brackets and
    blend weights are rebuilt in the plan's buffers, and the right-hand side and the
    reverse pass equal those of a plan created with the new thresholds (same kernels,
    same tiles: bit for bit), and the oracle at the new thresholds."""
    O = oracle
    t, cfg, g, ks, vf = _level_case(O)
    C = len(g)
    rng = np.random.default_rng(77)
    vf2 = rng.uniform(0.25, 1.05, C)               # also outside the table (clamped)
    vf2[:200] = 0.55                                # one crowded bracket
    gd = torch.tensor(g, device=DEV).view(-1)
    ksd = torch.tensor(ks, device=DEV)
    plan = G.Plan(t, C, precision=prec, vfrag=vf)
    print(f"set_vfrag {prec} C={C}", flush=True)
    # reverse-mode workspace first, so that it is rebuilt too
    st, gm = plan.rk_forward(gd.clone(), 1e-9, 1, kscale=ksd)
    plan.adjoint(st, gm, 1e-9, 1, torch.ones_like(gd), kscale=ksd)
    plan.set_vfrag(vf2)
    fresh = G.Plan(t, C, precision=prec, vfrag=vf2)
    r1, r2 = _raw(plan, gd, ksd), _raw(fresh, gd, ksd)
    assert torch.equal(r1, r2)
    idx = np.arange(0, C, 41)
    Yo, _, _ = O.rhs(cfg, g[idx], kscale=ks[idx], vfrag=vf2[idx])
    tol = 1e-12 if prec == "fp64" else 1e-6
    assert _eps(r1.view(C, -1)[idx].cpu().numpy(), Yo).max() <= tol
    outs = []
    for p in (plan, fresh):
        gg = gd.clone()
        st, gm = p.rk_forward(gg, 1e-9, 2, kscale=ksd)
        lam = torch.ones_like(gd)
        dks, dvf = p.adjoint(st, gm, 1e-9, 2, lam, kscale=ksd)
        outs.append((gg, lam, dks, dvf))
    for name, a, b in zip(("state", "dL/dg0", "dL/dkscale", "dL/dvfrag"), *outs):
        d = float((a - b).abs().max())
        print(f"  {name}: max |difference| {d:.3e} (scale {float(b.abs().max()):.3e})", flush=True)
        assert torch.equal(a, b), name
    # back to the original thresholds
    plan.set_vfrag(vf)
    assert torch.equal(_raw(plan, gd, ksd), _raw(G.Plan(t, C, precision=prec, vfrag=vf), gd, ksd))
    with pytest.raises(G.GDError):
        bad = vf.copy()
        bad[3] = np.nan
        plan.set_vfrag(bad)
    assert torch.equal(_raw(plan, gd, ksd), _raw(G.Plan(t, C, precision=prec, vfrag=vf), gd, ksd))


@pytest.mark.parametrize("prec", ["mixed", "fp64"])
def test_lanes_match_one_lane(oracle, prec):
    """gd_rk_step and gd_collision_rhs with the cells split into lanes (run side by
    side on streams of their own) against one lane, bit for bit: two groups (one with blended threshold
    brackets, one single-level), lane boundaries inside brackets and between groups,
    captured graphs and launches one by one, several calls with a change of dt."""
    O = oracle
    t1, cfg1, g1, ks1, vf1 = _level_case(O)
    N2, k2, C2 = 16, 2, 500
    t2 = G.Tensor(N2, k2, 1e-4, 1e8, kernel="ballistic", frag="powerlaw", levels=(0.5,), conservative=True)
    cfg2 = O.Config(N=N2, k=k2, xmin=1e-4, xmax=1e8, kernel="ballistic", frag="powerlaw", conservative=True,
                    levels=(0.5,))
    rng = np.random.default_rng(41)
    g2 = np.stack([O.project(cfg2, lambda x, mu=mu: W.lognormal_density(x, mu, 1.0, 1.0))
                   for mu in rng.uniform(np.log(30.0), np.log(3000.0), C2)])
    g1, _ = O.limit(cfg1, g1)
    g2, _ = O.limit(cfg2, g2)
    C1 = len(g1)
    ks = np.concatenate([ks1, np.exp(0.5 * rng.standard_normal(C2))])
    vf = np.concatenate([vf1, np.full(C2, 0.5)])
    g0 = torch.tensor(np.concatenate([g1.reshape(-1), g2.reshape(-1)]), device=DEV)
    ksd = torch.tensor(ks, device=DEV)
    dt = 2e-6
    ref_plan = G.Plan([t1, t2], [C1, C2], precision=prec, vfrag=vf)
    assert ref_plan.lanes()[0] == 1            # small plans take one lane by default
    raw_ref = torch.zeros(ref_plan.n_raw, dtype=torch.float64, device=DEV)
    rhs_ref = ref_plan.collision_rhs(g0, kscale=ksd, raw=raw_ref)
    ref = g0.clone()
    for n, d in ((2, dt), (1, 0.5 * dt)):
        ref_plan.rk_step(ref, d, n, kscale=ksd)
    torch.cuda.synchronize()
    for lanes in (2, 3, 5):
        for graph in (True, False):
            plan = G.Plan([t1, t2], [C1, C2], precision=prec, vfrag=vf)
            plan.set_lanes(lanes)
            plan.use_graph(graph)
            n_l, first = plan.lanes()
            assert n_l == lanes and first[0] == 0 and all(a < b for a, b in zip(first, first[1:])), first
            raw = torch.zeros(plan.n_raw, dtype=torch.float64, device=DEV)
            rhs = plan.collision_rhs(g0, kscale=ksd, raw=raw)
            torch.cuda.synchronize()
            assert torch.equal(rhs, rhs_ref) and torch.equal(raw, raw_ref), (lanes, "collision_rhs")
            g = g0.clone()
            junk = torch.zeros(1 << 20, device=DEV)
            for n, d in ((2, dt), (1, 0.5 * dt)):
                v = plan.rk_step(g, d, n, kscale=ksd, count_violations=True)
                junk += 1.0
                assert v == 0
            torch.cuda.synchronize()
            assert torch.equal(g, ref), (lanes, graph, float((g - ref).abs().max()))
    tiny = G.Plan(t2, 40, precision=prec)
    tiny.set_lanes(8)
    assert tiny.lanes()[0] == 2                # one lane per 32-slot tile at most
    tiny.set_lanes(0)
    assert tiny.lanes() == (1, [0])
