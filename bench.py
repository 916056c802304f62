#!/usr/bin/env python
"""Throughput of the collision-operator hot path on one MI355X.

One step is one SSP-RK3 step (three right-hand-side evaluations, each: limiter,
state split, contraction, flux assembly and stage combination) over the whole
batch of the workload; the reported value is right-hand-side evaluations per
second over all cells (cell-evals/s) in the split-FP16 precision.  The plain FP64
form runs the same steps on the same inputs for the speed ratio, and the two are
compared cell by cell for the accuracy line.

    python bench.py [--steps K] [--warmup W] [--workload c3_batched]

Prints one JSON line.  --gpus N with N > 1 exits: this build runs on one GPU.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "collision_rhs cell-evals/s, mixed vs FP64 GPU at 1e-6 rel err; adjoint/forward cost"
PEAK_F16_TFLOPS = 2500.0     # MI355X dense FP16 MFMA
PEAK_F64_TFLOPS = 78.6       # MI355X FP64 MFMA


def describe(w):
    if w.groups:
        shapes = "bins x order in {" + ", ".join(f"{n}x{k}" for n, k in w.groups) + "}"
    else:
        shapes = f"{w.bins} bins, order {w.order} (P={w.P})"
    per = ", per-cell kernel scale lognormal(0,0.5) and v_frag U[0.3,1.0]" if w.per_cell else ""
    return (f"{w.name}: {w.cells} cells, {shapes}, {w.kernel} kernel, {w.frag} fragmentation, "
            f"{'conservative' if w.conservative else 'non-conservative'} flux on [{w.x_min:g},{w.x_max:g}]{per}, "
            f"seeded lognormal initial states, dt={w.dt:g}")


def build_inputs(w, dev):
    """Tensors, per-group cell counts and the projected initial state of the workload
    (cells of an uneven batch sorted by group)."""
    import numpy as np
    import torch
    from paper_2607_13740_amd import gracedg as G
    from paper_2607_13740_amd import workloads as W

    params = W.lognormal_cells(w.cells, w.seed) if w.profile == "lognormal_cells" else None
    shapes = w.groups if w.groups else ((w.bins, w.order),)
    if w.groups:
        counts, order = W.uneven_groups(w)
    else:
        counts, order = np.array([w.cells]), np.arange(w.cells)
    t0 = time.perf_counter()
    tensors = [G.Tensor(N, k, w.x_min, w.x_max, kernel=w.kernel, frag=w.frag, levels=w.levels,
                        conservative=w.conservative) for N, k in shapes]
    t_init = time.perf_counter() - t0
    parts = []
    c0 = 0
    for t, n in zip(tensors, counts):
        ids = order[c0:c0 + n]
        c0 += n
        sub = None if params is None else {key: v[ids] for key, v in params.items()}
        smp = torch.tensor(W.samples(w, t.projection_points(), cells=int(n), params=sub), device=dev)
        parts.append(t.project(smp).reshape(-1))
        del smp
    g0 = torch.cat(parts)
    ks = vf = None
    if w.per_cell and params is not None:
        ks = torch.tensor(params["kscale"][order], device=dev)
        vf = np.asarray(params["vfrag"][order])
    return tensors, [int(c) for c in counts], g0, ks, vf, t_init, params


def time_steps(plan, g, w, ks, steps, warmup):
    """ms per RK step (the captured step replayed), then the average duration of the
    contraction kernel from HIP events on the plan's stream (launch by launch)."""
    import torch
    for _ in range(warmup):
        plan.rk_step(g, w.dt, 1, kscale=ks)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    plan.rk_step(g, w.dt, steps, kscale=ks)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    # distribution of single-step durations: HIP events around each replay on the
    # plan's stream (torch's current stream, on which the plan was created)
    ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(steps)]
    for a, b in ev:
        a.record()
        plan.rk_step(g, w.dt, 1, kscale=ks)
        b.record()
    torch.cuda.synchronize()
    per = sorted(a.elapsed_time(b) for a, b in ev)
    pct = lambda q: per[min(len(per) - 1, int(q * (len(per) - 1) + 0.5))]
    dist = {"p10": pct(0.1), "p50": pct(0.5), "p90": pct(0.9)}
    plan.timing(True)
    plan.rk_step(g, w.dt, max(2, steps // 4), kscale=ks)
    kms, launches = plan.contraction_time()
    sms, slaunches = plan.stage_time()
    plan.timing(False)
    return (t1 - t0) * 1e3 / steps, kms / max(1, launches), launches, sms / max(1, slaunches), dist


def cpu_baseline(w, params, seconds):
    """The FP64 oracle on the host cores, on a sample of the workload's cells (the
    first cells in the workload's own order, each evaluated with its group's shape)."""
    import numpy as np
    from oracle import oracle as O
    from paper_2607_13740_amd import workloads as W

    O.build(force=False)
    flags = O.use_native()
    shapes = w.groups if w.groups else ((w.bins, w.order),)
    cfgs = [O.Config(N=N, k=k, xmin=w.x_min, xmax=w.x_max, kernel=w.kernel, frag=w.frag,
                     conservative=w.conservative, vfrag=w.levels[0],
                     levels=w.levels if len(w.levels) > 1 else ()) for N, k in shapes]
    gid = np.zeros(w.cells, dtype=int)
    if w.groups:
        counts, order = W.uneven_groups(w)
        gid[order] = np.repeat(np.arange(len(shapes)), counts)

    def run(n):
        """oracle time of the first n cells"""
        tot = 0.0
        for gi, cfg in enumerate(cfgs):
            ids = np.nonzero(gid[:n] == gi)[0]
            if ids.size == 0:
                continue
            g = []
            for c in ids:
                if params is None:
                    f = W.xexp_density if w.profile == "xexp" else W.lognormal_density
                else:
                    f = (lambda mu, s, m: (lambda x: W.lognormal_density(x, mu, s, m)))(
                        params["mu"][c], params["sigma"][c], params["mass"][c])
                g.append(O.project(cfg, f))
            ks = params["kscale"][ids] if (params is not None and w.per_cell) else None
            vf = params["vfrag"][ids] if (params is not None and w.per_cell) else None
            t0 = time.perf_counter()
            O.rhs(cfg, np.array(g), kscale=ks, vfrag=vf)
            tot += time.perf_counter() - t0
        return tot

    cores = O.set_threads(0)
    n = max(1, min(cores, 16, w.cells))
    dt = run(n)
    m = int(min(4096, max(n, seconds / max(dt / n, 1e-9))))
    m = max(n, (m // cores) * cores) if m > cores else m
    m = min(m, w.cells)
    dt = run(m)
    # one thread, on a few cells (about a tenth of the budget)
    O.set_threads(1)
    m1 = int(max(1, min(m, 0.1 * seconds / max(dt * cores / m, 1e-9))))
    dt1 = run(m1)
    O.set_threads(cores)
    return {"value": m / dt, "unit": "cell-evals/s", "cores": cores, "kind": "oracle",
            "sample": f"first {m} cells of {w.name}, one right-hand-side evaluation each, FP64 nested "
                      f"Gauss-Legendre sums in C (gcc {flags}, OpenMP across cells), {dt:.1f} s",
            "one_thread": {"value": m1 / dt1, "sample": f"first {m1} cells, {dt1:.1f} s"},
            "cpu": host_cpu(), "host_cpus": os.cpu_count()}


def host_cpu():
    """What the host reports about its processor: the model string and family/model/
    stepping of /proc/cpuinfo, the vector extensions the native build can use, and the
    cores this process may run on."""
    info = {}
    try:
        with open("/proc/cpuinfo") as f:
            for ln in f:
                if ":" not in ln:
                    if info:
                        break
                    continue
                key, val = (x.strip() for x in ln.split(":", 1))
                if key in ("vendor_id", "model name", "cpu family", "model", "stepping", "cpu MHz", "flags") \
                        and key not in info:
                    info[key] = val
    except OSError:
        pass
    flags = set(info.pop("flags", "").split())
    info["vector_ext"] = [f for f in ("avx2", "fma", "avx512f", "avx512_bf16", "avx512vl") if f in flags]
    info["usable_cores"] = len(os.sched_getaffinity(0)) if hasattr(os, "sched_getaffinity") else os.cpu_count()
    return info


def cpu_blas_reference(t, g0, ks, vf, w, cells=2048):
    """A second CPU reference, not the oracle (it uses the library's host tensor): the
    FP64 contraction Y = s (1-theta) T_r (g x g) + s theta T_{r+1} (g x g) as BLAS
    matrix products over the materialised products g x g of a sample of cells, on the
    host cores.  It separates the algorithm's gain (the tensor form) from the
    hardware's."""
    import numpy as np
    lv = np.asarray(w.levels, dtype=np.float64)
    P, no = t.P, t.n_out
    T = [np.ascontiguousarray(t.export(r).reshape(no, P * P)) for r in range(len(lv))]
    m = min(cells, w.cells)
    g = g0.view(w.cells, P)[:m].cpu().numpy()
    s = ks[:m].cpu().numpy() if ks is not None else np.ones(m)
    v = vf[:m] if vf is not None else np.full(m, lv[0])
    r = np.clip(np.searchsorted(lv, v, side="right") - 1, 0, len(lv) - 1)
    nxt = np.minimum(r + 1, len(lv) - 1)
    th = np.where(nxt > r, np.clip((v - lv[r]) / (lv[nxt] - lv[r] + (nxt == r)), 0.0, 1.0), 0.0)
    t0 = time.perf_counter()
    X = np.einsum("cp,cq->pqc", g, g).reshape(P * P, m)
    Y = np.zeros((no, m))
    for b in np.unique(r):
        sel = np.nonzero(r == b)[0]
        Y[:, sel] = (T[b] @ X[:, sel]) * (1.0 - th[sel])
        if nxt[sel[0]] > b:
            Y[:, sel] += (T[b + 1] @ X[:, sel]) * th[sel]
    Y *= s
    dt = time.perf_counter() - t0
    return Y.T, {"value": m / dt, "unit": "cell-evals/s", "kind": "FP64 tensor contraction with BLAS (numpy "
                 "matmul over g x g, unfolded tensor), not the oracle", "cells": m, "seconds": dt}


def adaptive_bench(plan, g0, ks, w, n=20, warm=20):
    """Per-cell steps under the CFL bound (gd_rk_advance) on the same plan and inputs:
    ms per sub-step with one sub-step captured as a HIP graph and with the launches
    issued one by one, the adaptive stage kernel's average duration, and the fixed
    step issued one by one beside them (each timed after its own warm-up)."""
    import torch
    g = g0.clone()
    t = torch.zeros(plan.n_cells, dtype=torch.float64, device=g.device)
    kw = dict(kscale=ks, flux_floor=1e-4 if plan.precision == "mixed" else 0.0)

    def timed(fn):
        fn(warm)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        fn(n)
        torch.cuda.synchronize()
        return (time.perf_counter() - t0) * 1e3 / n

    advance = lambda m: plan.rk_advance(g, t, 1e30, 0.1, w.dt, m, **kw)
    plan.use_graph(False)
    ms_eager = timed(lambda m: plan.rk_step(g, w.dt, m, kscale=ks))
    ms_adapt_eager = timed(advance)
    plan.use_graph(True)
    ms_adapt = timed(advance)
    plan.timing(True)
    advance(4)
    sms, sl = plan.stage_time()     # 12 adaptive stages and the start limiter
    plan.timing(False)
    return {"ms_per_substep": ms_adapt, "ms_per_substep_eager": ms_adapt_eager,
            "eager_fixed_step_ms": ms_eager, "stage_kernel_ms": sms / max(1, sl),
            "cell_evals_per_s": 3.0 * plan.n_cells / (ms_adapt * 1e-3), "cfl": 0.1, "flux_floor": kw["flux_floor"]}


def mfma_counters(variant):
    """The committed rocprofv3 MFMA counters of the split contraction (SQ_INSTS_VALU_MFMA_MOPS_F16,
    SQ_VALU_MFMA_BUSY_CYCLES) when they were taken on the current kernel sources and variant."""
    import hashlib
    path = os.path.join(ROOT, "profiles", "k_contract_mixed_c3_batched_mfma.json")
    if not os.path.exists(path):
        return None
    rec = json.load(open(path))
    h = hashlib.sha256()
    for f in rec["source_files"]:
        h.update(open(os.path.join(ROOT, f), "rb").read())
    if h.hexdigest() != rec["source_sha256"]:
        return None
    key = f"{variant['waves']},{variant['tiles_per_wave']},{variant['rows']},{variant['xcd']}"
    v = rec["variants"].get(key)
    if v is None:
        # the XCD ordering changes the order of the work items, not the MFMA work
        key = next((k for k in rec["variants"] if k.rsplit(",", 1)[0] == key.rsplit(",", 1)[0]), None)
        if key is None:
            return None
        v = rec["variants"][key]
    return dict(v, measured_variant=key, fp64_kernel=rec.get("fp64_kernel"),
                file="profiles/k_contract_mfma_counters_c3_batched.md")


def measured_traffic(variant):
    """HBM bytes of one split-FP16 contraction launch in the given work-item variant,
    from the committed rocprofv3 FETCH_SIZE/WRITE_SIZE measurement scaled by the
    copy-kernel factors; None when the kernel source has changed since the counters
    were taken or the variant was not measured."""
    import hashlib
    path = os.path.join(ROOT, "profiles", "k_contract_mixed_c3_batched_traffic.json")
    if not os.path.exists(path):
        return None
    rec = json.load(open(path))
    h = hashlib.sha256()
    for f in rec["source_files"]:
        h.update(open(os.path.join(ROOT, f), "rb").read())
    if h.hexdigest() != rec["source_sha256"]:
        return None
    key = f"{variant['waves']},{variant['tiles_per_wave']},{variant['rows']},{variant['xcd']}"
    v = rec["variants"].get(key)
    return v["traffic_bytes_per_launch"] if v else None


def c2_precisions():
    """The single-cell workload (1000 steps) in both precisions against the oracle's
    states stored by tests/golden/make_c2_trajectory.py: per precision the normwise
    error of the bin masses after 100, 300 and 1000 steps, and the time per step."""
    import numpy as np
    import torch
    from paper_2607_13740_amd import gracedg as G
    path = os.path.join(ROOT, "tests", "golden", "c2_trajectory.json")
    gold = json.load(open(path))
    c = gold["config"]
    t = G.Tensor(c["N"], c["k"], c["xmin"], c["xmax"], kernel=c["kernel"], frag=c["frag"], levels=(c["vfrag"],),
                 conservative=c["conservative"])
    h = np.repeat(np.diff(t.edges()), c["k"] + 1)
    out = {"workload": f"c2_ballistic: 1 cell, {c['N']} bins, order {c['k']}, {c['kernel']} kernel, {c['frag']} "
                       f"fragmentation above v_frag={c['vfrag']}, conservative, LN(0,1) unit mass, dt={gold['dt']:g}",
           "reference": "FP64 oracle states (tests/golden/c2_trajectory.json)",
           "not_built": "FP32-state and bf16x3 precisions (the state is FP64 in every plan)"}
    for prec in ("fp64", "mixed"):
        plan = G.Plan(t, 1, precision=prec)
        g = torch.tensor(gold["g0"], dtype=torch.float64, device="cuda:0")
        errs, n, viol = {}, 0, 0
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for m in (100, 200, 700):
            viol += plan.rk_step(g, gold["dt"], m, count_violations=True)
            n += m
            ref = np.asarray(gold["states"][str(n)])
            errs[str(n)] = float(np.max(np.abs((g.cpu().numpy() - ref) * h)) / np.max(np.abs(ref * h)))
        dt = time.perf_counter() - t0
        out[prec] = {"state_error_vs_oracle": errs, "violations": int(viol), "ms_per_step": dt * 1e3 / n}
    return out


def moment_weights(t, pmax=3, R=32):
    """W[p][j*(k+1)+i] = integral over bin j of x^(p-1) P_i(xi(x)) dx, so that the
    moment M_p of a cell is W[p] . g (Gauss-Legendre with R points per bin)."""
    import numpy as np
    e = t.edges()
    s, wq = np.polynomial.legendre.leggauss(R)
    K1 = t.order + 1
    W = np.zeros((pmax + 1, t.bins * K1))
    for j in range(t.bins):
        a, b = e[j], e[j + 1]
        x = 0.5 * (a + b) + 0.5 * (b - a) * s
        for i in range(K1):
            Pi = np.polynomial.legendre.legval(s, [0] * i + [1])
            for p in range(pmax + 1):
                W[p, j * K1 + i] = 0.5 * (b - a) * np.sum(wq * x ** (p - 1) * Pi)
    return W


def adjoint_bench(steps_fraction=1.0):
    """Reverse-mode cost on the adjoint workload: the checkpointed forward (gd_rk_forward)
    and the adjoint (gd_adjoint) of its n_steps, seeded with the gradient of the
    moment loss sum_c sum_p ((M_p - M*_p)/M*_p)^2, p = 0..3, where M* are the moments
    of the unperturbed FP64 run times exp(0.1 eps), eps ~ N(0,1) (seeded)."""
    import numpy as np
    import torch
    from paper_2607_13740_amd import gracedg as G
    from paper_2607_13740_amd import workloads as W

    dev = "cuda:0"
    w = W.WORKLOADS["c5_adjoint"]
    n = max(1, int(w.n_steps * steps_fraction))
    tensors, counts, g0, ks, vf, _, _ = build_inputs(w, dev)
    t = tensors[0]
    C = w.cells
    Wm = torch.tensor(moment_weights(t), device=dev)              # [4, P]
    out = {"workload": f"c5_adjoint: {C} cells, {w.bins} bins, order {w.order} (P={w.P}), {n} steps of dt={w.dt:g}, "
                       "per-cell kernel scale and v_frag, moment loss p=0..3"}
    ref = g0.clone()
    G.Plan(tensors, counts, precision="fp64", vfrag=vf).rk_step(ref, w.dt, n, kscale=ks)
    Mref = ref.view(C, -1) @ Wm.T
    rng = np.random.default_rng(w.seed)
    Mstar = Mref * torch.tensor(np.exp(0.1 * rng.standard_normal((C, 4))), device=dev)
    for prec in ("mixed", "fp64"):
        plan = G.Plan(tensors, counts, precision=prec, vfrag=vf)
        g = g0.clone()
        plan.rk_step(g, w.dt, 2, kscale=ks)          # warm-up (graph capture, kernels)
        g = g0.clone()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        plan.rk_step(g, w.dt, n, kscale=ks)
        torch.cuda.synchronize()
        t_plain = time.perf_counter() - t0
        g = g0.clone()
        st, gm = plan.rk_forward(g, w.dt, 2, kscale=ks)
        lam = torch.zeros_like(g)
        plan.adjoint(st, gm, w.dt, 2, lam, kscale=ks)  # warm-up (reverse-mode workspace)
        del st, gm
        g = g0.clone()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        st, gm = plan.rk_forward(g, w.dt, n, kscale=ks)
        torch.cuda.synchronize()
        t_fwd = time.perf_counter() - t0
        M = g.view(C, -1) @ Wm.T
        loss = float((((M - Mstar) / Mstar) ** 2).sum())
        lam = ((2.0 * (M - Mstar) / Mstar ** 2) @ Wm).reshape(-1).contiguous()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        dks, dvf = plan.adjoint(st, gm, w.dt, n, lam, kscale=ks)
        torch.cuda.synchronize()
        t_adj = time.perf_counter() - t0
        out[prec] = {"forward_ms_per_step": t_plain * 1e3 / n, "checkpointed_forward_ms_per_step": t_fwd * 1e3 / n,
                     "adjoint_ms_per_step": t_adj * 1e3 / n, "adjoint_over_forward": t_adj / t_plain,
                     "adjoint_over_checkpointed_forward": t_adj / t_fwd, "loss": loss,
                     "grad_norm": float(lam.norm()), "dkscale_norm": float(dks.norm()),
                     "dvfrag_norm": float(dvf.norm())}
        print(f"# adjoint {prec}: forward {t_plain * 1e3 / n:.3f} ms/step (checkpointed {t_fwd * 1e3 / n:.3f}), "
              f"adjoint {t_adj * 1e3 / n:.3f} ms/step, ratio {t_adj / t_plain:.2f}", file=sys.stderr, flush=True)
        del st, gm
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--workload", default="c3_batched")
    ap.add_argument("--cpu-seconds", type=float, default=15.0)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-fp64", action="store_true")
    ap.add_argument("--no-adjoint", action="store_true")
    ap.add_argument("--variant", default=None,
                    help="waves,rows,xcd[,tiles_per_wave] of the contraction instead of the autotuner's choice")
    ap.add_argument("--lanes", type=int, default=0,
                    help="lanes of the RK step (cell ranges stepped side by side; 0 = the library's choice by size)")
    ap.add_argument("--copy-reference", action="store_true",
                    help="only copy a 512 MiB float64 buffer three times (the reference kernel that scales "
                         "rocprofv3's FETCH_SIZE/WRITE_SIZE counters to bytes) and exit")
    args = ap.parse_args()
    if args.copy_reference:
        import torch
        a = torch.ones(1 << 26, dtype=torch.float64, device="cuda:0")
        b = torch.empty_like(a)
        for _ in range(3):
            b.copy_(a)
        torch.cuda.synchronize()
        print("copied 3 x 512 MiB", flush=True)
        return
    if args.gpus != 1:
        print("bench.py runs on one GPU only: this build has no multi-GPU path (cells shard with no "
              "exchange; see the design notes)", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch
    from paper_2607_13740_amd import gracedg as G
    from paper_2607_13740_amd import workloads as W

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    dev = "cuda:0"
    w = W.WORKLOADS[args.workload]
    print(f"# workload {describe(w)}", file=sys.stderr, flush=True)
    tensors, counts, g0, ks, vf, t_init, params = build_inputs(w, dev)
    C = w.cells
    flops_launch = None
    res = {}
    for prec in (("mixed",) if args.no_fp64 else ("mixed", "fp64")):
        plan = G.Plan(tensors, counts, precision=prec, vfrag=vf)
        # 2 nnz per cell of its level's folded tensor (+ the level-difference part)
        flops_launch = plan.algorithmic_flops()
        g = g0.clone()
        if args.variant:
            vv = [int(x) for x in args.variant.split(",")] + [1]
            tp = vv[3] if prec == "mixed" else 1
            plan.set_variant(vv[0], vv[1], vv[2], tp)
            tune = {"waves": vv[0], "rows": vv[1], "xcd": vv[2], "tiles_per_wave": tp, "fixed": True}
        else:
            tune = plan.autotune(g, kscale=ks)
        one_lane_ms = None
        if args.lanes == 0 and plan.lanes()[0] > 1:
            # the same step with every launch over all cells, for comparison (not the metric)
            plan.set_lanes(1)
            one_lane_ms = time_steps(plan, g, w, ks, max(4, args.steps // 2), 2)[0]
        plan.set_lanes(args.lanes)
        ms, kms, launches, sms, dist = time_steps(plan, g, w, ks, args.steps, args.warmup)
        res[prec] = {"ms_per_step": ms, "kernel_ms": kms, "launches": launches, "plan": plan, "stage_ms": sms,
                     "variant": plan.variant(), "tune": tune, "step_ms_dist": dist, "lanes": plan.lanes(),
                     "one_lane_ms_per_step": one_lane_ms}
        print(f"# {prec}: {ms:.3f} ms/step, contraction {kms:.4f} ms/launch over {launches} launches, "
              f"stage kernel {sms:.4f} ms/launch, "
              f"variant {res[prec]['variant']}, lanes {res[prec]['lanes']}", file=sys.stderr, flush=True)
        # mass drift over the run (FP64 bookkeeping of the bin masses), cell by cell
        drift, voff = 0.0, 0
        for t, n in zip(tensors, counts):
            P, K1 = t.P, t.order + 1
            h = torch.tensor(np.diff(t.edges()), device=dev)
            gm = g[voff:voff + n * P].view(n, t.bins, K1)[:, :, 0] * h
            g0m = g0[voff:voff + n * P].view(n, t.bins, K1)[:, :, 0] * h
            if n:
                drift = max(drift, float(((gm.sum(1) - g0m.sum(1)).abs() / g0m.sum(1)).max()))
            voff += n * P
        res[prec]["mass_drift"] = drift
        res[prec]["adaptive"] = adaptive_bench(plan, g0, ks, w)
        print(f"# {prec} per-cell steps: {res[prec]['adaptive']['ms_per_substep']:.3f} ms/sub-step "
              f"(eager fixed step {res[prec]['adaptive']['eager_fixed_step_ms']:.3f})", file=sys.stderr, flush=True)

    # accuracy of the split contraction against the FP64 contraction on the full batch
    acc = {}
    if "fp64" in res:
        raws = {}
        for prec in ("mixed", "fp64"):
            raw = torch.zeros(res[prec]["plan"].n_raw, dtype=torch.float64, device=dev)
            res[prec]["plan"].collision_rhs(g0, kscale=ks, raw=raw)
            raws[prec] = raw
        eps, roff = [], 0
        for t, n in zip(tensors, counts):
            m = n * t.n_out
            a = raws["mixed"][roff:roff + m].view(n, -1)
            b = raws["fp64"][roff:roff + m].view(n, -1)
            if n:
                eps.append((a - b).abs().amax(1) / b.abs().amax(1))
            roff += m
        d = torch.cat(eps)
        # secondary metric: element-wise relative error on the entries above 1e-3 of
        # the cell's largest
        elem, roff = [], 0
        for t, n in zip(tensors, counts):
            m = n * t.n_out
            a = raws["mixed"][roff:roff + m].view(n, -1)
            b = raws["fp64"][roff:roff + m].view(n, -1)
            if n:
                big = b.abs() > 1e-3 * b.abs().amax(1, keepdim=True)
                elem.append(((a - b).abs() / b.abs())[big])
            roff += m
        e = torch.cat(elem)
        acc = {"eps_max": float(d.max()), "eps_median": float(d.median()),
               "definition": "per cell max_o |Y_mixed - Y_fp64| / max_o |Y_fp64| on the raw flux vector",
               "elementwise_max": float(e.max()), "elementwise_median": float(e.median()),
               "elementwise_definition": "|Y_mixed - Y_fp64| / |Y_fp64| over the entries with |Y_fp64| > 1e-3 "
                                         "max_o |Y_fp64| of their cell"}

    mixed = res["mixed"]
    cell_evals = 3.0 * C / (mixed["ms_per_step"] * 1e-3)
    exec_flops = mixed["variant"]["exec_flops"]
    achieved = flops_launch / (mixed["kernel_ms"] * 1e-3) / 1e12
    out = {
        "metric": METRIC,
        "value": cell_evals,
        "unit": "cell-evals/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": mixed["ms_per_step"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f16x3",
        "data": "synthetic",
        "config": {"workload": describe(w), "cells": C, "groups": len(tensors),
                   "P": [t.P for t in tensors] if len(tensors) > 1 else tensors[0].P,
                   "precision": "split FP16 (hi+lo, 3 MFMA products) with FP32 MFMA accumulation, FP64 p-sum, "
                                "FP64 state/limiter/RK",
                   "contraction_variant": mixed["variant"],
                   "lanes": {"count": mixed["lanes"][0], "first_tiles": mixed["lanes"][1],
                             "one_lane_ms_per_step": mixed["one_lane_ms_per_step"]},
                   "step": "one captured HIP graph per RK step and lane; lanes (cell ranges of equal cost) "
                           "step side by side on streams of their own and join at the end of the call"},
        "roofline": {"bound": "mfma", "achieved": achieved, "peak": PEAK_F16_TFLOPS, "unit": "TFLOP/s",
                     "frac": achieved / PEAK_F16_TFLOPS,
                     "traffic": measured_traffic(mixed["variant"]) if w.name == "c3_batched" else None,
                     "kernel": "k_contract_mixed", "kernel_ms": mixed["kernel_ms"],
                     "algorithmic_flops_per_launch": flops_launch,
                     "flops_per_cell_eval": flops_launch / C,
                     "executed_mfma_flops_per_launch": exec_flops,
                     "executed_mfma_tflops": exec_flops / (mixed["kernel_ms"] * 1e-3) / 1e12,
                     "mfma_utilisation": exec_flops / (mixed["kernel_ms"] * 1e-3) / 1e12 / PEAK_F16_TFLOPS,
                     "mfma_counters": mfma_counters(mixed["variant"]) if w.name == "c3_batched" else None},
        "stage_kernel_ms": mixed["stage_ms"],
        "step_ms_single_replays": mixed["step_ms_dist"],
        "tensor_init_s": t_init,
        "mass_drift_mixed": mixed["mass_drift"],
        "accuracy_vs_fp64_gpu": acc,
        "per_cell_steps": mixed["adaptive"],
    }
    if "fp64" in res:
        f = res["fp64"]
        f_evals = 3.0 * C / (f["ms_per_step"] * 1e-3)
        out["fp64_gpu"] = {"value": f_evals, "ms_per_step": f["ms_per_step"], "kernel_ms": f["kernel_ms"],
                           "step_ms_single_replays": f["step_ms_dist"],
                           "achieved_tflops": flops_launch / (f["kernel_ms"] * 1e-3) / 1e12,
                           "variant": f["variant"], "lanes": f["lanes"][0],
                           "one_lane_ms_per_step": f["one_lane_ms_per_step"],
                           "peak_tflops": PEAK_F64_TFLOPS, "mass_drift": f["mass_drift"],
                           "per_cell_steps": f["adaptive"]}
        out["speedup_mixed_vs_fp64"] = cell_evals / f_evals
    out["c2_precisions"] = c2_precisions()
    print(f"# c2: state error after 1000 steps fp64 {out['c2_precisions']['fp64']['state_error_vs_oracle']['1000']:.2e}, "
          f"split {out['c2_precisions']['mixed']['state_error_vs_oracle']['1000']:.2e}", file=sys.stderr, flush=True)
    if not args.no_adjoint:
        out["adjoint"] = adjoint_bench()
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(w, params, args.cpu_seconds)
        if len(tensors) == 1 and "fp64" in res:
            Yb, ref = cpu_blas_reference(tensors[0], g0, ks, vf, w)
            m = Yb.shape[0]
            Yg = raws["fp64"].view(C, -1)[:m].cpu().numpy()
            ref["max_rel_diff_vs_fp64_gpu"] = float((np.abs(Yb - Yg).max(1) / np.abs(Yg).max(1)).max())
            out["cpu_blas_reference"] = ref
            print(f"# cpu BLAS tensor contraction: {ref['value']:.0f} cell-evals/s on {m} cells "
                  f"(max rel diff vs FP64 GPU {ref['max_rel_diff_vs_fp64_gpu']:.1e})", file=sys.stderr, flush=True)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
