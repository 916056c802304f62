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
    import numpy as np
    import torch
    from paper_2607_13740_amd import gracedg as G
    from paper_2607_13740_amd import workloads as W

    t0 = time.perf_counter()
    t = G.Tensor(w.bins, w.order, w.x_min, w.x_max, kernel=w.kernel, frag=w.frag,
                 levels=w.levels, conservative=w.conservative)
    t_init = time.perf_counter() - t0
    params = W.lognormal_cells(w.cells, w.seed) if w.profile == "lognormal_cells" else None
    x = t.projection_points()
    smp = torch.tensor(W.samples(w, x, params=params), device=dev)
    g0 = t.project(smp).reshape(-1)
    del smp
    ks = vf = None
    if w.per_cell and params is not None:
        ks = torch.tensor(params["kscale"], device=dev)
        vf = np.asarray(params["vfrag"])
    return t, g0, ks, vf, t_init, params


def time_steps(plan, g, w, ks, steps, warmup):
    import torch
    for _ in range(warmup):
        plan.rk_step(g, w.dt, 1, kscale=ks)
    torch.cuda.synchronize()
    plan.timing(True)
    t0 = time.perf_counter()
    for _ in range(steps):
        plan.rk_step(g, w.dt, 1, kscale=ks)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    kms, launches = plan.contraction_time()
    plan.timing(False)
    return (t1 - t0) * 1e3 / steps, kms / max(1, launches), launches


def cpu_baseline(w, params, seconds):
    """The FP64 oracle on the host cores, on a sample of the workload's cells."""
    import numpy as np
    from oracle import oracle as O
    from paper_2607_13740_amd import workloads as W

    O.build(force=False)
    cfg = O.Config(N=w.bins, k=w.order, xmin=w.x_min, xmax=w.x_max, kernel=w.kernel, frag=w.frag,
                   conservative=w.conservative, vfrag=w.levels[0],
                   levels=w.levels if len(w.levels) > 1 else ())

    def states(n):
        out = []
        for c in range(n):
            if params is None:
                f = W.xexp_density if w.profile == "xexp" else W.lognormal_density
            else:
                f = (lambda mu, s, m: (lambda x: W.lognormal_density(x, mu, s, m)))(
                    params["mu"][c], params["sigma"][c], params["mass"][c])
            out.append(O.project(cfg, f))
        return np.array(out)

    cores = int(os.environ.get("OMP_NUM_THREADS", os.cpu_count() or 1))
    n = max(1, min(cores, 16))
    g = states(n)
    ks = params["kscale"][:n] if (params is not None and w.per_cell) else None
    vf = params["vfrag"][:n] if (params is not None and w.per_cell) else None
    t0 = time.perf_counter()
    O.rhs(cfg, g, kscale=ks, vfrag=vf)
    dt = time.perf_counter() - t0
    m = int(min(4096, max(n, seconds / max(dt / n, 1e-9))))
    m = max(n, (m // cores) * cores) if m > cores else m
    m = min(m, w.cells)
    g = states(m)
    ks = params["kscale"][:m] if (params is not None and w.per_cell) else None
    vf = params["vfrag"][:m] if (params is not None and w.per_cell) else None
    t0 = time.perf_counter()
    O.rhs(cfg, g, kscale=ks, vfrag=vf)
    dt = time.perf_counter() - t0
    return {"value": m / dt, "unit": "cell-evals/s", "cores": cores, "kind": "oracle",
            "sample": f"{m} cells of {w.name}, one right-hand-side evaluation each, FP64 nested "
                      f"Gauss-Legendre sums in C (gcc -O2, OpenMP across cells), {dt:.1f} s"}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--workload", default="c3_batched")
    ap.add_argument("--cpu-seconds", type=float, default=15.0)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-fp64", action="store_true")
    args = ap.parse_args()
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
    if w.groups:
        raise SystemExit("uneven batches are timed by bench_uneven (not built yet)")
    print(f"# workload {describe(w)}", file=sys.stderr, flush=True)
    t, g0, ks, vf, t_init, params = build_inputs(w, dev)
    info = t.info()
    C = w.cells
    res = {}
    for prec in (("mixed",) if args.no_fp64 else ("mixed", "fp64")):
        plan = G.Plan(t, C, precision=prec, vfrag=vf)
        g = g0.clone()
        ms, kms, launches = time_steps(plan, g, w, ks, args.steps, args.warmup)
        res[prec] = {"ms_per_step": ms, "kernel_ms": kms, "launches": launches, "plan": plan,
                     "stats": plan.schedule_stats(0)}
        print(f"# {prec}: {ms:.3f} ms/step, contraction {kms:.4f} ms/launch over {launches} launches",
              file=sys.stderr, flush=True)
        # mass drift over the timed run (FP64 bookkeeping of the bin masses)
        h = torch.tensor(np.repeat(np.diff(t.edges()), 1), device=dev)
        gm = g.view(C, w.bins, w.order + 1)[:, :, 0] * h
        g0m = g0.view(C, w.bins, w.order + 1)[:, :, 0] * h
        res[prec]["mass_drift"] = float(((gm.sum(1) - g0m.sum(1)).abs() / g0m.sum(1)).max())

    # accuracy of the split contraction against the FP64 contraction on the full batch
    acc = {}
    if "fp64" in res:
        raws = {}
        for prec in ("mixed", "fp64"):
            raw = torch.zeros(res[prec]["plan"].n_raw, dtype=torch.float64, device=dev)
            res[prec]["plan"].collision_rhs(g0, kscale=ks, raw=raw)
            raws[prec] = raw.view(C, -1)
        d = (raws["mixed"] - raws["fp64"]).abs().amax(1) / raws["fp64"].abs().amax(1)
        acc = {"eps_max": float(d.max()), "eps_median": float(d.median()),
               "definition": "per cell max_o |Y_mixed - Y_fp64| / max_o |Y_fp64| on the raw flux vector"}

    mixed = res["mixed"]
    cell_evals = 3.0 * C / (mixed["ms_per_step"] * 1e-3)
    # executed MFMA work of one launch: every stored fragment (32 rows x 16 K) of the
    # levels in use, 3 products, for every 32-cell tile of the bracket using it
    # (bracket sizes from the plan's slot count, fragments averaged over levels)
    st = mixed["stats"]
    n_levels = max(1, info["n_levels"])
    frags_per_level = st["frags_mixed"] / n_levels
    exec_flops = frags_per_level * 3 * (2 * 32 * 32 * 16) * (st["n_slots"] / 32)
    flops_launch = info["flops_per_eval"] * C
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
        "config": {"workload": describe(w), "cells": C, "P": w.P, "precision": "split FP16 (hi+lo, 3 MFMA "
                   "products) with FP32 MFMA accumulation, FP64 p-sum, FP64 state/limiter/RK"},
        "roofline": {"bound": "mfma", "achieved": achieved, "peak": PEAK_F16_TFLOPS, "unit": "TFLOP/s",
                     "frac": achieved / PEAK_F16_TFLOPS, "traffic": None,
                     "kernel": "k_contract_mixed", "kernel_ms": mixed["kernel_ms"],
                     "algorithmic_flops_per_launch": flops_launch,
                     "flops_per_cell_eval": info["flops_per_eval"],
                     "executed_mfma_tflops": exec_flops / (mixed["kernel_ms"] * 1e-3) / 1e12,
                     "mfma_utilisation": exec_flops / (mixed["kernel_ms"] * 1e-3) / 1e12 / PEAK_F16_TFLOPS},
        "tensor_init_s": t_init,
        "mass_drift_mixed": mixed["mass_drift"],
        "accuracy_vs_fp64_gpu": acc,
    }
    if "fp64" in res:
        f = res["fp64"]
        f_evals = 3.0 * C / (f["ms_per_step"] * 1e-3)
        out["fp64_gpu"] = {"value": f_evals, "ms_per_step": f["ms_per_step"], "kernel_ms": f["kernel_ms"],
                           "achieved_tflops": flops_launch / (f["kernel_ms"] * 1e-3) / 1e12,
                           "peak_tflops": PEAK_F64_TFLOPS, "mass_drift": f["mass_drift"]}
        out["speedup_mixed_vs_fp64"] = cell_evals / f_evals
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(w, params, args.cpu_seconds)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
