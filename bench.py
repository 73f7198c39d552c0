"""Benchmark of the phi-combination hot path on one MI355X.

Workload (one bench step): from the seeded level-6 state (solid-body zonal
flow u0 = 38.6 m/s, balanced depth, 120 m Gaussian bump; N = 40962 cells,
n = 163848 unknowns, FP64) run pexprb43 for 24 steps of 3600 s and exprb53
for 24 steps of 3600 s (tol 1e-10 relative, m_max 40).  That is 120
phipm_simul_iom2 evaluations per bench step.  value = evaluations per second
with all inputs resident in device memory.

Also reported: the roofline of the fused Jacobian-product/IOM2 kernel
(algorithmic bytes per launch over its HIP-event-timed average duration),
a per-kernel time breakdown, and the CPU oracle timed on a bounded sample of
the same workload.

Usage: python bench.py [--gpus 1] [--steps K] [--warmup W] [--no-cpu]
"""
import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = ("phi_k-combination evals/sec + Jv HBM GB/s (% peak); ensemble & adjoint vs plain, "
          "1e-11")
HBM_PEAK_GBS = 8000.0
# Algorithmic bytes per cell of one fused Jacobian product with the IOM2 dot
# epilogue: the plain product model (v 32 + Jv 32 + u_n 32 + eta_n 8 +
# neighbour ids 24 + centre/area 32 = 160 B) plus the second dot's read of
# v_{j-1} (32 B).
JV_IOM2_BYTES_PER_CELL = 192.0
STEPS_PER_METHOD = 24
DT = 3600.0
EVALS_PER_STEP = {"pexprb43": 2, "exprb53": 3}


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def run_pass(ctx, u, u0, torch):
    evals = 0
    stats = []
    for method in ("pexprb43", "exprb53"):
        ctx.reset_history()
        u.copy_(u0)
        for _ in range(STEPS_PER_METHOD):
            ctx.step(method, u, DT)
            evals += EVALS_PER_STEP[method]
            stats.append(ctx.step_stats())
    return evals, stats


def cpu_baseline(mesh, u0_host, steps):
    import oracle as O
    s = O.SWE(mesh)
    evals = 0
    t0 = time.perf_counter()
    for method in ("pexprb43", "exprb53"):
        st = O.swe_stepper(s, method)
        u = u0_host.copy()
        for _ in range(steps):
            u = st.step(u, DT)
            evals += EVALS_PER_STEP[method]
    t = time.perf_counter() - t0
    return {"value": evals / t, "unit": "phi-combination evals/s", "cores": 1, "kind": "oracle",
            "sample": "first %d steps of pexprb43 and of exprb53 (%d of the 120 evaluations of "
                      "one bench step), serial C oracle, %.1f s" % (steps, evals, t),
            "host_cpu": _cpu_model(), "host_nproc": os.cpu_count()}


def _cpu_model():
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--cpu-steps", type=int, default=6)
    ap.add_argument("--event-every", type=int, default=16,
                    help="time every N-th launch of each kernel with HIP events")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py measures one GPU only: this build has no multi-GPU path "
              "(--gpus %d requested)" % args.gpus, file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    import paper_1805_02144_amd as X
    from synth import fields as F
    from synth.mesh import get_mesh

    level = 6
    mesh = get_mesh(level)
    n = len(mesh["xyz"])
    u0_host = F.initial_state("c2_l6_24x3600")
    ctx = X.Context(mesh, "cuda:0", gamma_h=4e-4, tol=1e-10, m_max=40)
    u0 = torch.tensor(u0_host, dtype=torch.float64, device="cuda:0")
    u = torch.empty_like(u0)

    for _ in range(args.warmup):
        run_pass(ctx, u, u0, torch)
    torch.cuda.synchronize()

    ctx.profile(args.event_every)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    total_evals = 0
    all_stats = []
    for _ in range(args.steps):
        e, st = run_pass(ctx, u, u0, torch)
        total_evals += e
        all_stats += st
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    prof = ctx.profile_get()
    ctx.profile(0)
    elapsed = t1 - t0
    value = total_evals / elapsed

    # roofline of the fused Jacobian product + IOM2 dots
    ms, timed_n, all_n = prof["jv_iom2"]
    avg_s = ms * 1e-3 / max(timed_n, 1)
    achieved = JV_IOM2_BYTES_PER_CELL * n / avg_s / 1e9 if timed_n else 0.0
    roofline = {"bound": "hbm", "kernel": "k_jv<kEpiIom2>", "achieved": achieved,
                "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": achieved / HBM_PEAK_GBS,
                "traffic": None, "avg_us": avg_s * 1e6, "launches": all_n,
                "timed_launches": timed_n, "bytes_per_cell": JV_IOM2_BYTES_PER_CELL, "cells": n}
    avg = {k: (v[0] / v[1] if v[1] else 0.0) for k, v in prof.items()}
    counts = {k: v[2] for k, v in prof.items()}
    est = {k: avg[k] * counts[k] for k in prof}            # ms, all launches
    tot_ms = sum(est.values())
    kernels = {k: {"avg_us": 1e3 * avg[k], "launches": counts[k], "timed": prof[k][1],
                   "est_ms": est[k], "share": est[k] / tot_ms if tot_ms else 0.0} for k in prof}
    agg = {}
    for st in all_stats:
        for c in st:
            for k, v in c.items():
                if k in ("attempts", "rejected", "accepted", "matvecs", "expms", "sum_m"):
                    agg[k] = agg.get(k, 0) + v
    per_pass = {k: v / args.steps for k, v in agg.items()}

    cpu = None
    if not args.no_cpu:
        cpu = cpu_baseline(mesh, u0_host, args.cpu_steps)

    out = {
        "metric": METRIC,
        "value": value,
        "unit": "phi-combination evals/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": 1e3 * elapsed / args.steps,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic (seeded level-6 solid-body flow + Gaussian bump)",
        "config": {"workload": "pexprb43 and exprb53, 24 steps of 3600 s each, level-6 "
                               "icosahedral grid (N=40962, n=163848), FP64, tol 1e-10, m_max 40",
                   "grid_level": level, "cells": n, "unknowns": 4 * n,
                   "evals_per_step": sum(EVALS_PER_STEP.values()) * STEPS_PER_METHOD},
        "roofline": roofline,
        "cpu_baseline": cpu,
        "kernels": kernels,
        "krylov_per_step": per_pass,
        "device_time_fraction": (tot_ms * 1e-3) / elapsed,
    }
    print(json.dumps(out))
    ctx.close()


if __name__ == "__main__":
    main()
