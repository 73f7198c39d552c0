"""Benchmark of the phi-combination hot path on one MI355X.

Workload (one bench step): from the seeded level-6 state (solid-body zonal
flow u0 = 38.6 m/s, balanced depth, 120 m Gaussian bump; N = 40962 cells,
n = 163848 unknowns, FP64) run pexprb43 for 24 steps of 3600 s and exprb53
for 24 steps of 3600 s (tol 1e-10 relative, m_max 40).  That is 120
phipm_simul_iom2 evaluations per bench step.  value = evaluations per second
with all inputs resident in device memory.

Also reported: the roofline of the fused Jacobian-product/IOM2 kernel
(algorithmic bytes per launch over its HIP-event-timed average duration),
a per-kernel time breakdown, the CPU oracle timed on a bounded sample of
the same workload, and the other workloads' legs: one level-4 exprb42 step
(latency), the 64-member level-6 ensemble (batched vs per-member loop), the
level-8 jet (rooflines of the product and the update) and the level-7
adjoint twin experiment.

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
# IOM2 update per cell: read w, v_j, v_{j-1}, write v_{j+1} (4 x 32 B)
IOM2_BYTES_PER_CELL = 128.0
STEPS_PER_METHOD = 24
DT = 3600.0
EVALS_PER_STEP = {"pexprb43": 2, "exprb53": 3}


# Kernel sources of the roofline kernel: a PMC traffic figure in profiles/ is
# used only while these hash to the value it was taken on.
TRAFFIC_SOURCES = ["paper_1805_02144_amd/csrc/stencil.hip", "paper_1805_02144_amd/csrc/stencil_common.h",
                   "paper_1805_02144_amd/csrc/reduce.h", "paper_1805_02144_amd/csrc/xrb_internal.h"]
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "c2_l6_jv_iom2_traffic.md")


def kernel_source_hash():
    import hashlib
    h = hashlib.sha256()
    for f in TRAFFIC_SOURCES:
        with open(os.path.join(ROOT, f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def measured_traffic():
    """HBM bytes per launch of the roofline kernel from the committed PMC
    summary (FETCH_SIZE and WRITE_SIZE, each scaled by the factor a plain
    device copy of known size gives), or None if the kernel changed since."""
    try:
        kv = {}
        for line in open(TRAFFIC_FILE):
            if ":" in line and line.startswith("- "):
                k, v = line[2:].split(":", 1)
                kv[k.strip()] = v.strip().strip("`")
        if kv.get("source_sha") != kernel_source_hash():
            return None
        return float(kv["traffic_bytes_per_launch"])
    except (OSError, KeyError, ValueError):
        return None


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


def ensemble_leg(X, torch, mesh, reps=3):
    """64 level-6 members, exprb42, one step each: one batched launch sequence
    against the per-member loop of single steps (member-steps/s)."""
    import numpy as np
    from synth import fields as F
    U0, dts = F.ensemble_states(6, F.config_seed(3), 64)
    ctx = X.Context(mesh, "cuda:0", gamma_h=4e-4, tol=1e-10, m_max=40)
    tune = ctx.autotune(64)                      # launch shapes for this grid and batch
    Ub0 = torch.tensor(U0, dtype=torch.float64, device="cuda:0")
    Ub = Ub0.clone()
    ctx.reset_history()
    ctx.step_batch("exprb42", Ub, dts)          # warm-up (allocates the workspace)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(reps):
        Ub.copy_(Ub0)
        ctx.reset_history()
        ctx.step_batch("exprb42", Ub, dts)
    torch.cuda.synchronize()
    tb = (time.perf_counter() - t0) / reps
    u = torch.empty(Ub0.shape[1], dtype=torch.float64, device="cuda:0")
    u.copy_(Ub0[0])
    ctx.reset_history()
    ctx.step("exprb42", u, float(dts[0]))
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    last = None
    for k in range(64):
        u.copy_(Ub0[k])
        ctx.reset_history()
        ctx.step("exprb42", u, float(dts[k]))
        if k == 63:
            last = u.clone()
    torch.cuda.synchronize()
    tl = time.perf_counter() - t0
    same = bool(torch.equal(last, Ub[63]))
    ctx.close()
    return {"workload": "64 members, level-6 grid, exprb42, one step each, dt from "
                        "{600, 1200, 2400, 3600} s (seeded), FP64",
            "batched_member_steps_per_s": 64 / tb, "loop_member_steps_per_s": 64 / tl,
            "speedup": tl / tb, "batched_ms": 1e3 * tb, "loop_ms": 1e3 * tl,
            "last_member_bitwise_equal": same,
            "autotune": {"lanes": tune["lanes"], "lanes_batch": tune["lanes_batch"],
                         "single_us": tune["single_us"], "batch_us": tune["batch_us"]},
            "dt_mix": {str(int(d)): int((dts == d).sum()) for d in sorted(set(dts))}}


# the level-8 kernels last 20-150 us, so sampling every 16th launch costs
# little there and gives enough samples over six steps
JET_EVENT_EVERY = 16


def jet_leg(X, torch, event_every):
    """Level-8 jet (N = 655362, n = 2621448): exprb53, 6 steps of 1800 s,
    gamma_h = 1.25e-2 -- the bandwidth-bound roofline run of the Jacobian
    product and the IOM2 update."""
    from synth import fields as F
    from synth.mesh import get_mesh
    mesh = get_mesh(8)
    n = len(mesh["xyz"])
    u0 = torch.tensor(F.initial_state("c3_l8_jet"), dtype=torch.float64, device="cuda:0")
    ctx = X.Context(mesh, "cuda:0", gamma_h=1.25e-2, tol=1e-10, m_max=40)
    u = u0.clone()
    ctx.reset_history()
    ctx.step("exprb53", u, 1800.0)              # warm-up
    torch.cuda.synchronize()
    u.copy_(u0)
    ctx.reset_history()
    ctx.profile(event_every)
    t0 = time.perf_counter()
    for _ in range(6):
        ctx.step("exprb53", u, 1800.0)
    torch.cuda.synchronize()
    el = time.perf_counter() - t0
    prof = ctx.profile_get()
    ctx.profile(0)
    ctx.close()
    out = {"workload": "exprb53, 6 steps of 1800 s, level-8 jet + bump, N=655362, "
                       "n=2621448, FP64, gamma_h 1.25e-2",
           "phi_evals_per_s": 18 / el, "ms": 1e3 * el}
    for name, bpc in (("jv_iom2", JV_IOM2_BYTES_PER_CELL), ("iom2_update", IOM2_BYTES_PER_CELL)):
        ms, tn, an = prof[name]
        avg = ms * 1e-3 / max(tn, 1)
        ach = bpc * n / avg / 1e9 if tn else 0.0
        out["roofline_" + name] = {"bound": "hbm", "achieved": ach, "peak": HBM_PEAK_GBS,
                                   "unit": "GB/s", "frac": ach / HBM_PEAK_GBS,
                                   "avg_us": 1e6 * avg, "launches": an,
                                   "bytes_per_cell": bpc}
    return out


def c1_leg(X, torch, cpu=True, reps=100):
    """One exprb42 step of 900 s on the level-4 grid (N = 2562, n = 10248)
    from the seeded balanced state: a latency-bound single step (vectors of
    82 KB live in cache).  The state is reset before every step; reported
    are the median and mean microseconds per step over `reps` steps (HIP
    events around each step) and the phi-combination rate (two per step),
    plus the oracle's median over 5 steps."""
    import numpy as np
    import oracle as O
    from synth import fields as F
    from synth.mesh import get_mesh
    mesh = get_mesh(4)
    u0h = F.initial_state("c1_exprb42_l4")
    ctx = X.Context(mesh, "cuda:0", gamma_h=4e-4, tol=1e-10, m_max=40)
    u0 = torch.tensor(u0h, dtype=torch.float64, device="cuda:0")
    u = torch.empty_like(u0)
    for _ in range(10):
        u.copy_(u0)
        ctx.reset_history()
        ctx.step("exprb42", u, 900.0)
    torch.cuda.synchronize()
    ts = []
    for _ in range(reps):
        u.copy_(u0)
        ctx.reset_history()
        a = torch.cuda.Event(enable_timing=True)
        b = torch.cuda.Event(enable_timing=True)
        a.record()
        ctx.step("exprb42", u, 900.0)
        b.record()
        b.synchronize()
        ts.append(1e3 * a.elapsed_time(b))
    ctx.close()
    med = float(np.median(ts))
    out = {"workload": "exprb42, one step of 900 s, level-4 grid (N=2562, n=10248), FP64, "
                       "tol 1e-10, m_max 40, state reset before each step",
           "us_per_step_median": med, "us_per_step_mean": float(np.mean(ts)),
           "phi_evals_per_s": 2.0 / (med * 1e-6), "steps": reps}
    if cpu:
        s_ = O.SWE(mesh, gamma_h=4e-4)
        st = O.swe_stepper(s_, "exprb42")
        tc = []
        for _ in range(5):
            t0 = time.perf_counter()
            st.step(u0h, 900.0)
            tc.append(time.perf_counter() - t0)
        out["cpu_oracle_us_per_step_median"] = 1e6 * float(np.median(tc))
    return out


ADJ_STEPS, ADJ_DT, ADJ_OBS = 12, 1800.0, 5000


def adjoint_leg(X, torch, fd_dirs=4, cpu=True):
    """Level-7 twin experiment (N = 163842, n = 655368): the gradient of
    L = 1/2 sum (h - y)^2 over 5000 observations of a 12-step exprb42
    trajectory (1800 s steps) with respect to the whole initial state, by
    per-step vector-Jacobian products on the schedules recorded by the
    forward.  Reported: forward time (recording), reverse-sweep time (with
    its forward recomputation), their ratio, and central differences of the
    replayed forward along seeded directions."""
    import numpy as np
    import oracle as O
    from synth import fields as F
    from synth.mesh import get_mesh
    level = 7
    mesh = get_mesh(level)
    n = len(mesh["xyz"])
    u0h, uth, ost, oce, oer = F.adjoint_twin(level, F.config_seed(4), ADJ_STEPS, ADJ_OBS)
    dev = "cuda:0"
    ctx = X.Context(mesh, dev, gamma_h=4e-4, tol=1e-10, m_max=40)
    tune = ctx.autotune(1)                       # launch shapes for this grid
    cells = [torch.tensor(3 * n + oce[ost == k], device=dev) for k in range(ADJ_STEPS + 1)]
    errs = [torch.tensor(oer[ost == k], dtype=torch.float64, device=dev)
            for k in range(ADJ_STEPS + 1)]
    empty = np.zeros((0, 3))

    def run(u_init, record=False, scheds=None):
        u = u_init.clone()
        us, rec = [u.clone()], []
        ctx.reset_history()
        for k in range(ADJ_STEPS):
            if record or scheds is not None:
                ctx.schedule_set(empty if record else scheds[k])
                ctx.schedule_mode(X.RECORD if record else X.REPLAY)
            ctx.step("exprb42", u, ADJ_DT)
            if record or scheds is not None:
                ctx.schedule_mode(X.FREE)
            if record:
                rec.append(ctx.schedule_get())
            us.append(u.clone())
        return us, rec

    # truth and observations
    tru, _ = run(torch.tensor(uth, dtype=torch.float64, device=dev))
    ys = [tru[k][cells[k]] + errs[k] for k in range(ADJ_STEPS + 1)]

    def loss(us):
        return sum(0.5 * float(((us[k][cells[k]] - ys[k]) ** 2).sum())
                   for k in range(1, ADJ_STEPS + 1))

    u0 = torch.tensor(u0h, dtype=torch.float64, device=dev)

    def gradient(us, scheds, stats=None):
        g = torch.zeros(4 * n, dtype=torch.float64, device=dev)
        for k in range(ADJ_STEPS, 0, -1):
            g.index_add_(0, cells[k], us[k][cells[k]] - ys[k])
            if stats is None:
                g = ctx.step_vjp("exprb42", us[k - 1], ADJ_DT, g, sched=scheds[k - 1])
            else:
                g, st = ctx.step_vjp("exprb42", us[k - 1], ADJ_DT, g, sched=scheds[k - 1],
                                     return_stats=True)
                stats.append(st)
        return g

    us, scheds = run(u0, record=True)            # warm-up: workspaces, substep store
    gradient(us, scheds)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    us, scheds = run(u0, record=True)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    g = gradient(us, scheds)
    torch.cuda.synchronize()
    t2 = time.perf_counter()
    st = []
    gradient(us, scheds, st)
    L0 = loss(us)
    fwd, bwd = t1 - t0, t2 - t1
    # central differences of the replayed forward
    # central differences of the replayed forward.  eps = 1e-5 (times the
    # block RMS): at this size the replayed discrete map is not smooth below
    # ~1e-9 relative (IOM2 near-breakdowns; the oracle shows the same), so
    # smaller steps measure that roughness rather than the gradient.
    rng = np.random.default_rng(F.config_seed(4))
    scal = np.repeat([np.sqrt(np.mean(u0h[b * n:(b + 1) * n] ** 2)) for b in range(4)], n)
    fd = []
    eps = 1e-5
    for _ in range(fd_dirs):
        d = torch.tensor(rng.standard_normal(4 * n) * scal, device=dev)
        lp = loss(run(u0 + eps * d, scheds=scheds)[0])
        lm = loss(run(u0 - eps * d, scheds=scheds)[0])
        f = (lp - lm) / (2 * eps)
        a = float(g @ d)
        fd.append(abs(f - a) / abs(a))
    agg = {}
    for s2 in st:
        for c in s2:
            for k2 in ("attempts", "rejected", "accepted", "matvecs", "expms", "sum_m"):
                agg[k2] = agg.get(k2, 0) + c[k2]
    out = {"workload": "exprb42, 12 steps of 1800 s, level-7 grid (N=163842, n=655368), "
                       "5000 depth observations (twin experiment), FP64, tol 1e-10, m_max 40",
           "loss": L0, "forward_ms": 1e3 * fwd, "reverse_ms": 1e3 * bwd,
           "adjoint_over_forward": bwd / fwd, "fd_rel_err_max": max(fd) if fd else None,
           "fd_directions": fd_dirs, "fd_eps": eps, "adjoint_krylov": agg,
           "lanes": tune["lanes"]}
    if cpu:
        s = O.SWE(mesh, gamma_h=4e-4)
        gh = np.zeros(4 * n)
        gh[3 * n + oce[ost == ADJ_STEPS]] = 1.0
        tc = time.perf_counter()
        s.step_vjp("exprb42", u0h, ADJ_DT, gh, O.opts())
        out["cpu_oracle_step_vjp_s"] = time.perf_counter() - tc
        out["cpu_oracle_note"] = "one step vector-Jacobian product (forward recomputation " \
                                 "included), serial C oracle, free controller"
    ctx.close()
    return out


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
    ap.add_argument("--no-c1", action="store_true", help="skip the level-4 single-step leg")
    ap.add_argument("--lanes", type=int, default=0,
                    help="lanes per cell for the level-6 workload (0: the library's choice)")
    ap.add_argument("--autotune", action="store_true",
                    help="tune the level-6 context's lanes before measuring")
    ap.add_argument("--no-ensemble", action="store_true")
    ap.add_argument("--no-jet", action="store_true")
    ap.add_argument("--jet-only", action="store_true",
                    help="run only the level-8 leg (for profiling it alone)")
    ap.add_argument("--no-adjoint", action="store_true")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="end with three 64 MiB device-to-device copies (the reference "
                         "kernel for scaling PMC byte counters)")
    ap.add_argument("--adjoint-only", action="store_true",
                    help="run only the level-7 adjoint leg")
    ap.add_argument("--ensemble-only", action="store_true",
                    help="run only the 64-member level-6 ensemble leg")
    ap.add_argument("--event-every", type=int, default=64,
                    help="time every N-th launch of each kernel of the level-6 workload with HIP "
                         "events (each timed launch adds two event records; 16 costs the "
                         "measured rate about 5 %%, 64 is within noise of none)")
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

    if args.jet_only:
        print(json.dumps({"level8_jet": jet_leg(X, torch, JET_EVENT_EVERY)}))
        if args.copy_calibration:
            copy_calibration(torch)
        return
    if args.adjoint_only:
        print(json.dumps({"adjoint": adjoint_leg(X, torch, cpu=not args.no_cpu)}))
        return
    if args.ensemble_only:
        print(json.dumps({"ensemble": ensemble_leg(X, torch, get_mesh(6))}))
        return

    level = 6
    mesh = get_mesh(level)
    n = len(mesh["xyz"])
    u0_host = F.initial_state("c2_l6_24x3600")
    ctx = X.Context(mesh, "cuda:0", gamma_h=4e-4, tol=1e-10, m_max=40, lanes=args.lanes)
    tune = ctx.autotune(1) if args.autotune else None
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
    traffic = measured_traffic()
    roofline = {"bound": "hbm", "kernel": "k_jv<kEpiIom2>", "achieved": achieved,
                "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": achieved / HBM_PEAK_GBS,
                "traffic": traffic,
                "traffic_over_algorithmic": (traffic / (JV_IOM2_BYTES_PER_CELL * n)
                                             if traffic else None),
                "avg_us": avg_s * 1e6, "launches": all_n,
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

    c1 = None if args.no_c1 else c1_leg(X, torch, cpu=not args.no_cpu)
    ens = None if args.no_ensemble else ensemble_leg(X, torch, mesh)
    jet = None if args.no_jet else jet_leg(X, torch, JET_EVENT_EVERY)
    adj = None if args.no_adjoint else adjoint_leg(X, torch, cpu=not args.no_cpu)

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
        "lanes": {"requested": args.lanes, "autotuned": tune},
        "level4_c1": c1,
        "ensemble": ens,
        "level8_jet": jet,
        "adjoint": adj,
        "device_time_fraction": (tot_ms * 1e-3) / elapsed,
    }
    print(json.dumps(out))
    ctx.close()
    if args.copy_calibration:
        copy_calibration(torch)


def copy_calibration(torch):
    """Three 64 MiB device-to-device copies: the reference a profiler's byte
    counters are scaled by (a plain copy of known size), and the measured
    streaming bandwidth (read + write) of the part."""
    a = torch.ones(1 << 23, dtype=torch.float64, device="cuda:0")
    b = torch.empty_like(a)
    for _ in range(3):
        b.copy_(a)
    torch.cuda.synchronize()


if __name__ == "__main__":
    main()
