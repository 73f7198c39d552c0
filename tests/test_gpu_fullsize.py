"""Every workload compared with the oracle at its full size and full length
(Alg. 1 and the scheme mappings of Sec. 4.4; the adjoint is not in the
paper).  Replay mode -- the oracle's substep schedule consumed by the GPU --
is the binding 1e-11 check; free mode (the GPU's own controller) must take
the oracle's decisions, and then meet the same bar.

* level 6 (n = 163848): pexprb43 and exprb53, 24 steps of 3600 s each, every
  step's state and increment per variable block;
* level 8 (n = 2621448, jet, gamma_h = 1.25e-2): exprb53, all 6 steps of
  1800 s, one test per step so that progress shows;
* level 6 ensemble: all 64 members (one exprb42 step each, per-member step
  sizes) replayed from per-member oracle schedules and free-running, every
  member against the oracle, and the free batch bitwise equal to 64
  single-state steps;
* level 7 twin experiment: the 12-step exprb42 gradient of the observation
  misfit against the oracle's gradient on the same schedules.

The oracle runs its independent cell loops on several host threads here
(bitwise the serial result)."""
import os
import sys
from concurrent.futures import ThreadPoolExecutor

import numpy as np
import pytest

import oracle as O
from synth import fields as F
from synth.mesh import get_mesh

pytestmark = pytest.mark.gpu
TOL = 1e-11
THREADS = max(1, min(16, os.cpu_count() or 1))


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def X():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_1805_02144_amd as X
    X.lib()
    return X


@pytest.fixture(scope="module", autouse=True)
def oracle_threads():
    O.set_threads(THREADS)
    yield
    O.set_threads(1)


def blocks_rel(got, ref, n, base=None):
    base = ref if base is None else base
    out = []
    for b in range(4):
        sl = slice(b * n, (b + 1) * n)
        den = np.linalg.norm(base[sl])
        out.append(np.linalg.norm(got[sl] - ref[sl]) / den if den > 0 else np.linalg.norm(got[sl]))
    return max(out)


def to_np(t):
    import torch
    torch.cuda.synchronize()
    return t.cpu().numpy()


def decision_mismatches(gs, rs):
    """Attempts whose Krylov size or accept/land flags differ, plus any
    difference in the number of attempts."""
    k = min(len(gs), len(rs))
    return int(np.sum(np.any(gs[:k, 1:] != rs[:k, 1:], axis=1))) + abs(len(gs) - len(rs))


# ---------------------------------------------------------------- level 6
@pytest.mark.parametrize("method", ["pexprb43", "exprb53"])
def test_c2_full_length(X, method):
    """24 steps of 3600 s on the level-6 grid, replayed and free."""
    import torch
    mesh = get_mesh(6)
    s = O.SWE(mesh)
    n = s.n
    u0 = F.initial_state("c2_l6_24x3600")
    st = O.swe_stepper(s, method)
    refs, scheds = [u0], []
    for k in range(24):
        sch = O.new_schedule()
        refs.append(st.step(refs[-1], 3600.0, O.opts(mode=O.RECORD, sched=sch)))
        scheds.append(sch.as_array())
        if k % 6 == 5:
            say("C2 %s oracle step %d, attempts so far %d" % (method, k + 1,
                                                              sum(len(a) for a in scheds)))
    ctx = X.Context(mesh, "cuda:0")
    allsched = np.concatenate(scheds)
    # replay: the whole run's attempts in one schedule
    ctx.reset_history()
    ctx.schedule_set(allsched)
    ctx.schedule_mode(X.REPLAY)
    u = torch.tensor(u0, device="cuda:0")
    prev = u0
    e_state = e_inc = 0.0
    try:
        for k in range(24):
            ctx.step(method, u, 3600.0)
            g = to_np(u).copy()
            e_state = max(e_state, blocks_rel(g, refs[k + 1], n))
            e_inc = max(e_inc, blocks_rel(g - prev, refs[k + 1] - refs[k], n))
            prev = g
    finally:
        ctx.schedule_mode(X.FREE)
    say("C2 %s replay: worst state %.2e, worst increment %.2e over 24 steps"
        % (method, e_state, e_inc))
    assert e_state < TOL and e_inc < TOL
    # free: the GPU's controller decides
    ctx.reset_history()
    ctx.schedule_mode(X.RECORD)
    u = torch.tensor(u0, device="cuda:0")
    try:
        for k in range(24):
            ctx.step(method, u, 3600.0)
    finally:
        gs = ctx.schedule_get()
        ctx.schedule_mode(X.FREE)
    mis = decision_mismatches(gs, allsched)
    g = to_np(u)
    e_free = blocks_rel(g, refs[-1], n)
    e_free_inc = blocks_rel(g - u0, refs[-1] - u0, n)
    say("C2 %s free: %d attempts (oracle %d), %d decision mismatches, final state %.2e, "
        "increment over the run %.2e" % (method, len(gs), len(allsched), mis, e_free, e_free_inc))
    ctx.close()
    assert mis == 0
    assert e_free < TOL and e_free_inc < TOL


# ---------------------------------------------------------------- level 8
_C3 = {}


@pytest.mark.parametrize("k", range(1, 7))
def test_c3_full_length(X, k):
    """exprb53 step k of 6 (1800 s) on the level-8 jet, replayed from the
    oracle's schedule of that step; the GPU runs on its own trajectory."""
    import torch
    if k == 1:
        mesh = get_mesh(8)
        s = O.SWE(mesh, gamma_h=1.25e-2)
        u0 = F.initial_state("c3_l8_jet")
        _C3.clear()
        _C3.update(s=s, st=O.swe_stepper(s, "exprb53"), ref=u0, gpu_prev=u0,
                   ctx=X.Context(mesh, "cuda:0", gamma_h=1.25e-2),
                   u=torch.tensor(u0, device="cuda:0"), done=0)
        _C3["ctx"].reset_history()
    if _C3.get("done") != k - 1:
        pytest.skip("the previous level-8 step did not complete")
    s, ctx = _C3["s"], _C3["ctx"]
    sch = O.new_schedule()
    ref_prev = _C3["ref"]
    ref = _C3["st"].step(ref_prev, 1800.0, O.opts(mode=O.RECORD, sched=sch))
    say("C3 step %d: oracle attempts %d" % (k, sch.len))
    ctx.schedule_set(sch.as_array())
    ctx.schedule_mode(X.REPLAY)
    try:
        ctx.step("exprb53", _C3["u"], 1800.0)
    finally:
        ctx.schedule_mode(X.FREE)
    g = to_np(_C3["u"]).copy()
    e_state = blocks_rel(g, ref, s.n)
    e_inc = blocks_rel(g - _C3["gpu_prev"], ref - ref_prev, s.n)
    say("C3 step %d: state %.2e, increment %.2e" % (k, e_state, e_inc))
    _C3.update(ref=ref, gpu_prev=g)
    assert e_state < TOL and e_inc < TOL
    _C3["done"] = k
    if k == 6:
        ctx.close()
        _C3.clear()


# ---------------------------------------------------------------- ensemble
def _oracle_members(mesh, U, dts):
    """One recorded exprb42 step per member, members spread over host threads
    (each thread its own model, one oracle thread each)."""
    import threading
    local = threading.local()

    def one(k):
        if not hasattr(local, "s"):
            local.s = O.SWE(mesh)
        sch = O.new_schedule()
        u1 = O.swe_stepper(local.s, "exprb42").step(U[k], dts[k],
                                                    O.opts(mode=O.RECORD, sched=sch))
        return u1, sch.as_array()

    O.set_threads(1)
    try:
        with ThreadPoolExecutor(THREADS) as ex:
            out = list(ex.map(one, range(len(U))))
    finally:
        O.set_threads(THREADS)
    return [o[0] for o in out], [o[1] for o in out]


def test_c4_all_members(X):
    """All 64 level-6 members, one exprb42 step each with its own step size
    from {600, 1200, 2400, 3600} s: replayed per member, free per member,
    and the free batch bitwise equal to 64 single-state steps."""
    import torch
    mesh = get_mesh(6)
    U, dts = F.ensemble_states(6, F.config_seed(3), 64)
    n = len(mesh["xyz"])
    refs, scheds = _oracle_members(mesh, U, dts)
    say("C4 oracle: 64 members, %d attempts" % sum(len(a) for a in scheds))
    ctx = X.Context(mesh, "cuda:0")
    # replay, each member from its own schedule
    ctx.reset_history()
    for k in range(64):
        ctx.schedule_set_member(k, scheds[k])
    ctx.schedule_mode(X.REPLAY)
    Ub = torch.tensor(U, device="cuda:0")
    try:
        ctx.step_batch("exprb42", Ub, dts)
    finally:
        ctx.schedule_mode(X.FREE)
    got = to_np(Ub)
    e_rep = max(max(blocks_rel(got[k], refs[k], n), blocks_rel(got[k] - U[k], refs[k] - U[k], n))
                for k in range(64))
    say("C4 replay: worst member %.2e" % e_rep)
    assert e_rep < TOL
    # free, every member recording its own decisions
    ctx.reset_history()
    ctx.schedule_mode(X.RECORD)
    Ub = torch.tensor(U, device="cuda:0")
    try:
        ctx.step_batch("exprb42", Ub, dts)
    finally:
        gsch = [ctx.schedule_get_member(k) for k in range(64)]
        ctx.schedule_mode(X.FREE)
    got = to_np(Ub)
    mis = [decision_mismatches(gsch[k], scheds[k]) for k in range(64)]
    e_free = max(blocks_rel(got[k] - U[k], refs[k] - U[k], n) for k in range(64) if mis[k] == 0)
    say("C4 free: %d members with decision mismatches, worst member %.2e"
        % (sum(m > 0 for m in mis), e_free))
    assert sum(mis) == 0 and e_free < TOL
    # the batch is bitwise the per-member steps
    u = torch.empty(4 * n, dtype=torch.float64, device="cuda:0")
    for k in range(64):
        ctx.reset_history()
        u.copy_(torch.as_tensor(U[k], device="cuda:0"))
        ctx.step("exprb42", u, float(dts[k]))
        assert np.array_equal(to_np(u), got[k]), k
    ctx.close()


# ---------------------------------------------------------------- adjoint
_C5 = {}
C5_STEPS, C5_DT = 12, 1800.0


def test_c5_forward(X):
    """Level-7 twin experiment, forward: the truth run gives the observations
    (the same y for both sides), then 12 exprb42 steps of 1800 s recorded by
    the oracle and replayed on the GPU, every step's state compared."""
    import torch
    level = 7
    mesh = get_mesh(level)
    s = O.SWE(mesh)
    n = s.n
    u0, ut, ost, oce, oer = F.adjoint_twin(level, F.config_seed(4), C5_STEPS, 5000)
    st = O.swe_stepper(s, "exprb42")
    tru = [ut]
    for k in range(C5_STEPS):
        tru.append(st.step(tru[-1], C5_DT))
    y = np.array([tru[k][3 * n + c] for k, c in zip(ost, oce)]) + oer
    say("C5 truth run done")
    st = O.swe_stepper(s, "exprb42")
    refs, scheds = [u0], []
    for k in range(C5_STEPS):
        sch = O.new_schedule()
        refs.append(st.step(refs[-1], C5_DT, O.opts(mode=O.RECORD, sched=sch)))
        scheds.append(sch.as_array())
    say("C5 oracle forward done")
    ctx = X.Context(mesh, "cuda:0")
    ctx.autotune(1)                       # the adjoint workload's launch configuration
    us = [torch.tensor(u0, device="cuda:0")]
    ctx.reset_history()
    e = 0.0
    for k in range(C5_STEPS):
        ctx.schedule_set(scheds[k])
        ctx.schedule_mode(X.REPLAY)
        try:
            u = us[-1].clone()
            ctx.step("exprb42", u, C5_DT)
        finally:
            ctx.schedule_mode(X.FREE)
        us.append(u)
        e = max(e, blocks_rel(to_np(u), refs[k + 1], n))
    say("C5 forward: worst state %.2e" % e)
    cells = [3 * n + oce[ost == k] for k in range(C5_STEPS + 1)]
    ys = [y[ost == k] for k in range(C5_STEPS + 1)]
    L_ref = sum(0.5 * float(((refs[k][cells[k]] - ys[k]) ** 2).sum())
                for k in range(1, C5_STEPS + 1))
    L = sum(0.5 * float(((to_np(us[k])[cells[k]] - ys[k]) ** 2).sum())
            for k in range(1, C5_STEPS + 1))
    say("C5 loss %.12e (oracle %.12e)" % (L, L_ref))
    _C5.clear()
    _C5.update(s=s, ctx=ctx, us=us, refs=refs, scheds=scheds, cells=cells, ys=ys,
               g=np.zeros(4 * n), g_ref=np.zeros(4 * n), next=C5_STEPS)
    assert e < TOL
    assert abs(L - L_ref) <= TOL * abs(L_ref)


@pytest.mark.parametrize("k", range(C5_STEPS, 0, -1))
def test_c5_reverse(X, k):
    """Reverse step k of the twin experiment's gradient: the cotangent after
    adding step k's misfit, pulled back through step k by the GPU's
    vector-Jacobian product and by the oracle's, both on the recorded
    schedule (the per-step loop of the oracle's exprb42_loss_grad); each
    side carries its own running gradient, compared per variable block."""
    import torch
    if _C5.get("next") != k:
        pytest.skip("the forward run or a later reverse step did not complete")
    s, ctx = _C5["s"], _C5["ctx"]
    n = s.n
    refs, us, cells, ys = _C5["refs"], _C5["us"], _C5["cells"], _C5["ys"]
    g_ref = _C5["g_ref"]
    np.add.at(g_ref, cells[k], refs[k][cells[k]] - ys[k])
    g_ref, _ = s.step_vjp("exprb42", refs[k - 1], C5_DT, g_ref,
                          O.opts(mode=O.REPLAY, sched=O.schedule_from_array(_C5["scheds"][k - 1])))
    g = torch.tensor(_C5["g"], device="cuda:0")
    idx = torch.tensor(cells[k], device="cuda:0")
    g.index_add_(0, idx, us[k][idx] - torch.tensor(ys[k], device="cuda:0"))
    g = ctx.step_vjp("exprb42", us[k - 1], C5_DT, g, sched=_C5["scheds"][k - 1])
    got = to_np(g)
    e = blocks_rel(got, g_ref, n)
    say("C5 reverse step %d: gradient per block %.2e" % (k, e))
    _C5.update(g=got, g_ref=g_ref)
    assert e < TOL
    _C5["next"] = k - 1
    if k == 1:
        ctx.close()
        _C5.clear()


def test_c5_central_differences(X):
    """Central differences of the replayed level-7 twin experiment along 8
    seeded directions (eps = 1e-6 times each block's RMS) against the GPU
    gradient, with the Krylov tolerance at 1e-14 for the forward and the
    adjoint: at the workload's 1e-10 the replayed map carries the Krylov
    approximation error, whose variation along a direction is of order
    tol ||v|| / eps and swamps a 1e-6 comparison (the oracle shows the same
    roughness, and it shrinks with the tolerance)."""
    import torch
    level, steps, dt, eps = 7, 12, 1800.0, 1e-6
    mesh = get_mesh(level)
    n = len(mesh["xyz"])
    u0h, uth, ost, oce, oer = F.adjoint_twin(level, F.config_seed(4), steps, 5000)
    ctx = X.Context(mesh, "cuda:0", tol=1e-14)
    cells = [torch.tensor(3 * n + oce[ost == k], device="cuda:0") for k in range(steps + 1)]

    def run(u_init, record=False, scheds=None):
        u = torch.tensor(u_init, device="cuda:0") if isinstance(u_init, np.ndarray) \
            else u_init.clone()
        us, rec = [u.clone()], []
        ctx.reset_history()
        for k in range(steps):
            if record or scheds is not None:
                ctx.schedule_set(np.zeros((0, 3)) if record else scheds[k])
                ctx.schedule_mode(X.RECORD if record else X.REPLAY)
            try:
                ctx.step("exprb42", u, dt)
            finally:
                ctx.schedule_mode(X.FREE)
            if record:
                rec.append(ctx.schedule_get())
            us.append(u.clone())
        return us, rec

    tru, _ = run(uth)
    ys = [tru[k][cells[k]] + torch.tensor(oer[ost == k], device="cuda:0")
          for k in range(steps + 1)]

    def loss(us):
        return sum(0.5 * float(((us[k][cells[k]] - ys[k]) ** 2).sum())
                   for k in range(1, steps + 1))

    u0 = torch.tensor(u0h, device="cuda:0")
    us, scheds = run(u0, record=True)
    g = torch.zeros(4 * n, dtype=torch.float64, device="cuda:0")
    for k in range(steps, 0, -1):
        g.index_add_(0, cells[k], us[k][cells[k]] - ys[k])
        g = ctx.step_vjp("exprb42", us[k - 1], dt, g, sched=scheds[k - 1])
    rng = np.random.default_rng(F.config_seed(4))
    scal = np.repeat([np.sqrt(np.mean(u0h[b * n:(b + 1) * n] ** 2)) for b in range(4)], n)
    errs = []
    for _ in range(8):
        d = torch.tensor(rng.standard_normal(4 * n) * scal, device="cuda:0")
        lp = loss(run(u0 + eps * d, scheds=scheds)[0])
        lm = loss(run(u0 - eps * d, scheds=scheds)[0])
        a = float(g @ d)
        errs.append(abs((lp - lm) / (2 * eps) - a) / abs(a))
    say("C5 central differences (tol 1e-14, eps 1e-6):", " ".join("%.1e" % e for e in errs))
    ctx.close()
    assert max(errs) <= 1e-6
