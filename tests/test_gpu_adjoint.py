"""GPU parity of the adjoint path against the oracle: J^T and K stencils,
the exprb42 step vector-Jacobian product on the replayed forward (per
variable block, 1e-11 relative), a trajectory gradient, and a central-
difference check of the GPU gradient against the GPU's own replayed
forward."""
import sys

import numpy as np
import pytest

import oracle as O
from synth import fields as F
from synth.mesh import get_mesh

pytestmark = pytest.mark.gpu
TOL_STENCIL = 1e-12
TOL = 1e-11


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


_CACHE = {}


def setup(X, level):
    if level not in _CACHE:
        mesh = get_mesh(level)
        _CACHE[level] = (X.Context(mesh, "cuda:0"), O.SWE(mesh))
    return _CACHE[level]


def blocks_rel(got, ref, n):
    out = []
    for b in range(4):
        sl = slice(b * n, (b + 1) * n)
        den = np.linalg.norm(ref[sl])
        out.append(np.linalg.norm(got[sl] - ref[sl]) / den if den > 0 else np.linalg.norm(got[sl]))
    return max(out)


def to_np(t):
    import torch
    torch.cuda.synchronize()
    return t.cpu().numpy()


def rand_dir(n, seed, scale=(5.0, 50.0)):
    rng = np.random.default_rng(seed)
    return rng.standard_normal(4 * n) * np.r_[np.full(3 * n, scale[0]), np.full(n, scale[1])]


@pytest.mark.parametrize("level", [2, 4, 6])
def test_jtv_parity_and_dot(X, level):
    ctx, s = setup(X, level)
    u = F.initial_state("c2_l6_24x3600", level=level)
    w = rand_dir(s.n, level)
    v = rand_dir(s.n, level + 50)
    say("jtv level", level)
    got = to_np(ctx.jtv(u, w))
    assert blocks_rel(got, s.jtv(u, w), s.n) < TOL_STENCIL
    lhs = w @ to_np(ctx.jv(u, v))
    rhs = got @ v
    assert abs(lhs - rhs) <= 1e-12 * np.linalg.norm(w) * np.linalg.norm(to_np(ctx.jv(u, v)))


@pytest.mark.parametrize("level", [2, 5, 6])
def test_ktv_parity(X, level):
    """Levels 2 and 5 take the gather kernel, level 6 (chunk tables) the
    LDS-staged one."""
    ctx, s = setup(X, level)
    a = rand_dir(s.n, 7 + level)
    b = rand_dir(s.n, 8 + level)
    say("ktv level", level)
    assert blocks_rel(to_np(ctx.ktv(a, b)), s.ktv(a, b), s.n) < TOL_STENCIL


def _record_step(s, u0, dt, tol=1e-10):
    sch = O.new_schedule()
    u1 = O.swe_stepper(s, "exprb42").step(u0, dt, O.opts(tol=tol, mode=O.RECORD, sched=sch))
    return u1, sch.as_array()


@pytest.mark.parametrize("level,dt", [(3, 1800.0), (4, 3600.0)])
def test_step_vjp_parity(X, level, dt):
    ctx, s = setup(X, level)
    u0 = F.initial_state("c1_exprb42_l4", level=level)
    _, arr = _record_step(s, u0, dt)
    ubar = rand_dir(s.n, 31, (1.0, 1e-2))
    say("step_vjp level", level, "dt", dt, "attempts", len(arr))
    ref, ast = s.step_vjp("exprb42", u0, dt, ubar,
                          O.opts(mode=O.REPLAY, sched=O.schedule_from_array(arr)))
    got, gst = ctx.step_vjp("exprb42", u0, dt, ubar, sched=arr, return_stats=True)
    got = to_np(got)
    say("  oracle adjoint", ast, "\n  gpu adjoint", gst)
    for a, g in zip(ast, gst):
        assert (a["accepted"], a["sum_m"], a["attempts"]) == (g["accepted"], g["sum_m"], g["attempts"])
    assert blocks_rel(got, ref, s.n) < TOL
    assert blocks_rel(got - ubar, ref - ubar, s.n) < TOL


def test_step_vjp_in_place_and_zero(X):
    import torch
    ctx, s = setup(X, 3)
    u0 = F.initial_state("c1_exprb42_l4", level=3)
    _, arr = _record_step(s, u0, 1800.0)
    ubar = rand_dir(s.n, 32, (1.0, 1e-2))
    a = to_np(ctx.step_vjp("exprb42", u0, 1800.0, ubar, sched=arr))
    t = torch.tensor(ubar, device="cuda:0")
    lib = __import__("paper_1805_02144_amd").lib()
    ut = torch.tensor(u0, device="cuda:0")
    rc = lib.xrb_step_vjp(ctx.h, 0, ut.data_ptr(), 1800.0,
                          arr.ctypes.data_as(__import__("ctypes").POINTER(__import__("ctypes").c_double)),
                          len(arr), t.data_ptr(), t.data_ptr(), None)
    assert rc == 0
    assert np.array_equal(to_np(t), a)            # in place == out of place, bitwise
    z = to_np(ctx.step_vjp("exprb42", u0, 1800.0, np.zeros(4 * s.n), sched=arr))
    assert not np.any(z)


def test_trajectory_gradient_parity(X):
    import torch
    ctx, s = setup(X, 3)
    u0 = F.initial_state("c1_exprb42_l4", level=3)
    dt, steps = 1800.0, 3
    rng = np.random.default_rng(44)
    obs_step = rng.integers(1, steps + 1, 60)
    obs_cell = rng.choice(s.n, 60, replace=False)
    obs_val = u0[3 * s.n + obs_cell] + rng.normal(0.0, 5.0, 60)
    L, g_ref, scheds = O.exprb42_loss_grad(s, u0, dt, steps, obs_step, obs_cell, obs_val)
    # GPU: forward with recorded per-step schedules, then the reverse sweep
    us = [u0.copy()]
    gsch = []
    u = torch.tensor(u0, device="cuda:0")
    ctx.reset_history()
    for k in range(steps):
        ctx.schedule_set(np.zeros((0, 3)))
        ctx.schedule_mode(X.RECORD)
        ctx.step("exprb42", u, dt)
        ctx.schedule_mode(X.FREE)
        gsch.append(ctx.schedule_get())
        us.append(to_np(u).copy())
    for a, b in zip(gsch, scheds):
        assert len(a) == len(b) and np.array_equal(a[:, 1:], b[:, 1:])
    g = np.zeros(4 * s.n)
    for k in range(steps, 0, -1):
        sel = obs_step == k
        np.add.at(g, 3 * s.n + obs_cell[sel], us[k][3 * s.n + obs_cell[sel]] - obs_val[sel])
        g = to_np(ctx.step_vjp("exprb42", us[k - 1], dt, g, sched=scheds[k - 1]))
    say("trajectory gradient rel", blocks_rel(g, g_ref, s.n))
    assert blocks_rel(g, g_ref, s.n) < TOL


def test_step_vjp_central_difference_on_gpu(X):
    """<ubar, (Psi(u + e d) - Psi(u - e d)) / 2e> against <vjp(ubar), d>, the
    forward replayed on the GPU (level 5)."""
    import torch
    ctx, s = setup(X, 5)
    u0 = F.initial_state("c1_exprb42_l4", level=5)
    dt = 1800.0
    _, arr = _record_step(s, u0, dt)
    ubar = rand_dir(s.n, 51, (1.0, 1e-2))
    g = to_np(ctx.step_vjp("exprb42", u0, dt, ubar, sched=arr))
    scal = np.repeat([np.sqrt(np.mean(u0[b * s.n:(b + 1) * s.n] ** 2)) for b in range(4)], s.n)

    def psi(u):
        ctx.reset_history()
        ctx.schedule_set(arr)
        ctx.schedule_mode(X.REPLAY)
        try:
            t = torch.tensor(u, device="cuda:0")
            ctx.step("exprb42", t, dt)
            return to_np(t)
        finally:
            ctx.schedule_mode(X.FREE)

    rng = np.random.default_rng(52)
    eps = 1e-5
    for _ in range(2):
        d = rng.standard_normal(4 * s.n) * scal
        fd = ubar @ (psi(u0 + eps * d) - psi(u0 - eps * d)) / (2 * eps)
        say("  fd", fd, "adjoint", g @ d)
        assert abs(fd - g @ d) <= 1e-8 * abs(g @ d)


def test_level7_step_vjp_parity(X):
    """The adjoint workload's shape: level 7, an observation-like cotangent
    (depth at a seeded subset of cells), one exprb42 step of 1800 s, the
    forward replayed from the oracle's schedule."""
    mesh = get_mesh(7)
    s = O.SWE(mesh)
    n = s.n
    u0, _, ost, oce, oer = F.adjoint_twin(7, F.config_seed(4), 12, 5000)
    _, arr = _record_step(s, u0, 1800.0)
    ubar = np.zeros(4 * n)
    sel = oce[ost == 1]
    ubar[3 * n + sel] = oer[ost == 1]
    say("level 7 step_vjp, attempts", len(arr))
    ref, ast = s.step_vjp("exprb42", u0, 1800.0, ubar,
                          O.opts(mode=O.REPLAY, sched=O.schedule_from_array(arr)))
    ctx = X.Context(mesh, "cuda:0")
    got, gst = ctx.step_vjp("exprb42", u0, 1800.0, ubar, sched=arr, return_stats=True)
    got = to_np(got)
    for a, g in zip(ast, gst):
        assert (a["accepted"], a["sum_m"], a["attempts"]) == (g["accepted"], g["sum_m"], g["attempts"])
    say("  rel", blocks_rel(got, ref, n))
    assert blocks_rel(got, ref, n) < TOL
    ctx.close()


def test_autograd_trajectory(X):
    """X.trajectory as a torch.autograd.Function: the gradient of a loss on
    the states (observations of the depth) against the oracle's trajectory
    gradient, and the states themselves against plain steps."""
    import torch
    ctx, s = setup(X, 3)
    n = s.n
    u0h = F.initial_state("c1_exprb42_l4", level=3)
    dt, steps = 1800.0, 3
    rng = np.random.default_rng(45)
    obs_step = rng.integers(1, steps + 1, 50)
    obs_cell = rng.choice(n, 50, replace=False)
    obs_val = u0h[3 * n + obs_cell] + rng.normal(0.0, 5.0, 50)
    L_ref, g_ref, _ = O.exprb42_loss_grad(s, u0h, dt, steps, obs_step, obs_cell, obs_val)
    u0 = torch.tensor(u0h, device="cuda:0", requires_grad=True)
    states = X.trajectory(ctx, u0, [dt] * steps)
    y = torch.tensor(obs_val, device="cuda:0")
    r = states[torch.tensor(obs_step, device="cuda:0"), torch.tensor(3 * n + obs_cell, device="cuda:0")] - y
    loss = 0.5 * (r * r).sum()
    loss.backward()
    lv = float(loss.detach())
    say("autograd loss", lv, "oracle", L_ref)
    assert abs(lv - L_ref) <= 1e-9 * L_ref
    assert blocks_rel(u0.grad.detach().cpu().numpy(), g_ref, n) < TOL
    # the states equal plain steps
    u = torch.tensor(u0h, device="cuda:0")
    ctx.reset_history()
    for k in range(steps):
        ctx.step("exprb42", u, dt)
    assert np.array_equal(to_np(u), states[-1].detach().cpu().numpy())


def test_c5_level7_step_vjp(X):
    """C5 at full size (level 7, the twin-experiment state): one exprb42
    step VJP of 1800 s on the oracle's recorded schedule, in the adjoint
    workload's launch configuration (lanes chosen by the autotuner), against
    the oracle's VJP, per variable block."""
    import torch
    level, dt = 7, 1800.0
    mesh = get_mesh(level)
    s = O.SWE(mesh)
    n = s.n
    u0h, _, ost, oce, _ = F.adjoint_twin(level, F.config_seed(4), 12, 5000)
    sch = O.new_schedule()
    u1 = O.swe_stepper(s, "exprb42").step(u0h, dt, O.opts(mode=O.RECORD, sched=sch))
    arr = sch.as_array()
    rng = np.random.default_rng(3)
    ubar = np.zeros(4 * n)
    sel = oce[ost == 1]
    ubar[3 * n + sel] = rng.normal(0.0, 5.0, len(sel))
    gref, _ = s.step_vjp("exprb42", u0h, dt, ubar,
                         O.opts(mode=O.REPLAY, sched=O.schedule_from_array(arr)))
    ctx = X.Context(mesh, "cuda:0")
    try:
        tune = ctx.autotune(1)
        say("C5 level 7, lanes", tune["lanes"], "attempts", len(arr))
        ctx.reset_history()
        ctx.schedule_set(arr)
        ctx.schedule_mode(X.REPLAY)
        u = torch.tensor(u0h, device="cuda:0")
        ctx.step("exprb42", u, dt)
        ctx.schedule_mode(X.FREE)
        g1 = to_np(u)
        assert blocks_rel(g1, u1, n) < TOL
        assert blocks_rel(g1 - u0h, u1 - u0h, n) < TOL
        gg = to_np(ctx.step_vjp("exprb42", u0h, dt, ubar, sched=arr))
        err = blocks_rel(gg, gref, n)
        say("  vjp rel", err)
        assert err < TOL
    finally:
        ctx.close()
