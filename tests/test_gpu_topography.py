"""GPU parity with surface topography h_s (eq. sweqsinv's h_s, set through
xrb_set_topography): rhs and diagnostics against the oracle, the product
unchanged (J does not depend on h_s), the lake at rest steady, and replayed
exprb42 steps over a mountain at 1e-11."""
import sys

import numpy as np
import pytest

import oracle as O
from synth import fields as F
from synth.mesh import get_mesh

pytestmark = pytest.mark.gpu
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


def to_np(t):
    import torch
    torch.cuda.synchronize()
    return t.cpu().numpy()


def blocks_rel(got, ref, n, base=None):
    base = ref if base is None else base
    out = []
    for b in range(4):
        sl = slice(b * n, (b + 1) * n)
        den = np.linalg.norm(base[sl])
        out.append(np.linalg.norm(got[sl] - ref[sl]) / den if den > 0 else np.linalg.norm(got[sl]))
    return max(out)


@pytest.mark.parametrize("level", [4, 6])
def test_rhs_product_and_diagnostics_with_topography(X, level):
    """Rhs bar 1e-12 at level 4, 1e-11 (the method's parity bar) at level 6:
    the flow over the mountain is nearly balanced, so F is a residual of
    cancelling terms some 1e4 times larger, and rounding of the same relative
    size as elsewhere shows up larger relative to F."""
    bar = 1e-12 if level == 4 else 1e-11
    mesh = get_mesh(level)
    n = len(mesh["xyz"])
    hs = F.mountain(level, 7)
    u = F.mountain_flow_state(level, 7)
    v = np.random.default_rng(level).standard_normal(4 * n)
    ctx = X.Context(mesh, "cuda:0")
    s = O.SWE(mesh)
    s.set_topography(hs)
    say("topography level", level)
    jv_flat = to_np(ctx.jv(u, v))
    ctx.set_topography(hs)
    assert blocks_rel(to_np(ctx.rhs(u)), s.rhs(u), n) < bar
    assert np.array_equal(to_np(ctx.jv(u, v)), jv_flat)
    got, ref = ctx.diagnostics(u), s.diagnostics(u)
    for k in ref:
        assert abs(got[k] / ref[k] - 1) < 1e-12, k
    ctx.set_topography(None)
    assert blocks_rel(to_np(ctx.rhs(u)), O.SWE(mesh).rhs(u), n) < bar
    ctx.close()


def test_lake_at_rest_on_gpu(X):
    mesh = get_mesh(5)
    n = len(mesh["xyz"])
    hs = F.mountain(5, 7)
    ctx = X.Context(mesh, "cuda:0", gamma_h=0.0)
    ctx.set_topography(hs)
    lake = np.zeros(4 * n)
    lake[3 * n:] = 5000.0 - hs
    assert np.abs(to_np(ctx.rhs(lake))).max() < 1e-14
    ctx.close()


def test_replayed_steps_over_a_mountain(X):
    import torch
    level = 3
    mesh = get_mesh(level)
    n = len(mesh["xyz"])
    hs = F.mountain(level, 7)
    u0 = F.mountain_flow_state(level, 7)
    s = O.SWE(mesh)
    s.set_topography(hs)
    st = O.swe_stepper(s, "exprb42")
    sch = O.new_schedule()
    refs, ur = [], u0.copy()
    for _ in range(2):
        ur = st.step(ur, 1800.0, O.opts(mode=O.RECORD, sched=sch))
        refs.append(ur.copy())
    ctx = X.Context(mesh, "cuda:0")
    ctx.set_topography(hs)
    ctx.reset_history()
    ctx.schedule_set(sch.as_array())
    ctx.schedule_mode(X.REPLAY)
    u = torch.tensor(u0, dtype=torch.float64, device="cuda:0")
    prev = u0
    try:
        for r in refs:
            ctx.step("exprb42", u, 1800.0)
            g = to_np(u)
            assert blocks_rel(g, r, n) < TOL
            assert blocks_rel(g - prev, r - prev, n) < TOL
            prev = r
    finally:
        ctx.schedule_mode(X.FREE)
    ctx.close()
