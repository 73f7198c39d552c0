"""GPU parity of every lanes-per-cell variant of the stencil kernels (1, 2,
4, 8 lanes serve one cell; the automatic choice takes 8 on small grids and
fewer on large ones): stencils, a replayed phi combination, replayed exprb42
steps against the oracle, and batched == single bitwise for a few-lane
variant.  Level 7 covers the automatic choice for large grids."""
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


def rand_dir(n, seed):
    rng = np.random.default_rng(seed)
    return rng.standard_normal(4 * n) * np.r_[np.full(3 * n, 5.0), np.full(n, 50.0)]


@pytest.mark.parametrize("lanes", [1, 2, 4, 8])
@pytest.mark.parametrize("level", [2, 5])
def test_stencils_every_lane_count(X, lanes, level):
    mesh = get_mesh(level)
    s = O.SWE(mesh)
    ctx = X.Context(mesh, "cuda:0", lanes=lanes)
    u = F.initial_state("c2_l6_24x3600", level=level)
    v = rand_dir(s.n, level + lanes)
    say("lanes", lanes, "level", level)
    assert blocks_rel(to_np(ctx.rhs(u)), s.rhs(u), s.n) < TOL_STENCIL
    assert blocks_rel(to_np(ctx.jv(u, v)), s.jv(u, v), s.n) < TOL_STENCIL
    ctx.close()


@pytest.mark.parametrize("lanes", [1, 2, 4])
def test_phi_and_steps_every_lane_count(X, lanes):
    import torch
    level = 3
    mesh = get_mesh(level)
    s = O.SWE(mesh)
    ctx = X.Context(mesh, "cuda:0", lanes=lanes)
    u0 = F.initial_state("c1_exprb42_l4", level=level)
    say("lanes", lanes, "phi + exprb42 replay")
    # phi combination, replayed
    v = [None, s.rhs(u0) * 1800.0, None, rand_dir(s.n, 9) * 1e-3]
    sch = O.new_schedule()
    ref, _, _ = s.phi_combo(u0, 1800.0, v, [0.5, 1.0], O.opts(mode=O.RECORD, sched=sch))
    ctx.schedule_set(sch.as_array())
    ctx.schedule_mode(X.REPLAY)
    try:
        W = ctx.phi_combo(u0, 1800.0, v, [0.5, 1.0])
    finally:
        ctx.schedule_mode(X.FREE)
    for w, r in zip(W, ref):
        assert blocks_rel(to_np(w), r, s.n) < TOL
    # two exprb42 steps, replayed
    st = O.swe_stepper(s, "exprb42")
    sch = O.new_schedule()
    refs, ur = [], u0.copy()
    for _ in range(2):
        ur = st.step(ur, 1800.0, O.opts(mode=O.RECORD, sched=sch))
        refs.append(ur.copy())
    ctx.reset_history()
    ctx.schedule_set(sch.as_array())
    ctx.schedule_mode(X.REPLAY)
    u = torch.tensor(u0, dtype=torch.float64, device="cuda:0")
    prev = u0
    try:
        for r in refs:
            ctx.step("exprb42", u, 1800.0)
            g = to_np(u)
            assert blocks_rel(g, r, s.n) < TOL
            assert blocks_rel(g - prev, r - prev, s.n) < TOL
            prev = r
    finally:
        ctx.schedule_mode(X.FREE)
    ctx.close()


def test_batched_equals_single_with_two_lanes(X):
    import torch
    level, nm = 3, 3
    mesh = get_mesh(level)
    U, _ = F.ensemble_states(level, 1805021447, nm)
    dts = np.array([600.0, 2400.0, 3600.0])
    ctx = X.Context(mesh, "cuda:0", lanes=2)
    Ub = torch.tensor(U, device="cuda:0")
    ctx.reset_history()
    ctx.step_batch("exprb42", Ub, dts)
    got = Ub.cpu().numpy()
    for k in range(nm):
        ctx.reset_history()
        u = torch.tensor(U[k], device="cuda:0")
        ctx.step("exprb42", u, dts[k])
        assert np.array_equal(u.cpu().numpy(), got[k]), k
    ctx.close()


def test_level7_automatic_lanes(X):
    """Bar 1e-11 here (the parity bar of the method): the rounding of the
    fourth-order dissipation nu L(L x), a difference of differences, grows
    with the grid, and at level 7 reaches ~1e-12 of the block norms for
    two correct summation orders."""
    mesh = get_mesh(7)
    s = O.SWE(mesh)
    ctx = X.Context(mesh, "cuda:0")
    u = F.initial_state("c5_l7_adjoint")
    v = rand_dir(s.n, 77)
    say("level 7 automatic lanes")
    assert blocks_rel(to_np(ctx.rhs(u)), s.rhs(u), s.n) < TOL
    assert blocks_rel(to_np(ctx.jv(u, v)), s.jv(u, v), s.n) < TOL
    ctx.close()


@pytest.mark.parametrize("level", [4, 5])
def test_two_and_eight_lanes_bitwise(X, level):
    """Two and eight lanes per cell place the edge slots and output
    components so that the group sums add the same pairs, and accumulate
    without contraction: rhs, products and whole free-running steps agree
    bit for bit (eight lanes on these grids also form L x inside the
    product, two lanes use the separate Laplacian pass).  This is what lets
    ensemble batches take two lanes while single states take eight on grids
    without chunk tables (up to 16384 cells)."""
    import torch
    mesh = get_mesh(level)
    n = len(mesh["xyz"])
    u0 = F.initial_state("c2_l6_24x3600", level=level)
    v = rand_dir(n, 40 + level)
    res = {}
    for lanes in (2, 8):
        ctx = X.Context(mesh, "cuda:0", lanes=lanes)
        say("lanes", lanes, "level", level, "bitwise")
        out = [to_np(ctx.rhs(u0)), to_np(ctx.jv(u0, v))]
        u = torch.tensor(u0, dtype=torch.float64, device="cuda:0")
        ctx.reset_history()
        for _ in range(2):
            ctx.step("pexprb43", u, 3600.0)
        out.append(to_np(u))
        res[lanes] = out
        ctx.close()
    for a, b in zip(res[2], res[8]):
        assert np.array_equal(a, b)


def test_level6_lds_product_matches_eight_lanes(X):
    """Level 6 (40962 cells) carries chunk tables, so two lanes take the
    LDS-staged Laplacian and product, which form the edge weights from the
    chord by series and fuse their accumulations: their products agree with
    the eight-lane gather kernels to rounding, not bit for bit, and a
    batched two-lane step still equals the single one bit for bit."""
    import torch
    level = 6
    mesh = get_mesh(level)
    s = O.SWE(mesh)
    u0 = F.initial_state("c2_l6_24x3600", level=level)
    v = rand_dir(s.n, 46)
    ref = s.jv(u0, v)
    res = {}
    for lanes in (2, 8):
        ctx = X.Context(mesh, "cuda:0", lanes=lanes)
        say("lanes", lanes, "level 6 product")
        res[lanes] = to_np(ctx.jv(u0, v))
        assert blocks_rel(res[lanes], ref, s.n) < TOL_STENCIL
        ctx.close()
    assert blocks_rel(res[2], res[8], s.n, base=ref) < TOL_STENCIL
    nm = 3
    U, dts = F.ensemble_states(level, 1805021446, nm)
    ctx = X.Context(mesh, "cuda:0", lanes=2)
    say("level 6 two-lane batch vs single")
    Ub = torch.tensor(U, device="cuda:0")
    ctx.reset_history()
    ctx.step_batch("exprb42", Ub, dts)
    got = Ub.cpu().numpy()
    for k in range(nm):
        ctx.reset_history()
        u = torch.tensor(U[k], device="cuda:0")
        ctx.step("exprb42", u, dts[k])
        assert np.array_equal(u.cpu().numpy(), got[k]), k
    ctx.close()


def test_level7_batched_equals_single(X):
    """Level 7 (641 chunks) takes the chunked IOM2 update with one norm
    partial per block of a shared 512-block grid: the single state's update
    fused with the next Laplacian and the batch's chunked update must still
    give the same bits, step for step."""
    import torch
    level, nm = 7, 2
    mesh = get_mesh(level)
    U, dts = F.ensemble_states(level, 1805021447, nm)
    ctx = X.Context(mesh, "cuda:0", lanes=2)
    say("level 7 two-lane batch vs single")
    Ub = torch.tensor(U, device="cuda:0")
    ctx.reset_history()
    ctx.step_batch("exprb42", Ub, dts)
    got = Ub.cpu().numpy()
    for k in range(nm):
        ctx.reset_history()
        u = torch.tensor(U[k], device="cuda:0")
        ctx.step("exprb42", u, dts[k])
        assert np.array_equal(u.cpu().numpy(), got[k]), k
    ctx.close()
