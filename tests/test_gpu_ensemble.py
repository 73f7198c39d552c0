"""Batched ensemble (many members, each its own step size, Krylov sizes and
substeps, in one batched sequence of launches) against (a) the same members
stepped one at a time through xrb_step -- bitwise, since both run the same
kernels with the same reduction order -- and (b) the CPU oracle at 1e-11."""
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


def blocks_rel(got, ref, n, base=None):
    base = ref if base is None else base
    out = []
    for b in range(4):
        sl = slice(b * n, (b + 1) * n)
        den = np.linalg.norm(base[sl])
        out.append(np.linalg.norm(got[sl] - ref[sl]) / den if den > 0 else np.linalg.norm(got[sl]))
    return max(out)


def members(level, nm, seed=1805021443):
    mesh = get_mesh(level)
    U, dts = F.ensemble_states(level, seed, nm)
    return mesh, U, dts


@pytest.mark.parametrize("method", ["exprb42", "exprb53", "epi3"])
def test_batched_equals_single_bitwise(X, method):
    import torch
    level, nm = 3, 4
    mesh, U, dts = members(level, nm)
    dts = np.array([600.0, 1200.0, 2400.0, 3600.0])
    say("ensemble bitwise", method)
    ctx = X.Context(mesh, "cuda:0")
    Ub = torch.tensor(U, device="cuda:0")
    ctx.reset_history()
    for _ in range(2):
        ctx.step_batch(method, Ub, dts)
    got = Ub.cpu().numpy()
    for k in range(nm):
        ctx.reset_history()
        u = torch.tensor(U[k], device="cuda:0")
        for _ in range(2):
            ctx.step(method, u, dts[k])
        assert np.array_equal(u.cpu().numpy(), got[k]), k
    ctx.close()


def test_batched_matches_oracle(X):
    import torch
    level, nm = 4, 3
    mesh, U, dts = members(level, nm)
    dts = np.array([600.0, 2400.0, 3600.0])
    say("ensemble vs oracle")
    ctx = X.Context(mesh, "cuda:0")
    Ub = torch.tensor(U, device="cuda:0")
    ctx.reset_history()
    ctx.step_batch("exprb42", Ub, dts)
    got = Ub.cpu().numpy()
    s = O.SWE(mesh)
    n = s.n
    for k in range(nm):
        ref = O.swe_stepper(s, "exprb42").step(U[k], dts[k])
        assert blocks_rel(got[k], ref, n) < TOL
        assert blocks_rel(got[k] - U[k], ref - U[k], n) < TOL
    ctx.close()


def test_c4_level6_members_bitwise(X):
    """C4 shape: level-6 members with step sizes from {600, 1200, 2400, 3600} s
    (8 of the 64 members here), batched == single, first member vs oracle."""
    import torch
    level, nm = 6, 8
    mesh, U, dts = members(level, nm)
    say("C4 members", dts)
    ctx = X.Context(mesh, "cuda:0")
    Ub = torch.tensor(U, device="cuda:0")
    ctx.reset_history()
    _, st = ctx.step_batch("exprb42", Ub, dts, return_stats=True)
    got = Ub.cpu().numpy()
    for k in (0, nm - 1):
        ctx.reset_history()
        u = torch.tensor(U[k], device="cuda:0")
        ctx.step("exprb42", u, dts[k])
        assert np.array_equal(u.cpu().numpy(), got[k])
    s = O.SWE(mesh)
    ref = O.swe_stepper(s, "exprb42").step(U[0], dts[0])
    assert blocks_rel(got[0] - U[0], ref - U[0], s.n) < TOL
    assert len(st) == nm and all(c[0]["accepted"] >= 1 for c in st)
    ctx.close()


def test_c4_six_launches(X):
    """C4 parity run: all 64 level-6 members through 6 batched launches
    (one exprb42 step each, step sizes from {600, 1200, 2400, 3600} s);
    the first and last members equal 6 single-state steps bit for bit, and
    the first member matches the oracle's free-running 6 steps at 1e-11 on
    the increment per block."""
    import torch
    level, nm = 6, 64
    mesh, U, dts = members(level, nm)
    say("C4 six launches, 64 members")
    ctx = X.Context(mesh, "cuda:0")
    Ub = torch.tensor(U, device="cuda:0")
    ctx.reset_history()
    for _ in range(6):
        ctx.step_batch("exprb42", Ub, dts)
    got = Ub.cpu().numpy()
    for k in (0, nm - 1):
        ctx.reset_history()
        u = torch.tensor(U[k], device="cuda:0")
        for _ in range(6):
            ctx.step("exprb42", u, dts[k])
        assert np.array_equal(u.cpu().numpy(), got[k]), k
    ctx.close()
    s = O.SWE(mesh)
    st = O.swe_stepper(s, "exprb42")
    ref = U[0].copy()
    for _ in range(6):
        ref = st.step(ref, dts[0])
    assert blocks_rel(got[0] - U[0], ref - U[0], s.n) < TOL


def test_batch_with_a_resting_member_bitwise(X):
    """A member whose inputs are all zero (a resting ocean: F = 0, so every
    phi-combination input vanishes) takes the zero-output path of a batched
    call while the others iterate; its outputs must be exact zeros, not the
    previous step's values left in its buffers.  Step 1 runs three perturbed
    members, then member 1 is replaced by a resting ocean for step 2; each
    member must equal the same sequence of single-state steps bitwise."""
    import torch
    level, nm = 4, 3
    mesh, U, dts = members(level, nm)
    n = len(mesh["xyz"])
    dts = np.array([1200.0, 2400.0, 3600.0])
    rest = np.concatenate([np.zeros(3 * n), np.full(n, 5000.0)])
    say("ensemble with a resting member")
    ctx = X.Context(mesh, "cuda:0")
    Ub = torch.tensor(U, device="cuda:0")
    ctx.reset_history()
    ctx.step_batch("exprb42", Ub, dts)
    Ub[1] = torch.as_tensor(rest, device="cuda:0")
    ctx.step_batch("exprb42", Ub, dts)
    got = Ub.cpu().numpy()
    assert np.array_equal(got[1], rest)
    for k in range(nm):
        ctx.reset_history()
        u = torch.tensor(U[k], device="cuda:0")
        ctx.step("exprb42", u, dts[k])
        if k == 1:
            u.copy_(torch.as_tensor(rest, device="cuda:0"))
        ctx.step("exprb42", u, dts[k])
        assert np.array_equal(u.cpu().numpy(), got[k]), k
    ctx.close()
