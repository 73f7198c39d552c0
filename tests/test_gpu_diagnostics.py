"""GPU conserved-quantity diagnostics (mass, total energy, potential
enstrophy; Sec. 6 conservation paragraph) through the C-ABI: parity with the
oracle, and the paper's conservation behaviour reproduced on the level-6
grid -- mass to rounding and energy and potential enstrophy within 0.1 %
over 15 days of pexprb43 with 4.8 h steps."""
import sys

import numpy as np
import pytest

import oracle as O
from synth import fields as F
from synth.mesh import get_mesh

pytestmark = pytest.mark.gpu


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


@pytest.mark.parametrize("level", [4, 6])
def test_diagnostics_parity(X, level):
    mesh = get_mesh(level)
    ctx = X.Context(mesh, "cuda:0")
    s = O.SWE(mesh)
    u = F.initial_state("c2_l6_24x3600", level=level)
    say("diagnostics parity level", level)
    got, ref = ctx.diagnostics(u), s.diagnostics(u)
    for k in ref:
        assert abs(got[k] / ref[k] - 1) < 1e-12, (k, got[k], ref[k])
    assert ctx.diagnostics(u) == got     # fixed summation order
    ctx.close()


def test_level6_fifteen_days_conservation(X):
    import torch
    mesh = get_mesh(6)
    ctx = X.Context(mesh, "cuda:0")
    u = torch.tensor(F.initial_state("c2_l6_24x3600"), dtype=torch.float64, device="cuda:0")
    d0 = ctx.diagnostics(u)
    ctx.reset_history()
    say("level 6: 75 pexprb43 steps of 4.8 h")
    for _ in range(75):
        ctx.step("pexprb43", u, 4.8 * 3600.0)
    d = ctx.diagnostics(u)
    rel = {k: d[k] / d0[k] - 1 for k in d}
    say("normalised conservation errors", rel)
    assert abs(rel["mass"]) < 1e-12
    assert abs(rel["energy"]) < 1e-3 and abs(rel["enstrophy"]) < 1e-3
    ctx.close()
