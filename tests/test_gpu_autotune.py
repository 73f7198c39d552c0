"""The lanes-per-cell autotuner (xrb_autotune): it times every candidate on
the context's grid, and the pair it keeps preserves bitwise equality of
batched members with single runs -- checked by running both after tuning."""
import sys

import numpy as np
import pytest

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


def test_autotune_level6_keeps_batched_equal_to_single(X):
    import torch
    level, nm = 6, 8
    mesh = get_mesh(level)
    ctx = X.Context(mesh, "cuda:0")
    r = ctx.autotune(nm)
    say("autotune level 6", r)
    assert all(t > 0 for t in r["single_us"].values()) and all(t > 0 for t in r["batch_us"].values())
    a, b = r["lanes"], r["lanes_batch"]
    assert a in (1, 2, 4, 8) and b in (1, 2, 4, 8)
    assert a == b or {a, b} <= {2, 8}
    U, dts = F.ensemble_states(level, 1805021443, nm)
    Ub = torch.tensor(U, device="cuda:0")
    ctx.reset_history()
    ctx.step_batch("exprb42", Ub, dts)
    got = Ub.cpu().numpy()
    for k in (0, nm - 1):
        ctx.reset_history()
        u = torch.tensor(U[k], device="cuda:0")
        ctx.step("exprb42", u, dts[k])
        assert np.array_equal(u.cpu().numpy(), got[k]), k
    ctx.close()


def test_autotune_large_grid_keeps_one_lane_count(X):
    """Above 65536 cells the reducing products accumulate per lane, so only
    equal lane counts keep batched runs bitwise equal to single ones."""
    mesh = get_mesh(7)
    ctx = X.Context(mesh, "cuda:0")
    r = ctx.autotune(2)
    say("autotune level 7", r)
    assert r["lanes"] == r["lanes_batch"]
    ctx.close()
