"""The launch-shape autotuner (xrb_autotune): it times every candidate on
the context's grid; the lanes pair it keeps preserves bitwise equality of
batched members with single runs, and the block shapes it picks change no
result bit -- checked by running steps before and after tuning."""
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
    U, dts = F.ensemble_states(level, 1805021443, nm)
    # before tuning: the built-in shapes (two lanes on this grid)
    u0 = torch.tensor(U[0], device="cuda:0")
    ctx.reset_history()
    ctx.step("exprb42", u0, dts[0])
    before = u0.cpu().numpy()
    r = ctx.autotune(nm)
    say("autotune level 6", r)
    assert all(t > 0 for t in r["single_us"].values()) and all(t > 0 for t in r["batch_us"].values())
    a, b = r["lanes"], r["lanes_batch"]
    assert a in (1, 2, 4, 8) and b in (1, 2, 4, 8)
    # this grid carries chunk tables: two lanes take the LDS-staged kernels,
    # so only equal lane counts keep batched members equal to single runs
    assert a == b
    if a == 2:   # LDS-staged product (fixed block), LDS Laplacian over a tuned grid
        assert r["jv_block"] == 0 and r["jv_block_batch"] == 0
        assert r["lap_grid"] in (0, 512, 1024, 2048)
    else:
        assert set(r["jv_threads_single_us"]) and all(t > 0 for t in r["jv_threads_single_us"].values())
        assert r["jv_block"] in [0] + list(r["jv_threads_single_us"])
        assert r["lap_block"] in (0, 64, 128, 256)
    Ub = torch.tensor(U, device="cuda:0")
    ctx.reset_history()
    ctx.step_batch("exprb42", Ub, dts)
    got = Ub.cpu().numpy()
    for k in (0, nm - 1):
        ctx.reset_history()
        u = torch.tensor(U[k], device="cuda:0")
        ctx.step("exprb42", u, dts[k])
        assert np.array_equal(u.cpu().numpy(), got[k]), k
    # the tuned block and grid shapes give the bits of the built-in ones
    if a == 2:
        assert np.array_equal(got[0], before)
    else:
        assert np.max(np.abs(got[0] - before)) <= 1e-10 * np.max(np.abs(before))
    ctx.close()


def test_autotune_large_grid_keeps_one_lane_count(X):
    """Above 65536 cells the reducing products accumulate per lane, so only
    equal lane counts keep batched runs bitwise equal to single ones."""
    import torch
    mesh = get_mesh(7)
    ctx = X.Context(mesh, "cuda:0")
    u0 = F.initial_state("c1_exprb42_l4", level=7)
    u = torch.tensor(u0, device="cuda:0")
    ctx.step("exprb42", u, 900.0)
    before = u.cpu().numpy()
    r = ctx.autotune(2)
    say("autotune level 7", r)
    assert r["lanes"] == r["lanes_batch"]
    if r["lanes"] == 2:   # the LDS-staged kernels: their grid shapes change no bit
        assert r["lap_grid"] in (0, 512, 1024, 2048)
        u = torch.tensor(u0, device="cuda:0")
        ctx.reset_history()
        ctx.step("exprb42", u, 900.0)
        assert np.array_equal(u.cpu().numpy(), before)
    ctx.close()
