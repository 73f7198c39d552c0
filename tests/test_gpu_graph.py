"""The batched ensemble step captured as one HIP graph (replay mode): the
host walks the members' recorded schedules without waiting for decisions,
the stream is captured, and every launch of the graph must give the bits
of the eager replayed batched step -- which equal the free-running batched
step whose decisions were recorded.  The graph is launched several times,
with eager work and synchronisations between launches, and every launch is
checked.  Also: capture is refused outside replay mode."""
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


@pytest.mark.parametrize("level,method", [(4, "exprb42"), (5, "exprb53"), (4, "epi3")])
def test_captured_batched_step_is_bitwise(X, level, method):
    import torch
    nm = 6
    mesh = get_mesh(level)
    U, dts = F.ensemble_states(level, 1805021443, nm)
    say("graph: level %d, %s, %d members, dt %s" % (level, method, nm, list(dts)))
    ctx = X.Context(mesh, "cuda:0")
    # free run, recording every member's decisions
    ctx.reset_history()
    ctx.schedule_mode(X.RECORD)
    Uf = torch.tensor(U, device="cuda:0")
    ctx.step_batch(method, Uf, dts)
    ctx.schedule_mode(X.FREE)
    free = Uf.cpu().numpy()
    scheds = [ctx.schedule_get_member(k) for k in range(nm)]
    say("  attempts per member", [len(s) for s in scheds])

    def load_schedules():
        for k in range(nm):
            ctx.schedule_set_member(k, scheds[k])

    # eager replay
    ctx.reset_history()
    load_schedules()
    ctx.schedule_mode(X.REPLAY)
    Ue = torch.tensor(U, device="cuda:0")
    ctx.step_batch(method, Ue, dts)
    eager = Ue.cpu().numpy()
    assert np.array_equal(eager, free)
    # captured
    ctx.reset_history()
    load_schedules()
    Ug = torch.tensor(U, device="cuda:0")
    ctx.step_batch_capture(method, Ug, dts)
    ctx.schedule_mode(X.FREE)
    assert np.array_equal(Ug.cpu().numpy(), U), "capture must not run the step"
    U0 = torch.tensor(U, device="cuda:0")
    for rep in range(3):
        Ug.copy_(U0)
        torch.cuda.synchronize()
        ctx.graph_launch()
        got = Ug.cpu().numpy()
        ndiff = int(np.sum(got != eager))
        say("  launch %d: %d values differ from the eager replay" % (rep, ndiff))
        assert ndiff == 0
        # eager work between launches
        x = torch.tensor(U[0], device="cuda:0")
        ctx.rhs(x)
        torch.cuda.synchronize()
    ctx.close()


def test_capture_needs_replay_mode(X):
    import torch
    level, nm = 3, 2
    mesh = get_mesh(level)
    U, dts = F.ensemble_states(level, 7, nm)
    ctx = X.Context(mesh, "cuda:0")
    Ug = torch.tensor(U, device="cuda:0")
    with pytest.raises(X.ExprbError):
        ctx.step_batch_capture("exprb42", Ug, dts)
    with pytest.raises(X.ExprbError):
        lib = X.lib()
        ctx._check(lib.xrb_graph_launch(ctx.h))
    ctx.close()
