"""The allocation-free Jacobian product xrb_jv_static, called through the
C-ABI: the same bits as xrb_jv on the same context, on consecutive calls
that share the library's static device scratch -- a level-6 grid (separate
Laplacian pass, two lanes per cell), then a smaller level-3 grid (the
product forms L v itself, eight lanes), then the level-6 grid again -- and
within the stencil bar of the oracle's J(u) v (eqs. dynjs-dynjc)."""
import ctypes as C
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


def blocks_rel(got, ref, n):
    out = []
    for b in range(4):
        sl = slice(b * n, (b + 1) * n)
        out.append(np.linalg.norm(got[sl] - ref[sl]) / np.linalg.norm(ref[sl]))
    return max(out)


def case(level, seed):
    mesh = get_mesh(level)
    n = len(mesh["xyz"])
    u0 = F.initial_state("c1_exprb42_l4", level=level)
    rng = np.random.default_rng(seed)
    v = rng.standard_normal(4 * n) * np.r_[np.full(3 * n, 5.0), np.full(n, 50.0)]
    return mesh, n, u0, v


def test_static_product_matches_the_allocating_one(X):
    import torch
    L = X.lib()
    ctxs = {}
    for level, seed in ((6, 61), (3, 31), (6, 62)):
        mesh, n, u0, v = case(level, seed)
        if level not in ctxs:
            ctxs[level] = X.Context(mesh, "cuda:0")
        ctx = ctxs[level]
        say("jv_static: level %d (%d cells), seed %d" % (level, n, seed))
        u = torch.tensor(u0, dtype=torch.float64, device="cuda:0")
        vv = torch.tensor(v, dtype=torch.float64, device="cuda:0")
        ref = torch.empty(4 * n, dtype=torch.float64, device="cuda:0")
        got = torch.full((4 * n,), float("nan"), dtype=torch.float64, device="cuda:0")
        ctx._stream()
        assert L.xrb_jv(ctx.h, C.c_void_p(u.data_ptr()), C.c_void_p(vv.data_ptr()),
                        C.c_void_p(ref.data_ptr())) == X.OK
        assert L.xrb_jv_static(ctx.h, C.c_void_p(u.data_ptr()), C.c_void_p(vv.data_ptr()),
                               C.c_void_p(got.data_ptr())) == X.OK
        assert L.xrb_sync(ctx.h) == X.OK
        g, r = got.cpu().numpy(), ref.cpu().numpy()
        assert np.array_equal(g, r), "level %d: %d values differ" % (level, int(np.sum(g != r)))
        orc = O.SWE(mesh).jv(u0, v)
        e = blocks_rel(g, orc, n)
        say("  bitwise equal to xrb_jv; oracle %.2e" % e)
        assert e < 1e-12
    for c in ctxs.values():
        c.close()


def test_static_product_rejects_bad_pointers(X):
    import torch
    L = X.lib()
    mesh, n, u0, v = case(3, 5)
    ctx = X.Context(mesh, "cuda:0")
    u = torch.tensor(u0, dtype=torch.float64, device="cuda:0")
    ctx._stream()
    assert L.xrb_jv_static(ctx.h, C.c_void_p(u.data_ptr()), C.c_void_p(u.data_ptr()),
                           C.c_void_p(u.data_ptr())) == X.EINVAL
    assert L.xrb_jv_static(ctx.h, None, C.c_void_p(u.data_ptr()),
                           C.c_void_p(u.data_ptr())) == X.EINVAL
    ctx.close()
