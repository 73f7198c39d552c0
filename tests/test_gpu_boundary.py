"""The C-ABI boundary: vectors cross it in the paper's component-major layout
[u_x | u_y | u_z | h] at any 8-byte alignment (the library converts them into
its own cell-major, 16-byte aligned buffers) with the same bits as aligned
ones.  Also the argument checks of the phi-combination entry point that the
conversion relies on (distinct outputs)."""
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


def to_np(t):
    import torch
    torch.cuda.synchronize()
    return t.cpu().numpy()


def shifted(a):
    """A contiguous device copy of a that starts 8 bytes past a 16-byte boundary."""
    import torch
    buf = torch.zeros(len(a) + 1, dtype=torch.float64, device="cuda:0")
    assert buf.data_ptr() % 16 == 0
    buf[1:] = torch.as_tensor(a, dtype=torch.float64, device="cuda:0")
    v = buf[1:]
    assert v.is_contiguous() and v.data_ptr() % 16 == 8
    return v


def test_unaligned_vectors_give_the_same_bits(X):
    import torch
    level = 4
    mesh = get_mesh(level)
    n = len(mesh["xyz"])
    ctx = X.Context(mesh, "cuda:0")
    u0 = F.initial_state("c1_exprb42_l4", level=level)
    rng = np.random.default_rng(12)
    v = rng.standard_normal(4 * n) * np.r_[np.full(3 * n, 5.0), np.full(n, 50.0)]
    say("boundary: aligned vs 8-byte shifted vectors, level", level)
    ref = [to_np(ctx.rhs(u0)), to_np(ctx.jv(u0, v))]
    ref += [to_np(w) for w in ctx.phi_combo(u0, 900.0, [None, v * 1e-3], [0.5, 1.0])]
    got = [to_np(ctx.rhs(shifted(u0))), to_np(ctx.jv(shifted(u0), shifted(v)))]
    got += [to_np(w) for w in ctx.phi_combo(shifted(u0), 900.0, [None, shifted(v * 1e-3)],
                                            [0.5, 1.0])]
    for a, b in zip(ref, got):
        assert np.array_equal(a, b)
    # in/out state of a step
    ua = torch.tensor(u0, device="cuda:0")
    ctx.reset_history()
    ctx.step("exprb42", ua, 900.0)
    us = shifted(u0)
    ctx.reset_history()
    ctx.step("exprb42", us, 900.0)
    assert np.array_equal(to_np(ua), to_np(us))
    ctx.close()


def test_phi_combo_rejects_aliased_outputs(X):
    import torch
    level = 2
    mesh = get_mesh(level)
    n = len(mesh["xyz"])
    ctx = X.Context(mesh, "cuda:0")
    lib = X.lib()
    import ctypes as C
    u = torch.tensor(F.initial_state("c1_exprb42_l4", level=level), device="cuda:0")
    v = torch.ones(4 * n, dtype=torch.float64, device="cuda:0")
    out = torch.empty(4 * n, dtype=torch.float64, device="cuda:0")
    va = (C.c_void_p * 2)(None, v.data_ptr())
    oa = (C.c_void_p * 2)(out.data_ptr(), out.data_ptr())
    rho = np.array([0.5, 1.0])
    rc = lib.xrb_phi_combo(ctx.h, C.c_double(600.0), C.c_void_p(u.data_ptr()), 1, va, 2,
                           rho.ctypes.data_as(C.POINTER(C.c_double)), oa, None)
    assert rc == -1   # XRB_EINVAL
    ctx.close()


def test_mesh_info_and_latched_errors(X):
    """xrb_mesh_info returns the grid the context was made from (centres as
    given, areas summing to the sphere's); a device-side failure (a NaN
    input met by a norm) is returned by the call and again, once, by the
    next xrb_sync."""
    import ctypes as C
    level = 3
    mesh = get_mesh(level)
    ctx = X.Context(mesh, "cuda:0")
    n, xyz, area = ctx.mesh_info()
    assert n == len(mesh["xyz"])
    assert np.array_equal(xyz, np.asarray(mesh["xyz"], dtype=np.float64))
    a = 6.371e6
    assert abs(area.sum() / (4 * np.pi * a * a) - 1.0) < 1e-12 and np.all(area > 0)
    lib = X.lib()
    assert lib.xrb_sync(ctx.h) == 0
    u = F.initial_state("c1_exprb42_l4", level=level)
    bad = np.ones(4 * n)
    bad[3] = np.nan
    with pytest.raises(X.ExprbError):
        ctx.phi_combo(u, 600.0, [None, bad], [1.0])
    assert lib.xrb_sync(ctx.h) == -5      # XRB_ENAN, latched
    assert lib.xrb_sync(ctx.h) == 0       # and cleared
    ctx.sync()
    n2 = C.c_int64()
    assert lib.xrb_mesh_info(ctx.h, C.byref(n2), None, None) == 0 and n2.value == n
    ctx.close()
