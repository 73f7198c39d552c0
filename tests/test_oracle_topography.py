"""Pins of the oracle's surface topography h_s (the h_s in the energy
E = |u|^2/2 + g (h + h_s) of eq. sweqsinv):
  * a zero h_s reproduces the flat model bit for bit;
  * h_s enters F only through the energy gradient: F with h_s minus F
    without is -g G(h_s) in the velocity and zero in the depth;
  * a lake at rest (u = 0, h + h_s constant) is steady without dissipation;
  * over a mountain the inviscid total energy sum A (h|u|^2/2 + g h^2/2 +
    g h h_s) is kept to 1e-7 over five days, while the same sum without the
    g h h_s term is not (so the diagnostic's terrain term is pinned too),
    and mass is conserved to rounding."""
import numpy as np

import oracle as O
from synth import fields as F
from synth.mesh import get_mesh


def test_zero_topography_is_flat_bitwise():
    mesh = get_mesh(3)
    s = O.SWE(mesh)
    u = F.mountain_flow_state(3, 7)
    f0 = s.rhs(u)
    s.set_topography(np.zeros(s.n))
    assert np.array_equal(s.rhs(u), f0)


def test_topography_enters_through_the_energy_gradient_only():
    mesh = get_mesh(4)
    s = O.SWE(mesh)
    n = s.n
    u = F.mountain_flow_state(4, 7)
    hs = F.mountain(4, 7)
    f0 = s.rhs(u)
    s.set_topography(hs)
    f1 = s.rhs(u)
    gx, gy, gz = s.grad(hs).T
    d = f1 - f0
    scale = 9.80616 * max(np.abs(gx).max(), np.abs(gy).max(), np.abs(gz).max())
    for b, gb in enumerate((gx, gy, gz)):
        assert np.abs(d[b * n:(b + 1) * n] + 9.80616 * gb).max() < 1e-10 * scale
    assert np.array_equal(f1[3 * n:], f0[3 * n:])


def test_lake_at_rest_is_steady():
    mesh = get_mesh(4)
    s = O.SWE(mesh, gamma_h=0.0)
    n = s.n
    hs = F.mountain(4, 7)
    s.set_topography(hs)
    lake = np.zeros(4 * n)
    lake[3 * n:] = 5000.0 - hs
    assert np.abs(s.rhs(lake)).max() < 1e-14


def test_energy_with_terrain_term_conserved_over_a_mountain():
    level = 3
    mesh = get_mesh(level)
    s = O.SWE(mesh, gamma_h=0.0)
    n = s.n
    hs = F.mountain(level, 7)
    s.set_topography(hs)
    area = np.asarray(s.area)
    u = F.mountain_flow_state(level, 7)
    d0 = s.diagnostics(u)
    st = O.swe_stepper(s, "pexprb43")
    for _ in range(25):
        u = st.step(u, 4.8 * 3600.0)
    d = s.diagnostics(u)
    assert abs(d["mass"] / d0["mass"] - 1) < 1e-13
    assert abs(d["energy"] / d0["energy"] - 1) < 1e-7
    # without the terrain term the sum is not an invariant
    u0 = F.mountain_flow_state(level, 7)
    t0 = d0["energy"] - 9.80616 * np.sum(area * u0[3 * n:] * hs)
    t1 = d["energy"] - 9.80616 * np.sum(area * u[3 * n:] * hs)
    assert abs(t1 / t0 - 1) > 1e-5
