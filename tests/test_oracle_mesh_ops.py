"""Pins of the oracle's grid, discrete operators, F(u) and J(u)v against
mathematics that does not depend on the oracle's own code (Sec. 2).

* grid: Euler characteristic, 12 pentagons, total area 4 pi a^2;
* operators: exact continuous results (gradient of a linear function,
  Laplacian eigenfunctions, Stokes vorticity of solid-body rotation, a
  divergence-free field) converge with grid level;
* F: rest state is a fixed point bitwise, mass is conserved, the balanced
  solid-body flow (an exact steady solution of the continuous equations) is
  steady up to a residual that shrinks with the grid;
* J: F is exactly quadratic, so a central difference of F equals J v for any
  step (checks every block of eqs. dynja-dynjc, including the row-2 signs of
  J_r); the transpose passes the dot test.
"""
import numpy as np
import pytest

import oracle as O
from synth import fields as F
from synth.mesh import get_mesh, n_cells

A = 6.371e6


@pytest.mark.parametrize("level", [0, 1, 2, 3, 4])
def test_grid_topology(level):
    m = get_mesh(level)
    N = n_cells(level)
    assert len(m["xyz"]) == N
    assert int((m["deg"] == 5).sum()) == 12
    E = int(m["deg"].sum()) // 2
    Fc = len(m["tri"])
    assert N - E + Fc == 2
    nb, dg = m["nbr"], m["deg"]
    for i in range(0, N, max(1, N // 200)):
        for s in range(dg[i]):
            j = nb[i, s]
            assert i in nb[j, :dg[j]]


def _reverse_slots(m):
    nb, dg = m["nbr"], m["deg"]
    rev = np.full(nb.shape, -1)
    for i in range(len(nb)):
        for s in range(dg[i]):
            j = nb[i, s]
            rev[i, s] = list(nb[j, :dg[j]]).index(i)
    return rev


@pytest.mark.parametrize("level", [2, 4])
def test_geometry_area_and_antisymmetry(level):
    m = get_mesh(level)
    s = O.SWE(m)
    assert abs(s.area.sum() / (4 * np.pi * A * A) - 1.0) < 1e-12
    L, D, Nn = s.edge_len(), s.edge_dist(), s.edge_nrm()
    rev = _reverse_slots(m)
    nb, dg = m["nbr"], m["deg"]
    for i in range(len(nb)):
        for k in range(dg[i]):
            j, kk = nb[i, k], rev[i, k]
            assert L[i, k] == L[j, kk]
            assert D[i, k] == D[j, kk]
            assert np.all(Nn[i, k] == -Nn[j, kk])
    # normals are unit and tangent at the edge midpoint direction
    x = m["xyz"]
    for i in range(0, len(nb), 7):
        for k in range(dg[i]):
            rm = x[i] + x[nb[i, k]]
            assert abs(np.dot(Nn[i, k], rm)) < 1e-14
            assert abs(np.linalg.norm(Nn[i, k]) - 1) < 1e-15


def _op_errors(level):
    m = get_mesh(level)
    s = O.SWE(m, gamma_h=0.0)
    x = m["xyz"]
    g = np.array([0.3, -0.5, 0.8])
    G = s.grad(A * (x @ g))
    ex = g - (x @ g)[:, None] * x
    e_grad = np.sqrt(((G - ex) ** 2).sum(1).mean() / (ex ** 2).sum(1).mean())
    Y = F.sh_eval({(3, 2): 1.0}, x, 3)
    e_lap = np.sqrt(((s.lap(Y) + 12.0 / A ** 2 * Y) ** 2).mean() / ((12.0 / A ** 2 * Y) ** 2).mean())
    w = np.array([1e-5, -2e-5, 3e-5])
    u = np.cross(w, A * x)
    z = s.curl(u[:, 0], u[:, 1], u[:, 2])
    e_curl = np.sqrt(((z - 2 * (x @ w)) ** 2).mean()) / np.linalg.norm(2 * w)
    d = s.div(u[:, 0], u[:, 1], u[:, 2])
    e_div = np.sqrt((d ** 2).mean()) / (np.abs(u).max() / A)
    return np.array([e_grad, e_lap, e_curl, e_div])


def test_operators_converge():
    errs = np.array([_op_errors(l) for l in (3, 4, 5)])
    # every operator converges at least at first order, and is accurate at L5
    assert np.all(errs[1] < 0.6 * errs[0])
    assert np.all(errs[2] < 0.6 * errs[1])
    assert np.all(errs[2] < 5e-3)


@pytest.mark.parametrize("level", [2, 4])
def test_rest_state_bitwise_fixed_point(level):
    m = get_mesh(level)
    s = O.SWE(m)
    n = s.n
    rest = np.concatenate([np.zeros(3 * n), np.full(n, 5123.25)])
    f = s.rhs(rest)
    assert np.all(f == 0.0)
    assert np.all(s.rhs(np.zeros(4 * n)) == 0.0)


@pytest.mark.parametrize("level", [2, 4])
def test_mass_conservation_of_rhs(level):
    m = get_mesh(level)
    s = O.SWE(m)
    n = s.n
    u = F.initial_state("c1_exprb42_l4", level=level)
    hdot = s.rhs(u)[3 * n:]
    a = s.area
    assert abs(np.dot(a, hdot)) <= 1e-14 * np.dot(a, np.abs(hdot))


def test_balanced_solid_body_is_steady_in_the_limit():
    res = []
    for level in (3, 4, 5):
        m = get_mesh(level)
        s = O.SWE(m, gamma_h=0.0)
        x = m["xyz"]
        n = len(x)
        vel, h = F.solid_body(x, 38.6, 5000.0)
        f = s.rhs(F.pack(vel, h))
        fu = f[:3 * n].reshape(3, n).T
        res.append([np.sqrt((fu ** 2).sum(1).mean()) / (7.292e-5 * 38.6),
                    np.sqrt((f[3 * n:] ** 2).mean()) / (38.6 * 1906.0 / A)])
    res = np.array(res)
    assert np.all(res[1] < 0.6 * res[0]) and np.all(res[2] < 0.6 * res[1])
    assert np.all(res[2] < 5e-3)


@pytest.mark.parametrize("level", [2, 3])
def test_jv_is_exact_central_difference(level):
    m = get_mesh(level)
    s = O.SWE(m)
    n = s.n
    u = F.initial_state("c1_exprb42_l4", level=level)
    rng = np.random.default_rng(level)
    v = rng.standard_normal(4 * n) * np.r_[np.full(3 * n, 10.0), np.full(n, 100.0)]
    jv = s.jv(u, v)
    for eps in (0.5, 1.0, 4.0):
        fd = (s.rhs(u + eps * v) - s.rhs(u - eps * v)) / (2 * eps)
        for b in range(4):
            sl = slice(b * n, (b + 1) * n)
            assert np.linalg.norm(fd[sl] - jv[sl]) <= 1e-12 * np.linalg.norm(jv[sl])


def test_jtv_dot_test():
    m = get_mesh(3)
    s = O.SWE(m)
    u = F.initial_state("c1_exprb42_l4", level=3)
    rng = np.random.default_rng(7)
    for _ in range(3):
        a = rng.standard_normal(s.N)
        b = rng.standard_normal(s.N)
        lhs = a @ s.jv(u, b)
        rhs = s.jtv(u, a) @ b
        assert abs(lhs - rhs) <= 1e-13 * (np.abs(a) @ np.abs(s.jv(u, np.abs(b))) + abs(lhs))


def test_dense_jacobian_transpose():
    m = get_mesh(1)
    s = O.SWE(m)
    u = F.initial_state("c1_exprb42_l4", level=1)
    J = s.dense_jacobian(u)
    JT = np.empty_like(J)
    e = np.zeros(s.N)
    for k in range(s.N):
        e[k] = 1.0
        JT[:, k] = s.jtv(u, e)
        e[k] = 0.0
    assert np.abs(JT - J.T).max() <= 1e-13 * np.abs(J).max()
