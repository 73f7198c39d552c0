"""Pins of the oracle's adjoint (no GPU): the K operator against the
Jacobian-vector product, the adjoint of one phi-combination against the
exact gradient of the dense augmented-matrix definition (SciPy's Frechet
derivative of expm), and the exprb42 step and trajectory vector-Jacobian
products against central differences of the replayed forward."""
import numpy as np
import pytest
import scipy.linalg as sl

import oracle as O
from synth import fields as F
from synth.mesh import get_mesh


@pytest.fixture(scope="module")
def swe2():
    return O.SWE(get_mesh(2))


@pytest.mark.parametrize("level", [2, 3])
def test_ktv_matches_jacobian_difference(level):
    """<d, K(a, b)> = <a, (J(d) - J(0)) b>: K is the u-gradient of <a, J(u) b>."""
    s = O.SWE(get_mesh(level))
    rng = np.random.default_rng(level)
    for _ in range(3):
        a, b, d = (rng.standard_normal(s.N) for _ in range(3))
        lhs = d @ s.ktv(a, b)
        rhs = a @ (s.jv(d, b) - s.jv(np.zeros(s.N), b))
        assert abs(lhs - rhs) <= 1e-12 * (abs(rhs) + np.linalg.norm(a) * np.linalg.norm(b))


def test_ktv_is_bilinear_and_independent_of_state(swe2):
    s = swe2
    rng = np.random.default_rng(7)
    a, a2, b = (rng.standard_normal(s.N) for _ in range(3))
    k = s.ktv(a, b)
    assert np.allclose(s.ktv(2.0 * a + a2, b), 2.0 * k + s.ktv(a2, b), rtol=1e-12, atol=1e-12 * np.abs(k).max())
    # (J(u + e) - J(u))^T a = K(a, e) for any u: F is quadratic
    u = F.initial_state("c1_exprb42_l4", level=2)
    e = rng.standard_normal(s.N)
    lhs = s.jtv(u + e, a) - s.jtv(u, a)
    assert np.linalg.norm(lhs - s.ktv(a, e)) <= 1e-11 * np.linalg.norm(lhs)


def _aug(A, vs, p):
    n = A.shape[0]
    M = np.zeros((n + p, n + p))
    M[:n, :n] = A
    for j in range(1, p + 1):
        if vs[j] is not None:
            M[:n, n + p - j] = vs[j]
    for k in range(p - 1):
        M[n + k, n + k + 1] = 1.0
    x0 = np.zeros(n + p)
    if vs[0] is not None:
        x0[:n] = vs[0]
    x0[n + p - 1] = 1.0
    return M, x0


def _exact_vjp(A, vs, rho, wbars):
    """W_i = [I 0] expm(rho_i M) x0 (eq. 3.15 as a linear ODE in augmented
    form); its gradient through the Frechet derivative of expm, whose adjoint
    is the Frechet derivative at the transpose."""
    n = A.shape[0]
    p = len(vs) - 1
    M, x0 = _aug(A, vs, p)
    Ab = np.zeros((n, n))
    vb = [np.zeros(n) for _ in range(p + 1)]
    Ws = []
    for r, wb in zip(rho, wbars):
        E = sl.expm(r * M)
        Ws.append((E @ x0)[:n])
        Wb = np.zeros(n + p)
        Wb[:n] = wb
        _, L = sl.expm_frechet(r * M.T, np.outer(Wb, x0))
        Ab += r * L[:n, :n]
        for j in range(1, p + 1):
            vb[j] += r * L[:n, n + p - j]
        vb[0] += (E.T @ Wb)[:n]
    return Ws, vb, Ab


@pytest.mark.parametrize("case", [
    dict(n=30, p=1, rho=[0.75], v0=False, scale=0.6, tol=1e-13, bound=1e-12),
    dict(n=30, p=3, rho=[0.5, 1.0], v0=True, scale=0.6, tol=1e-13, bound=1e-12),
    dict(n=40, p=4, rho=[0.3, 0.9], v0=False, scale=1.0, tol=1e-13, bound=1e-12),
    dict(n=150, p=3, rho=[1.0], v0=False, scale=0.5, tol=1e-11, bound=1e-8),
])
def test_phi_adjoint_against_frechet(case):
    rng = np.random.default_rng(case["n"] + case["p"])
    n, p = case["n"], case["p"]
    A = rng.standard_normal((n, n)) * case["scale"] * (4.0 / np.sqrt(n))
    vs = [rng.standard_normal(n) if case["v0"] else None]
    vs += [rng.standard_normal(n) if (j % 2 == 1 or j == p) else None for j in range(1, p + 1)]
    wbars = [rng.standard_normal(n) for _ in case["rho"]]
    o = O.opts(tol=case["tol"], m_max=40)
    W, vb, Ab, fs, ast = O.phi_vjp_dense(A, vs, case["rho"], wbars, o)
    We, vbe, Abe = _exact_vjp(A, vs, case["rho"], wbars)
    for w, we in zip(W, We):
        assert np.linalg.norm(w - we) <= case["bound"] * np.linalg.norm(we)
    assert np.linalg.norm(Ab - Abe) <= case["bound"] * np.linalg.norm(Abe)
    for j in range(p + 1):
        assert np.linalg.norm(vb[j] - vbe[j]) <= case["bound"] * np.linalg.norm(vbe[j]), j
    assert ast["accepted"] == fs["accepted"]          # one adjoint substep per forward substep


def test_phi_adjoint_zero_inputs_and_zero_cotangent():
    """Zero forward inputs (no forward substeps): the adjoint still returns
    vbar_l = sum_i rho_i^l phi_l(rho_i A^T) Wbar_i, and no A-term (y = 0);
    a zero cotangent gives zero everything."""
    rng = np.random.default_rng(3)
    n, p = 25, 3
    A = rng.standard_normal((n, n)) * 0.5
    vs = [None, np.zeros(n), None, np.zeros(n)]
    wb = [rng.standard_normal(n)]
    W, vb, Ab, fs, ast = O.phi_vjp_dense(A, vs, [1.0], wb, O.opts(tol=1e-13))
    _, vbe, _ = _exact_vjp(A, vs, [1.0], wb)
    assert fs["accepted"] == 0 and not np.any(W[0]) and not np.any(Ab)
    for j in range(p + 1):
        assert np.linalg.norm(vb[j] - vbe[j]) <= 1e-12 * np.linalg.norm(vbe[j])
    vs = [None, rng.standard_normal(n), None, rng.standard_normal(n)]
    W, vb, Ab, fs, ast = O.phi_vjp_dense(A, vs, [1.0], [np.zeros(n)], O.opts(tol=1e-13))
    assert not np.any(Ab) and all(not np.any(v) for v in vb)


def _replay(arr, tol):
    return O.opts(tol=tol, mode=O.REPLAY, sched=O.schedule_from_array(arr))


@pytest.mark.parametrize("tol", [1e-10, 1e-12])
def test_step_vjp_against_central_differences(swe2, tol):
    s = swe2
    u0 = F.initial_state("c1_exprb42_l4", level=2)
    dt = 900.0
    sch = O.new_schedule()
    O.swe_stepper(s, "exprb42").step(u0, dt, O.opts(tol=tol, mode=O.RECORD, sched=sch))
    arr = sch.as_array()
    rng = np.random.default_rng(11)
    ubar = rng.standard_normal(s.N) * np.repeat([1.0, 1.0, 1.0, 1e-2], s.n)
    g, ast = s.step_vjp("exprb42", u0, dt, ubar, _replay(arr, tol))
    scal = np.repeat([np.sqrt(np.mean(u0[b * s.n:(b + 1) * s.n] ** 2)) for b in range(4)], s.n)

    def psi(u):
        return O.swe_stepper(s, "exprb42").step(u, dt, _replay(arr, tol))

    eps = 1e-5
    for _ in range(4):
        d = rng.standard_normal(s.N) * scal
        fd = ubar @ (psi(u0 + eps * d) - psi(u0 - eps * d)) / (2 * eps)
        assert abs(fd - g @ d) <= 1e-9 * abs(g @ d)


def test_trajectory_gradient_against_central_differences(swe2):
    s = swe2
    u0 = F.initial_state("c1_exprb42_l4", level=2)
    dt, steps = 1800.0, 3
    rng = np.random.default_rng(12)
    obs_step = rng.integers(1, steps + 1, 40)
    obs_cell = rng.choice(s.n, 40, replace=False)
    obs_val = u0[3 * s.n + obs_cell] + rng.normal(0.0, 5.0, 40)
    L, g, scheds = O.exprb42_loss_grad(s, u0, dt, steps, obs_step, obs_cell, obs_val, tol=1e-11)

    def loss(u):
        us = [u]
        for k in range(steps):
            us.append(O.swe_stepper(s, "exprb42").step(us[-1], dt, _replay(scheds[k], 1e-11)))
        r = np.array([us[k][3 * s.n + c] for k, c in zip(obs_step, obs_cell)]) - obs_val
        return 0.5 * r @ r

    assert abs(loss(u0) - L) <= 1e-12 * L
    scal = np.repeat([np.sqrt(np.mean(u0[b * s.n:(b + 1) * s.n] ** 2)) for b in range(4)], s.n)
    eps = 1e-6
    for _ in range(3):
        d = rng.standard_normal(s.N) * scal
        fd = (loss(u0 + eps * d) - loss(u0 - eps * d)) / (2 * eps)
        assert abs(fd - g @ d) <= 1e-7 * abs(g @ d)
