"""Pins of the oracle's phipm_simul_iom2 (Alg. 1) against the plain
definition W_i = sum_l rho_i^l phi_l(rho_i A) v_l = y(rho_i) of eq. 3.15,
evaluated independently as a dense exponential of the augmented matrix
[[A, (v_p, ..., v_1)], [0, N_p]] (scipy.linalg.expm), plus exact special
cases, the zero-skip counts of Sec. 4.3 and record/replay determinism."""
import math

import numpy as np
import pytest
import scipy.linalg as sl

import oracle as O
from synth import fields as F
from synth.mesh import get_mesh


def dense_combo(A, vs, rho):
    """y(rho) of y' = A y + sum_j t^(j-1)/(j-1)! v_j, y(0) = v_0."""
    n = A.shape[0]
    p = len(vs) - 1
    if p == 0:
        return [sl.expm(r * A) @ vs[0] for r in rho]
    Ah = np.zeros((n + p, n + p))
    Ah[:n, :n] = A
    for j in range(1, p + 1):
        if vs[j] is not None:
            Ah[:n, n + p - j] = vs[j]
    for k in range(p - 1):
        Ah[n + k, n + k + 1] = 1.0
    x0 = np.zeros(n + p)
    if vs[0] is not None:
        x0[:n] = vs[0]
    x0[n + p - 1] = 1.0
    return [(sl.expm(r * Ah) @ x0)[:n] for r in rho]


def rel(a, b):
    return np.linalg.norm(a - b) / np.linalg.norm(b)


def test_zero_matrix_is_polynomial():
    n = 6
    rng = np.random.default_rng(0)
    vs = [rng.standard_normal(n) for _ in range(5)]
    rho = [0.25, 0.6, 1.0]
    W, st, _ = O.phi_combo_dense(np.zeros((n, n)), vs, rho)
    for r, w in zip(rho, W):
        ref = sum(r ** l * vs[l] / math.factorial(l) for l in range(5))
        assert np.allclose(w, ref, rtol=1e-14, atol=1e-15)


def test_scalar_matrix_phi_functions():
    for z in (-4.0, -0.5, 2.0):
        vs = [np.array([1.5]), np.array([-0.5]), None, np.array([2.0])]
        rho = [0.3, 1.0]
        W, _, _ = O.phi_combo_dense(np.array([[z]]), vs, rho, O.opts(tol=1e-14))
        for r, w in zip(rho, W):
            ph = math.exp(r * z)
            phis = [ph]
            for j in range(3):
                ph = (ph - 1.0 / math.factorial(j)) / (r * z)
                phis.append(ph)
            ref = 1.5 * phis[0] - 0.5 * r * phis[1] + 2.0 * r ** 3 * phis[3]
            assert abs(w[0] - ref) <= 1e-12 * abs(ref)


def test_zero_input_gives_exact_zero():
    A = np.random.default_rng(1).standard_normal((5, 5))
    W, st, _ = O.phi_combo_dense(A, [None, np.zeros(5), None], [0.5, 1.0])
    assert all(np.all(w == 0.0) for w in W) and st["attempts"] == 0


@pytest.fixture(scope="module")
def swe162():
    m = get_mesh(2)
    s = O.SWE(m)
    u = F.initial_state("c1_exprb42_l4", level=2)
    return s, u


@pytest.mark.parametrize("p", [1, 2, 3, 4])
def test_dense_check_162_cells(swe162, p):
    s, u = swe162
    dt = 900.0
    A = dt * s.dense_jacobian(u)
    rng = np.random.default_rng(10 + p)
    scale = np.r_[np.full(3 * s.n, 1.0), np.full(s.n, 10.0)]
    vs = [None] + [rng.standard_normal(s.N) * scale for _ in range(p)]
    if p >= 2:
        vs[1] = None
    rho = [0.5, 0.9]
    W, st, _ = s.phi_combo(u, dt, vs, rho, O.opts(tol=1e-10))
    ref = dense_combo(A, vs, rho)
    for w, r in zip(W, ref):
        assert rel(w, r) < 1e-9
    assert st["rejected"] >= 1  # cold start at m = 1 has to grow


def test_dense_check_large_norm_substeps(swe162):
    s, u = swe162
    dt = 14400.0
    A = dt * s.dense_jacobian(u)
    rng = np.random.default_rng(3)
    vs = [rng.standard_normal(s.N), rng.standard_normal(s.N), None, rng.standard_normal(s.N)]
    rho = [0.75, 1.0]
    W, st, _ = s.phi_combo(u, dt, vs, rho, O.opts(tol=1e-10, m_max=8))
    ref = dense_combo(A, vs, rho)
    for w, r in zip(W, ref):
        assert rel(w, r) < 1e-9
    assert st["accepted"] > 3  # several substeps


def test_skew_symmetric_matrix():
    rng = np.random.default_rng(5)
    n = 60
    S = rng.standard_normal((n, n))
    S = 3.0 * (S - S.T) / np.linalg.norm(S - S.T, 2)
    vs = [rng.standard_normal(n), rng.standard_normal(n)]
    W, _, _ = O.phi_combo_dense(S, vs, [1.0], O.opts(tol=1e-12, m_max=20))
    assert rel(W[0], dense_combo(S, vs, [1.0])[0]) < 1e-10


def test_zero_skip_counts_and_invariance(swe162):
    s, u = swe162
    dt = 900.0
    rng = np.random.default_rng(4)
    v1 = rng.standard_normal(s.N)
    v3 = 1e-2 * rng.standard_normal(s.N)
    # exprb42 call (ii) shape: p = 3, v_0 = v_2 = 0
    W, st, _ = s.phi_combo(u, dt, [None, v1, None, v3], [1.0])
    assert st["rec_matvecs"] == 2 + 3 * (st["accepted"] - 1)
    # an explicit zero v_0 disables the skip but not the result
    W2, st2, _ = s.phi_combo(u, dt, [np.zeros(s.N), v1, None, v3], [1.0])
    assert st2["rec_matvecs"] == 3 * st2["accepted"]
    assert np.array_equal(W[0], W2[0])
    # pexprb43 call (ii) shape: p = 4, only v_3, v_4
    v4 = rng.standard_normal(s.N)
    W, st, _ = s.phi_combo(u, dt, [None, None, None, v3, v4], [1.0])
    assert st["rec_matvecs"] == 1 + 4 * (st["accepted"] - 1)


def test_record_replay_bitwise(swe162):
    s, u = swe162
    dt = 3600.0
    rng = np.random.default_rng(6)
    vs = [None, rng.standard_normal(s.N), None, rng.standard_normal(s.N)]
    sch = O.new_schedule()
    W, st, _ = s.phi_combo(u, dt, vs, [0.5, 1.0], O.opts(mode=O.RECORD, sched=sch))
    arr = sch.as_array()
    assert len(arr) == st["attempts"]
    assert int((arr[:, 2].astype(int) & 1).sum()) == st["accepted"]
    rep = O.schedule_from_array(arr)
    W2, st2, _ = s.phi_combo(u, dt, vs, [0.5, 1.0], O.opts(mode=O.REPLAY, sched=rep))
    assert rep.pos == len(arr)
    for a, b in zip(W, W2):
        assert np.array_equal(a, b)


def test_nan_input_is_reported():
    v = np.ones(4)
    v[2] = np.nan
    with pytest.raises(RuntimeError):
        O.phi_combo_dense(np.eye(4), [None, v], [1.0])
