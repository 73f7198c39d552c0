"""Pins of the oracle's Pade-13 scaling-and-squaring exponential: closed
forms, an independent library routine (scipy.linalg.expm), and the
augmented-matrix identity that Alg. 1 relies on (columns of
exp(tau [[H, e_1 e_1^T], [0, N]]) are tau^k phi_k(tau H) e_1)."""
import math

import numpy as np
import pytest
import scipy.linalg as sl

import oracle as O


def test_rotation_closed_form():
    for th in (0.1, 1.0, 3.0, 25.0):
        X, _ = O.expm(np.array([[0.0, th], [-th, 0.0]]))
        ref = np.array([[math.cos(th), math.sin(th)], [-math.sin(th), math.cos(th)]])
        assert np.abs(X - ref).max() < 1e-13 * max(1.0, th)


def test_nilpotent_and_diagonal():
    K = 7
    N = np.diag(np.ones(K - 1), 1)
    X, _ = O.expm(2.0 * N)
    ref = sum(np.linalg.matrix_power(2.0 * N, k) / math.factorial(k) for k in range(K))
    assert np.abs(X - ref).max() < 1e-13 * np.abs(ref).max()
    d = np.array([-30.0, -1.0, 0.0, 0.5, 2.0])
    X, s = O.expm(np.diag(d))
    assert s > 0
    assert np.allclose(np.diag(X), np.exp(d), rtol=1e-13, atol=0)


@pytest.mark.parametrize("K,scale", [(5, 1e-3), (12, 0.5), (20, 4.0), (45, 10.0), (45, 60.0)])
def test_against_scipy(K, scale):
    rng = np.random.default_rng(K)
    A = rng.standard_normal((K, K))
    A = scale * A / np.abs(A).sum(0).max()
    X, _ = O.expm(A)
    ref = sl.expm(A)
    assert np.linalg.norm(X - ref) <= 1e-12 * np.linalg.norm(ref) * max(1.0, scale)


def _phi_scalar(k, z):
    """phi_k(z) by eq. 3.7's recursion from phi_0 = e^z (|z| not tiny)."""
    ph = math.exp(z)
    for j in range(k):
        ph = (ph - 1.0 / math.factorial(j)) / z
    return ph


def test_augmented_matrix_gives_phi_columns():
    # 1x1 "Hessenberg" H = [z], p = 4: column k of the upper-right block is
    # tau^k phi_k(tau z)
    p = 4
    for z in (-3.0, -0.7, 1.3):
        for tau in (0.5, 1.0):
            K = 1 + p + 1
            Hh = np.zeros((K, K))
            Hh[0, 0] = z
            Hh[0, 1] = 1.0
            for k in range(p):
                Hh[1 + k, 2 + k] = 1.0
            X, _ = O.expm(tau * Hh)
            for k in range(1, p + 2):
                ref = tau ** k * _phi_scalar(k, tau * z)
                assert abs(X[0, k] - ref) <= 1e-12 * abs(ref)
