"""Pins of the two oracle parts that the dense checks cannot reach.

* eq. cost (Sec. 4.3): the work estimate C(tau, m) the step-size / Krylov-size
  controller compares.  Checked against values worked out by hand from the
  printed formula, with cases chosen so that the plausible slips fail: the
  nearest-integer bracket rounding half away from zero (2.5 -> 3, where
  half-even or floor give 2), the substep count floored at 1, the log2 term
  clamped at 0 (a negative log2 would lower the price), the log2 term rounded
  to the nearest integer (log2 3 -> 2, where floor gives 1), and every
  additive term present.
* eq. niu with eq. swdis: the hyperdissipation D_f = -nu L^2 with
  nu = gamma_h dxbar^4 / dt_e, dxbar^2 = 4 pi a^2 / N.  At a resting ocean
  the depth row of J is D_f alone, and spherical harmonics are eigenfunctions
  of the continuous Laplacian (L Y_lm = -l(l+1)/a^2 Y_lm), so
  (J v)_h = -nu (l(l+1)/a^2)^2 Y_lm up to the grid's discretisation error,
  which must fall at second order with the level.  A wrong power of dxbar,
  a wrong dt_e or gamma_h, a wrong sign or a single L instead of L^2 fails.
"""
import numpy as np
import pytest

import oracle as O
from synth import fields as F
from synth.mesh import get_mesh

A = 6.371e6


@pytest.mark.parametrize("args, expected", [
    # tau, m, p, t_out - t, n, ||tau Hhat||_1
    # nint(2.5/1) = 3 substeps: 3*5*(100 + 4000) = 61500; 2(p-1)(n_A + n) = 8200;
    # M = 44/3 + 2*nint(log2(8)) = 62/3, (m+p+1)^3 = 512 -> 31744/3; (2p+1) n = 500
    ((1.0, 5, 2, 2.5, 100.0, 42.96), 61500.0 + 8200.0 + 31744.0 / 3.0 + 500.0),
    # the same with ||tau Hhat|| = 1: log2(1/5.37) < 0 is clamped, M = 44/3 -> 22528/3
    ((1.0, 5, 2, 2.5, 100.0, 1.0), 61500.0 + 8200.0 + 22528.0 / 3.0 + 500.0),
    # nint(0.3) = 0 substeps floored at 1: 1*10*4100 = 41000; p = 1: no recurrence term;
    # log2(16.11/5.37) = log2 3 -> 2, M = 56/3, (12)^3 = 1728 -> 32256; (2p+1) n = 300
    ((1.0, 10, 1, 0.3, 100.0, 16.11), 41000.0 + 0.0 + 32256.0 + 300.0),
    # level-6 size: n = 163848, n_A = 6553920; nint(1/0.3) = 3 substeps of m = 40:
    # 3*40*6717768 = 806132160; 2*3*6717768 = 40306608; log2(171.84/5.37) = 5 ->
    # M = 74/3, 45^3 = 91125 -> 2247750; 9 n = 1474632
    ((0.3, 40, 4, 1.0, 163848.0, 171.84), 806132160.0 + 40306608.0 + 2247750.0 + 1474632.0),
])
def test_cost_hand_values(args, expected):
    got = O.phi_cost(*args)
    assert got == pytest.approx(expected, rel=1e-14, abs=0.0)


def test_cost_is_increasing_in_work():
    # more substeps, a larger Krylov size or a larger ||tau Hhat|| never cost less
    base = O.phi_cost(0.5, 8, 3, 1.0, 1000.0, 40.0)
    assert O.phi_cost(0.25, 8, 3, 1.0, 1000.0, 40.0) > base
    assert O.phi_cost(0.5, 9, 3, 1.0, 1000.0, 40.0) > base
    assert O.phi_cost(0.5, 8, 3, 1.0, 1000.0, 4 * 40.0) > base


def _dissipation_error(level, l, mm, gamma_h=4e-4, dt_e=240.0):
    m = get_mesh(level)
    s = O.SWE(m, gamma_h=gamma_h, dt_e=dt_e)
    n = s.n
    area = s.area
    Y = F.sh_eval({(l, mm): 1.0}, m["xyz"], l)
    rest = np.concatenate([np.zeros(3 * n), np.full(n, 5000.0)])
    v = np.concatenate([np.zeros(3 * n), Y])
    jh = s.jv(rest, v)[3 * n:]
    got = (area * Y) @ jh / ((area * Y) @ Y)
    nu = gamma_h * (4.0 * np.pi * A * A / n) ** 2 / dt_e      # eq. niu
    lam = -nu * (l * (l + 1) / A ** 2) ** 2                   # D_f = -nu L^2 on Y_lm
    return got / lam - 1.0


@pytest.mark.parametrize("l, mm", [(2, 1), (4, 3)])
def test_hyperdissipation_eigenvalue(l, mm):
    errs = np.array([_dissipation_error(level, l, mm) for level in (3, 4, 5)])
    # second-order convergence of the grid's L^2 on smooth eigenfunctions
    assert np.all(np.abs(errs[1:]) < 0.3 * np.abs(errs[:-1]))
    assert abs(errs[-1]) < 5e-3


def test_hyperdissipation_scales_with_its_constants():
    # gamma_h and dt_e enter nu as gamma_h / dt_e: the same eigenvalue error
    e0 = _dissipation_error(4, 2, 1)
    e1 = _dissipation_error(4, 2, 1, gamma_h=1.25e-2, dt_e=600.0)
    assert abs(e0 - e1) < 1e-12
