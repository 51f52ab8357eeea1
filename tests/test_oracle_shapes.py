"""Pins of the oracle for the round-square scatterer of Sec. 4.

* The curve: its polygon area converges at second order to the area the
  paper states, 23 pi r^2 / 2, and the farthest point is 4 r from the centre
  (on the diagonals).
* The whole system with non-circular chords: no scattered field without
  contrast, block-size invariance (M_H = 1 against M_H = 2) and the flux
  balance over the propagating Bragg orders converging under refinement.
"""
import math

import numpy as np

import workloads as W
from oracle import fields as fl
from oracle import system as sy
from oracle.geometry import ROUND_SQUARE, boundary_curve


def _round_square(M_L, M_H, N, r, ka, th):
    wl = W.small_square(M_L, M_H, N, r, ka, th)
    wl.shape = W.ROUND_SQUARE
    return wl


def test_round_square_area_and_reach():
    errs = []
    for N in (256, 1024):
        t = 2 * np.pi * np.arange(N) / N
        p = boundary_curve(ROUND_SQUARE, 0.07, t)
        x, y = p[:, 0], p[:, 1]
        area = 0.5 * np.sum(x * np.roll(y, -1) - np.roll(x, -1) * y)
        errs.append(abs(area / (23 * math.pi * 0.07 ** 2 / 2) - 1))
        assert abs(np.max(np.hypot(x, y)) - 4 * 0.07) < 1e-15
    assert errs[1] < 1e-5 and 14 < errs[0] / errs[1] < 18       # second order


def test_round_square_no_contrast_no_scattering():
    wl = _round_square(1, 1, 128, 0.07, 2.0, 0.4)
    wl.rho_fiber, wl.c_fiber = wl.rho_matrix, wl.c_matrix
    pb = sy.problem_from_workload(wl, 2.0, 0.4)
    psi, _, _ = sy.solve(pb)
    n, kap, gam, R, T = fl.bragg(pb, psi, 3)
    prop = np.abs(gam.imag) < 1e-14
    assert np.max(np.abs(R[prop])) < 1e-5 and np.max(np.abs(T[prop])) < 1e-5


def test_round_square_block_size_invariance():
    ka, th = 2.5, 0.35
    p1 = sy.problem_from_workload(_round_square(1, 1, 64, 0.07, ka, th), ka, th)
    p2 = sy.problem_from_workload(_round_square(1, 2, 64, 0.07, ka, th), ka, th)
    s1, _, _ = sy.solve(p1)
    s2, _, _ = sy.solve(p2)
    n = 2 * 64
    aa = np.exp(1j * ka * math.sin(th))
    assert np.linalg.norm(s2[:n] - s1) < 1e-10 * np.linalg.norm(s1)
    assert np.linalg.norm(s2[n:] - aa * s1) < 1e-10 * np.linalg.norm(s1)


def test_round_square_energy_balance_converges():
    res = []
    for N in (64, 128):
        pb = sy.problem_from_workload(_round_square(1, 1, N, 0.08, 3.0, 0.3), 3.0, 0.3)
        psi, _, _ = sy.solve(pb)
        res.append(abs(fl.energy_residual(pb, psi)))
    assert res[1] < 5e-3
    assert 1.6 < res[0] / res[1] < 2.4
