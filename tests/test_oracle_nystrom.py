"""Pins for the oracle's spectral Nystrom discretisation (oracle/nystrom.py).

Quadrature level: the logarithmic weights integrate ln(4 sin^2) times
trigonometric polynomials exactly (closed form), the differentiation matrix
differentiates them exactly.  Operator level: on a circle every layer
operator is diagonal in the Fourier modes with eigenvalues in closed form
from Graf's addition theorem (the Nystrom S, D, K, T against them).  System
level: the Mie series for one fibre (spectral convergence), block-size
invariance of the periodic system, the flux balance, and the multiple
scattering solution of the same array of circles; the round square of
Sec. 4 by its own convergence and the flux balance.
"""
import math

import numpy as np
import pytest
from scipy.special import hankel1, h1vp, jv, jvp

import workloads as W
from analytic import mie_scattered, mst_periodic
from oracle import fields as fl
from oracle import lattice as la
from oracle import nystrom as ny
from oracle import system as sy


@pytest.mark.parametrize("N", [8, 16, 32])
def test_log_weights_integrate_trig_polynomials(N):
    """int_0^{2 pi} ln(4 sin^2((t - tau)/2)) e^{i m tau} dtau = -(2 pi/|m|) e^{i m t}
    (m != 0), 0 (m = 0), exactly for |m| < N/2."""
    tj = 2 * np.pi * np.arange(N) / N
    for t in (0.0, 0.37, 2.9):
        w = ny.kress_weights(N, t - tj)
        for m in range(-(N // 2) + 1, N // 2):
            got = np.sum(w * np.exp(1j * m * tj))
            ref = 0.0 if m == 0 else -(2 * np.pi / abs(m)) * np.exp(1j * m * t)
            assert abs(got - ref) < 1e-12, (N, t, m, got, ref)
        # and cos(N tau / 2), the one Nyquist function the nodes see
        got = np.sum(w * np.cos(0.5 * N * tj))
        assert abs(got + (4 * np.pi / N) * np.cos(0.5 * N * t)) < 1e-12


def test_differentiation_matrix():
    N = 32
    t = 2 * np.pi * np.arange(N) / N
    D = ny.diff_matrix(N)
    for m in (1, 3, 15):
        assert np.max(np.abs(D @ np.sin(m * t) - m * np.cos(m * t))) < 1e-12 * m
    assert np.max(np.abs(D @ np.cos(16 * t))) < 1e-12        # the Nyquist mode has no derivative


@pytest.mark.parametrize("kappa", [0.7, 2.1, 6.0])
def test_circle_layer_operators_match_their_eigenvalues(kappa):
    """Circle of radius a: by Graf's theorem H0(k|x - y|) = sum_m J_m(ka) H_m(ka) e^{i m (t - tau)},
    so S e^{i m t} = (i pi a/2) J_m H_m, D and K (principal values: the mean of
    the two one-sided derivatives) (i pi k a/4)(J_m H_m' + J_m' H_m), and
    T = (i pi k^2 a/2) J_m' H_m' times e^{i m t}."""
    a, N = 0.3, 64
    wl = W.tiny()
    wl.radii = np.array([a])
    wl.n_elem = N
    bd = ny.discretise(wl.lattice, wl.a, 1, 1, N, wl.radii)
    S, D, K, T = ny.self_matrices(bd, 0, kappa)
    t = 2 * np.pi * np.arange(N) / N
    z = kappa * a
    for m in (0, 1, 4, 9, 15):
        v = np.exp(1j * m * t)
        J, Jp, Hm, Hp = jv(m, z), jvp(m, z), hankel1(m, z), h1vp(m, z)
        lam = {"S": 0.5j * np.pi * a * J * Hm,
               "D": 0.25j * np.pi * kappa * a * (J * Hp + Jp * Hm),
               "K": 0.25j * np.pi * kappa * a * (J * Hp + Jp * Hm),
               "T": 0.5j * np.pi * kappa ** 2 * a * Jp * Hp}
        for name, Mx in (("S", S), ("D", D), ("K", K), ("T", T)):
            got = Mx @ v
            err = np.max(np.abs(got - lam[name] * v)) / max(abs(lam[name]), 1e-3)
            assert err < 1e-10, (name, m, err)


def _mie_error(N):
    wl = W.tiny()
    wl.n_elem = N
    pb = ny.problem_from_workload(wl, 2.0, math.pi / 4, periodic=False)
    A = ny.dense_matrix(pb)
    psi = np.linalg.solve(A, sy.rhs(pb))
    c = pb.bd.centres[0]
    ang = np.linspace(0, 2 * np.pi, 13)[:-1]
    pts = c + 0.6 * np.stack([np.cos(ang), np.sin(ang)], 1)
    us = ny.potential(pb, psi, pts)
    um = mie_scattered(pb.k, pb.k1, 0.3, wl.rho_fiber, wl.rho_matrix, pb.theta, c, pts)
    return np.max(np.abs(us - um)) / np.max(np.abs(um))


def test_mie_series_spectral_convergence():
    """One fibre in free space: the error falls faster than any power of N
    (the element discretisation: first order)."""
    e = [_mie_error(N) for N in (16, 32, 64)]
    assert e[2] < 1e-11
    assert e[0] / e[1] > 100 and e[1] / e[2] > 100


def test_block_size_invariance():
    ka, th = 2.0, 0.35
    p1 = ny.problem_from_workload(W.small_square(1, 1, 32, 0.3, ka, th), ka, th)
    p2 = ny.problem_from_workload(W.small_square(1, 2, 32, 0.3, ka, th), ka, th)
    s1 = np.linalg.solve(ny.dense_matrix(p1), sy.rhs(p1))
    s2 = np.linalg.solve(ny.dense_matrix(p2), sy.rhs(p2))
    n = 2 * 32
    aa = np.exp(1j * ka * math.sin(th))
    assert np.linalg.norm(s2[:n] - s1) < 1e-10 * np.linalg.norm(s1)
    assert np.linalg.norm(s2[n:] - aa * s1) < 1e-10 * np.linalg.norm(s1)


@pytest.mark.parametrize("case", ["one_fibre", "two_fibres"])
def test_periodic_system_matches_multiple_scattering(case):
    """Bragg amplitudes of the periodic Nystrom system against the multiple
    scattering solution of the same array of circles (spectral in both)."""
    if case == "one_fibre":
        wl, ka, th = W.tiny(), 2.0, math.pi / 4
    else:
        wl, ka, th = W.small_square(2, 1, 64, radii=np.array([0.3, 0.22])), 4.0, 0.7
    errs = []
    for N in (16, 32):
        wl.n_elem = N
        pb = ny.problem_from_workload(wl, ka, th)
        psi = np.linalg.solve(ny.dense_matrix(pb), sy.rhs(pb))
        _, _, gam, R, T = fl.bragg(pb, psi, 3, G=1)
        ls = lambda ox, oy, nu, ex: la.lattice_sum_orders(pb.k, pb.bd.H, th, ox, oy, nu, exclude=ex)
        _, Rm, Tm, _ = mst_periodic(pb.k, pb.k1, wl.rho_fiber, wl.rho_matrix, th, pb.bd.H,
                                    pb.bd.centres, wl.radii, 16, ls)
        prop = np.abs(gam.imag) < 1e-14
        errs.append(max(np.max(np.abs(R - Rm)[prop]), np.max(np.abs(T - Tm)[prop])))
        assert abs(fl.energy_residual(pb, psi)) < (1e-5 if N == 16 else 1e-11)
    # spectral: from 16 to 32 nodes per fibre the error drops to rounding
    assert errs[1] < 1e-11, errs
    assert errs[0] / errs[1] > 1e3, errs


def test_round_square_converges():
    """The round square of Sec. 4 (no closed form): Bragg amplitudes at N = 64
    and 128 agree far beyond the element method, and the flux balances."""
    wl = W.bandgap_block("round_square_square", 0.35, n_elem=64, M_L=1, M_H=1)
    ka, th = 2.0, 0.3
    amps = []
    for N in (64, 128):
        wl.n_elem = N
        pb = ny.problem_from_workload(wl, ka, th)
        psi = np.linalg.solve(ny.dense_matrix(pb), sy.rhs(pb))
        _, _, gam, R, T = fl.bragg(pb, psi, 3, G=1)
        amps.append(np.concatenate([R, T]))
        assert abs(fl.energy_residual(pb, psi)) < 1e-6
    assert np.max(np.abs(amps[0] - amps[1])) < 1e-7
