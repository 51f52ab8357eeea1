"""Pins for the oracle's element integrals and dense system (Sec. 2, eqs. 6-9).

Element level: the Struve closed form against adaptive quadrature, the
Laplace limit of the self hypersingular term, the Maue identity against the
directly integrated hypersingular kernel, and kernel derivatives against
finite differences.  System level: the Mie series for one fibre in free space
(first-order convergence under refinement), vanishing scattered field without
contrast, block-size invariance of the periodic system and the flux balance
over the propagating Bragg orders.
"""
import math

import numpy as np
import pytest
from scipy.integrate import quad
from scipy.special import hankel1

import workloads as W
from analytic import mie_scattered
from oracle import elements as el
from oracle import fields as fl
from oracle import system as sy
from oracle.kernels import grad_x_phi, kernels_sdkt, phi


def test_int_h0_closed_form():
    for x in (1e-4, 0.01, 0.3, 2.0, 7.5):
        re = quad(lambda t: hankel1(0, t).real, 0, x, epsabs=1e-15, epsrel=1e-14, limit=200)[0]
        im = quad(lambda t: hankel1(0, t).imag, 0, x, epsabs=1e-15, epsrel=1e-14, limit=200)[0]
        assert abs(el.int_h0(x) - (re + 1j * im)) < 1e-12 * abs(re + 1j * im)


def test_self_T_laplace_limit():
    """kappa -> 0: the finite part of the Laplace hypersingular operator on a
    straight chord at its midpoint is -2/(pi h)."""
    h = 0.01
    _, _, _, T = el.self_terms(1e-7, np.array([h]))
    assert abs(T[0].real - (-2.0 / (math.pi * h))) < 1e-6 * 2.0 / (math.pi * h)


def test_self_T_is_limit_off_element():
    """T_self is the limit of the Maue form of T_e(x) as x approaches the midpoint."""
    kap, h = 3.0, 0.02
    a = np.array([-h / 2, 0.0])
    b = np.array([h / 2, 0.0])
    n_e = np.array([0.0, -1.0])           # tangent (1,0) -> normal (t_y, -t_x)
    nu = n_e
    vals = []
    for eps in (1e-3 * h, 5e-4 * h):
        x = np.array([0.0, 0.0]) + eps * nu
        # exact S_e(x) by quadrature, gradients at the chord ends in closed form
        Sre = quad(lambda s: phi(kap, x[0] - s, x[1]).real, -h / 2, h / 2, points=[0.0],
                   epsabs=1e-16, epsrel=1e-13, limit=400)[0]
        Sim = quad(lambda s: phi(kap, x[0] - s, x[1]).imag, -h / 2, h / 2, points=[0.0],
                   epsabs=1e-16, epsrel=1e-13, limit=400)[0]
        gb = np.array(grad_x_phi(kap, x[0] - b[0], x[1] - b[1]))
        ga = np.array(grad_x_phi(kap, x[0] - a[0], x[1] - a[1]))
        tau = np.array([-nu[1], nu[0]])
        vals.append(kap ** 2 * (Sre + 1j * Sim) - tau @ (gb - ga))
    ext = 2 * vals[1] - vals[0]            # linear extrapolation to eps = 0
    _, _, _, T = el.self_terms(kap, np.array([h]))
    assert abs(ext - T[0]) < 1e-5 * abs(T[0])


def test_maue_identity_vs_direct_hypersingular_integral():
    """Near pairs: integrating the T kernel equals the Maue form."""
    kap = 2.5
    wl = W.tiny()
    pb = sy.problem_from_workload(wl, 2.0, 0.3, periodic=False)
    bd = pb.bd
    for tgt, src in ((10, 11), (10, 12), (40, 38)):
        x, nu = bd.mid[tgt], bd.nrm[tgt]
        nr = el.near_rule([kap], x[None], nu[None], bd.mid[[src]], bd.tan[[src]], bd.nrm[[src]],
                          bd.h[[src]])
        S, T = nr[0, 0, 0], nr[0, 3, 0]
        gb = np.array(grad_x_phi(kap, *(x - bd.b_pt[src])))
        ga = np.array(grad_x_phi(kap, *(x - bd.a_pt[src])))
        tau = np.array([-nu[1], nu[0]])
        maue = kap ** 2 * (nu @ bd.nrm[src]) * S - tau @ (gb - ga)
        assert abs(maue - T) < 1e-11 * abs(T)


def test_kernel_derivatives_finite_difference():
    kap = 1.7
    x = np.array([0.3, -0.2])
    y = np.array([-0.1, 0.25])
    nu = np.array([0.6, 0.8])
    n = np.array([-0.28, 0.96])
    eps = 1e-5
    S, D, K, T = kernels_sdkt(kap, *(x - y), *nu, *n)
    s = lambda xx, yy: phi(kap, *(xx - yy))
    D_fd = (s(x, y + eps * n) - s(x, y - eps * n)) / (2 * eps)
    K_fd = (s(x + eps * nu, y) - s(x - eps * nu, y)) / (2 * eps)
    d = lambda xx: kernels_sdkt(kap, *(xx - y), *nu, *n)[1]
    T_fd = (d(x + eps * nu) - d(x - eps * nu)) / (2 * eps)
    assert abs(D - D_fd) < 1e-8 * abs(D)
    assert abs(K - K_fd) < 1e-8 * abs(K)
    assert abs(T - T_fd) < 1e-7 * abs(T)


def _mie_error(N):
    wl = W.tiny()
    wl.n_elem = N
    pb = sy.problem_from_workload(wl, 2.0, math.pi / 4, periodic=False)
    psi, _, _ = sy.solve(pb)
    c = pb.bd.centres[0]
    ang = np.linspace(0, 2 * np.pi, 13)[:-1]
    pts = c + 0.6 * np.stack([np.cos(ang), np.sin(ang)], 1)
    us = sy.potential(pb, psi, pts)
    um = mie_scattered(pb.k, pb.k1, 0.3, wl.rho_fiber, wl.rho_matrix, pb.theta, c, pts)
    return np.max(np.abs(us - um)) / np.max(np.abs(um))


def test_mie_series_first_order_convergence():
    e = [_mie_error(N) for N in (64, 128, 256)]
    assert e[2] < 8e-3
    for a, b in zip(e, e[1:]):
        assert 1.8 < a / b < 2.2


def test_no_contrast_no_scattering():
    wl = W.tiny()
    wl.n_elem = 128
    wl.rho_fiber, wl.c_fiber = wl.rho_matrix, wl.c_matrix
    pb = sy.problem_from_workload(wl, 2.0, math.pi / 4)
    psi, _, B = sy.solve(pb)
    n, kap, gam, R, T = fl.bragg(pb, psi, 3)
    prop = np.abs(gam.imag) < 1e-14
    assert np.max(np.abs(R[prop])) < 1e-5 and np.max(np.abs(T[prop])) < 1e-5


def test_block_size_invariance():
    """The same crystal solved with M_H = 1 and M_H = 2: the second row of
    fibres carries exactly alpha_a = exp(i k a sin theta) times the first."""
    ka, th = 2.0, 0.35
    w1 = W.small_square(1, 1, 64, 0.3, ka, th)
    w2 = W.small_square(1, 2, 64, 0.3, ka, th)
    p1 = sy.problem_from_workload(w1, ka, th)
    p2 = sy.problem_from_workload(w2, ka, th)
    s1, _, _ = sy.solve(p1)
    s2, _, _ = sy.solve(p2)
    n = 2 * 64
    aa = np.exp(1j * ka * math.sin(th))
    assert np.linalg.norm(s2[:n] - s1) < 1e-10 * np.linalg.norm(s1)
    assert np.linalg.norm(s2[n:] - aa * s1) < 1e-10 * np.linalg.norm(s1)


def test_energy_balance_converges():
    res = []
    for N in (64, 128):
        wl = W.tiny()
        wl.n_elem = N
        pb = sy.problem_from_workload(wl, 2.0, math.pi / 4)
        psi, _, _ = sy.solve(pb)
        res.append(abs(fl.energy_residual(pb, psi)))
    assert res[1] < 3e-3
    assert 1.7 < res[0] / res[1] < 2.3


def test_free_space_self_blocks_are_circulant():
    """A fibre is a circle cut into N equal chords; rotating by one chord maps
    element a to a + 1 together with its normal, quadrature points and self
    term, so without images every 2x2 block of a fibre's elements a, b
    depends only on (b - a) mod N (the symmetry behind the circulant self
    rows of the near field).  Two fibres of different radii in free space."""
    wl = W.small_square(2, 1, 32, radii=np.array([0.3, 0.22]))
    pb = sy.problem_from_workload(wl, 2.5, 0.4, periodic=False)
    A = sy.dense_matrix(pb)
    bd = pb.bd
    N = bd.N
    for f in range(bd.M):
        e = f * N + np.arange(N)
        rot = f * N + (np.arange(N) + 1) % N
        for rows in (sy.col_phi, sy.col_varphi):
            for cols in (sy.col_phi, sy.col_varphi):
                blk = A[np.ix_(rows(bd, e), cols(bd, e))]
                shifted = A[np.ix_(rows(bd, rot), cols(bd, rot))]
                assert np.max(np.abs(shifted - blk)) < 1e-11 * np.max(np.abs(blk))
    # with the images the diagonal blocks lose the symmetry: the periodic
    # system differs from the free-space one there
    Ap = sy.dense_matrix(sy.problem_from_workload(wl, 2.5, 0.4, periodic=True))
    e0 = np.arange(N)
    d = Ap[np.ix_(sy.col_phi(bd, e0), sy.col_phi(bd, e0))] - A[np.ix_(sy.col_phi(bd, e0), sy.col_phi(bd, e0))]
    assert np.max(np.abs(d[1:, 1:] - d[:-1, :-1])) > 1e-6


def test_fibre_self_blocks_are_the_free_space_diagonal():
    """The preconditioner blocks are the diagonal fibre blocks of the
    free-space system: for one fibre the whole free-space matrix, for two
    fibres the diagonal blocks of theirs (the cross-fibre blocks left out),
    the same at every angle, and different from the periodic system's
    diagonal blocks, which carry the images."""
    wl1 = W.small_square(1, 1, 32, r=0.3)
    pb1 = sy.problem_from_workload(wl1, 2.5, 0.4, periodic=False)
    blk1 = sy.fibre_self_blocks(sy.problem_from_workload(wl1, 2.5, 0.4))
    assert np.max(np.abs(blk1[0] - sy.dense_matrix(pb1))) == 0.0
    wl = W.small_square(2, 1, 32, radii=np.array([0.3, 0.22]))
    pb = sy.problem_from_workload(wl, 2.5, 0.4)
    blk = sy.fibre_self_blocks(pb)
    Af = sy.dense_matrix(sy.problem_from_workload(wl, 2.5, 0.4, periodic=False))
    Ap = sy.dense_matrix(pb)
    N = wl.n_elem
    for f in range(2):
        seg = slice(2 * f * N, 2 * f * N + 2 * N)
        assert np.max(np.abs(blk[f] - Af[seg, seg])) == 0.0
        assert np.max(np.abs(blk[f] - Ap[seg, seg])) > 1e-6
    assert np.max(np.abs(Af[0:2 * N, 2 * N:4 * N])) > 1e-3      # the left-out coupling is real
    blk_th = sy.fibre_self_blocks(sy.problem_from_workload(wl, 2.5, 1.1))
    assert np.max(np.abs(blk_th - blk)) == 0.0
    x = W.random_density(4 * N, 5)
    y = sy.precond_apply(pb, x, inverse=True, blocks=blk)
    assert np.linalg.norm(sy.precond_apply(pb, y, inverse=False, blocks=blk) - x) < 1e-12 * np.linalg.norm(x)


def test_fibre_self_block_is_diagonalised_by_the_dft():
    """Block-circulant structure, checked with numpy's FFT: with R(d) the 2x2
    block of element 0 with element d (identity removed) and
    L(kappa) = sum_d R(d) w^{kappa d}, w = exp(2 pi i / N), the block maps x
    to the inverse DFT of (I + L(kappa)) xhat(kappa)."""
    wl = W.small_square(1, 1, 32, r=0.35)
    pb = sy.problem_from_workload(wl, 3.0, 0.2)
    P = sy.fibre_self_blocks(pb)[0]
    N = wl.n_elem
    R = np.stack([[P[0, :N], P[0, N:]], [P[N, :N], P[N, N:]]])      # [2, 2, N] over source offset d
    R[0, 0, 0] -= 1.0
    R[1, 1, 0] -= 1.0
    L = np.fft.ifft(R, axis=-1) * N                                   # sum_d R(d) w^{+kappa d}
    x = W.random_density(2 * N, 9)
    xh = np.stack([np.fft.fft(x[:N]), np.fft.fft(x[N:])])
    yh = xh + np.einsum("ijk,jk->ik", L, xh)
    y = np.concatenate([np.fft.ifft(yh[0]), np.fft.ifft(yh[1])])
    assert np.linalg.norm(y - P @ x) < 1e-12 * np.linalg.norm(P @ x)
