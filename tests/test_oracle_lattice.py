"""Pins for the oracle's quasi-periodic image sums (Sec. 3.3, eqs. 17-18).

Each check compares against something other than the oracle's own formula:
the spectral (Rayleigh) series, the exact identity between tails of
different cut-offs, the adaptive rule, quasi-periodicity, and Graf's
addition theorem (eq. 10) for the higher-order lattice sums.
"""
import math

import numpy as np
import pytest
from scipy.special import hankel1, jv

from analytic import spectral_h0_sum
from oracle import lattice as lt
from oracle.kernels import kernels_sdkt

CASES = [  # k, H, theta
    (2.0, 1.0, math.pi / 4),
    (0.7, 2.0, 0.3),
    (5.0, 1.0, 0.0),
    (3.1, 4.0, -0.4),
]


def _direct_h0(k, H, beta, X, Y, q, deriv):
    out = 0.0
    for m in range(-q, q + 1):
        Ym = Y - m * H
        r = np.hypot(X, Ym)
        if deriv == (0, 0):
            f = hankel1(0, k * r)
        elif deriv == (1, 0):
            f = -k * hankel1(1, k * r) * X / r
        else:
            f = -k * hankel1(1, k * r) * Ym / r
        out = out + np.exp(1j * m * beta) * f
    return out


@pytest.mark.parametrize("k,H,theta", CASES)
@pytest.mark.parametrize("deriv", [(0, 0), (1, 0), (0, 1)])
def test_tails_match_spectral_series(k, H, theta, deriv):
    rng = np.random.default_rng(1)
    beta = k * H * math.sin(theta)
    X = rng.uniform(0.1, 0.9, 12) * H * rng.choice([-1, 1], 12)
    Y = rng.uniform(-0.9, 0.9, 12) * H
    q = lt.choose_q(k, H, float(np.max(np.abs(X))), float(np.max(np.abs(Y))))
    fac = {(0, 0): lambda it, mu: np.ones_like(X) + 0 * it,
           (1, 0): lambda it, mu: it * np.ones_like(X),
           (0, 1): lambda it, mu: mu * np.ones_like(X)}[deriv]
    got = _direct_h0(k, H, beta, X, Y, q, deriv) + lt.tails(k, H, beta, X, Y, q, fac)
    ref = spectral_h0_sum(k, H, beta, X, Y, deriv=deriv)
    assert np.max(np.abs(got - ref) / np.abs(ref)) < 1e-12


def test_tail_cutoff_identity():
    """tails(q1) - tails(q2) equals the direct images q1 < |m| <= q2 exactly."""
    k, H, theta = 2.3, 1.0, 0.5
    beta = k * H * math.sin(theta)
    X = np.array([0.0, 0.2, -0.45, 0.3])
    Y = np.array([0.0, 0.1, 0.4, -0.7])
    one = lambda it, mu: np.ones_like(X) + 0 * it
    t3 = lt.tails(k, H, beta, X, Y, 3, one)
    t7 = lt.tails(k, H, beta, X, Y, 7, one)
    mid = sum(np.exp(1j * m * beta) * hankel1(0, k * np.hypot(X, Y - m * H))
              for m in list(range(-7, -3)) + list(range(4, 8)))
    assert np.max(np.abs((t3 - t7) - mid)) < 1e-13 * np.max(np.abs(mid))


def test_separable_tails_match_adaptive():
    k, H, theta = 2.0, 1.0, math.pi / 4
    beta = k * H * math.sin(theta)
    rng = np.random.default_rng(3)
    xt = rng.uniform(0.2, 0.8, (5, 2))
    ys = rng.uniform(0.2, 0.8, (7, 2))
    a1 = rng.uniform(0, 2 * np.pi, 5)
    a2 = rng.uniform(0, 2 * np.pi, 7)
    nut = np.stack([np.cos(a1), np.sin(a1)], 1)
    nys = np.stack([np.cos(a2), np.sin(a2)], 1)
    q = 3
    rule = lt.tail_rule(k, H, beta, q, 1.0, 1.0)
    sep = lt.tails_separable(k, H, beta, q, xt, nut, ys, nys, rule)
    X = xt[:, None, 0] - ys[None, :, 0]
    Y = xt[:, None, 1] - ys[None, :, 1]
    nx, ny = nut[:, None, 0], nut[:, None, 1]
    mx, my = nys[None, :, 0], nys[None, :, 1]

    def fac(it, muY):
        gn = mx * it + my * muY
        gv = nx * it + ny * muY
        one = np.ones_like(X)
        return np.stack([one + 0 * gn, -gn * one, gv * one, -gv * gn])

    ad = lt.tails(k, H, beta, X, Y, q, fac)
    assert np.max(np.abs(sep - ad)) < 1e-12 * np.max(np.abs(ad))


@pytest.mark.parametrize("k,H,theta", CASES[:3])
def test_periodic_kernel_quasi_periodic(k, H, theta):
    """sum_m alpha^m K(d + h - m h) = alpha sum_m alpha^m K(d - m h) (eq. 3)."""
    rng = np.random.default_rng(4)
    xt = rng.uniform(0.1, 0.9, (4, 2)) * H
    ys = rng.uniform(0.1, 0.9, (6, 2)) * H
    nut = np.tile([[0.6, 0.8]], (4, 1))
    nys = np.tile([[-0.8, 0.6]], (6, 1))
    beta = k * H * math.sin(theta)

    def full(xt):
        per = lt.periodic_offzero_kernels(k, H, theta, xt, nut, ys, nys, x_max=H, y_max=2 * H)
        dx = xt[:, None, 0] - ys[None, :, 0]
        dy = xt[:, None, 1] - ys[None, :, 1]
        m0 = kernels_sdkt(k, dx, dy, nut[:, None, 0], nut[:, None, 1], nys[None, :, 0], nys[None, :, 1])
        return [p + z for p, z in zip(per, m0)]

    a = full(xt)
    b = full(xt + np.array([0.0, H]))
    for u, v in zip(a, b):
        assert np.max(np.abs(v - np.exp(1j * beta) * u)) < 1e-11 * np.max(np.abs(u))


def test_lattice_orders_low_orders_vs_spectral():
    k, H, theta = 2.0, 1.0, math.pi / 4
    beta = k * H * math.sin(theta)
    ox, oy = 0.3, 0.1
    S = lt.lattice_sum_orders(k, H, theta, ox, oy, 2)
    X, Y = np.array([ox]), np.array([oy])
    g = spectral_h0_sum(k, H, beta, X, Y)[0]
    gx = spectral_h0_sum(k, H, beta, X, Y, deriv=(1, 0))[0]
    gy = spectral_h0_sum(k, H, beta, X, Y, deriv=(0, 1))[0]
    gxx = spectral_h0_sum(k, H, beta, X, Y, deriv=(2, 0))[0]
    gxy = spectral_h0_sum(k, H, beta, X, Y, deriv=(1, 1))[0]
    gyy = spectral_h0_sum(k, H, beta, X, Y, deriv=(0, 2))[0]
    ref = {0: g,
           1: (-1 / k) * (gx + 1j * gy),
           -1: (1 / k) * (gx - 1j * gy),
           2: (1 / k ** 2) * (gxx + 2j * gxy - gyy),
           -2: (1 / k ** 2) * (gxx - 2j * gxy - gyy)}
    for nu, v in ref.items():
        assert abs(S[nu + 2] - v) < 1e-11 * abs(v), nu


def test_lattice_orders_graf_shift():
    """High orders: shifting the offset by a small delta obeys Graf (eq. 10),
    S_nu(o + delta) = sum_l S_{nu+l}(o) J_l(k|delta|) e^{-i l arg(-delta)}."""
    k, H, theta = 1.5, 1.0, 0.2
    o = (0.0, 2.0)
    exclude = (-1, 0, 1, 2, 3)
    dl = np.array([0.05, -0.03])
    nmax, lmax = 12, 14
    S0 = lt.lattice_sum_orders(k, H, theta, o[0], o[1], nmax + lmax, exclude=exclude)
    S1 = lt.lattice_sum_orders(k, H, theta, o[0] + dl[0], o[1] + dl[1], nmax, exclude=exclude)
    r = math.hypot(*dl)
    ang = math.atan2(-dl[1], -dl[0])
    off = nmax + lmax
    for nu in range(-nmax, nmax + 1):
        v = sum(S0[off + nu + l] * jv(l, k * r) * np.exp(-1j * l * ang)
                for l in range(-lmax, lmax + 1))
        assert abs(v - S1[nu + nmax]) < 1e-10 * abs(S1[nu + nmax]), nu
