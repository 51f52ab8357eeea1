"""Pins of the oracle's FMM moments, energy transmission coefficient and
whole periodic system against quantities fixed by the mathematics.

* Moments (Sec. 3.2, multipole moment of eq. 11 and Graf's theorem, eq. 10):
  the multipole expansion sum_n Hp_n(k(x - O)) M_n about a cell centre O must
  reproduce the field of the cell's density combination D phi - i eta S varphi
  at a far point, summed directly with the free-space kernels at the same
  Gauss points; the truncation error falls like tau^p with
  tau = max|y - O| / |x - O| (Theorems 1-2).
* ETC (Sec. 4): without scattering, du/dx1 of the incident wave has modulus
  k cos(theta) everywhere, so ETC = cos(theta) exactly; with one transmitted
  order it is cos(theta)|1 + T_0|, with two propagating orders the mean of
  |A + B e^{i phi}| over a period is (2/pi)(|A| + |B|) E(m),
  m = 4|A||B|/(|A| + |B|)^2 (complete elliptic integral of the second kind).
* Whole periodic system (Sec. 2, eqs. 1-3 and 9): the Bragg amplitudes of the
  BEM solution converge at first order in the element size to those of the
  multiple-scattering solution of the same array of circles (tests/analytic.py),
  and the Richardson extrapolation of two refinements agrees to a few 1e-4.
"""
import math

import numpy as np
import pytest
from scipy.special import ellipe

import oracle.fmmdefs as fd
import workloads as W
from analytic import mst_periodic
from oracle import fields as fl
from oracle import lattice as la
from oracle import system as sy
from oracle.geometry import gauss_points
from oracle.kernels import kernels_sdkt
from scipy.special import hankel1


def _direct_field(pb, psi, elems, x, kappa, G=4):
    """Field of D phi - i eta S varphi of the elements `elems` at the point x,
    by direct summation of the kernels at the Gauss points."""
    bd = pb.bd
    phi_d, vphi = sy.split_density(pb, psi)
    pts, wts = gauss_points(bd, G)
    tot = 0.0 + 0.0j
    for e in elems:
        d = x[None, :] - pts[e]
        S, D, _, _ = kernels_sdkt(kappa, d[:, 0], d[:, 1], 0.0, 0.0, bd.nrm[e, 0], bd.nrm[e, 1])
        tot += np.sum(wts[e] * (D * phi_d[e] - 1j * pb.eta * S * vphi[e]))
    return tot


def _expansion_field(M, centre, x, kappa):
    p = (M.size - 1) // 2
    n = np.arange(-p, p + 1)
    v = x - centre
    r, t = math.hypot(*v), math.atan2(v[1], v[0])
    return np.sum(hankel1(n, kappa * r) * np.exp(1j * n * t) * M)


@pytest.mark.parametrize("channel", [0, 1])
def test_moments_reproduce_far_field(channel):
    """A 16-element arc of a fibre, its moments about the arc's centroid, and
    far points at three times the arc's radius in several directions."""
    wl = W.small_square(1, 1, 64, r=0.3)
    pb = sy.problem_from_workload(wl, 3.0, 0.4)
    kappa = pb.k if channel == 0 else pb.k1
    psi = W.random_density(pb.n, 21)
    elems = np.arange(5, 21)
    bd = pb.bd
    O = bd.mid[elems].mean(0)
    rad = np.max(np.hypot(*(np.concatenate([bd.a_pt[elems], bd.b_pt[elems]]) - O).T))
    errs = {}
    for p in (8, 16, 24):
        M = fd.moments(pb, psi, O, elems, kappa, p)
        e = 0.0
        for ang in (0.3, 1.9, 3.5, 5.0):
            x = O + 3.0 * rad * np.array([math.cos(ang), math.sin(ang)])
            ref = _direct_field(pb, psi, elems, x, kappa)
            e = max(e, abs(_expansion_field(M, O, x, kappa) - ref) / abs(ref))
        errs[p] = e
    assert errs[24] < 1e-10
    # geometric decay, at least tau = 1/3 per order on average
    assert errs[16] < errs[8] * 3.0 ** -6 and errs[24] < errs[16] * 3.0 ** -6


def test_moments_pin_catches_a_flipped_radial_derivative(monkeypatch):
    """Planted mistake: the sign of dJ_n/drho in the normal derivative."""
    wl = W.small_square(1, 1, 64, r=0.3)
    pb = sy.problem_from_workload(wl, 3.0, 0.4)
    psi = W.random_density(pb.n, 21)
    elems = np.arange(5, 21)
    O = pb.bd.mid[elems].mean(0)
    x = O + np.array([0.5, 0.2])
    ref = _direct_field(pb, psi, elems, x, pb.k)
    good = _expansion_field(fd.moments(pb, psi, O, elems, pb.k, 24), O, x, pb.k)
    orig = fd.jvp
    monkeypatch.setattr(fd, "jvp", lambda n, z: -orig(n, z))
    bad = _expansion_field(fd.moments(pb, psi, O, elems, pb.k, 24), O, x, pb.k)
    assert abs(good - ref) < 1e-10 * abs(ref)
    assert abs(bad - ref) > 1e-2 * abs(ref)


@pytest.mark.parametrize("theta", [0.0, 0.3, math.pi / 4, 1.2])
def test_etc_without_scattering_is_cos_theta(theta):
    """Psi = 0: no scattered field, the incident wave alone gives cos(theta)."""
    for wl in (W.small_square(2, 3, 16, r=0.3), W.small_square(3, 2, 16, r=0.25, lattice=W.HEXAGON)):
        pb = sy.problem_from_workload(wl, 2.7, theta)
        v = fl.etc(pb, np.zeros(pb.n, dtype=np.complex128))
        assert abs(v - math.cos(theta)) < 1e-13


def test_etc_modal_closed_forms():
    k, H, L, th = 2.3, 3.5, 2.0, 0.5
    n = np.arange(-3, 4)
    kap = k * math.sin(th) + 2 * math.pi * n / H
    gam = np.sqrt((k * k - kap * kap).astype(np.complex128))
    gam = np.where(gam.imag < 0, -gam, gam)
    prop = np.abs(gam.imag) < 1e-14
    assert prop.sum() == 2          # orders 0 and -1 propagate
    # one transmitted order
    T = np.zeros(n.size, dtype=np.complex128)
    T[3] = -0.4 + 0.3j
    assert abs(fl.etc_from_modes(k, H, L, n, kap, gam, T) - math.cos(th) * abs(1 + T[3])) < 1e-13
    # two propagating orders: mean of |A + B e^{i phi}|
    T[2] = 0.35 - 0.2j
    A = abs(gam[3] * (1 + T[3]))
    B = abs(gam[2] * T[2])
    m = 4 * A * B / (A + B) ** 2
    ref = (2 / math.pi) * (A + B) * ellipe(m) / k
    assert abs(fl.etc_from_modes(k, H, L, n, kap, gam, T, n_pts=2048) - ref) < 1e-10


def test_etc_of_the_no_contrast_system():
    """The whole chain (solve, Bragg amplitudes, ETC) on a block without
    contrast: ETC equals cos(theta) up to the discretisation error."""
    wl = W.tiny()
    wl.n_elem = 128
    wl.rho_fiber, wl.c_fiber = wl.rho_matrix, wl.c_matrix
    pb = sy.problem_from_workload(wl, 2.0, math.pi / 4)
    psi, _, _ = sy.solve(pb)
    assert abs(fl.etc(pb, psi) - math.cos(math.pi / 4)) < 1e-5


def _bem_amplitudes(wl, ka, th, N):
    wl.n_elem = N
    pb = sy.problem_from_workload(wl, ka, th)
    psi, _, _ = sy.solve(pb)
    _, _, gam, R, T = fl.bragg(pb, psi, 3)
    return pb, gam, R, T


@pytest.mark.parametrize("case", ["one_fibre", "two_fibres"])
def test_periodic_system_converges_to_multiple_scattering(case):
    if case == "one_fibre":
        wl, ka, th = W.tiny(), 2.0, math.pi / 4
    else:
        wl, ka, th = W.small_square(2, 1, 64, radii=np.array([0.3, 0.22])), 4.0, 0.7
    res = [_bem_amplitudes(wl, ka, th, N) for N in (64, 128)]
    pb, gam = res[0][0], res[0][1]
    ls = lambda ox, oy, nu, ex: la.lattice_sum_orders(pb.k, pb.bd.H, th, ox, oy, nu, exclude=ex)
    _, Rm, Tm, _ = mst_periodic(pb.k, pb.k1, wl.rho_fiber, wl.rho_matrix, th, pb.bd.H,
                                pb.bd.centres, wl.radii, 12, ls)
    prop = np.abs(gam.imag) < 1e-14
    assert prop.sum() == (1 if case == "one_fibre" else 2)
    e = [max(np.max(np.abs(R - Rm)[prop]), np.max(np.abs(T - Tm)[prop])) for _, _, R, T in res]
    assert e[1] < 1.5e-2
    assert 1.8 < e[0] / e[1] < 2.2                     # first order in the element size
    (_, _, R1, T1), (_, _, R2, T2) = res
    ext = max(np.max(np.abs(2 * R2 - R1 - Rm)[prop]), np.max(np.abs(2 * T2 - T1 - Tm)[prop]))
    assert ext < 1e-3
