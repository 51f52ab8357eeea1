"""Reflected/transmitted Bragg amplitudes and the energy transmission
coefficient (oracle; test infrastructure only).

With the spectral form of the quasi-periodic kernel,
    sum_m alpha^m Phi(x, y + m h) = (i / (2H)) sum_n e^{i kappa_n (x2 - y2) + i gamma_n |x1 - y1|} / gamma_n,
    kappa_n = k sin(theta) + 2 pi n / H,  gamma_n = sqrt(k^2 - kappa_n^2), Im >= 0,
the scattered field of the representation (eq. 4 with eq. 7) is, right of the
block, sum_n T_n e^{i(gamma_n x1 + kappa_n x2)} and, left of it,
sum_n R_n e^{i(-gamma_n x1 + kappa_n x2)}, with
    T_n = 1/(2 H gamma_n) int e^{-i(gamma_n y1 + kappa_n y2)} [(gamma_n n1 + kappa_n n2) phi + eta varphi] ds
    R_n = 1/(2 H gamma_n) int e^{ i(gamma_n y1 - kappa_n y2)} [-(gamma_n n1 - kappa_n n2) phi + eta varphi] ds.
The n = 0 mode of the total field on the right carries the incident wave.
ETC is the quantity of Sec. 4, (1/(kH)) int_0^H |du/dx1 (L, x2)| dx2, taken on
the modal expansion with the trapezoid rule in x2.  For lossless media the
flux balance sum_prop gamma_n (|R_n|^2 + |delta_n0 + T_n|^2) = k cos(theta)
holds for the exact solution and serves as a check.
"""
from __future__ import annotations

import math

import numpy as np

from .geometry import gauss_points
from .system import Problem, split_density


def bragg(pb: Problem, psi, n_orders: int, G: int | None = None):
    """Bragg orders, their wavenumbers and amplitudes R_n, T_n.  The boundary
    integrals use the 8-point Gauss rule on every chord, or for the Nystrom
    boundary (nystrom.py, nodes and trapezoid weights) the nodes themselves."""
    bd = pb.bd
    if G is None:
        G = 1 if getattr(bd, "speed", None) is not None else 8
    phi_d, vphi = split_density(pb, psi)
    gp, gw = gauss_points(bd, G)
    n = np.arange(-n_orders, n_orders + 1)
    kap = pb.k * math.sin(pb.theta) + 2 * math.pi * n / bd.H
    gam = np.sqrt((pb.k ** 2 - kap ** 2).astype(np.complex128))
    gam = np.where(gam.imag < 0, -gam, gam)
    y1 = gp[..., 0][None]
    y2 = gp[..., 1][None]
    n1 = bd.nrm[None, :, None, 0]
    n2 = bd.nrm[None, :, None, 1]
    g = gam[:, None, None]
    kk = kap[:, None, None]
    ph = phi_d[None, :, None]
    vp = vphi[None, :, None]
    ew = gw[None]
    T = (np.exp(-1j * (g * y1 + kk * y2)) * ((g * n1 + kk * n2) * ph + pb.eta * vp) * ew).sum((1, 2))
    R = (np.exp(1j * (g * y1 - kk * y2)) * (-(g * n1 - kk * n2) * ph + pb.eta * vp) * ew).sum((1, 2))
    T = T / (2 * bd.H * gam)
    R = R / (2 * bd.H * gam)
    return n, kap, gam, R, T


def energy_residual(pb: Problem, psi, n_orders: int = 20):
    n, kap, gam, R, T = bragg(pb, psi, n_orders)
    prop = np.abs(gam.imag) < 1e-14
    t0 = T + (n == 0)
    flux = np.sum(gam[prop].real * (np.abs(R[prop]) ** 2 + np.abs(t0[prop]) ** 2))
    return flux / (pb.k * math.cos(pb.theta)) - 1.0


def etc_from_modes(k: float, H: float, L: float, n, kap, gam, T, n_pts: int = 512):
    """ETC of Sec. 4 from the transmitted Bragg amplitudes T_n (orders n,
    wavenumbers kap, gam): right of the block the total field is
    sum_n (delta_n0 + T_n) e^{i(gam_n x1 + kap_n x2)}, so
    du/dx1 (L, x2) = sum_n i gam_n (delta_n0 + T_n) e^{i(gam_n L + kap_n x2)};
    its modulus is averaged over one period in x2 by the trapezoid rule
    (spectrally accurate for the periodic integrand) and divided by k."""
    x2 = np.arange(n_pts) * H / n_pts
    t0 = np.asarray(T) + (np.asarray(n) == 0)
    du = (1j * gam[:, None] * t0[:, None]
          * np.exp(1j * (gam[:, None] * L + kap[:, None] * x2[None, :]))).sum(0)
    return float(np.mean(np.abs(du)) * H / (k * H))


def etc(pb: Problem, psi, n_orders: int = 30, n_pts: int = 512):
    n, kap, gam, R, T = bragg(pb, psi, n_orders)
    return etc_from_modes(pb.k, pb.bd.H, pb.bd.L, n, kap, gam, T, n_pts)
