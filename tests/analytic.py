"""Closed-form and series solutions used to pin the oracle.

These are independent representations of quantities the oracle computes by
the paper's own route; none of them is used by the oracle itself.

* Spectral (Rayleigh) series of the quasi-periodic sum of H0: Poisson
  summation of the Fourier transform of the free-space kernel along y,
      sum_m e^{i m beta} H0(k|(X, Y - mH)|)
          = (2/H) sum_n e^{i kappa_n Y + i gamma_n |X|} / gamma_n,
  kappa_n = (beta + 2 pi n)/H, gamma_n = sqrt(k^2 - kappa_n^2), Im >= 0,
  exponentially convergent for X != 0.
* Mie series for transmission through one circular fibre (free space): the
  separated solution of eqs. (1)-(2) for a disc, with
  u_inc = sum i^n J_n(kr) e^{in(phi - theta)},
  u_s   = sum a_n H_n(kr) e^{in(phi - theta)}.
"""
from __future__ import annotations

import math

import numpy as np
from scipy.special import hankel1, h1vp, jv, jvp


def spectral_h0_sum(k, H, beta, X, Y, n_terms=None, deriv=(0, 0)):
    """Quasi-periodic sum of H0 and its (dX^a dY^b) derivative, X != 0."""
    X = np.asarray(X, dtype=np.float64)
    Y = np.asarray(Y, dtype=np.float64)
    if n_terms is None:
        xm = max(float(np.min(np.abs(X))), 1e-3)
        n_terms = int(60.0 * H / (2 * math.pi * xm)) + int(k * H / (2 * math.pi)) + 10
    n = np.arange(-n_terms, n_terms + 1)
    kap = (beta + 2 * math.pi * n) / H
    gam = np.sqrt((k * k - kap * kap).astype(np.complex128))
    gam = np.where(gam.imag < 0, -gam, gam)
    sx = np.sign(X)[..., None]
    a, b = deriv
    ph = np.exp(1j * kap * Y[..., None] + 1j * gam * np.abs(X)[..., None])
    fac = (1j * gam * sx) ** a * (1j * kap) ** b
    return (2.0 / H) * np.sum(fac * ph / gam, axis=-1)


def mie_coefficients(k, k1, R, rho_fiber, rho_matrix, n_max):
    n = np.arange(-n_max, n_max + 1)
    num = (k / rho_matrix) * jvp(n, k * R) * jv(n, k1 * R) \
        - (k1 / rho_fiber) * jvp(n, k1 * R) * jv(n, k * R)
    den = (k1 / rho_fiber) * jvp(n, k1 * R) * hankel1(n, k * R) \
        - (k / rho_matrix) * h1vp(n, k * R) * jv(n, k1 * R)
    return n, (1j ** n) * num / den


def mie_scattered(k, k1, R, rho_fiber, rho_matrix, theta, centre, pts, n_max=60):
    n, an = mie_coefficients(k, k1, R, rho_fiber, rho_matrix, n_max)
    d = np.asarray(pts) - np.asarray(centre)[None, :]
    r = np.hypot(d[:, 0], d[:, 1])
    ph = np.arctan2(d[:, 1], d[:, 0])
    # the incident wave seen from the fibre centre carries exp(i k c . d)
    shift = np.exp(1j * k * (centre[0] * math.cos(theta) + centre[1] * math.sin(theta)))
    return shift * np.sum(an[None, :] * hankel1(n[None, :], k * r[:, None])
                          * np.exp(1j * n[None, :] * (ph[:, None] - theta)), axis=1)
