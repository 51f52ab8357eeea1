"""Free-space Helmholtz kernels (oracle; test infrastructure only).

Fundamental solution Phi(x, y) = (i/4) H0^(1)(kappa |x - y|) (Sec. 2), and the
kernels of the four layer operators of eq. (6), written in d = x - y:
  S: Phi
  D: d Phi / d n_y          (double layer, normal at the source)
  K: d Phi / d nu_x         (normal at the target)
  T: d^2 Phi / d nu_x d n_y (hypersingular)
Derivatives use H0' = -H1 and H1'(z) = H0(z) - H1(z)/z.
"""
from __future__ import annotations

import numpy as np
from scipy.special import hankel1


def kernels_sdkt(kappa: float, dx, dy, nx_x, nx_y, ny_x, ny_y):
    """Return S, D, K, T kernels for separations d = (dx, dy).

    nx = target normal nu_x, ny = source normal n_y.  Arrays broadcast."""
    r = np.hypot(dx, dy)
    z = kappa * r
    h0 = hankel1(0, z)
    h1 = hankel1(1, z)
    d_nx = dx * nx_x + dy * nx_y
    d_ny = dx * ny_x + dy * ny_y
    nn = nx_x * ny_x + nx_y * ny_y
    S = 0.25j * h0
    D = 0.25j * kappa * h1 * d_ny / r
    K = -0.25j * kappa * h1 * d_nx / r
    T = 0.25j * kappa * ((kappa * h0 / r - 2.0 * h1 / r ** 2) * d_nx * d_ny / r + h1 * nn / r)
    return S, D, K, T


def phi(kappa: float, dx, dy):
    return 0.25j * hankel1(0, kappa * np.hypot(dx, dy))


def grad_x_phi(kappa: float, dx, dy):
    """Gradient of Phi with respect to the target point x."""
    r = np.hypot(dx, dy)
    g = -0.25j * kappa * hankel1(1, kappa * r) / r
    return g * dx, g * dy
