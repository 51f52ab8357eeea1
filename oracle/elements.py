"""Element integrals of the layer kernels (oracle; test infrastructure only).

The paper divides each boundary into N elements (Sec. 3.2) but does not say
how the element integrals are taken.  Reading used here, which defines the
discrete operator that the fast method approximates:

  * far rule   G-point Gauss-Legendre on the chord; used for every pair
               except the ones below, and for every periodic image m != 0;
  * near rule  the exact chord integral (adaptive quadrature to ~1e-14),
               for same-fibre pairs with cyclic index distance 1 or 2, m = 0;
  * self       the chord's own collocation point, m = 0:
                 S_self = (i/4) 2 int_0^{h/2} H0(kappa s) ds, by the Struve
                 closed form of int_0^x J0 and int_0^x Y0;
                 D_self = K_self = 0 (straight chord, principal value);
                 T_self = kappa^2 S_self - (i kappa / 2) H1(kappa h / 2),
               the finite part given by the straight-element Maue identity
                 T_e(x) = kappa^2 (nu_x . n_e) S_e(x)
                          - tau_x . grad_x [Phi(x, b_e) - Phi(x, a_e)],
                 tau_x = (-nu_x2, nu_x1),
               evaluated at the chord midpoint.
"""
from __future__ import annotations

import numpy as np
from scipy.integrate import quad_vec
from scipy.special import hankel1, j0, j1, struve, y0, y1

from .kernels import kernels_sdkt

NEAR_BAND = 2     # same-fibre cyclic index distance handled by the near rule


def int_h0(x):
    """int_0^x H0^(1)(t) dt via the Struve-function closed forms."""
    x = np.asarray(x, dtype=np.float64)
    s0, s1 = struve(0, x), struve(1, x)
    ij = x * j0(x) + 0.5 * np.pi * x * (j1(x) * s0 - j0(x) * s1)
    iy = x * y0(x) + 0.5 * np.pi * x * (y1(x) * s0 - y0(x) * s1)
    return ij + 1j * iy


def self_terms(kappa, h):
    """(S, D, K, T) of a chord of length h at its own midpoint."""
    h = np.asarray(h, dtype=np.float64)
    S = 0.5j / kappa * int_h0(0.5 * kappa * h)
    T = kappa ** 2 * S - 0.5j * kappa * hankel1(1, 0.5 * kappa * h)
    z = np.zeros_like(S)
    return S, z, z, T


def far_rule(kappa, x, nu, pts, wts, nrm):
    """Gauss-Legendre element integrals.

    x [..., 2] targets with normals nu [..., 2]; pts [..., G, 2], wts [..., G]
    the element's nodes and weights; nrm [..., 2] the element normals.
    Leading dimensions broadcast.  Returns S, D, K, T of shape [...]."""
    dx = x[..., None, 0] - pts[..., 0]
    dy = x[..., None, 1] - pts[..., 1]
    S, D, K, T = kernels_sdkt(kappa, dx, dy, nu[..., None, 0], nu[..., None, 1],
                              nrm[..., None, 0], nrm[..., None, 1])
    return ((S * wts).sum(-1), (D * wts).sum(-1), (K * wts).sum(-1), (T * wts).sum(-1))


def near_rule(kappas, x, nu, mid, tan, nrm, h, epsrel=1e-14):
    """Exact chord integrals for a batch of (target, element) pairs.

    x, nu, mid, tan, nrm: [P, 2]; h: [P].  Returns an array [len(kappas), 4, P]
    holding S, D, K, T for each wavenumber."""
    x = np.asarray(x)

    def integrand(xi):
        y = mid + (0.5 * h * xi)[:, None] * tan
        out = []
        for kap in kappas:
            S, D, K, T = kernels_sdkt(kap, x[:, 0] - y[:, 0], x[:, 1] - y[:, 1],
                                      nu[:, 0], nu[:, 1], nrm[:, 0], nrm[:, 1])
            out.append(np.stack([S, D, K, T]) * (0.5 * h))
        return np.stack(out)

    val, _ = quad_vec(integrand, -1.0, 1.0, epsabs=1e-300, epsrel=epsrel, norm="max",
                      limit=20000)
    return val
