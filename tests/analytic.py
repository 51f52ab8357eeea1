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


def mst_periodic(k, k1, rho_fiber, rho_matrix, theta, H, centres, radii, n_max, lattice_sums,
                 n_orders=3):
    """Multiple scattering by a quasi-periodic array of circles (the "MST" the
    paper lists among the methods for phononic crystals, Sec. 1): the exact
    continuous solution of eqs. (1)-(3) for circular fibres, truncated in the
    multipole order.

    Fibre j scatters sum_n b_jn H_n(k|x - c_j|) e^{i n arg(x - c_j)}; its image
    at c_j + m h carries alpha^m b_j (eq. 3).  Every fibre answers the regular
    field reaching it, sum_n A_in J_n(k r_i) e^{i n phi_i}, through the Mie
    factor of a disc, b_in = s_in A_in.  Graf's theorem (eq. 10) moves the
    field of fibre j and its images to the centre of fibre i,
        A_il = A_il^inc + sum_j sum_n b_jn S_{n-l}(c_i - c_j),
    with the lattice sums S_nu(o) = sum_m alpha^m H_nu(k|o - m h|) e^{i nu arg(o - m h)}
    (the term o - m h = 0 left out), supplied by `lattice_sums(ox, oy, nu_max,
    exclude)`.  The incident wave gives A_il^inc = e^{i k d.c_i} i^l e^{-i l theta}.

    The Bragg amplitudes follow from the spectral form of the quasi-periodic
    sum of H_0 and the order-raising identities after eq. (17): right of the
    array (x1 > c_jx), sum_m alpha^m H_n e^{i n arg} of the image column is
    (2/H) sum_q e^{i(gamma_q X + kappa_q Y)} ((kappa_q - i gamma_q)/k)^n / gamma_q,
    left of it the same with ((kappa_q + i gamma_q)/k)^n and -gamma_q X.
    Returns (orders q, R_q, T_q, b)."""
    centres = np.asarray(centres, dtype=np.float64).reshape(-1, 2)
    M = centres.shape[0]
    n = np.arange(-n_max, n_max + 1)
    P = n.size
    s = np.zeros((M, P), dtype=np.complex128)
    for j in range(M):
        R = radii[j]
        num = (k / rho_matrix) * jvp(n, k * R) * jv(n, k1 * R) \
            - (k1 / rho_fiber) * jvp(n, k1 * R) * jv(n, k * R)
        den = (k1 / rho_fiber) * jvp(n, k1 * R) * hankel1(n, k * R) \
            - (k / rho_matrix) * h1vp(n, k * R) * jv(n, k1 * R)
        s[j] = num / den
    Tm = np.zeros((M * P, M * P), dtype=np.complex128)
    for i in range(M):
        for j in range(M):
            o = centres[i] - centres[j]
            S = lattice_sums(o[0], o[1], 2 * n_max, (0,) if i == j else ())
            # rows l, columns n: S_{n - l}, index (n - l) + 2 n_max
            idx = n[None, :] - n[:, None] + 2 * n_max
            Tm[i * P:(i + 1) * P, j * P:(j + 1) * P] = S[idx]
    d = np.array([math.cos(theta), math.sin(theta)])
    Ainc = np.concatenate([np.exp(1j * k * (centres[i] @ d)) * (1j ** n) * np.exp(-1j * n * theta)
                           for i in range(M)])
    sd = s.reshape(-1)
    b = np.linalg.solve(np.eye(M * P) - sd[:, None] * Tm, sd * Ainc).reshape(M, P)

    q = np.arange(-n_orders, n_orders + 1)
    kap = k * math.sin(theta) + 2 * math.pi * q / H
    gam = np.sqrt((k * k - kap * kap).astype(np.complex128))
    gam = np.where(gam.imag < 0, -gam, gam)
    Tq = np.zeros(q.size, dtype=np.complex128)
    Rq = np.zeros(q.size, dtype=np.complex128)
    for j in range(M):
        cx, cy = centres[j]
        right = ((kap[:, None] - 1j * gam[:, None]) / k) ** n[None, :]
        left = ((kap[:, None] + 1j * gam[:, None]) / k) ** n[None, :]
        Tq += np.exp(-1j * (gam * cx + kap * cy)) * (right @ b[j])
        Rq += np.exp(1j * (gam * cx - kap * cy)) * (left @ b[j])
    Tq *= 2.0 / (H * gam)
    Rq *= 2.0 / (H * gam)
    return q, Rq, Tq, b
