"""FMM stage definitions by direct summation (oracle; test infrastructure only).

Sec. 3.2 of the paper writes the kernel of the representation through Graf's
theorem (eq. 10): for |y - O| < |x - O|,
    H0(k|x - y|) = sum_n Hp_n(k(x - O)) Jm_n(k(y - O)),
    Hp_n(v) = H_n(|v|) e^{i n arg v},  Jm_n(v) = J_n(|v|) e^{-i n arg v},
so the field of the density combination D phi - i eta S varphi of a cell C is
sum_n Hp_n(k(x - O_C)) M_n(C) with the multipole moment (the MM of S-bar and
D-bar in Sec. 3.2, combined as in the representation and with the factor i/4
of Phi folded in):
    M_n(C) = (i/4) sum_{e in C} sum_g w_g [ dJm_n(k(y_g - O_C))/dn_y phi_e
                                            - i eta Jm_n(k(y_g - O_C)) varphi_e ].
The normal derivative is taken in polar form,
    grad_y [J_n(k rho) e^{-i n t}] = k J_n'(k rho) e^{-i n t} rho_hat
                                     - i n J_n(k rho) e^{-i n t} t_hat / rho,
independently of the recurrence form used by the library.  Moments moved up
the tree by M2M equal the moments taken directly about the parent centre up
to the truncation error of eq. (10).
"""
from __future__ import annotations

import numpy as np
from scipy.special import jv, jvp

from .geometry import gauss_points
from .system import Problem, split_density


def moments(pb: Problem, psi, centre, elems, kappa: float, p: int, G: int = 4):
    """Direct moments M_n, n = -p..p, of the elements `elems` about `centre`."""
    bd = pb.bd
    phi_d, vphi = split_density(pb, psi)
    pts, wts = gauss_points(bd, G)
    elems = np.asarray(elems)
    y = pts[elems].reshape(-1, 2)
    w = wts[elems].reshape(-1)
    nrm = np.repeat(bd.nrm[elems], G, axis=0)
    ph = np.repeat(phi_d[elems], G)
    vp = np.repeat(vphi[elems], G)
    d = y - np.asarray(centre)[None, :]
    rho = np.hypot(d[:, 0], d[:, 1])
    t = np.arctan2(d[:, 1], d[:, 0])
    rh = np.stack([np.cos(t), np.sin(t)], 1)
    th = np.stack([-np.sin(t), np.cos(t)], 1)
    n_rh = (nrm * rh).sum(1)
    n_th = (nrm * th).sum(1)
    out = np.zeros(2 * p + 1, dtype=np.complex128)
    for i, n in enumerate(range(-p, p + 1)):
        e = np.exp(-1j * n * t)
        J = jv(n, kappa * rho)
        dJ = kappa * jvp(n, kappa * rho) * e * n_rh - 1j * n * J * e * n_th / rho
        out[i] = 0.25j * np.sum(w * (dJ * ph - 1j * pb.eta * J * e * vp))
    return out
