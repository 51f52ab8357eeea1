"""Spectral Nystrom discretisation of the same boundary-integral system
(oracle; test infrastructure only).

The paper builds on Kress's boundary integral equations (Sec. 1, refs. 2 and
4) and solves them with constant elements; this module is the other
discretisation those references give: densities at the nodes t_j = 2 pi j / N
of each fibre's parametrisation x(t) (counter-clockwise, outward normal
nu = (x2', -x1') / |x'|), the trapezoidal rule for every smooth kernel
(pairs of different fibres, every periodic image), and for each fibre's own
operators at image 0 the logarithmic splitting

    F(t, tau) = F1(t, tau) ln(4 sin^2((t - tau)/2)) + F2(t, tau),
    int F phi dtau ~ sum_j [ R_j(t) F1(t, t_j) + (2 pi / N) F2(t, t_j) ] phi_j,
    R_j(t) = -(4 pi / N) sum_{m=1}^{N/2-1} cos(m (t - t_j)) / m - (4 pi / N^2) cos(N (t - t_j) / 2),

the weights that integrate the logarithm times trigonometric polynomials of
degree below N/2 exactly.  The log coefficients follow from the series of Y0
and Y1 (DLMF 10.8.1-10.8.2); the diagonal values F2(t, t) from the limits:
  S: F = (i/4) H0(k r) |x'(tau)|,   F1 = -J0(k r) |x'(tau)| / (4 pi),
     F2(t, t) = (i/4 - C/(2 pi) - ln(k |x'(t)| / 2) / (2 pi)) |x'(t)|, C Euler's constant;
  D: F = (i k/4) H1(k r) (x(t) - x(tau)) . nt(tau) / r,  nt = nu |x'|,
     F1 = -(k / (4 pi)) J1(k r) (x(t) - x(tau)) . nt(tau) / r,  F2(t, t) = x''(t) . nt(t) / (4 pi |x'(t)|^2);
  K: F = -(i k/4) H1(k r) (x(t) - x(tau)) . nu(t) / r |x'(tau)|, F1 its J1 part, the same F2(t, t);
  T: Maue's identity, T phi = (1/|x'(t)|) d/dt S0 (d phi / dtau) + k^2 S_nu phi, with S0 the
     kernel (i/4) H0 (no |x'|) and S_nu the kernel (i/4) H0 nu(t) . nt(tau), both split as S,
     and d/dt the trigonometric differentiation of the nodal values (eigenvalue i q on mode q,
     0 on the Nyquist mode).
D and K are the principal values (their jumps are the identity terms of eq. 8), as for the
elements.  The rows of (I - A) are those of eq. 9 (system.py), with these matrices in place of
the element integrals; the right-hand side, the Bragg amplitudes and ETC are the element
formulas with the nodes as points and the trapezoid weights |x'(t_j)| 2 pi / N as lengths.
"""
from __future__ import annotations

import dataclasses
import math

import numpy as np
from scipy.special import hankel1, j0, j1

from .geometry import Boundary, fibre_centres
from .lattice import choose_q, periodic_offzero_kernels
from .kernels import kernels_sdkt
from .system import Problem, col_phi, col_varphi

EULER_C = 0.5772156649015329


def curve_derivatives(shape: int, r: float, t):
    """x(t) - c, x'(t), x''(t) of a fibre's boundary curve (circle or the round
    square of Sec. 4), each [len(t), 2]."""
    t = np.asarray(t, dtype=np.float64)
    c, s = np.cos(t), np.sin(t)
    if shape == 0:
        x = r * np.stack([c, s], -1)
        d1 = r * np.stack([-s, c], -1)
        d2 = -x
        return x, d1, d2
    if shape == 1:
        # r ((3 + 2 sin^2 t) cos t, (3 + 2 cos^2 t) sin t)
        x = r * np.stack([(3 + 2 * s * s) * c, (3 + 2 * c * c) * s], -1)
        d1 = r * np.stack([4 * s * c * c - (3 + 2 * s * s) * s, -4 * c * s * s + (3 + 2 * c * c) * c], -1)
        # derivatives of 4 s c^2 - 3 s - 2 s^3 and -4 c s^2 + 3 c + 2 c^3
        d2 = r * np.stack([4 * c ** 3 - 8 * s * s * c - 3 * c - 6 * s * s * c,
                           4 * s ** 3 - 8 * c * c * s - 3 * s - 6 * c * c * s], -1)
        return x, d1, d2
    raise ValueError("shape must be 0 (circle) or 1 (round square)")


@dataclasses.dataclass
class NystromBoundary(Boundary):
    """Nodes as the points (mid), unit tangents, outward normals, trapezoid
    weights |x'| 2 pi / N as h, plus the speed |x'| and x'' at every node."""
    speed: np.ndarray = None     # [E]
    acc: np.ndarray = None       # [E, 2] x''(t_j)


def discretise(lattice: int, a: float, M_L: int, M_H: int, N: int, radii, shape: int = 0) -> NystromBoundary:
    if N % 2:
        raise ValueError("N must be even")
    centres, L, H = fibre_centres(lattice, a, M_L, M_H)
    M = M_L * M_H
    radii = np.asarray(radii, dtype=np.float64).reshape(M)
    t = 2.0 * np.pi * np.arange(N) / N
    pts = np.zeros((M * N, 2))
    d1 = np.zeros((M * N, 2))
    d2 = np.zeros((M * N, 2))
    for f in range(M):
        x, v, w = curve_derivatives(shape, radii[f], t)
        pts[f * N:(f + 1) * N] = centres[f] + x
        d1[f * N:(f + 1) * N] = v
        d2[f * N:(f + 1) * N] = w
    speed = np.hypot(d1[:, 0], d1[:, 1])
    tan = d1 / speed[:, None]
    nrm = np.stack([tan[:, 1], -tan[:, 0]], axis=1)
    h = speed * 2.0 * np.pi / N
    fibre = np.repeat(np.arange(M), N)
    local = np.tile(np.arange(N), M)
    return NystromBoundary(M, N, centres, radii, L, H, pts.copy(), pts.copy(), pts, tan, nrm, h, fibre, local,
                           speed=speed, acc=d2)


def problem_from_workload(wl, ka: float, theta: float, periodic: bool = True, eta: float | None = None) -> Problem:
    bd = discretise(wl.lattice, wl.a, wl.M_L, wl.M_H, wl.n_elem, wl.radii, getattr(wl, "shape", 0))
    k = ka / wl.a
    k1 = k * wl.c_matrix / wl.c_fiber
    varrho = wl.rho_matrix / wl.rho_fiber
    if eta is None:
        eta = wl.eta if wl.eta > 0 else k
    # G = 1: the point rule at the nodes with weight h (gauss_points(bd, 1))
    return Problem(bd, k, k1, varrho, eta, theta, 1, periodic)


def kress_weights(N: int, s):
    """R(s) of the logarithmic quadrature: the weight of node t_j for target
    t is R(t - t_j)."""
    s = np.asarray(s, dtype=np.float64)
    m = np.arange(1, N // 2)
    out = -(4.0 * np.pi / N) * (np.cos(np.multiply.outer(s, m)) / m).sum(-1)
    return out - (4.0 * np.pi / N ** 2) * np.cos(0.5 * N * s)


def diff_matrix(N: int):
    """Trigonometric differentiation of N (even) equispaced nodal values:
    D[i, j] = (1/2) (-1)^(i - j) cot((t_i - t_j) / 2), D[i, i] = 0."""
    i = np.arange(N)
    d = i[:, None] - i[None, :]
    with np.errstate(divide="ignore", invalid="ignore"):
        D = 0.5 * np.where(d % 2 == 0, 1.0, -1.0) / np.tan(np.pi * d / N)
    D[i, i] = 0.0
    return D


def _split(F, F1, diag, R, N):
    """sum_j [R_ij F1_ij + (2 pi / N) F2_ij] with F2 = F - F1 ln(4 sin^2) off the
    diagonal and F2_ii = diag."""
    n = F.shape[0]
    t = 2.0 * np.pi * np.arange(n) / N
    dt = t[:, None] - t[None, :]
    off = ~np.eye(n, dtype=bool)
    lg = np.zeros_like(dt)
    lg[off] = np.log(4.0 * np.sin(0.5 * dt[off]) ** 2)
    F2 = np.where(off, F - F1 * lg, 0.0)
    F2[np.arange(n), np.arange(n)] = diag
    return R * F1 + (2.0 * np.pi / N) * F2


def self_matrices(bd: NystromBoundary, f: int, kappa: float):
    """The Nystrom matrices [N, N] of S, D, K, T (principal values) of fibre
    f's own boundary at wavenumber kappa (image 0)."""
    N = bd.N
    sl = slice(f * N, (f + 1) * N)
    x, sp, nu, acc = bd.mid[sl], bd.speed[sl], bd.nrm[sl], bd.acc[sl]
    nt = nu * sp[:, None]
    t = 2.0 * np.pi * np.arange(N) / N
    R = kress_weights(N, t[:, None] - t[None, :])
    dx = x[:, None, 0] - x[None, :, 0]
    dy = x[:, None, 1] - x[None, :, 1]
    r = np.hypot(dx, dy)
    off = ~np.eye(N, dtype=bool)
    rr = np.where(off, r, 1.0)
    z = kappa * rr
    H0 = np.where(off, hankel1(0, z), 0.0)
    H1 = np.where(off, hankel1(1, z), 0.0)
    J0 = np.where(off, j0(z), 1.0)
    J1r = np.where(off, j1(z) / rr, 0.5 * kappa)          # J1(k r)/r -> k/2
    dnt = dx * nt[None, :, 0] + dy * nt[None, :, 1]        # (x_i - x_j) . nt_j
    dnu = dx * nu[:, None, 0] + dy * nu[:, None, 1]        # (x_i - x_j) . nu_i
    lnk = 0.25j - EULER_C / (2 * np.pi) - np.log(0.5 * kappa * sp) / (2 * np.pi)
    curv = np.einsum("ij,ij->i", acc, nt) / (4 * np.pi * sp ** 2)
    # S
    F = 0.25j * H0 * sp[None, :]
    F1 = -J0 * sp[None, :] / (4 * np.pi)
    S = _split(F, F1, lnk * sp, R, N)
    # D
    F = 0.25j * kappa * H1 * dnt / rr
    F1 = -(kappa / (4 * np.pi)) * J1r * dnt
    D = _split(F, F1, curv, R, N)
    # K
    F = -0.25j * kappa * H1 * dnu / rr * sp[None, :]
    F1 = (kappa / (4 * np.pi)) * J1r * dnu * sp[None, :]
    K = _split(F, F1, curv, R, N)
    # T by Maue's identity
    F = 0.25j * H0
    F1 = -J0 / (4 * np.pi)
    S0 = _split(F, F1, lnk, R, N)
    nn = nu @ nt.T                                         # nu_i . nt_j
    F = 0.25j * H0 * nn
    F1 = -J0 * nn / (4 * np.pi)
    Snu = _split(F, F1, lnk * sp, R, N)
    Dm = diff_matrix(N)
    T = (Dm @ S0 @ Dm) / sp[:, None] + kappa ** 2 * Snu
    return S, D, K, T


def layer_rows(pb: Problem, targets):
    """As system.layer_rows for the Nystrom discretisation: interior (k1,
    own fibre) and exterior (k, every fibre and image) S, D, K, T [len(targets), E]."""
    bd = pb.bd
    targets = np.asarray(targets)
    E, N = bd.E, bd.N
    x = bd.mid[targets]
    nu = bd.nrm[targets]
    dx = x[:, None, 0] - bd.mid[None, :, 0]
    dy = x[:, None, 1] - bd.mid[None, :, 1]
    same = bd.fibre[targets][:, None] == bd.fibre[None, :]
    with np.errstate(divide="ignore", invalid="ignore"):
        ext = list(kernels_sdkt(pb.k, dx, dy, nu[:, None, 0], nu[:, None, 1], bd.nrm[None, :, 0],
                                bd.nrm[None, :, 1]))
    for c in range(4):
        ext[c] = np.where(same, 0.0, ext[c] * bd.h[None, :])
    inn = [np.zeros_like(ext[0]) for _ in range(4)]
    for f in np.unique(bd.fibre[targets]):
        rows = np.nonzero(bd.fibre[targets] == f)[0]
        loc = bd.local[targets[rows]]
        cols = f * N + np.arange(N)
        se = self_matrices(bd, f, pb.k)
        si = self_matrices(bd, f, pb.k1)
        for c in range(4):
            ext[c][np.ix_(rows, cols)] = se[c][loc]
            inn[c][np.ix_(rows, cols)] = si[c][loc]
    if pb.periodic:
        q = choose_q(pb.k, bd.H, bd.L, bd.H)
        per = periodic_offzero_kernels(pb.k, bd.H, pb.theta, x, nu, bd.mid, bd.nrm, q=q, x_max=bd.L, y_max=bd.H)
        for c in range(4):
            ext[c] = ext[c] + per[c] * bd.h[None, :]
    names = "SDKT"
    return ({f"int_{names[c]}": inn[c] for c in range(4)},
            {f"ext_{names[c]}": ext[c] for c in range(4)})


def operator_rows(pb: Problem, targets):
    """Rows of (I - A) of eq. 9 in the Nystrom discretisation for the nodes
    `targets`: (R1, R2), each [len(targets), 2E], the row-1 and row-2
    equations (as system.operator_rows)."""
    bd = pb.bd
    targets = np.asarray(targets)
    inn, ext = layer_rows(pb, targets)
    R1 = np.zeros((len(targets), pb.n), dtype=np.complex128)
    R2 = np.zeros_like(R1)
    c = 2.0 / (1j * pb.eta * (1.0 + pb.varrho))
    allp, allv = col_phi(bd, np.arange(bd.E)), col_varphi(bd, np.arange(bd.E))
    R1[:, allp] = ext["ext_D"] - inn["int_D"]
    R1[:, allv] = -1j * pb.eta * (ext["ext_S"] - inn["int_S"])
    R2[:, allp] = c * (ext["ext_T"] - pb.varrho * inn["int_T"])
    R2[:, allv] = c * (-1j * pb.eta) * (ext["ext_K"] - pb.varrho * inn["int_K"])
    r = np.arange(len(targets))
    R1[r, col_phi(bd, targets)] += 1.0
    R2[r, col_varphi(bd, targets)] += 1.0
    return R1, R2


def dense_matrix(pb: Problem) -> np.ndarray:
    """(I - A) of eq. 9 in the Nystrom discretisation (rows as system.operator_rows)."""
    bd = pb.bd
    tg = np.arange(bd.E)
    R1, R2 = operator_rows(pb, tg)
    A = np.zeros((pb.n, pb.n), dtype=np.complex128)
    A[col_phi(bd, tg)] = R1
    A[col_varphi(bd, tg)] = R2
    return A


def potential(pb: Problem, psi, pts):
    """Scattered field (eq. 4 with eq. 7) at points away from the boundary, by
    the trapezoidal rule at the nodes."""
    bd = pb.bd
    e = np.arange(bd.E)
    phi_d, vphi = psi[col_phi(bd, e)], psi[col_varphi(bd, e)]
    pts = np.asarray(pts, dtype=np.float64)
    dx = pts[:, None, 0] - bd.mid[None, :, 0]
    dy = pts[:, None, 1] - bd.mid[None, :, 1]
    z = np.zeros_like(dx)
    S, D, _, _ = kernels_sdkt(pb.k, dx, dy, z, z, bd.nrm[None, :, 0], bd.nrm[None, :, 1])
    if pb.periodic:
        xm = max(bd.L, float(np.max(np.abs(dx))))
        ym = max(bd.H, float(np.max(np.abs(dy))))
        per = periodic_offzero_kernels(pb.k, bd.H, pb.theta, pts, np.zeros_like(pts), bd.mid, bd.nrm,
                                       x_max=xm, y_max=ym)
        S = S + per[0]
        D = D + per[1]
    return (D * bd.h[None, :]) @ phi_d - 1j * pb.eta * ((S * bd.h[None, :]) @ vphi)
