"""Dense boundary-integral system (I - A) Psi = B (oracle; test infrastructure only).

Follows Sec. 2 of the paper: Kress representation (eqs. 4-5) with the
quasi-periodic exterior potentials (eqs. 7-8) and the row scaling of eq. (9):

  row 1 at x in Gamma_i:
    phi_i - D1 phi_i + i eta S1 varphi_i + sum_j (Dbar2 phi_j - i eta Sbar2 varphi_j) = -u_inc
  row 2 (eq. 6 second line times 2/(i eta (1 + varrho))):
    varphi_i + c [ sum_j (Tbar2 phi_j - i eta Kbar2 varphi_j) - varrho (T1 phi_i - i eta K1 varphi_i) ]
      = (2i / (eta (1 + varrho))) d u_inc / d nu,      c = 2 / (i eta (1 + varrho))

with phi the double-layer and varphi the single-layer density, unknown order
Psi = (phi_1, varphi_1, ..., phi_M, varphi_M) (each block N long, eq. 9),
varrho = rho_matrix / rho_fibre, k = omega / c_matrix, k1 = omega / c_fibre,
incident plane wave u_inc = exp(i k x . d), d = (cos theta, sin theta).

Readings: eta = k unless given (the paper only says 'a real constant');
element integrals as in elements.py; the exterior kernel is the full image
sum: the m = 0 term by the far/near/self rules, every m != 0 by the far rule
with the image sums of lattice.py.  `periodic=False` drops all images
(fibres in free space), used to pin the oracle against the Mie series and
to define the fibres' free-space self blocks (the GMRES preconditioner).
"""
from __future__ import annotations

import dataclasses
import math

import numpy as np
import scipy.linalg

from . import elements as el
from .geometry import Boundary, discretise, gauss_points
from .lattice import choose_q, periodic_offzero_kernels


@dataclasses.dataclass
class Problem:
    bd: Boundary
    k: float
    k1: float
    varrho: float
    eta: float
    theta: float
    G: int = 4
    periodic: bool = True

    @property
    def n(self) -> int:
        return 2 * self.bd.E

    @property
    def alpha(self) -> complex:
        return complex(np.exp(1j * self.k * self.bd.H * math.sin(self.theta)))


def problem_from_workload(wl, ka: float, theta: float, G: int = 4, periodic: bool = True,
                          eta: float | None = None) -> Problem:
    bd = discretise(wl.lattice, wl.a, wl.M_L, wl.M_H, wl.n_elem, wl.radii, getattr(wl, "shape", 0))
    k = ka / wl.a
    k1 = k * wl.c_matrix / wl.c_fiber
    varrho = wl.rho_matrix / wl.rho_fiber
    if eta is None:
        eta = wl.eta if wl.eta > 0 else k
    return Problem(bd, k, k1, varrho, eta, theta, G, periodic)


def col_phi(bd: Boundary, e):
    """Column of the double-layer density of global element e."""
    e = np.asarray(e)
    return 2 * (e // bd.N) * bd.N + (e % bd.N)


def col_varphi(bd: Boundary, e):
    e = np.asarray(e)
    return 2 * (e // bd.N) * bd.N + bd.N + (e % bd.N)


def layer_rows(pb: Problem, targets):
    """Element integrals for target collocation points `targets` against all elements.

    Returns dicts int_[S,D,K,T] (interior, wavenumber k1, same fibre only, zero
    elsewhere) and ext_[S,D,K,T] (exterior, wavenumber k, all images), each
    [len(targets), E]."""
    bd = pb.bd
    targets = np.asarray(targets)
    E, N = bd.E, bd.N
    pts, wts = gauss_points(bd, pb.G)
    x = bd.mid[targets]
    nu = bd.nrm[targets]
    T_ = len(targets)
    same = bd.fibre[targets][:, None] == bd.fibre[None, :]
    dloc = np.abs(bd.local[targets][:, None] - bd.local[None, :])
    dloc = np.minimum(dloc, N - dloc)
    is_self = same & (dloc == 0)
    is_near = same & (dloc >= 1) & (dloc <= el.NEAR_BAND)

    xb = np.broadcast_to(x[:, None, :], (T_, E, 2))
    nub = np.broadcast_to(nu[:, None, :], (T_, E, 2))
    ext = list(el.far_rule(pb.k, xb, nub, pts[None], wts[None], bd.nrm[None]))
    inn = list(el.far_rule(pb.k1, xb, nub, pts[None], wts[None], bd.nrm[None]))

    ti, ej = np.nonzero(is_near)
    if ti.size:
        nr = el.near_rule([pb.k, pb.k1], x[ti], nu[ti], bd.mid[ej], bd.tan[ej], bd.nrm[ej], bd.h[ej])
        for c in range(4):
            ext[c][ti, ej] = nr[0, c]
            inn[c][ti, ej] = nr[1, c]
    ti, ej = np.nonzero(is_self)
    if ti.size:
        se = el.self_terms(pb.k, bd.h[ej])
        si = el.self_terms(pb.k1, bd.h[ej])
        for c in range(4):
            ext[c][ti, ej] = se[c]
            inn[c][ti, ej] = si[c]
    for c in range(4):
        inn[c] = np.where(same, inn[c], 0.0)

    if pb.periodic:
        G = pb.G
        ys = pts.reshape(E * G, 2)
        nys = np.repeat(bd.nrm, G, axis=0)
        q = choose_q(pb.k, bd.H, bd.L, bd.H)
        per = periodic_offzero_kernels(pb.k, bd.H, pb.theta, x, nu, ys, nys, q=q,
                                       x_max=bd.L, y_max=bd.H)
        for c in range(4):
            ext[c] = ext[c] + (per[c].reshape(T_, E, G) * wts[None]).sum(-1)
    names = "SDKT"
    return ({f"int_{names[c]}": inn[c] for c in range(4)},
            {f"ext_{names[c]}": ext[c] for c in range(4)})


def operator_rows(pb: Problem, targets, chunk: int = 0):
    """Rows of (I - A) for the collocation points `targets`.

    Returns (R1, R2), each [len(targets), 2E]: the row-1 and row-2 equations."""
    bd = pb.bd
    targets = np.asarray(targets)
    if chunk <= 0:
        chunk = max(1, int(2_000_000 // (bd.E * pb.G)))
    R1 = np.zeros((len(targets), pb.n), dtype=np.complex128)
    R2 = np.zeros_like(R1)
    c = 2.0 / (1j * pb.eta * (1.0 + pb.varrho))
    allc_phi = col_phi(bd, np.arange(bd.E))
    allc_vphi = col_varphi(bd, np.arange(bd.E))
    for s in range(0, len(targets), chunk):
        tg = targets[s:s + chunk]
        inn, ext = layer_rows(pb, tg)
        r = np.arange(s, s + len(tg))
        R1[np.ix_(r, allc_phi)] = ext["ext_D"] - inn["int_D"]
        R1[np.ix_(r, allc_vphi)] = -1j * pb.eta * (ext["ext_S"] - inn["int_S"])
        R2[np.ix_(r, allc_phi)] = c * (ext["ext_T"] - pb.varrho * inn["int_T"])
        R2[np.ix_(r, allc_vphi)] = c * (-1j * pb.eta) * (ext["ext_K"] - pb.varrho * inn["int_K"])
        R1[r, col_phi(bd, tg)] += 1.0
        R2[r, col_varphi(bd, tg)] += 1.0
    return R1, R2


def dense_matrix(pb: Problem, chunk: int = 0) -> np.ndarray:
    bd = pb.bd
    tg = np.arange(bd.E)
    R1, R2 = operator_rows(pb, tg, chunk)
    A = np.zeros((pb.n, pb.n), dtype=np.complex128)
    A[col_phi(bd, tg)] = R1
    A[col_varphi(bd, tg)] = R2
    return A


def fibre_self_blocks(pb: Problem) -> np.ndarray:
    """Blocks of the block-Jacobi preconditioner of GMRES (Sec. 4 names the
    solver a preconditioned GMRES): for each fibre f, its free-space self
    block of (I - A), the rows and columns of its own densities with every
    periodic image left out (and so independent of theta).  Returns
    [M, 2N, 2N], rows and columns in the order (phi_f, varphi_f) of Psi."""
    free = dataclasses.replace(pb, periodic=False)
    bd = pb.bd
    N = bd.N
    out = np.zeros((bd.M, 2 * N, 2 * N), dtype=np.complex128)
    for f in range(bd.M):
        e = f * N + np.arange(N)
        R1, R2 = operator_rows(free, e)
        cols = np.concatenate([col_phi(bd, e), col_varphi(bd, e)])
        out[f, :N] = R1[:, cols]
        out[f, N:] = R2[:, cols]
    return out


def precond_apply(pb: Problem, x, inverse: bool = True, blocks=None) -> np.ndarray:
    """P^{-1} x (inverse) or P x for the block-diagonal P of fibre_self_blocks."""
    if blocks is None:
        blocks = fibre_self_blocks(pb)
    N = pb.bd.N
    x = np.asarray(x, dtype=np.complex128)
    y = np.empty_like(x)
    for f in range(pb.bd.M):
        seg = slice(2 * f * N, 2 * f * N + 2 * N)
        y[seg] = np.linalg.solve(blocks[f], x[seg]) if inverse else blocks[f] @ x[seg]
    return y


def rhs(pb: Problem) -> np.ndarray:
    """B of eq. (9): (-u_inc, 2i/(eta(1+varrho)) du_inc/dnu) per fibre."""
    bd = pb.bd
    d = np.array([math.cos(pb.theta), math.sin(pb.theta)])
    uinc = np.exp(1j * pb.k * (bd.mid @ d))
    dn = 1j * pb.k * (bd.nrm @ d) * uinc
    B = np.zeros(pb.n, dtype=np.complex128)
    e = np.arange(bd.E)
    B[col_phi(bd, e)] = -uinc
    B[col_varphi(bd, e)] = 2j / (pb.eta * (1.0 + pb.varrho)) * dn
    return B


def solve(pb: Problem, A=None, B=None):
    """Dense LU solve of (I - A) Psi = B.  Returns (Psi, A, B)."""
    if A is None:
        A = dense_matrix(pb)
    if B is None:
        B = rhs(pb)
    lu = scipy.linalg.lu_factor(A)
    return scipy.linalg.lu_solve(lu, B), A, B


def split_density(pb: Problem, psi):
    """Psi -> (phi [E], varphi [E]) in global element order."""
    bd = pb.bd
    e = np.arange(bd.E)
    return psi[col_phi(bd, e)], psi[col_varphi(bd, e)]


def potential(pb: Problem, psi, pts, exterior: bool = True):
    """Field at points off the boundary: u_s (exterior, all images) or the
    interior field of the fibres (eqs. 4-5), by the far rule."""
    bd = pb.bd
    phi_d, vphi = split_density(pb, psi)
    gp, gw = gauss_points(bd, 16)
    pts = np.asarray(pts, dtype=np.float64)
    kap = pb.k if exterior else pb.k1
    dx = pts[:, None, None, 0] - gp[None, :, :, 0]
    dy = pts[:, None, None, 1] - gp[None, :, :, 1]
    z = np.zeros_like(dx)
    from .kernels import kernels_sdkt
    S, D, _, _ = kernels_sdkt(kap, dx, dy, z, z, bd.nrm[None, :, None, 0], bd.nrm[None, :, None, 1])
    if exterior and pb.periodic:
        from .lattice import periodic_offzero_kernels
        G = gp.shape[1]
        ys = gp.reshape(-1, 2)
        nys = np.repeat(bd.nrm, G, axis=0)
        xm = max(bd.L, float(np.max(np.abs(dx))))
        ym = max(bd.H, float(np.max(np.abs(dy))))
        per = periodic_offzero_kernels(pb.k, bd.H, pb.theta, pts, np.zeros_like(pts), ys, nys,
                                       x_max=xm, y_max=ym)
        S = S + per[0].reshape(S.shape)
        D = D + per[1].reshape(S.shape)
    Se = (S * gw[None]).sum(-1)
    De = (D * gw[None]).sum(-1)
    return De @ phi_d - 1j * pb.eta * (Se @ vphi)
