"""Fibre lattice and boundary discretisation (oracle; test infrastructure only).

Fundamental block (Sec. 2, eq. 3; Fig. 1): M_H rows by M_L columns of fibres,
periodic along y with period H = M_H * a, quasi-periodic phase
alpha = exp(i k H sin(theta)).

Readings where the paper is silent:
  * Square lattice: centre of fibre (col i, row j) at ((i+1/2)a, (j+1/2)a).
  * Hexagon lattice (figure missing): columns at x_i = (i+1/2)(sqrt(3)/2)a,
    rows at y = (j + 1/2 + (i mod 2)/2) a, so H = M_H a, L = M_L (sqrt(3)/2) a.
  * Fibre index f = j * M_L + i.
  * Each boundary is cut into N straight chords between nodes
    c + gamma(r, t_e), t_e = 2 pi e / N (counter-clockwise), with
    piecewise-constant densities and collocation at chord midpoints; the
    outward normal of a chord with unit tangent t is (t_y, -t_x).
  * Boundary curves gamma: the circle r (cos t, sin t), and the round square
    of Sec. 4, r ((3 + 2 sin^2 t) cos t, (3 + 2 cos^2 t) sin t).
"""
from __future__ import annotations

import dataclasses
import math

import numpy as np

SQUARE = 0
HEXAGON = 1
CIRCLE = 0
ROUND_SQUARE = 1


def boundary_curve(shape: int, r: float, t):
    """Points gamma(r, t) of a fibre's boundary relative to its centre."""
    t = np.asarray(t, dtype=np.float64)
    if shape == CIRCLE:
        return np.stack([r * np.cos(t), r * np.sin(t)], axis=-1)
    if shape == ROUND_SQUARE:
        # Sec. 4: the round-square scatterer
        return np.stack([r * (3.0 + 2.0 * np.sin(t) ** 2) * np.cos(t),
                         r * (3.0 + 2.0 * np.cos(t) ** 2) * np.sin(t)], axis=-1)
    raise ValueError("shape must be CIRCLE or ROUND_SQUARE")


def fibre_centres(lattice: int, a: float, M_L: int, M_H: int):
    """Centres [M, 2] and the block size (L, H)."""
    cs = np.zeros((M_L * M_H, 2))
    for j in range(M_H):
        for i in range(M_L):
            f = j * M_L + i
            if lattice == SQUARE:
                cs[f] = ((i + 0.5) * a, (j + 0.5) * a)
            elif lattice == HEXAGON:
                cs[f] = ((i + 0.5) * math.sqrt(3.0) / 2.0 * a,
                         (j + 0.5 + 0.5 * (i % 2)) * a)
            else:
                raise ValueError("lattice must be SQUARE or HEXAGON")
    if lattice == SQUARE:
        L = M_L * a
    else:
        L = M_L * math.sqrt(3.0) / 2.0 * a
    return cs, L, M_H * a


@dataclasses.dataclass
class Boundary:
    """Chord elements of all fibres, in fibre-major natural order."""
    M: int
    N: int                 # elements per fibre
    centres: np.ndarray    # [M, 2]
    radii: np.ndarray      # [M]
    L: float
    H: float
    a_pt: np.ndarray       # [E, 2] chord start node
    b_pt: np.ndarray       # [E, 2] chord end node
    mid: np.ndarray        # [E, 2] collocation point
    tan: np.ndarray        # [E, 2] unit tangent (a -> b)
    nrm: np.ndarray        # [E, 2] outward unit normal
    h: np.ndarray          # [E] chord length
    fibre: np.ndarray      # [E] fibre index of each element
    local: np.ndarray      # [E] element index within its fibre

    @property
    def E(self) -> int:
        return self.M * self.N


def discretise(lattice: int, a: float, M_L: int, M_H: int, N: int, radii, shape: int = CIRCLE) -> Boundary:
    centres, L, H = fibre_centres(lattice, a, M_L, M_H)
    M = M_L * M_H
    radii = np.asarray(radii, dtype=np.float64).reshape(M)
    t = 2.0 * np.pi * np.arange(N) / N
    t1 = 2.0 * np.pi * (np.arange(N) + 1) / N
    a_pt = np.zeros((M * N, 2))
    b_pt = np.zeros((M * N, 2))
    for f in range(M):
        c, r = centres[f], radii[f]
        a_pt[f * N:(f + 1) * N] = c + boundary_curve(shape, r, t)
        b_pt[f * N:(f + 1) * N] = c + boundary_curve(shape, r, t1)
    d = b_pt - a_pt
    h = np.hypot(d[:, 0], d[:, 1])
    tan = d / h[:, None]
    nrm = np.stack([tan[:, 1], -tan[:, 0]], axis=1)
    mid = 0.5 * (a_pt + b_pt)
    fibre = np.repeat(np.arange(M), N)
    local = np.tile(np.arange(N), M)
    return Boundary(M, N, centres, radii, L, H, a_pt, b_pt, mid, tan, nrm, h, fibre, local)


def gauss_points(bd: Boundary, G: int):
    """G-point Gauss-Legendre nodes on every chord: points [E, G, 2], weights [E, G]."""
    xi, w = np.polynomial.legendre.leggauss(G)
    pts = bd.mid[:, None, :] + 0.5 * bd.h[:, None, None] * xi[None, :, None] * bd.tan[:, None, :]
    wts = 0.5 * bd.h[:, None] * w[None, :]
    return pts, wts
