"""Seeded synthetic inputs shared by the oracle, the tests and the benchmark.

This module only draws and names inputs: lattice type and size, fibre radii,
materials, frequency/angle grids, expansion settings and random density
vectors.  It holds none of the method's arithmetic (no geometry, kernels,
expansions or solves), so that the CPU oracle and the GPU library can both be
fed from it without sharing any computation.

The workloads mirror the phononic-crystal experiments of the paper (Sec. 4):
circular fibres on a square or hexagon lattice, a mercury/water contrast, and
a fundamental block of M_H rows by M_L columns (Sec. 2, eq. 3).
"""
from __future__ import annotations

import dataclasses
import math
from typing import List, Optional

import numpy as np

SQUARE = 0
HEXAGON = 1
CIRCLE = 0
ROUND_SQUARE = 1

# Mercury fibres in water, the contrast used by the benchmark workloads.
MERCURY = dict(rho=13500.0, c=1450.0)
WATER = dict(rho=1000.0, c=1490.0)


@dataclasses.dataclass
class Workload:
    name: str
    lattice: int            # SQUARE or HEXAGON
    a: float                # lattice constant
    M_L: int                # fibre columns (x)
    M_H: int                # fibre rows (y), period H = M_H * a
    n_elem: int             # boundary elements per fibre
    radii: np.ndarray       # [M] fibre radii, fibre f = row * M_L + col
    rho_fiber: float
    c_fiber: float
    rho_matrix: float
    c_matrix: float
    ka: List[float]
    theta: List[float]
    p: int                  # expansion truncation (-p..p)
    leaf_max: int           # max elements per quadtree leaf
    tol: float = 1e-8       # GMRES relative residual
    eta: float = 0.0        # coupling constant; <= 0 means eta = k
    shape: int = 0          # CIRCLE, or ROUND_SQUARE (radii are then the curve's size parameter r)

    @property
    def M(self) -> int:
        return self.M_L * self.M_H

    @property
    def n_unknowns(self) -> int:
        return 2 * self.M * self.n_elem


def _full(M, r):
    return np.full(M, float(r))


def tiny(seed: int = 0) -> Workload:
    """Square lattice, one mercury fibre r=0.3a, 256 elements (512 unknowns),
    ka=2, theta=pi/4, p=16, leaf<=32."""
    return Workload("tiny_square_M1_N256", SQUARE, 1.0, 1, 1, 256, _full(1, 0.3),
                    MERCURY["rho"], MERCURY["c"], WATER["rho"], WATER["c"],
                    [2.0], [math.pi / 4], 16, 32)


def square_8x8(seed: int = 2) -> Workload:
    """Square 8x8 block, radii U[0.2,0.35]a (seeded), 512 elements per fibre:
    32768 elements, 65536 unknowns; p=24, leaf<=64; ka = 32 evenly spaced values
    in [0.5, 6.0] at theta=0; GMRES tolerance 1e-8."""
    rng = np.random.default_rng(seed)
    radii = rng.uniform(0.2, 0.35, size=64)
    return Workload("square_8x8_N512", SQUARE, 1.0, 8, 8, 512, radii,
                    MERCURY["rho"], MERCURY["c"], WATER["rho"], WATER["c"],
                    list(np.linspace(0.5, 6.0, 32)), [0.0], 24, 64)


def hexagon_16x16(seed: int = 3) -> Workload:
    """Hexagon 16x16 block, radii 0.25a(1 +- 2%) (seeded), 256 elements per
    fibre: 65536 elements, 131072 unknowns; p=24, leaf<=64; ka=2, theta=pi/6."""
    rng = np.random.default_rng(seed)
    radii = 0.25 * (1.0 + 0.02 * rng.uniform(-1.0, 1.0, size=256))
    return Workload("hexagon_16x16_N256", HEXAGON, 1.0, 16, 16, 256, radii,
                    MERCURY["rho"], MERCURY["c"], WATER["rho"], WATER["c"],
                    [2.0], [math.pi / 6], 24, 64)


def square_4x4_sweep(seed: int = 4) -> Workload:
    """Square 4x4 block, r=0.3a, 256 elements per fibre (8192 unknowns per
    solve); 64 ka values in [0.2, 8.0] times 8 theta values j*pi/16."""
    return Workload("square_4x4_N256_sweep", SQUARE, 1.0, 4, 4, 256, _full(16, 0.3),
                    MERCURY["rho"], MERCURY["c"], WATER["rho"], WATER["c"],
                    list(np.linspace(0.2, 8.0, 64)), [j * math.pi / 16 for j in range(8)],
                    24, 64)


def small_square(M_L: int = 2, M_H: int = 2, n_elem: int = 64, r: float = 0.3,
                 ka: float = 2.0, theta: float = math.pi / 6, p: int = 16,
                 leaf_max: int = 16, radii: Optional[np.ndarray] = None,
                 lattice: int = SQUARE) -> Workload:
    """Reduced multi-fibre block used for full dense-solve parity."""
    M = M_L * M_H
    rad = _full(M, r) if radii is None else np.asarray(radii, dtype=np.float64)
    return Workload(f"small_{'sq' if lattice == SQUARE else 'hex'}_{M_L}x{M_H}_N{n_elem}",
                    lattice, 1.0, M_L, M_H, n_elem, rad,
                    MERCURY["rho"], MERCURY["c"], WATER["rho"], WATER["c"],
                    [ka], [theta], p, leaf_max)


def random_density(n_unknowns: int, seed: int) -> np.ndarray:
    """Complex128 vector with independent standard normal real/imag parts."""
    rng = np.random.default_rng(seed)
    return rng.standard_normal(n_unknowns) + 1j * rng.standard_normal(n_unknowns)


def warm_start_draws(n: int, seed: int) -> np.ndarray:
    """[n, 5] draws of (ka, theta, radius/a, rho_fiber/rho_matrix, c_fiber/c_matrix)
    uniform over ka in [0.2, 8], theta in [0, pi/2), r in [0.15, 0.4],
    density ratio in [0.5, 20] and speed ratio in [0.5, 2]."""
    rng = np.random.default_rng(seed)
    lo = np.array([0.2, 0.0, 0.15, 0.5, 0.5])
    hi = np.array([8.0, math.pi / 2, 0.4, 20.0, 2.0])
    return lo + (hi - lo) * rng.random((n, 5))


def warm_start_groups(n_groups: int, per_group: int, seed: int):
    """Draws of the warm-start study grouped by geometry and frequency:
    [n_groups, 4] of (ka, r/a, rho_fiber/rho_matrix, c_fiber/c_matrix) uniform
    over the ranges of warm_start_draws, and [n_groups, per_group] angles
    uniform in [0, pi/2); group g with angle j is the draw
    (ka_g, theta_gj, r_g, rho_g, c_g).  The block is a square 4 x 4 of equal
    fibres with 256 elements each, matrix water."""
    rng = np.random.default_rng(seed)
    lo = np.array([0.2, 0.15, 0.5, 0.5])
    hi = np.array([8.0, 0.4, 20.0, 2.0])
    g = lo + (hi - lo) * rng.random((n_groups, 4))
    th = (math.pi / 2) * rng.random((n_groups, per_group))
    return g, th


def warm_start_block(r: float, rho_ratio: float, c_ratio: float) -> Workload:
    """The square 4 x 4 block of the warm-start study for one draw."""
    return Workload("square_4x4_N256_warm", SQUARE, 1.0, 4, 4, 256, _full(16, r),
                    rho_ratio * WATER["rho"], c_ratio * WATER["c"], WATER["rho"], WATER["c"],
                    [], [], 24, 32)


# The liquid phononic crystals of the band-gap experiments (Sec. 4): water
# fibres (rho 1000, c 1500) in a mercury matrix (rho 13600, c 1450), lattice
# constant a = 0.5, M_H = 6 rows by M_L = 4 columns, 256 points per fibre,
# incidence along +x (theta = 0), filling fractions 35 % and 50 %.
WATER_SEC4 = dict(rho=1000.0, c=1500.0)
MERCURY_SEC4 = dict(rho=13600.0, c=1450.0)
BANDGAP_CASES = ("circle_square", "circle_triangle", "round_square_square")


def bandgap_block(case: str, filling: float, n_elem: int = 256, M_L: int = 4, M_H: int = 6,
                  p: int = 24, leaf_max: int = 64) -> Workload:
    """Block of one band-gap case.  The size parameter follows from the
    filling fraction: the fibre area (pi r^2 for a circle, 23 pi r^2 / 2 for
    the round square) over the lattice cell area (a^2 square, sqrt(3)/2 a^2
    for the hexagonal, i.e. triangular, lattice)."""
    a = 0.5
    if case == "circle_square":
        lattice, shape, r = SQUARE, CIRCLE, a * math.sqrt(filling / math.pi)
    elif case == "circle_triangle":
        lattice, shape, r = HEXAGON, CIRCLE, a * math.sqrt(filling * math.sqrt(3.0) / (2.0 * math.pi))
    elif case == "round_square_square":
        lattice, shape, r = SQUARE, ROUND_SQUARE, a * math.sqrt(2.0 * filling / (23.0 * math.pi))
    else:
        raise ValueError(case)
    return Workload(f"bandgap_{case}_ff{int(round(100 * filling))}", lattice, a, M_L, M_H, n_elem,
                    _full(M_L * M_H, r), WATER_SEC4["rho"], WATER_SEC4["c"], MERCURY_SEC4["rho"],
                    MERCURY_SEC4["c"], [], [0.0], p, leaf_max, shape=shape)


def bandgap_frequencies(n: int = 150, f_max: float = 1.5) -> np.ndarray:
    """Normalised frequencies ka / (2 pi) of the ETC sweep, cell-centred on
    (0, f_max] so that none falls on a Wood anomaly of the 6-row block at
    theta = 0 (ka / (2 pi) = j / 6)."""
    return (np.arange(n) + 0.5) * f_max / n
