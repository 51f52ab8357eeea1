"""Write the stored dense-LU solutions that the GPU parity tests compare with.

Each file holds the solution Psi of (I - A) Psi = B (eq. 9) for one block and
one (ka, theta), computed by the oracle alone: the dense FP64 matrix with the
exact quasi-periodic kernel and an LU solve.  The blocks are too large for the
oracle to assemble inside a test (minutes of CPU time), so the solutions are
stored once.  Run from the repository root:

    python tests/golden/make_golden.py square_2x2_N512     # about 2 minutes
    python tests/golden/make_golden.py square_4x4_N256     # about 15 minutes

Only `oracle/` and `workloads.py` (seeded inputs) are used.
"""
from __future__ import annotations

import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

import workloads as W  # noqa: E402
from oracle import system as sy  # noqa: E402


def golden_cases():
    """name -> (workload, [(ka, theta), ...]).  The 2 x 2 block takes four
    fibres of the square 8x8 benchmark block (radii from its seed, 512
    elements per fibre, p = 24, leaf 64) at the frequency of that block's
    sweep that the apply benchmark uses (ka = 3.339, theta = 0; Wood margin
    0.063 for the 2 x 2 period); the 4 x 4 block is the band-sweep block
    (r = 0.3a, 256 elements per fibre) at two angles of one frequency of its
    grid (ka = 4.41, theta = pi/16 and 3 pi/16; Wood margins 0.26 and 0.25)."""
    w8 = W.square_8x8()
    sw = W.square_4x4_sweep()
    return {
        "square_2x2_N512": (W.small_square(2, 2, 512, radii=w8.radii[[0, 1, 8, 9]], p=24, leaf_max=64),
                            [(float(w8.ka[16]), 0.0)]),
        "square_4x4_N256": (sw, [(float(sw.ka[34]), float(sw.theta[1])), (float(sw.ka[34]), float(sw.theta[3]))]),
    }


def path(name: str) -> str:
    return os.path.join(HERE, name + ".npz")


def make(name: str) -> None:
    wl, waves = golden_cases()[name]
    sols, kas, ths = [], [], []
    for ka, th in waves:
        t = time.time()
        pb = sy.problem_from_workload(wl, ka, th)
        psi, _, _ = sy.solve(pb)
        sols.append(psi)
        kas.append(ka)
        ths.append(th)
        print(f"{name}: ka={ka:.6f} theta={th:.6f} solved in {time.time() - t:.1f} s", flush=True)
    np.savez(path(name), psi=np.stack(sols), ka=np.array(kas), theta=np.array(ths),
             radii=np.asarray(wl.radii), n_elem=wl.n_elem, M_L=wl.M_L, M_H=wl.M_H)


if __name__ == "__main__":
    for n in sys.argv[1:] or list(golden_cases()):
        make(n)
