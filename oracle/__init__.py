"""CPU oracle for the periodic FM-BEM transmission problem.

TEST INFRASTRUCTURE ONLY.  Only ``tests/``, ``__graft_entry__.smoke()`` and
the ``cpu_baseline`` leg of ``bench.py`` may import this package.  The GPU
library never calls it and shares no code with it.

The oracle is the plain, slow definition of what the fast method computes:
the dense FP64 matrix (I - A) of the discrete boundary integral system
(paper Sec. 2, eq. 9) with the exact quasi-periodic exterior kernel, solved
by LU.  The fast multipole method approximates exactly this matrix.

Modules:
  geometry  fibre lattice and chord discretisation
  kernels   free-space Helmholtz kernels S, D, K, T (Sec. 2)
  lattice   quasi-periodic image sums: direct part plus the two Fourier
            integral tails (Sec. 3.3, eqs. 17-18, corrected)
  elements  element integrals: far rule, near rule, self element
  system    dense (I - A), right-hand side B, LU solve
  fields    Bragg amplitudes, energy transmission coefficient (Sec. 4)
  fmmdefs   FMM stage definitions by direct summation (Sec. 3.2)
  warmstart learned warm start: features, MLP with MSE gradients, Adam,
            per-fibre modal transform of the densities (not from the paper)
"""
