"""pfmbem: periodic fast-multipole BEM for 2D acoustic transmission in
periodic fibre media, written for AMD MI355X (gfx950).

The computation lives in the HIP library libpfmbem.so (C ABI in
include/pfmbem.h); `pfm` is its thin ctypes binding.
"""
from .pfm import Problem, PfmError, bessel01, lib, SUPPORTED_P  # noqa: F401
