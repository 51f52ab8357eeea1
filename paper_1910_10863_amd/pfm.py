"""ctypes binding of libpfmbem.so (argument marshalling only).

Device memory and streams come from PyTorch: vectors are complex128 CUDA
tensors of length 2*M*N in the unknown order of eq. (9),
Psi = (phi_1, varphi_1, ..., phi_M, varphi_M).  Every computation runs in
the HIP library; this module has no fallback path.
"""
from __future__ import annotations

import ctypes
import os
from typing import Optional

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libpfmbem.so")
_lib = None

SUPPORTED_P = (8, 12, 16, 20, 24, 32, 40)
CIRCLE = 0
ROUND_SQUARE = 1


class PfmError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"pfmbem error {code}: {msg}")
        self.code = code


class Geometry(ctypes.Structure):
    _fields_ = [("lattice", ctypes.c_int), ("a", ctypes.c_double), ("M_L", ctypes.c_int),
                ("M_H", ctypes.c_int), ("n_elem", ctypes.c_int),
                ("radii", ctypes.POINTER(ctypes.c_double)), ("r0", ctypes.c_double), ("shape", ctypes.c_int)]


class Material(ctypes.Structure):
    _fields_ = [("rho_fiber", ctypes.c_double), ("c_fiber", ctypes.c_double),
                ("rho_matrix", ctypes.c_double), ("c_matrix", ctypes.c_double),
                ("eta", ctypes.c_double)]


class Options(ctypes.Structure):
    _fields_ = [("p", ctypes.c_int), ("leaf_max", ctypes.c_int), ("mac", ctypes.c_double),
                ("g_far", ctypes.c_int), ("restart", ctypes.c_int), ("max_iter", ctypes.c_int),
                ("tol", ctypes.c_double), ("wood_margin", ctypes.c_double),
                ("precision", ctypes.c_int), ("inner_tol", ctypes.c_double),
                ("max_batch", ctypes.c_int), ("use_graph", ctypes.c_int),
                ("p2p_blocks_per_cu", ctypes.c_int), ("p2p_unroll", ctypes.c_int),
                ("store_self_blocks", ctypes.c_int), ("p2p_cached_rows", ctypes.c_int),
                ("direct_lattice_m2l", ctypes.c_int), ("precond", ctypes.c_int),
                ("self_mode", ctypes.c_int), ("tree_on_host", ctypes.c_int),
                ("m2l_vector", ctypes.c_int), ("discretisation", ctypes.c_int),
                ("tree_shape", ctypes.c_int)]


class Info(ctypes.Structure):
    _fields_ = [("status", ctypes.c_int), ("iters", ctypes.c_int), ("matvecs", ctypes.c_int),
                ("rel_residual", ctypes.c_double), ("t_solve_s", ctypes.c_double),
                ("outer", ctypes.c_int), ("fallback", ctypes.c_int), ("matvecs_mixed", ctypes.c_int)]


class Stats(ctypes.Structure):
    _fields_ = [("M", ctypes.c_int), ("N", ctypes.c_int), ("E", ctypes.c_int),
                ("n_unknowns", ctypes.c_int), ("n_cells", ctypes.c_int), ("n_leaves", ctypes.c_int),
                ("depth", ctypes.c_int), ("n_m2l_ext", ctypes.c_int), ("n_m2l_int", ctypes.c_int),
                ("n_near_pairs", ctypes.c_int), ("n_near_entries", ctypes.c_longlong),
                ("n_near_cols", ctypes.c_longlong),
                ("n_root_offsets", ctypes.c_int), ("n_m2l_offsets", ctypes.c_int),
                ("near_bytes", ctypes.c_double), ("k", ctypes.c_double), ("k1", ctypes.c_double),
                ("eta", ctypes.c_double), ("varrho", ctypes.c_double), ("theta", ctypes.c_double),
                ("lattice_q", ctypes.c_int), ("p2p_split", ctypes.c_int), ("n_near_computed", ctypes.c_int),
                ("n_near_stored", ctypes.c_longlong), ("n_near_circulant", ctypes.c_longlong),
                ("p2p_window_leaves", ctypes.c_int), ("p2p_window_max", ctypes.c_int),
                ("lattice_m2l_grid", ctypes.c_int), ("workspace_bytes", ctypes.c_double),
                ("workspace_bound", ctypes.c_int), ("batch_capacity", ctypes.c_int),
                ("n_device_allocs", ctypes.c_longlong), ("device_alloc_bytes", ctypes.c_double),
                ("self_fft", ctypes.c_int), ("tree_on_device", ctypes.c_int), ("spectral_roots", ctypes.c_int),
                ("n_spectral_fibres", ctypes.c_int), ("m2l_mfma_items", ctypes.c_int),
                ("m2l_vector_chunks", ctypes.c_int), ("m2l_mfma_entries", ctypes.c_int),
                ("precond_in_apply", ctypes.c_int)]


CHORDS = 0
NYSTROM = 1
TREE_SQUARE = 0
TREE_TRIANGLE = 1
FP64 = 0
MIXED = 1

MAX_BATCH = 16

EXPORTS = ["pfm_create", "pfm_set_stream", "pfm_set_wave", "pfm_matvec", "pfm_matvec_mixed", "pfm_rhs", "pfm_solve",
           "pfm_precond_apply", "pfm_fields", "pfm_get_stats", "pfm_matvec_timed", "pfm_last_error", "pfm_destroy",
           "pfm_set_batch", "pfm_matvec_batch", "pfm_rhs_batch", "pfm_solve_batch", "pfm_sweep",
           "pfm_matvec_batch_timed", "pfm_workspace_size", "pfm_bind", "pfm_matvec_static",
           "pfm_matvec_stage_timed",
           "pfm_test_bessel", "pfm_test_lattice", "pfm_test_moments", "pfm_test_plan_digest"]


def lib():
    """Load libpfmbem.so; raise if it has not been built."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"{LIB_PATH} is missing: build it with __graft_entry__.build()")
    L = ctypes.CDLL(LIB_PATH)
    P = ctypes.c_void_p
    vp = ctypes.c_void_p
    L.pfm_create.argtypes = [ctypes.POINTER(Geometry), ctypes.POINTER(Material), ctypes.POINTER(Options),
                             ctypes.POINTER(P)]
    L.pfm_set_stream.argtypes = [P, vp]
    L.pfm_set_wave.argtypes = [P, ctypes.c_double, ctypes.c_double]
    L.pfm_matvec.argtypes = [P, vp, vp]
    L.pfm_matvec_mixed.argtypes = [P, vp, vp]
    L.pfm_matvec_static.argtypes = [P, vp, vp]
    L.pfm_workspace_size.argtypes = [P, ctypes.c_int, ctypes.POINTER(ctypes.c_size_t)]
    L.pfm_bind.argtypes = [P, vp, ctypes.c_size_t, vp]
    dp = ctypes.POINTER(ctypes.c_double)
    L.pfm_set_batch.argtypes = [P, ctypes.c_double, ctypes.c_int, dp]
    L.pfm_matvec_batch.argtypes = [P, vp, vp]
    L.pfm_rhs_batch.argtypes = [P, vp]
    L.pfm_solve_batch.argtypes = [P, vp, vp, ctypes.c_int, ctypes.POINTER(Info)]
    L.pfm_sweep.argtypes = [P, ctypes.c_int, dp, ctypes.c_int, dp, vp, ctypes.POINTER(Info)]
    L.pfm_matvec_batch_timed.argtypes = [P, vp, vp, ctypes.c_int, dp, dp]
    L.pfm_matvec_stage_timed.argtypes = [P, vp, ctypes.c_int, ctypes.c_int, dp]
    L.pfm_rhs.argtypes = [P, vp]
    L.pfm_solve.argtypes = [P, vp, vp, ctypes.c_int, ctypes.POINTER(Info)]
    L.pfm_precond_apply.argtypes = [P, vp, vp, ctypes.c_int]
    L.pfm_fields.argtypes = [P, vp, ctypes.c_int, ctypes.POINTER(ctypes.c_double),
                             ctypes.POINTER(ctypes.c_double), ctypes.POINTER(ctypes.c_double),
                             ctypes.POINTER(ctypes.c_double)]
    L.pfm_get_stats.argtypes = [P, ctypes.POINTER(Stats)]
    L.pfm_matvec_timed.argtypes = [P, vp, vp, ctypes.c_int, ctypes.POINTER(ctypes.c_double),
                                   ctypes.POINTER(ctypes.c_double)]
    L.pfm_last_error.argtypes = [P]
    L.pfm_last_error.restype = ctypes.c_char_p
    L.pfm_destroy.argtypes = [P]
    L.pfm_destroy.restype = None
    L.pfm_test_bessel.argtypes = [vp, ctypes.c_int, vp]
    L.pfm_test_lattice.argtypes = [P, ctypes.POINTER(ctypes.c_double), ctypes.POINTER(ctypes.c_double),
                                   ctypes.POINTER(ctypes.c_int)]
    L.pfm_test_moments.argtypes = [P, vp, ctypes.POINTER(ctypes.c_double), ctypes.POINTER(ctypes.c_double),
                                   ctypes.POINTER(ctypes.c_int), ctypes.POINTER(ctypes.c_int)]
    L.pfm_test_plan_digest.argtypes = [P, ctypes.POINTER(ctypes.c_ulonglong)]
    for name in EXPORTS:
        if name not in ("pfm_last_error", "pfm_destroy"):
            getattr(L, name).restype = ctypes.c_int
    _lib = L
    return L


def _ptr(t):
    import torch
    if not (isinstance(t, torch.Tensor) and t.is_cuda):
        raise TypeError("expected a CUDA tensor")
    if not t.is_contiguous():
        raise ValueError("tensor must be contiguous")
    return ctypes.c_void_p(t.data_ptr())


def _dptr(a: np.ndarray):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def _iptr(a: np.ndarray):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_int))


class Problem:
    """One fundamental block of fibres with its FMM plan."""

    def __init__(self, lattice: int, a: float, M_L: int, M_H: int, n_elem: int, radii,
                 rho_fiber: float, c_fiber: float, rho_matrix: float, c_matrix: float, shape: int = CIRCLE,
                 eta: float = 0.0, p: int = 16, leaf_max: int = 32, mac: float = 0.65,
                 g_far: int = 4, restart: int = 200, max_iter: int = 4000, tol: float = 1e-8,
                 wood_margin: float = 0.0, precision: int = FP64, inner_tol: float = 0.0,
                 max_batch: int = 1, use_graph: bool = False, p2p_blocks_per_cu: int = 0, p2p_unroll: int = 0,
                 store_self_blocks: bool = False, p2p_cached_rows: bool = False,
                 direct_lattice_m2l: bool = False, precond: bool = False, self_fft: bool = True,
                 tree_on_host: bool = False, spectral_roots: bool = True, m2l_vector: bool = False,
                 nystrom: bool = False, triangle_tree: bool = False):
        import torch
        L = lib()
        self._L = L
        self._h = ctypes.c_void_p()
        rad = np.ascontiguousarray(np.asarray(radii, dtype=np.float64).reshape(-1))
        self._radii = rad
        geo = Geometry(lattice, a, M_L, M_H, n_elem, _dptr(rad), 0.0, shape)
        mat = Material(rho_fiber, c_fiber, rho_matrix, c_matrix, eta)
        opt = Options(p, leaf_max, mac, g_far, restart, max_iter, tol, wood_margin, precision, inner_tol,
                      max_batch, 1 if use_graph else 0, p2p_blocks_per_cu, p2p_unroll,
                      1 if store_self_blocks else 0, 1 if p2p_cached_rows else 0,
                      1 if direct_lattice_m2l else 0, 1 if precond else 0,
                      (0 if spectral_roots else 2) if self_fft else 1,
                      1 if tree_on_host else 0, 1 if m2l_vector else 0, NYSTROM if nystrom else CHORDS,
                      TREE_TRIANGLE if triangle_tree else TREE_SQUARE)
        code = L.pfm_create(ctypes.byref(geo), ctypes.byref(mat), ctypes.byref(opt), ctypes.byref(self._h))
        if code != 0:
            msg = L.pfm_last_error(self._h).decode() if self._h else "?"
            if self._h:
                L.pfm_destroy(self._h)
            self._h = None
            raise PfmError(code, msg)
        self.n = 2 * M_L * M_H * n_elem
        self.M = M_L * M_H
        self.N = n_elem
        self.p = p
        self.max_batch = max(1, max_batch)
        self.B = 0
        self.set_stream(torch.cuda.current_stream())

    @classmethod
    def from_workload(cls, wl, **kw):
        args = dict(lattice=wl.lattice, a=wl.a, M_L=wl.M_L, M_H=wl.M_H, n_elem=wl.n_elem,
                    radii=wl.radii, rho_fiber=wl.rho_fiber, c_fiber=wl.c_fiber,
                    rho_matrix=wl.rho_matrix, c_matrix=wl.c_matrix, shape=wl.shape, eta=wl.eta, p=wl.p,
                    leaf_max=wl.leaf_max, tol=wl.tol)
        args.update(kw)
        return cls(**args)

    def _check(self, code):
        if code != 0:
            raise PfmError(code, self._L.pfm_last_error(self._h).decode())

    def close(self):
        if self._h:
            self._L.pfm_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def set_stream(self, stream):
        self._stream = stream
        self._check(self._L.pfm_set_stream(self._h, ctypes.c_void_p(stream.cuda_stream)))

    def set_wave(self, ka: float, theta: float):
        self._check(self._L.pfm_set_wave(self._h, float(ka), float(theta)))

    def empty(self):
        import torch
        return torch.empty(self.n, dtype=torch.complex128, device="cuda")

    def matvec(self, psi, out=None):
        if psi.numel() != self.n:
            raise ValueError("psi has the wrong length")
        y = self.empty() if out is None else out
        self._check(self._L.pfm_matvec(self._h, _ptr(psi), _ptr(y)))
        return y

    def matvec_mixed(self, psi, out=None):
        if psi.numel() != self.n:
            raise ValueError("psi has the wrong length")
        y = self.empty() if out is None else out
        self._check(self._L.pfm_matvec_mixed(self._h, _ptr(psi), _ptr(y)))
        return y

    def matvec_static(self, psi, out=None):
        """The apply with its scratch in the library's fixed device array."""
        if psi.numel() != self.n:
            raise ValueError("psi has the wrong length")
        y = self.empty() if out is None else out
        self._check(self._L.pfm_matvec_static(self._h, _ptr(psi), _ptr(y)))
        return y

    def workspace_size(self, batch: int = 0) -> int:
        n = ctypes.c_size_t()
        self._check(self._L.pfm_workspace_size(self._h, int(batch), ctypes.byref(n)))
        return n.value

    def bind(self, workspace=None, stream=None):
        """Move the library's workspace into `workspace` (a uint8 CUDA tensor the
        caller keeps alive), or back into a library-owned block (None)."""
        import torch
        st = torch.cuda.current_stream() if stream is None else stream
        if workspace is None:
            code = self._L.pfm_bind(self._h, None, 0, ctypes.c_void_p(st.cuda_stream))
        else:
            if workspace.dtype != torch.uint8:
                raise TypeError("workspace must be a uint8 tensor")
            code = self._L.pfm_bind(self._h, _ptr(workspace), workspace.numel(), ctypes.c_void_p(st.cuda_stream))
        self._check(code)
        self._stream = st
        self._workspace = workspace

    def rhs(self):
        b = self.empty()
        self._check(self._L.pfm_rhs(self._h, _ptr(b)))
        return b

    @staticmethod
    def _mode(x0, fallback, augment):
        if x0 is None:
            return 0
        return 3 if augment else (2 if fallback else 1)

    def solve(self, b=None, x0=None, raise_on_noconv: bool = False, fallback: bool = False, augment: bool = False):
        """x0: start vector (fallback: replaced by zero when it does not beat
        zero) or, with augment, a guess that augments the first GMRES cycle."""
        import torch
        x = self.empty() if x0 is None else x0.clone()
        info = Info()
        code = self._L.pfm_solve(self._h, _ptr(b) if b is not None else None, _ptr(x),
                                 self._mode(x0, fallback, augment), ctypes.byref(info))
        if code != 0 and (code != 4 or raise_on_noconv):
            self._check(code)
        return x, {"status": info.status, "iters": info.iters, "matvecs": info.matvecs,
                   "rel_residual": info.rel_residual, "t_solve_s": info.t_solve_s, "outer": info.outer,
                   "fallback": info.fallback, "matvecs_mixed": info.matvecs_mixed}

    def precond_apply(self, x, inverse: bool = True, out=None):
        """P^{-1} x (inverse) or P x, P the fibres' free-space self blocks."""
        if x.numel() != self.n:
            raise ValueError("x has the wrong length")
        y = self.empty() if out is None else out
        self._check(self._L.pfm_precond_apply(self._h, _ptr(x), _ptr(y), 1 if inverse else 0))
        return y

    def fields(self, psi, n_orders: int = 10):
        no = 2 * n_orders + 1
        R = np.zeros(2 * no)
        T = np.zeros(2 * no)
        etc = ctypes.c_double()
        en = ctypes.c_double()
        self._check(self._L.pfm_fields(self._h, _ptr(psi), n_orders, _dptr(R), _dptr(T),
                                       ctypes.byref(etc), ctypes.byref(en)))
        return R[0::2] + 1j * R[1::2], T[0::2] + 1j * T[1::2], etc.value, en.value

    def stats(self) -> dict:
        st = Stats()
        self._check(self._L.pfm_get_stats(self._h, ctypes.byref(st)))
        return {f: getattr(st, f) for f, _ in Stats._fields_}

    def stage_timed(self, psi, stage: str, reps: int = 200) -> float:
        """Mean milliseconds of one launch of a chain stage ("p2m", "m2m",
        "m2l", "down_l2p") repeated reps times back to back."""
        ms = ctypes.c_double()
        idx = ["p2m", "m2m", "m2l", "down_l2p"].index(stage)
        self._check(self._L.pfm_matvec_stage_timed(self._h, _ptr(psi), idx, reps, ctypes.byref(ms)))
        return ms.value

    def plan_digest(self) -> list:
        """Eight 64-bit digests of the plan's tree and lists (pfm_test_plan_digest)."""
        out = (ctypes.c_ulonglong * 8)()
        self._check(self._L.pfm_test_plan_digest(self._h, out))
        return list(out)

    def matvec_timed(self, psi, reps: int = 10):
        y = self.empty()
        stage = np.zeros(6)
        tot = ctypes.c_double()
        self._check(self._L.pfm_matvec_timed(self._h, _ptr(psi), _ptr(y), reps, _dptr(stage),
                                             ctypes.byref(tot)))
        names = ["p2m", "m2m", "m2l", "down_l2p", "p2p", "combine"]
        return dict(zip(names, stage.tolist())), tot.value, y

    # ---- batched sweep: B angles at one frequency, vectors [B, n] ----
    def set_batch(self, ka: float, thetas):
        th = np.ascontiguousarray(np.asarray(thetas, dtype=np.float64).reshape(-1))
        self._check(self._L.pfm_set_batch(self._h, float(ka), th.size, _dptr(th)))
        self.B = th.size

    def empty_batch(self):
        import torch
        return torch.empty((self.B, self.n), dtype=torch.complex128, device="cuda")

    def matvec_batch(self, psi, out=None):
        if psi.numel() != self.B * self.n:
            raise ValueError("psi must hold B * n values")
        y = self.empty_batch() if out is None else out
        self._check(self._L.pfm_matvec_batch(self._h, _ptr(psi), _ptr(y)))
        return y

    def rhs_batch(self):
        b = self.empty_batch()
        self._check(self._L.pfm_rhs_batch(self._h, _ptr(b)))
        return b

    @staticmethod
    def _infos(arr):
        return [{"status": i.status, "iters": i.iters, "matvecs": i.matvecs, "rel_residual": i.rel_residual,
                 "t_solve_s": i.t_solve_s, "fallback": i.fallback} for i in arr]

    def solve_batch(self, b=None, x0=None, fallback: bool = False, augment: bool = False):
        x = self.empty_batch() if x0 is None else x0.clone()
        infos = (Info * self.B)()
        code = self._L.pfm_solve_batch(self._h, _ptr(b) if b is not None else None, _ptr(x),
                                       self._mode(x0, fallback, augment), infos)
        if code not in (0, 4, 6):
            self._check(code)
        return x, self._infos(infos)

    def sweep(self, kas, thetas):
        """Solve every (ka, theta) pair; returns x [n_ka, B, n] and infos [n_ka][B]."""
        import torch
        ka = np.ascontiguousarray(np.asarray(kas, dtype=np.float64).reshape(-1))
        th = np.ascontiguousarray(np.asarray(thetas, dtype=np.float64).reshape(-1))
        x = torch.empty((ka.size, th.size, self.n), dtype=torch.complex128, device="cuda")
        infos = (Info * (ka.size * th.size))()
        code = self._L.pfm_sweep(self._h, ka.size, _dptr(ka), th.size, _dptr(th), _ptr(x), infos)
        if code not in (0, 4, 5, 6):
            self._check(code)
        self.B = th.size
        flat = self._infos(infos)
        return x, [flat[i * th.size:(i + 1) * th.size] for i in range(ka.size)]

    def matvec_batch_timed(self, psi, reps: int = 10):
        y = self.empty_batch()
        stage = np.zeros(6)
        tot = ctypes.c_double()
        self._check(self._L.pfm_matvec_batch_timed(self._h, _ptr(psi), _ptr(y), reps, _dptr(stage),
                                                   ctypes.byref(tot)))
        names = ["p2m", "m2m", "m2l", "down_l2p", "p2p", "combine"]
        return dict(zip(names, stage.tolist())), tot.value, y

    # ---- test hooks ----
    def lattice_sums(self):
        st = self.stats()
        nr = st["n_root_offsets"]
        NT = 4 * self.p + 1
        sums = np.zeros(2 * nr * NT)
        offs = np.zeros(2 * nr)
        mr = np.zeros(2 * nr, dtype=np.int32)
        self._check(self._L.pfm_test_lattice(self._h, _dptr(sums), _dptr(offs), _iptr(mr)))
        return (sums[0::2] + 1j * sums[1::2]).reshape(nr, NT), offs.reshape(nr, 2), mr.reshape(nr, 2)

    def moments(self, psi):
        st = self.stats()
        nc = st["n_cells"]
        NP = 2 * self.p + 1
        mom = np.zeros(2 * nc * 2 * NP)
        cen = np.zeros(2 * nc)
        info = np.zeros(4 * nc, dtype=np.int32)
        order = np.zeros(st["E"], dtype=np.int32)
        self._check(self._L.pfm_test_moments(self._h, _ptr(psi), _dptr(mom), _dptr(cen), _iptr(info),
                                             _iptr(order)))
        return ((mom[0::2] + 1j * mom[1::2]).reshape(nc, 2, NP), cen.reshape(nc, 2),
                info.reshape(nc, 4), order)


def bessel01(x):
    """J0, J1, Y0, Y1 of a float64 CUDA tensor, computed by the library's device code."""
    import torch
    out = torch.empty(4 * x.numel(), dtype=torch.float64, device="cuda")
    code = lib().pfm_test_bessel(_ptr(x), x.numel(), _ptr(out))
    if code != 0:
        raise PfmError(code, "pfm_test_bessel failed")
    return out.view(-1, 4)
