"""ctypes binding of the learned warm start (include/pfmwarm.h): argument
marshalling only.

Every arithmetic step runs in libpfmbem.so: features, target statistics and
standardisation, the MLP forward / backward / Adam steps in FP32, the
validation shrink, BF16 inference on the matrix cores, the modal analysis of
solved densities and the synthesis of start vectors.  PyTorch holds the
device memory.  Data generation, the training loop and the evaluation are in
warm_train.py.
"""
from __future__ import annotations

import ctypes
import math
import time
from dataclasses import dataclass
from typing import Dict, List, Optional, Sequence

import numpy as np

from . import pfm

EXPORTS = ["pfm_mlp_create", "pfm_mlp_destroy", "pfm_mlp_set_stream", "pfm_mlp_n_params", "pfm_mlp_buffers",
           "pfm_mlp_get_params", "pfm_mlp_set_params", "pfm_mlp_get_grads", "pfm_mlp_scale_output",
           "pfm_mlp_forward", "pfm_mlp_backward_mse", "pfm_mlp_adam", "pfm_mlp_to_bf16", "pfm_mlp_infer_bf16",
           "pfm_warm_features", "pfm_modes_analyse", "pfm_modes_synthesise", "pfm_mlp_target_stats",
           "pfm_mlp_standardise", "pfm_mlp_validation_shrink"]

SIZES = (5, 256, 256, 256, 2048)      # (ka, theta, r, rho ratio, c ratio) -> 16 fibres x 2 x 32 modes x re/im
N_MODES = 32

_bound = False


def lib():
    global _bound
    L = pfm.lib()
    if _bound:
        return L
    P = ctypes.c_void_p
    fp = ctypes.c_void_p
    L.pfm_mlp_create.argtypes = [ctypes.POINTER(ctypes.c_int), ctypes.c_int, ctypes.c_int, ctypes.c_ulonglong,
                                 ctypes.POINTER(P)]
    L.pfm_mlp_destroy.argtypes = [P]
    L.pfm_mlp_destroy.restype = None
    L.pfm_mlp_set_stream.argtypes = [P, P]
    L.pfm_mlp_n_params.argtypes = [P]
    L.pfm_mlp_n_params.restype = ctypes.c_longlong
    L.pfm_mlp_buffers.argtypes = [P, ctypes.POINTER(fp), ctypes.POINTER(fp)]
    L.pfm_mlp_get_params.argtypes = [P, fp]
    L.pfm_mlp_set_params.argtypes = [P, fp]
    L.pfm_mlp_get_grads.argtypes = [P, fp]
    L.pfm_mlp_scale_output.argtypes = [P, fp, fp]
    L.pfm_mlp_target_stats.argtypes = [P, fp, ctypes.c_int, fp, fp]
    L.pfm_mlp_standardise.argtypes = [P, fp, ctypes.c_int, fp, fp, fp]
    L.pfm_mlp_validation_shrink.argtypes = [P, fp, fp, ctypes.c_int, fp, ctypes.POINTER(ctypes.c_float)]
    L.pfm_mlp_forward.argtypes = [P, fp, ctypes.c_int, fp]
    L.pfm_mlp_backward_mse.argtypes = [P, fp, ctypes.c_int, ctypes.POINTER(ctypes.c_float)]
    L.pfm_mlp_adam.argtypes = [P, ctypes.c_float, ctypes.c_float, ctypes.c_float, ctypes.c_float, ctypes.c_int]
    L.pfm_mlp_to_bf16.argtypes = [P]
    L.pfm_mlp_infer_bf16.argtypes = [P, fp, ctypes.c_int, fp]
    L.pfm_warm_features.argtypes = [fp, ctypes.c_int, fp, P]
    dp = ctypes.POINTER(ctypes.c_double)
    L.pfm_modes_analyse.argtypes = [P, ctypes.c_int, ctypes.c_int, dp, fp, fp]
    L.pfm_modes_synthesise.argtypes = [P, ctypes.c_int, ctypes.c_int, dp, fp, fp]
    _bound = True
    return L


def _ptr(t):
    return ctypes.c_void_p(t.data_ptr())


def _check(code, what):
    if code != 0:
        raise pfm.PfmError(code, what)


class MLP:
    """The warm-start network (FP32 parameters on the device)."""

    def __init__(self, sizes: Sequence[int] = SIZES, max_batch: int = 1024, seed: int = 1):
        import torch
        L = lib()
        self._L = L
        self.sizes = tuple(int(s) for s in sizes)
        self.max_batch = max_batch
        arr = (ctypes.c_int * len(self.sizes))(*self.sizes)
        self._h = ctypes.c_void_p()
        _check(L.pfm_mlp_create(arr, len(self.sizes) - 1, max_batch, seed, ctypes.byref(self._h)), "pfm_mlp_create")
        self.n_params = L.pfm_mlp_n_params(self._h)
        _check(L.pfm_mlp_set_stream(self._h, ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)), "stream")

    def close(self):
        if self._h:
            self._L.pfm_mlp_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def params(self):
        import torch
        p = torch.empty(self.n_params, dtype=torch.float32, device="cuda")
        _check(self._L.pfm_mlp_get_params(self._h, _ptr(p)), "get_params")
        return p

    def set_params(self, p):
        _check(self._L.pfm_mlp_set_params(self._h, _ptr(p.contiguous())), "set_params")

    def grads(self):
        import torch
        g = torch.empty(self.n_params, dtype=torch.float32, device="cuda")
        _check(self._L.pfm_mlp_get_grads(self._h, _ptr(g)), "get_grads")
        return g

    def forward(self, x, out=None):
        import torch
        y = out if out is not None else torch.empty((x.shape[0], self.sizes[-1]), dtype=torch.float32, device="cuda")
        _check(self._L.pfm_mlp_forward(self._h, _ptr(x), x.shape[0], _ptr(y)), "forward")
        return y

    def backward_mse(self, t, want_loss: bool = False) -> Optional[float]:
        loss = ctypes.c_float()
        _check(self._L.pfm_mlp_backward_mse(self._h, _ptr(t), t.shape[0], ctypes.byref(loss) if want_loss else None),
               "backward")
        return loss.value if want_loss else None

    def adam(self, lr: float, t: int, b1: float = 0.9, b2: float = 0.999, eps: float = 1e-8):
        _check(self._L.pfm_mlp_adam(self._h, lr, b1, b2, eps, t), "adam")

    def scale_output(self, scale, shift):
        _check(self._L.pfm_mlp_scale_output(self._h, _ptr(scale), _ptr(shift)), "scale_output")

    def target_stats(self, t):
        """Per-column mean and standard deviation of targets t [n, width]."""
        import torch
        w = self.sizes[-1]
        mean = torch.empty(w, dtype=torch.float32, device="cuda")
        std = torch.empty(w, dtype=torch.float32, device="cuda")
        _check(self._L.pfm_mlp_target_stats(self._h, _ptr(t), t.shape[0], _ptr(mean), _ptr(std)), "target_stats")
        return mean, std

    def standardise(self, t, mean, std):
        import torch
        out = torch.empty_like(t)
        _check(self._L.pfm_mlp_standardise(self._h, _ptr(t), t.shape[0], _ptr(mean), _ptr(std), _ptr(out)),
               "standardise")
        return out

    def validation_shrink(self, x, t):
        """Shrink of the outputs from held-back rows, folded into the last
        layer; returns (shrink, relative error after it)."""
        import torch
        shrink = torch.empty(self.sizes[-1], dtype=torch.float32, device="cuda")
        err = ctypes.c_float()
        _check(self._L.pfm_mlp_validation_shrink(self._h, _ptr(x), _ptr(t), x.shape[0], _ptr(shrink),
                                                 ctypes.byref(err)), "validation_shrink")
        return shrink, err.value

    def to_bf16(self):
        _check(self._L.pfm_mlp_to_bf16(self._h), "to_bf16")

    def infer_bf16(self, x, out=None):
        import torch
        y = out if out is not None else torch.empty((x.shape[0], self.sizes[-1]), dtype=torch.float32, device="cuda")
        _check(self._L.pfm_mlp_infer_bf16(self._h, _ptr(x), x.shape[0], _ptr(y)), "infer_bf16")
        return y


def features(draws):
    """draws: float64 CUDA tensor [B, 5] -> float32 [B, 5] network inputs."""
    import torch
    L = lib()
    x = torch.empty(draws.shape, dtype=torch.float32, device="cuda")
    _check(L.pfm_warm_features(_ptr(draws), draws.shape[0], _ptr(x),
                               ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)), "features")
    return x


def modes_analyse(prob: "pfm.Problem", K: int, thetas, psi):
    import torch
    L = lib()
    th = np.ascontiguousarray(np.asarray(thetas, dtype=np.float64).reshape(-1))
    B = th.size
    vec = torch.empty((B, 4 * prob.M * K), dtype=torch.float32, device="cuda")
    _check(L.pfm_modes_analyse(prob._h, K, B, th.ctypes.data_as(ctypes.POINTER(ctypes.c_double)), _ptr(psi),
                               _ptr(vec)), "modes_analyse")
    return vec


def modes_synthesise(prob: "pfm.Problem", K: int, thetas, vec):
    import torch
    L = lib()
    th = np.ascontiguousarray(np.asarray(thetas, dtype=np.float64).reshape(-1))
    B = th.size
    psi = torch.empty((B, prob.n), dtype=torch.complex128, device="cuda")
    _check(L.pfm_modes_synthesise(prob._h, K, B, th.ctypes.data_as(ctypes.POINTER(ctypes.c_double)),
                                  _ptr(vec.contiguous()), _ptr(psi)), "modes_synthesise")
    return psi
