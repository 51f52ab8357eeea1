"""Learned warm start, plain definitions (oracle; test infrastructure only).

The warm start maps the parameters of a solve to the low Fourier modes of
the solution densities of every fibre and seeds GMRES with the synthesised
densities.  Nothing here comes from the paper: the network, the modal
representation and the training are this project's own choices, written as
their textbook definitions so that the GPU kernels can be checked against
them:

  features   (ka, theta, r/a, rho_f/rho_m, c_f/c_m) scaled to [-1, 1] by the
             sampling ranges
  mlp        multilayer perceptron h_{l+1} = tanh(W_l h_l + b_l) on the hidden
             layers, linear output layer; W_l is [out, in], row-major
  mse        L = (1 / (B n_out)) sum (y - t)^2 over a batch of B rows,
             gradients by the chain rule written out layer by layer
  adam       the update of Kingma & Ba (2015) with bias correction
  modes      per fibre f and density s (phi, varphi), with the incident
             phase at the fibre centre removed,
               c_{f,s,n} = (1/N) sum_e psi_{f,s}(e) e^{-2 pi i n e / N} e^{-i k c_f.d},
             n = -K/2 .. K/2 - 1, and the synthesis
               psi_{f,s}(e) = e^{i k c_f.d} sum_n c_{f,s,n} e^{2 pi i n e / N}
             network output layout: [f][s][n][re, im].
"""
from __future__ import annotations

import math
from typing import List, Sequence, Tuple

import numpy as np

LO = np.array([0.2, 0.0, 0.15, 0.5, 0.5])
HI = np.array([8.0, math.pi / 2, 0.4, 20.0, 2.0])


def features(draws: np.ndarray) -> np.ndarray:
    """[B, 5] raw draws -> [B, 5] inputs in [-1, 1]."""
    return 2.0 * (np.asarray(draws, dtype=np.float64) - LO) / (HI - LO) - 1.0


def init_params(sizes: Sequence[int], seed: int) -> List[Tuple[np.ndarray, np.ndarray]]:
    """Uniform(-1/sqrt(in), 1/sqrt(in)) weights and biases (the usual default)."""
    rng = np.random.default_rng(seed)
    out = []
    for a, b in zip(sizes[:-1], sizes[1:]):
        s = 1.0 / math.sqrt(a)
        out.append((rng.uniform(-s, s, (b, a)), rng.uniform(-s, s, b)))
    return out


def forward(params, X: np.ndarray) -> List[np.ndarray]:
    """Activations [X, h_1, ..., y]; tanh on every layer but the last."""
    acts = [np.asarray(X, dtype=np.float64)]
    for li, (W, b) in enumerate(params):
        z = acts[-1] @ W.T + b
        acts.append(np.tanh(z) if li < len(params) - 1 else z)
    return acts


def mse_and_grads(params, X: np.ndarray, T: np.ndarray):
    """Loss and [(dW, db)] per layer, by backpropagation."""
    acts = forward(params, X)
    y = acts[-1]
    Bn = y.shape[0] * y.shape[1]
    loss = float(np.sum((y - T) ** 2) / Bn)
    d = 2.0 * (y - T) / Bn                 # dL/dz of the linear output layer
    grads = [None] * len(params)
    for li in range(len(params) - 1, -1, -1):
        W, _ = params[li]
        h = acts[li]
        grads[li] = (d.T @ h, d.sum(axis=0))
        if li > 0:
            d = (d @ W) * (1.0 - acts[li] ** 2)     # through tanh of layer li
    return loss, grads


def adam(param: np.ndarray, grad: np.ndarray, m: np.ndarray, v: np.ndarray, t: int,
         lr: float, b1: float = 0.9, b2: float = 0.999, eps: float = 1e-8):
    """One Adam step (t >= 1); returns the new (param, m, v)."""
    m = b1 * m + (1.0 - b1) * grad
    v = b2 * v + (1.0 - b2) * grad * grad
    mh = m / (1.0 - b1 ** t)
    vh = v / (1.0 - b2 ** t)
    return param - lr * mh / (np.sqrt(vh) + eps), m, v


def incident_phase(k: float, theta: float, centres: np.ndarray) -> np.ndarray:
    """e^{i k c_f . d} per fibre, d = (cos theta, sin theta)."""
    c = np.asarray(centres, dtype=np.float64).reshape(-1, 2)
    return np.exp(1j * k * (c[:, 0] * math.cos(theta) + c[:, 1] * math.sin(theta)))


def density_modes(psi: np.ndarray, M: int, N: int, K: int, k: float, theta: float,
                  centres: np.ndarray) -> np.ndarray:
    """[M, 2, K] modal coefficients of Psi (order of eq. 9: phi_f, varphi_f per fibre)."""
    P = np.asarray(psi).reshape(M, 2, N)
    e = np.arange(N)
    n = np.arange(-K // 2, K // 2)
    F = np.exp(-2j * np.pi * np.outer(n, e) / N) / N          # [K, N]
    c = np.einsum("kn,fsn->fsk", F, P)
    return c / incident_phase(k, theta, centres)[:, None, None]


def modes_density(coef: np.ndarray, M: int, N: int, K: int, k: float, theta: float,
                  centres: np.ndarray) -> np.ndarray:
    """Psi [2 M N] from [M, 2, K] coefficients."""
    c = np.asarray(coef).reshape(M, 2, K) * incident_phase(k, theta, centres)[:, None, None]
    e = np.arange(N)
    n = np.arange(-K // 2, K // 2)
    G = np.exp(2j * np.pi * np.outer(e, n) / N)               # [N, K]
    return np.einsum("nk,fsk->fsn", G, c).reshape(-1)


def modes_to_vector(coef: np.ndarray) -> np.ndarray:
    """[M, 2, K] complex -> network layout [M*2*K*2] real ([f][s][n][re, im])."""
    c = np.asarray(coef)
    return np.stack([c.real, c.imag], axis=-1).reshape(-1)


def vector_to_modes(v: np.ndarray, M: int, K: int) -> np.ndarray:
    a = np.asarray(v, dtype=np.float64).reshape(M, 2, K, 2)
    return a[..., 0] + 1j * a[..., 1]
