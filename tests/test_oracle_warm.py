"""Pins of the warm-start oracle: gradients against central differences, the
least-squares stationarity of a linear layer, the first Adam step in closed
form, and the modal transform against its defining properties."""
import math

import numpy as np
import pytest

from oracle import warmstart as ws


def _flat(params):
    return np.concatenate([np.concatenate([W.ravel(), b]) for W, b in params])


def _unflat(v, sizes):
    out, o = [], 0
    for a, b in zip(sizes[:-1], sizes[1:]):
        W = v[o:o + a * b].reshape(b, a)
        o += a * b
        out.append((W, v[o:o + b]))
        o += b
    return out


@pytest.mark.parametrize("sizes", [(3, 4, 5), (5, 6, 6, 6, 7)])
def test_gradients_match_central_differences(sizes):
    rng = np.random.default_rng(1)
    params = ws.init_params(sizes, 2)
    X = rng.standard_normal((9, sizes[0]))
    T = rng.standard_normal((9, sizes[-1]))
    _, grads = ws.mse_and_grads(params, X, T)
    g = _flat([(dW, db) for dW, db in grads])
    v0 = _flat(params)
    h = 1e-6
    num = np.zeros_like(v0)
    for i in range(v0.size):
        vp, vm = v0.copy(), v0.copy()
        vp[i] += h
        vm[i] -= h
        num[i] = (ws.mse_and_grads(_unflat(vp, sizes), X, T)[0] -
                  ws.mse_and_grads(_unflat(vm, sizes), X, T)[0]) / (2 * h)
    assert np.max(np.abs(num - g)) < 1e-8 * max(1.0, np.max(np.abs(g)))


def test_linear_layer_is_stationary_at_least_squares():
    rng = np.random.default_rng(3)
    X = rng.standard_normal((40, 5))
    T = rng.standard_normal((40, 3))
    Xa = np.hstack([X, np.ones((40, 1))])
    sol, *_ = np.linalg.lstsq(Xa, T, rcond=None)
    params = [(sol[:5].T.copy(), sol[5].copy())]
    loss, grads = ws.mse_and_grads(params, X, T)
    assert np.max(np.abs(grads[0][0])) < 1e-13 and np.max(np.abs(grads[0][1])) < 1e-13
    # the loss is the mean squared least-squares residual
    assert abs(loss - np.mean((Xa @ sol - T) ** 2)) < 1e-14


def test_first_adam_step_is_lr_times_sign():
    g = np.array([3.0, -1e-3, 2.5e-4, -7.0])
    p, m, v = ws.adam(np.zeros(4), g, np.zeros(4), np.zeros(4), 1, lr=0.01, eps=0.0)
    assert np.allclose(p, -0.01 * np.sign(g), rtol=0, atol=1e-15)
    assert np.allclose(m, 0.1 * g) and np.allclose(v, 0.001 * g * g)


def test_features_map_ranges_to_unit_interval():
    f = ws.features(np.stack([ws.LO, ws.HI, 0.5 * (ws.LO + ws.HI)]))
    assert np.allclose(f, [[-1] * 5, [1] * 5, [0] * 5], atol=1e-15)


def test_modes_of_a_single_harmonic_and_round_trip():
    M, N, K = 3, 64, 16
    k, th = 2.3, 0.4
    cen = np.array([[0.5, 0.5], [1.5, 0.5], [0.5, 1.5]])
    e = np.arange(N)
    ph = ws.incident_phase(k, th, cen)
    psi = np.zeros((M, 2, N), complex)
    psi[1, 0] = 2.0 * np.exp(2j * np.pi * 5 * e / N) * ph[1]          # mode +5 of phi_2
    psi[2, 1] = -1j * np.exp(-2j * np.pi * 8 * e / N) * ph[2]         # mode -8 of varphi_3
    c = ws.density_modes(psi.ravel(), M, N, K, k, th, cen)
    ref = np.zeros((M, 2, K), complex)
    ref[1, 0, 5 + K // 2] = 2.0
    ref[2, 1, -8 + K // 2] = -1j
    assert np.max(np.abs(c - ref)) < 1e-14
    # band-limited densities are reproduced exactly
    rng = np.random.default_rng(4)
    cr = rng.standard_normal((M, 2, K)) + 1j * rng.standard_normal((M, 2, K))
    back = ws.density_modes(ws.modes_density(cr, M, N, K, k, th, cen), M, N, K, k, th, cen)
    assert np.max(np.abs(back - cr)) < 1e-13
    # the analysis agrees with the FFT of the de-rotated densities
    x = (rng.standard_normal(2 * M * N) + 1j * rng.standard_normal(2 * M * N)).reshape(M, 2, N)
    cx = ws.density_modes(x.ravel(), M, N, K, k, th, cen)
    fx = np.fft.fft(x / ph[:, None, None], axis=-1) / N
    idx = np.arange(-K // 2, K // 2) % N
    assert np.max(np.abs(cx - fx[..., idx])) < 1e-14


def test_vector_layout_round_trip():
    rng = np.random.default_rng(5)
    c = rng.standard_normal((4, 2, 8)) + 1j * rng.standard_normal((4, 2, 8))
    v = ws.modes_to_vector(c)
    assert v.shape == (4 * 2 * 8 * 2,)
    assert v[0] == c[0, 0, 0].real and v[1] == c[0, 0, 0].imag and v[2] == c[0, 0, 1].real
    assert np.array_equal(ws.vector_to_modes(v, 4, 8), c)
