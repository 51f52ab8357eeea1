"""GPU parity of the spectral Nystrom discretisation (PFM_NYSTROM) against
the oracle's Nystrom system, through the C ABI.

The device path changes only the geometry (nodes instead of chord
midpoints), the point rule for every smooth kernel, and the circulant rows of
each fibre's own block (Kress's logarithmic splitting, T by Maue's identity
with the trigonometric differentiation done in Fourier space); the tree, the
roots by Fourier modes, the matrix-core M2L and GMRES are the element
method's.  Checked: the apply against the dense Nystrom matrix (separated and
close fibres, square and hexagonal blocks, both forms of the roots), the
GMRES solution against LU, the Bragg amplitudes and flux balance against the
oracle's, and the spectral accuracy against the multiple scattering solution
of the same array of circles.
"""
import functools
import math
import sys

import numpy as np
import pytest

import workloads as W

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


def _say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def pfm():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1910_10863_amd import pfm as m
    m.lib()
    return m


_WL = {
    "tiny": (W.tiny, 2.0, math.pi / 4),
    "sq2x2": (lambda: W.small_square(2, 2, 32, 0.3, 2.0, math.pi / 6), 2.0, math.pi / 6),
    "hex2x2": (lambda: W.small_square(2, 2, 32, 0.3, 3.0, 0.3, lattice=W.HEXAGON), 3.0, 0.3),
    "sq2x1radii": (lambda: W.small_square(2, 1, 64, radii=np.array([0.3, 0.22])), 4.0, 0.7),
    # close fibres: stored near blocks between neighbours and across the
    # periodic boundary, point rule there too
    "sq2x2close": (lambda: W.small_square(2, 2, 64, 0.45, 2.0, 0.4), 2.0, 0.4),
}


def _wl(key, n_elem=None):
    make, ka, th = _WL[key]
    wl = make()
    if n_elem is not None:
        wl.n_elem = n_elem
    return wl, ka, th


@functools.lru_cache(maxsize=8)
def _oracle(key, n_elem=None):
    from oracle import nystrom as ny
    from oracle import system as sy
    wl, ka, th = _wl(key, n_elem)
    pb = ny.problem_from_workload(wl, ka, th)
    A = ny.dense_matrix(pb)
    return pb, A, sy.rhs(pb)


def _gpu(pfm, key, n_elem=None, p=40, leaf=16, **kw):
    wl, ka, th = _wl(key, n_elem)
    prob = pfm.Problem.from_workload(wl, p=p, leaf_max=leaf, nystrom=True, **kw)
    prob.set_wave(ka, th)
    return prob


@pytest.mark.parametrize("spectral", [True, False])
@pytest.mark.parametrize("key", ["tiny", "sq2x2", "hex2x2", "sq2x1radii", "sq2x2close"])
def test_nystrom_matvec_vs_dense_oracle(pfm, key, spectral):
    pb, A, B = _oracle(key)
    _say("nystrom matvec:", key, "spectral roots:", spectral)
    prob = _gpu(pfm, key, spectral_roots=spectral)
    st = prob.stats()
    assert st["self_fft"] == 1 and st["n_near_circulant"] == 0
    psi = W.random_density(prob.n, 7)
    y = prob.matvec(torch.tensor(psi, device="cuda")).cpu().numpy()
    ref = A @ psi
    err = np.linalg.norm(y - ref) / np.linalg.norm(ref)
    _say("  rel err", err, "near pairs", st["n_near_pairs"], "spectral fibres", st["n_spectral_fibres"])
    if key == "sq2x2close":
        assert st["n_near_pairs"] > 0
    assert err < 1e-10


def test_nystrom_rhs_and_self_rows(pfm):
    """The right-hand side at the nodes, and the own block's rows alone
    (one fibre, no neighbours within reach but its images)."""
    pb, A, B = _oracle("tiny")
    prob = _gpu(pfm, "tiny")
    b = prob.rhs().cpu().numpy()
    assert np.linalg.norm(b - B) < 1e-13 * np.linalg.norm(B)
    # unit vectors: columns of (I - A)
    for j in (0, 5, 64 + 3):
        e = np.zeros(prob.n, dtype=np.complex128)
        e[j] = 1.0
        col = prob.matvec(torch.tensor(e, device="cuda")).cpu().numpy()
        err = np.max(np.abs(col - A[:, j])) / np.max(np.abs(A[:, j]))
        assert err < 1e-10, (j, err)


@pytest.mark.parametrize("key", ["tiny", "sq2x2", "hex2x2"])
def test_nystrom_solve_vs_dense_lu(pfm, key):
    pb, A, B = _oracle(key)
    ref = np.linalg.solve(A, B)
    _say("nystrom solve:", key)
    prob = _gpu(pfm, key, tol=1e-12, restart=100)
    x, info = prob.solve()
    _say("  ", info)
    assert info["status"] == 0
    err = np.linalg.norm(x.cpu().numpy() - ref) / np.linalg.norm(ref)
    assert err < 1e-9


def test_nystrom_preconditioned_solve(pfm):
    """The block-Jacobi preconditioner built from the Nystrom own blocks:
    P^{-1} P x = x, and the preconditioned solve reaches LU's solution."""
    pb, A, B = _oracle("sq2x2")
    ref = np.linalg.solve(A, B)
    prob = _gpu(pfm, "sq2x2", tol=1e-12, restart=100, precond=True)
    x = torch.tensor(W.random_density(prob.n, 3), device="cuda")
    back = prob.precond_apply(prob.precond_apply(x, inverse=False), inverse=True)
    assert torch.linalg.norm(back - x) < 1e-12 * torch.linalg.norm(x)
    # P is the own blocks of (I - A) at wavenumbers k and k1 without images:
    # on one fibre's rows and columns, the free-space Nystrom self block
    from oracle import nystrom as ny
    wl, ka, th = _wl("sq2x2")
    fb = ny.problem_from_workload(wl, ka, th, periodic=False)
    Af = ny.dense_matrix(fb)
    N = wl.n_elem
    idx = np.arange(2 * N)                      # fibre 0's phi, then its varphi
    v = np.zeros(prob.n, dtype=np.complex128)
    v[idx] = W.random_density(2 * N, 4)
    Pv = prob.precond_apply(torch.tensor(v, device="cuda"), inverse=False).cpu().numpy()
    refv = Af[np.ix_(idx, idx)] @ v[idx]
    assert np.linalg.norm(Pv[idx] - refv) < 1e-10 * np.linalg.norm(refv)
    sol, info = prob.solve()
    assert info["status"] == 0
    assert np.linalg.norm(sol.cpu().numpy() - ref) < 1e-9 * np.linalg.norm(ref)


def test_nystrom_fields_vs_oracle(pfm):
    from oracle import fields as fl
    pb, A, B = _oracle("sq2x1radii")
    psi = np.linalg.solve(A, B)
    prob = _gpu(pfm, "sq2x1radii")
    R, T, etc, en = prob.fields(torch.tensor(psi, device="cuda"), 5)
    n, kap, gam, Rr, Tr = fl.bragg(pb, psi, 5, G=1)
    assert np.max(np.abs(R - Rr)) < 1e-12 * max(1.0, np.max(np.abs(Rr)))
    assert np.max(np.abs(T - Tr)) < 1e-10 * np.max(np.abs(Tr))
    assert abs(en - fl.energy_residual(pb, psi, n_orders=5)) < 1e-12


@pytest.mark.parametrize("key", ["tiny", "sq2x1radii"])
def test_nystrom_spectral_accuracy_vs_multiple_scattering(pfm, key):
    """GMRES on the device, Bragg amplitudes against the multiple scattering
    solution of the same array of circles: rounding level from 32 nodes per
    fibre, where the element method at 32 chords is off in the second digit."""
    from analytic import mst_periodic
    from oracle import lattice as la
    from oracle import nystrom as ny
    wl, ka, th = _wl(key, 32)
    pb = ny.problem_from_workload(wl, ka, th)
    ls = lambda ox, oy, nu, ex: la.lattice_sum_orders(pb.k, pb.bd.H, th, ox, oy, nu, exclude=ex)
    q, Rm, Tm, _ = mst_periodic(pb.k, pb.k1, wl.rho_fiber, wl.rho_matrix, th, pb.bd.H, pb.bd.centres, wl.radii,
                                16, ls)
    kap = pb.k * math.sin(th) + 2 * math.pi * np.asarray(q) / pb.bd.H
    prop = kap ** 2 < pb.k ** 2
    errs = {}
    for nys in (True, False):
        prob = pfm.Problem.from_workload(wl, p=40, leaf_max=16, nystrom=nys, tol=1e-12, restart=100)
        prob.set_wave(ka, th)
        x, info = prob.solve()
        assert info["status"] == 0
        R, T, etc, en = prob.fields(x, 3)
        errs[nys] = max(np.max(np.abs(R - Rm)[prop]), np.max(np.abs(T - Tm)[prop]))
        _say("  mst:", key, "nystrom" if nys else "chords", errs[nys], "energy", en)
        if nys:
            assert abs(en) < 1e-10
    assert errs[True] < 1e-10
    assert errs[False] > 1e3 * errs[True]


def test_nystrom_rejects_what_it_cannot_do(pfm):
    wl = W.tiny()
    wl.n_elem = 96
    with pytest.raises(pfm.PfmError):
        pfm.Problem.from_workload(wl, nystrom=True)
    wl = W.bandgap_block("round_square_square", 0.35, n_elem=64, M_L=1, M_H=1)
    with pytest.raises(pfm.PfmError):
        pfm.Problem.from_workload(wl, nystrom=True)
    wl = W.tiny()
    with pytest.raises(pfm.PfmError):
        pfm.Problem.from_workload(wl, nystrom=True, self_fft=False)


@pytest.mark.parametrize("n_elem,ka", [(64, 3.338709677419355), (128, 3.338709677419355), (512, 6.0)])
def test_nystrom_square_8x8_rows(pfm, n_elem, ka):
    """The square 8x8 block (64 fibres, seeded radii) at node counts the
    Nystrom benchmark leg uses and at the benchmark's 512, in its launch
    configuration (p = 32, leaf 64; at 64 nodes every fibre is one leaf):
    sampled rows of the oracle's Nystrom system applied to a random
    density, among them rows of the fibres with close neighbours."""
    from oracle import nystrom as ny
    from oracle import system as sy
    wl = W.square_8x8()
    wl.n_elem = n_elem
    prob = pfm.Problem.from_workload(wl, p=32, leaf_max=64, nystrom=True)
    prob.set_wave(ka, 0.0)
    psi = W.random_density(prob.n, 13)
    y = prob.matvec(torch.tensor(psi, device="cuda")).cpu().numpy()
    pb = ny.problem_from_workload(wl, ka, 0.0)
    rng = np.random.default_rng(13)
    close = np.array([25, 33, 52, 53]) * n_elem + n_elem // 3     # pairs of fibres 0.33a and 0.34a apart
    tg = np.unique(np.concatenate([rng.choice(pb.bd.E, 6, replace=False), close]))
    R1, R2 = ny.operator_rows(pb, tg)
    r = np.concatenate([R1 @ psi, R2 @ psi])
    g = np.concatenate([y[sy.col_phi(pb.bd, tg)], y[sy.col_varphi(pb.bd, tg)]])
    err = np.max(np.abs(g - r)) / np.sqrt(np.mean(np.abs(r) ** 2))
    _say("nystrom square 8x8 rows:", n_elem, ka, err, prob.stats()["n_spectral_fibres"])
    assert err < 1e-9


def test_nystrom_square_8x8_converges(pfm):
    """Spectral convergence on the square 8x8 block: the propagating Bragg
    amplitudes of the device solves at 64 and 128 nodes per fibre agree to
    1e-9, and the flux balances."""
    wl = W.square_8x8()
    ka, H = 3.338709677419355, wl.M_H * wl.a
    q = np.arange(-10, 11)
    prop = np.abs(2 * math.pi * q / H) < ka / wl.a          # theta = 0
    amps = []
    for n in (64, 128):
        wl.n_elem = n
        prob = pfm.Problem.from_workload(wl, p=32, leaf_max=64, nystrom=True, tol=1e-12, restart=200)
        prob.set_wave(ka, 0.0)
        x, info = prob.solve()
        assert info["status"] == 0
        R, T, etc, en = prob.fields(x, 10)        # period 8: orders up to +-4 propagate
        amps.append(np.concatenate([R[prop], T[prop]]))
        _say("  nystrom square 8x8 N =", n, "iters", info["iters"], "energy", en)
        assert abs(en) < 1e-9
    assert np.max(np.abs(amps[0] - amps[1])) < 1e-9
