"""GPU parity of the HIP path against the CPU oracle, through the C ABI.

Stages: device Bessel functions, lattice sums of the top-level M2L, the
upward pass (P2M + M2M) against direct moments, the full operator apply
against the dense oracle matrix (square and hexagon blocks), and the GMRES
solution against the dense LU solution.
"""
import functools
import math
import sys

import numpy as np
import pytest
from scipy.special import j0, j1, y0, y1

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


@functools.lru_cache(maxsize=8)
def _oracle(key):
    from oracle import system as sy
    wl, ka, th = _WL[key]
    pb = sy.problem_from_workload(wl, ka, th)
    A = sy.dense_matrix(pb)
    return pb, A, sy.rhs(pb)


_WL = {
    "tiny": (W.tiny(), 2.0, math.pi / 4),
    "sq2x2": (W.small_square(2, 2, 64, 0.3, 2.0, math.pi / 6), 2.0, math.pi / 6),
    "hex2x2": (W.small_square(2, 2, 64, 0.3, 3.0, 0.3, lattice=W.HEXAGON), 3.0, 0.3),
    "sq3x1": (W.small_square(3, 1, 96, 0.25, 5.0, 0.2, radii=np.array([0.2, 0.3, 0.25])), 5.0, 0.2),
    # close equal fibres: near pairs between neighbours, also across the
    # periodic boundary (image m = +-1), share stored near regions
    "sq2x2close": (W.small_square(2, 2, 64, 0.45, 2.0, 0.4), 2.0, 0.4),
    # four columns: the two inner columns' leaves read shared near regions
    "sq4x2close": (W.small_square(4, 2, 64, 0.45, 2.0, 0.3), 2.0, 0.3),
}


def _gpu_problem(pfm, key, p, leaf, **kw):
    wl, ka, th = _WL[key]
    prob = pfm.Problem.from_workload(wl, p=p, leaf_max=leaf, **kw)
    prob.set_wave(ka, th)
    return prob


def test_device_bessel(pfm):
    x = np.concatenate([np.logspace(-5, 1.9, 400), [24.9, 25.0, 25.1, 30.0]])
    _say("bessel: n =", x.size)
    out = pfm.bessel01(torch.tensor(x, dtype=torch.float64, device="cuda")).cpu().numpy()
    for c, f in enumerate((j0, j1, y0, y1)):
        ref = f(x)
        err = np.abs(out[:, c] - ref) / np.maximum(np.abs(ref), 1e-3)
        assert err.max() < 1e-12, (c, x[err.argmax()], err.max())


@pytest.mark.parametrize("key,p", [("tiny", 24), ("sq2x2", 24), ("hex2x2", 24)])
def test_lattice_sums_vs_oracle(pfm, key, p):
    from oracle.lattice import lattice_sum_orders
    wl, ka, th = _WL[key]
    _say("lattice sums:", key, "p =", p)
    prob = _gpu_problem(pfm, key, p, 32)
    S, offs, mr = prob.lattice_sums()
    k = ka / wl.a
    H = wl.M_H * wl.a
    for o in range(S.shape[0]):
        ex = tuple(range(mr[o, 0], mr[o, 1] + 1))
        ref = lattice_sum_orders(k, H, th, offs[o, 0], offs[o, 1], 2 * p, exclude=ex)
        # scale of each order: the largest of it and its neighbours (orders that
        # vanish by symmetry are compared against their neighbours' size)
        mag = np.abs(ref)
        scale = np.maximum(mag, np.maximum(np.roll(mag, 1), np.roll(mag, -1)))
        err = np.abs(S[o] - ref) / scale
        assert err.max() < 1e-10, (o, offs[o], np.argmax(err) - 2 * p, err.max())


@pytest.mark.parametrize("key,p,leaf", [("tiny", 24, 16), ("sq2x2", 20, 16)])
def test_upward_pass_vs_direct_moments(pfm, key, p, leaf):
    from oracle import fmmdefs
    pb, A, B = _oracle(key)
    wl, ka, th = _WL[key]
    _say("moments:", key, "p =", p, "leaf =", leaf)
    prob = _gpu_problem(pfm, key, p, leaf)
    psi = W.random_density(prob.n, 11)
    mom, cen, info, order = prob.moments(torch.tensor(psi, device="cuda"))
    for c in range(mom.shape[0]):
        elems = order[info[c, 2]:info[c, 3]]
        for ch, kap in ((0, pb.k), (1, pb.k1)):
            ref = fmmdefs.moments(pb, psi, cen[c], elems, kap, p)
            err = np.max(np.abs(mom[c, ch] - ref)) / np.max(np.abs(ref))
            assert err < 1e-11, (c, ch, info[c], err)


def _matvec_err(pfm, key, p, leaf, seed=5, **kw):
    pb, A, B = _oracle(key)
    prob = _gpu_problem(pfm, key, p, leaf, **kw)
    psi = W.random_density(prob.n, seed)
    y = prob.matvec(torch.tensor(psi, device="cuda")).cpu().numpy()
    ref = A @ psi
    return np.linalg.norm(y - ref) / np.linalg.norm(ref), prob


@pytest.mark.parametrize("form", ["spectral", "fft_tree", "tree"])
@pytest.mark.parametrize("key,p,leaf,tol", [
    ("tiny", 40, 32, 1e-10),
    ("tiny", 16, 32, 1e-5),
    ("sq2x2", 40, 16, 1e-10),
    ("hex2x2", 40, 16, 1e-10),
    ("sq3x1", 40, 16, 1e-10),
    ("sq2x2close", 40, 16, 1e-10),
    ("sq4x2close", 40, 16, 1e-10),
    # one leaf per fibre with close neighbours: the root is a leaf with near
    # pairs (its far part comes from the roots' synthesis alone)
    ("sq2x2close", 40, 64, 1e-10),
    ("sq4x2close", 40, 64, 1e-10),
])
def test_matvec_vs_dense_oracle(pfm, key, p, leaf, tol, form):
    """The three forms of a fibre's own image-0 block and of the fibre roots:
    own block by FFT with the roots by Fourier modes when only root-to-root
    pairs remain (the default), own block by FFT with every other pair in the
    tree, and every pair in the tree."""
    self_fft, spectral = form != "tree", form == "spectral"
    _say("matvec:", key, "p =", p, "leaf =", leaf, "form =", form)
    err, prob = _matvec_err(pfm, key, p, leaf, self_fft=self_fft, spectral_roots=spectral)
    st = prob.stats()
    _say("  rel err", err, st)
    # the FFT form needs a power of two elements per fibre (sq3x1 has 96)
    n = _WL[key][0].n_elem
    eligible = self_fft and 8 <= n <= 512 and n & (n - 1) == 0
    assert st["self_fft"] == (1 if eligible else 0)
    if eligible:
        assert st["n_m2l_int"] == 0 and st["n_near_circulant"] == 0
    # fibres farther apart than the admissibility ratio allows: only root
    # pairs, every fibre spectral; close fibres keep their trees
    separated = key in ("tiny", "sq2x2", "hex2x2")
    M = _WL[key][0].M
    assert st["spectral_roots"] == (1 if spectral and eligible else 0)
    if st["spectral_roots"] and separated:
        assert st["n_near_pairs"] == 0 and st["n_spectral_fibres"] == M
    if st["spectral_roots"] and not separated:
        assert st["n_near_pairs"] > 0 and st["n_spectral_fibres"] < M
    assert err < tol


@pytest.mark.parametrize("form", ["spectral", "tree"])
@pytest.mark.parametrize("key", ["tiny", "hex2x2", "sq3x1", "sq4x2close"])
def test_m2l_matrix_cores_vs_dense_oracle(pfm, key, form):
    """The M2L entries on the matrix cores (products of one translation with
    up to 16 sources' moments) against the dense oracle and against every
    entry on the vector ALU: both forms of the own blocks (every pair in the
    tree: interior and exterior channels, leaf entries with images)."""
    self_fft = form == "spectral"
    err_m, prob_m = _matvec_err(pfm, key, 40, 16, self_fft=self_fft)
    err_v, prob_v = _matvec_err(pfm, key, 40, 16, self_fft=self_fft, m2l_vector=True)
    sm, sv = prob_m.stats(), prob_v.stats()
    _say("m2l mfma vs vector:", key, form, err_m, err_v, sm["m2l_mfma_items"], sm["m2l_vector_chunks"],
         sv["m2l_vector_chunks"])
    assert sm["m2l_mfma_items"] > 0 and sv["m2l_mfma_items"] == 0
    assert sv["m2l_vector_chunks"] >= sm["m2l_mfma_items"]
    assert err_m < 1e-10 and err_v < 1e-10
    assert abs(err_m - err_v) < 1e-12


@pytest.mark.parametrize("key", ["sq3x1", "sq2x2close", "hex2x2"])
def test_circulant_self_rows_equal_stored_blocks(pfm, key):
    """The near pairs of a fibre with itself from one circulant row per fibre
    equal their stored blocks (the chords of a circle are rotations of each
    other); pairs with other fibres or images stay stored either way."""
    wl, ka, th = _WL[key]
    psi = W.random_density(2 * wl.M * wl.n_elem, 21)
    ys, st = [], []
    for store in (False, True):
        prob = pfm.Problem.from_workload(wl, p=24, leaf_max=16, store_self_blocks=store, self_fft=False)
        prob.set_wave(ka, th)
        ys.append(prob.matvec(torch.tensor(psi, device="cuda")).cpu().numpy())
        st.append(prob.stats())
    _say("circulant vs stored:", key, [(s["n_near_circulant"], s["n_near_stored"], s["n_near_entries"]) for s in st])
    assert st[0]["n_near_circulant"] > 0 and st[1]["n_near_circulant"] == 0
    assert st[0]["n_near_circulant"] + st[0]["n_near_stored"] <= st[0]["n_near_entries"]
    # stored: every pair has a block (equal fibres may share regions)
    assert 0 < st[1]["n_near_stored"] <= st[1]["n_near_entries"]
    assert np.max(np.abs(ys[0] - ys[1])) < 1e-12 * np.max(np.abs(ys[1]))


@pytest.mark.parametrize("key,leaf", [("sq3x1", 16), ("sq2x2close", 16), ("hex2x2", 16), ("tiny", 32), ("tiny", 64)])
def test_p2p_row_windows_equal_cached_rows(pfm, key, leaf):
    """P2P reading each target leaf's window of the circulant rows from LDS
    gives exactly the sums of reading every entry through the caches (the
    same entries, FMAs and order); leaves whose window would exceed the LDS
    cap take the cached path within the same launch."""
    wl, ka, th = _WL[key]
    psi = W.random_density(2 * wl.M * wl.n_elem, 23)
    ys, st = [], []
    for cached in (False, True):
        prob = pfm.Problem.from_workload(wl, p=24, leaf_max=leaf, p2p_cached_rows=cached, self_fft=False)
        prob.set_wave(ka, th)
        ys.append(prob.matvec(torch.tensor(psi, device="cuda")).cpu().numpy())
        st.append(prob.stats())
    _say("row windows:", key, leaf, st[0]["n_leaves"], st[0]["p2p_window_leaves"], st[0]["p2p_window_max"])
    assert st[0]["p2p_window_leaves"] > 0 and 0 < st[0]["p2p_window_max"] <= 320
    assert st[1]["p2p_window_leaves"] == 0 and st[1]["p2p_window_max"] == 0
    assert np.array_equal(ys[0], ys[1])


def test_matvec_error_decreases_with_p(pfm):
    """Through the tree the truncation error of eq. 10 falls with p (Theorems
    1-2); with the own blocks applied by FFT only the pairs between fibres
    and with images carry it, so the error there is never larger."""
    errs = [(_matvec_err(pfm, "sq2x2", p, 16, self_fft=False)[0]) for p in (8, 16, 24, 32)]
    errs_fft = [(_matvec_err(pfm, "sq2x2", p, 16)[0]) for p in (8, 16, 24, 32)]
    _say("matvec error vs p:", errs, "own blocks by FFT:", errs_fft)
    for a, b in zip(errs, errs[1:]):
        assert b < a
    for a, b in zip(errs_fft, errs):
        assert a <= 1.5 * b


@pytest.mark.parametrize("key", ["tiny", "sq2x2", "hex2x2"])
def test_solve_vs_dense_lu(pfm, key):
    pb, A, B = _oracle(key)
    ref = np.linalg.solve(A, B)
    _say("solve:", key)
    prob = _gpu_problem(pfm, key, 40, 16 if key != "tiny" else 32, tol=1e-12, restart=100)
    b = prob.rhs().cpu().numpy()
    assert np.linalg.norm(b - B) < 1e-13 * np.linalg.norm(B)
    x, info = prob.solve()
    _say("  ", info)
    assert info["status"] == 0
    err = np.linalg.norm(x.cpu().numpy() - ref) / np.linalg.norm(ref)
    _say("  rel err vs LU", err)
    assert err < 1e-8


def test_fields_vs_oracle(pfm):
    from oracle import fields as fl
    pb, A, B = _oracle("tiny")
    psi = np.linalg.solve(A, B)
    prob = _gpu_problem(pfm, "tiny", 24, 32)
    R, T, etc, en = prob.fields(torch.tensor(psi, device="cuda"), 6)
    n, kap, gam, Rr, Tr = fl.bragg(pb, psi, 6)
    assert np.max(np.abs(R - Rr)) < 1e-12 * max(1.0, np.max(np.abs(Rr)))
    assert np.max(np.abs(T - Tr)) < 1e-10 * np.max(np.abs(Tr))
    assert abs(etc - fl.etc(pb, psi, n_orders=6)) < 1e-12
    assert abs(en - fl.energy_residual(pb, psi, n_orders=6)) < 1e-12


@pytest.mark.parametrize("p", [8, 12, 16, 20, 32])
def test_m2l_matrix_cores_every_order(pfm, p):
    """The matrix-core M2L at every supported expansion order: with the last
    order on the vector ALU (p = 8, 16, 32: 2p + 1 = 16 q + 1) and without
    (p = 12, 20), single angle and a batch of two, against the same apply
    with every entry on the vector ALU (same truncation: rounding only),
    on a block with close fibres (in-tree entries, leaf and cell moments
    from their weights) and with separated ones (root pairs only)."""
    for key in ("sq2x2close", "hex2x2"):
        wl, ka, th = _WL[key]
        ys = []
        for vec in (False, True):
            prob = pfm.Problem.from_workload(wl, p=p, leaf_max=16, m2l_vector=vec, max_batch=2)
            psi = torch.tensor(np.stack([W.random_density(prob.n, 31 + b) for b in range(2)]), device="cuda")
            prob.set_wave(ka, th)
            y1 = prob.matvec(psi[0].contiguous()).cpu().numpy()
            prob.set_batch(ka, [th, th + 0.4])
            yb = prob.matvec_batch(psi).cpu().numpy()
            ys.append((y1, yb))
            if not vec:
                assert prob.stats()["m2l_mfma_items"] > 0
        d1 = np.linalg.norm(ys[0][0] - ys[1][0]) / np.linalg.norm(ys[1][0])
        db = np.linalg.norm(ys[0][1] - ys[1][1]) / np.linalg.norm(ys[1][1])
        _say("m2l every order:", key, "p", p, d1, db)
        assert d1 < 1e-12 and db < 1e-12


# ---- mixed precision: complex64 near field inside FP64 iterative refinement ----

@pytest.mark.parametrize("key", ["tiny", "sq2x2", "hex2x2", "sq2x2close"])
def test_mixed_matvec_vs_dense_oracle(pfm, key):
    """The mixed apply differs from the exact operator by the FP32 rounding of
    the near blocks and densities: relative error a few times 2^-24."""
    pb, A, B = _oracle(key)
    _say("mixed matvec:", key)
    # complex64 concerns stored blocks: store the self pairs too
    prob = _gpu_problem(pfm, key, 40, 16 if key != "tiny" else 32, precision=pfm.MIXED, store_self_blocks=True)
    psi = W.random_density(prob.n, 5)
    t = torch.tensor(psi, device="cuda")
    y32 = prob.matvec_mixed(t).cpu().numpy()
    y64 = prob.matvec(t).cpu().numpy()
    ref = A @ psi
    e32 = np.linalg.norm(y32 - ref) / np.linalg.norm(ref)
    e64 = np.linalg.norm(y64 - ref) / np.linalg.norm(ref)
    _say("  rel err mixed", e32, "fp64", e64)
    assert e64 < 1e-10
    assert 1e-9 < e32 < 2e-6


@pytest.mark.parametrize("key", ["sq2x2", "hex2x2"])
def test_mixed_solve_vs_dense_lu(pfm, key):
    pb, A, B = _oracle(key)
    ref = np.linalg.solve(A, B)
    _say("mixed solve:", key)
    prob = _gpu_problem(pfm, key, 40, 16, tol=1e-12, restart=100, precision=pfm.MIXED, store_self_blocks=True)
    x, info = prob.solve()
    _say("  ", info)
    # relaxed inner applies: FP64 first, complex64 once the residual is small
    assert info["status"] == 0 and info["outer"] >= 1
    assert 0 < info["matvecs_mixed"] < info["matvecs"]
    xs = x.cpu().numpy()
    # the true residual of the refined solution with the exact dense operator
    res = np.linalg.norm(B - A @ xs) / np.linalg.norm(B)
    err = np.linalg.norm(xs - ref) / np.linalg.norm(ref)
    _say("  dense residual", res, "rel err vs LU", err)
    assert res < 1e-10
    assert err < 1e-8


def test_mixed_requires_mixed_handle(pfm):
    prob = _gpu_problem(pfm, "tiny", 16, 32)
    with pytest.raises(RuntimeError):
        prob.matvec_mixed(prob.empty())
