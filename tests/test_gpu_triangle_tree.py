"""The triangle quadtree of the hexagonal lattice (Sec. 3.1, Fig. 5;
pfm_options.tree_shape = PFM_TREE_TRIANGLE): the apply against the dense
oracle in every form of the own blocks and roots (the oracle's matrix does
not depend on the tree), the solve against LU, the hexagon 16x16 block in
the tree form against sampled oracle rows and against the square tree, the
tree's structure (six triangles under each hexagonal root, four under each
triangle), and the errors of the option."""
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
    "hex2x2": (lambda: W.small_square(2, 2, 64, 0.3, 3.0, 0.3, lattice=W.HEXAGON), 3.0, 0.3),
    # close fibres: near pairs and M2L between triangles of neighbours and images
    "hex2x2close": (lambda: W.small_square(2, 2, 64, 0.45, 2.0, 0.4, lattice=W.HEXAGON), 2.0, 0.4),
    "hex3x2radii": (lambda: W.small_square(3, 2, 96, lattice=W.HEXAGON,
                                           radii=np.array([0.2, 0.45, 0.3, 0.4, 0.25, 0.35])), 4.0, 0.2),
}


@functools.lru_cache(maxsize=4)
def _oracle(key):
    from oracle import system as sy
    make, ka, th = _WL[key]
    pb = sy.problem_from_workload(make(), ka, th)
    return pb, sy.dense_matrix(pb), sy.rhs(pb)


def _prob(pfm, key, **kw):
    make, ka, th = _WL[key]
    prob = pfm.Problem.from_workload(make(), **kw)
    prob.set_wave(ka, th)
    return prob


@pytest.mark.parametrize("form", ["spectral", "fft_tree", "tree"])
@pytest.mark.parametrize("key,leaf", [("hex2x2", 16), ("hex2x2close", 8), ("hex2x2close", 64), ("hex3x2radii", 16)])
def test_triangle_tree_matvec_vs_dense_oracle(pfm, key, leaf, form):
    pb, A, B = _oracle(key)
    kw = dict(self_fft=form != "tree", spectral_roots=form == "spectral")
    _say("triangle tree matvec:", key, "leaf", leaf, form)
    prob = _prob(pfm, key, p=40, leaf_max=leaf, triangle_tree=True, **kw)
    st = prob.stats()
    assert st["tree_on_device"] == 0
    psi = W.random_density(prob.n, 3)
    y = prob.matvec(torch.tensor(psi, device="cuda")).cpu().numpy()
    ref = A @ psi
    err = np.linalg.norm(y - ref) / np.linalg.norm(ref)
    _say("  rel err", err, "cells", st["n_cells"], "leaves", st["n_leaves"], "m2l", st["n_m2l_ext"],
         st["n_m2l_int"], "near", st["n_near_pairs"])
    assert err < 1e-10


def test_triangle_tree_structure(pfm):
    """hex2x2close, leaf 8, 64 chords per fibre: the root (hexagon) has six
    triangle children, every deeper cell at most four; the cell centres of
    level 1 are the centroids of the six triangles, a/3 from the fibre
    centre at 30 + 60 j degrees."""
    make, ka, th = _WL["hex2x2close"]
    wl = make()
    prob = _prob(pfm, "hex2x2close", p=16, leaf_max=8, triangle_tree=True)
    mom, cen, info, order = prob.moments(torch.tensor(W.random_density(prob.n, 1), device="cuda"))
    st = prob.stats()
    M = wl.M
    lvl = info[:, 0]
    assert np.sum(lvl == 0) == M and np.sum(lvl == 1) == 6 * M
    from oracle import system as sy
    pb = sy.problem_from_workload(wl, ka, th)
    c0 = pb.bd.centres[0]
    l1 = cen[(lvl == 1) & (info[:, 1] == 0)] - c0
    ang = np.sort(np.mod(np.degrees(np.arctan2(l1[:, 1], l1[:, 0])), 360.0))
    assert np.allclose(np.hypot(l1[:, 0], l1[:, 1]), wl.a / 3, atol=1e-12)
    assert np.allclose(ang, 30.0 + 60.0 * np.arange(6), atol=1e-9)
    assert st["depth"] >= 2


@pytest.mark.parametrize("key", ["hex2x2", "hex2x2close"])
def test_triangle_tree_solve_vs_dense_lu(pfm, key):
    pb, A, B = _oracle(key)
    ref = np.linalg.solve(A, B)
    prob = _prob(pfm, key, p=40, leaf_max=16, triangle_tree=True, tol=1e-12, restart=100, self_fft=False)
    x, info = prob.solve()
    assert info["status"] == 0
    assert np.linalg.norm(x.cpu().numpy() - ref) < 1e-9 * np.linalg.norm(ref)


def test_triangle_tree_hexagon_16x16_rows(pfm):
    """The hexagon 16x16 block (256 fibres, 131072 unknowns, p = 24, leaf 64)
    with every pair in the triangle trees: sampled oracle rows, and the same
    apply with the square trees (both FMM approximations of one matrix)."""
    from oracle import system as sy
    wl = W.hexagon_16x16()
    ka, th = 2.0, math.pi / 6
    psi = W.random_density(2 * wl.M * wl.n_elem, 29)
    ys = {}
    for tri in (True, False):
        prob = pfm.Problem.from_workload(wl, restart=50, triangle_tree=tri, self_fft=False)
        prob.set_wave(ka, th)
        ys[tri] = prob.matvec(torch.tensor(psi, device="cuda")).cpu().numpy()
        st = prob.stats()
        _say("hexagon 16x16 tree form, triangle" if tri else "square", st["n_cells"], st["n_m2l_ext"],
             st["n_m2l_int"], st["n_near_pairs"])
        prob.close()
    pb = sy.problem_from_workload(wl, ka, th)
    rng = np.random.default_rng(29)
    tg = np.sort(rng.choice(pb.bd.E, 8, replace=False))
    R1, R2 = sy.operator_rows(pb, tg)
    r = np.concatenate([R1 @ psi, R2 @ psi])
    g = np.concatenate([ys[True][sy.col_phi(pb.bd, tg)], ys[True][sy.col_varphi(pb.bd, tg)]])
    err = np.max(np.abs(g - r)) / np.sqrt(np.mean(np.abs(r) ** 2))
    diff = np.linalg.norm(ys[True] - ys[False]) / np.linalg.norm(ys[False])
    _say("  rows", err, "triangle vs square", diff)
    assert err < 1e-8 and diff < 1e-8


def test_triangle_tree_errors(pfm):
    wl = W.small_square(2, 2, 64, 0.3)                 # square lattice
    with pytest.raises(pfm.PfmError):
        pfm.Problem.from_workload(wl, triangle_tree=True)
