"""GPU parity at the benchmark sizes and in the launch configuration that
bench.py times, on outputs the oracle computes one by one: sampled rows of
(I - A) applied to a random density, and the lattice sums of every fibre
offset.  Plus edge cases (smallest element count, one-element leaves, ragged
leaves), determinism and the error paths of the C ABI.
"""
import math
import sys

import numpy as np
import pytest

import workloads as W

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


def _say(*a):
    print(*a, flush=True)


@pytest.fixture(scope="module")
def pfm():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1910_10863_amd import pfm as m
    m.lib()
    return m


def _rows_parity(pfm, wl, ka, th, n_rows, seed, **kw):
    from oracle import system as sy
    prob = pfm.Problem.from_workload(wl, **kw)
    prob.set_wave(ka, th)
    psi = W.random_density(prob.n, seed)
    y = prob.matvec(torch.tensor(psi, device="cuda")).cpu().numpy()
    pb = sy.problem_from_workload(wl, ka, th)
    rng = np.random.default_rng(seed)
    tg = np.sort(rng.choice(pb.bd.E, n_rows, replace=False))
    R1, R2 = sy.operator_rows(pb, tg)
    r = np.concatenate([R1 @ psi, R2 @ psi])
    g = np.concatenate([y[sy.col_phi(pb.bd, tg)], y[sy.col_varphi(pb.bd, tg)]])
    err = np.max(np.abs(g - r)) / np.sqrt(np.mean(np.abs(r) ** 2))
    return err, prob


# square 8x8 block, 65536 unknowns, p = 24, leaf 64: the benchmark workload
@pytest.mark.parametrize("ka", [0.5, 3.338709677419355, 6.0])
def test_square_8x8_rows(pfm, ka):
    wl = W.square_8x8()
    _say("square 8x8 rows, ka =", ka)
    err, prob = _rows_parity(pfm, wl, ka, 0.0, 8, 21, restart=200)
    _say("  max row error / rms", err)
    assert err < 1e-8


def test_square_8x8_one_leaf_per_fibre_rows(pfm):
    """64 chords per fibre with leaf 64: every fibre is one leaf, and the
    fibres with close neighbours have roots that are leaves with near pairs
    (their far part must come from the roots' synthesis alone).  Rows of
    those fibres and of others against the oracle."""
    from oracle import system as sy
    wl = W.square_8x8()
    wl.n_elem = 64
    ka = 3.338709677419355
    prob = pfm.Problem.from_workload(wl, p=32, leaf_max=64)
    prob.set_wave(ka, 0.0)
    st = prob.stats()
    assert st["spectral_roots"] == 1 and 0 < st["n_spectral_fibres"] < 64 and st["n_near_pairs"] > 0
    psi = W.random_density(prob.n, 17)
    y = prob.matvec(torch.tensor(psi, device="cuda")).cpu().numpy()
    pb = sy.problem_from_workload(wl, ka, 0.0)
    tg = np.array([25, 33, 52, 53, 2, 60]) * 64 + np.array([3, 40, 10, 60, 5, 33])
    R1, R2 = sy.operator_rows(pb, tg)
    r = np.concatenate([R1 @ psi, R2 @ psi])
    g = np.concatenate([y[sy.col_phi(pb.bd, tg)], y[sy.col_varphi(pb.bd, tg)]])
    err = np.max(np.abs(g - r)) / np.sqrt(np.mean(np.abs(r) ** 2))
    _say("square 8x8, one leaf per fibre: max row error / rms", err)
    assert err < 1e-10


def test_hexagon_16x16_rows(pfm):
    wl = W.hexagon_16x16()
    _say("hexagon 16x16 rows")
    err, prob = _rows_parity(pfm, wl, wl.ka[0], wl.theta[0], 6, 22)
    _say("  max row error / rms", err, prob.stats()["n_near_entries"])
    assert err < 1e-8


@pytest.mark.parametrize("ka,th", [(0.2, 0.0), (4.0, 3 * math.pi / 16), (8.0, 7 * math.pi / 16)])
def test_square_4x4_rows(pfm, ka, th):
    wl = W.square_4x4_sweep()
    _say("square 4x4 rows", ka, th)
    err, prob = _rows_parity(pfm, wl, ka, th, 8, 23)
    _say("  max row error / rms", err)
    assert err < 1e-8


def test_lattice_sums_square_8x8(pfm):
    from oracle.lattice import lattice_sum_orders
    wl = W.square_8x8()
    prob = pfm.Problem.from_workload(wl)
    for ka in (0.5, 6.0):
        prob.set_wave(ka, 0.0)
        S, offs, mr = prob.lattice_sums()
        _say("lattice 8x8 ka", ka, "offsets", S.shape[0])
        for o in range(0, S.shape[0], 16):
            ex = tuple(range(mr[o, 0], mr[o, 1] + 1))
            ref = lattice_sum_orders(ka, 8.0, 0.0, offs[o, 0], offs[o, 1], 2 * wl.p, exclude=ex)
            mag = np.abs(ref)
            scale = np.maximum(mag, np.maximum(np.roll(mag, 1), np.roll(mag, -1)))
            assert np.max(np.abs(S[o] - ref) / scale) < 1e-10, offs[o]


@pytest.mark.parametrize("case", ["n8_leaf1", "ragged_hex", "one_leaf"])
def test_edge_cases_dense(pfm, case):
    from oracle import system as sy
    if case == "n8_leaf1":
        wl = W.small_square(1, 1, 8, 0.3, 1.5, 0.4, p=8, leaf_max=1)
        kw = dict(p=32, leaf_max=1, mac=0.4)
    elif case == "ragged_hex":
        wl = W.small_square(3, 2, 100, 0.3, 2.5, -0.3, lattice=W.HEXAGON,
                            radii=np.array([0.3, 0.25, 0.28, 0.31, 0.22, 0.3]))
        kw = dict(p=32, leaf_max=13)
    else:
        wl = W.small_square(2, 1, 40, 0.3, 3.0, 0.2)
        kw = dict(p=32, leaf_max=64)
    ka, th = wl.ka[0], wl.theta[0]
    prob = pfm.Problem.from_workload(wl, **kw)
    prob.set_wave(ka, th)
    psi = W.random_density(prob.n, 4)
    y = prob.matvec(torch.tensor(psi, device="cuda")).cpu().numpy()
    pb = sy.problem_from_workload(wl, ka, th)
    ref = sy.dense_matrix(pb) @ psi
    err = np.linalg.norm(y - ref) / np.linalg.norm(ref)
    _say(case, "rel err", err, prob.stats()["depth"])
    assert err < 1e-9


def test_apply_is_deterministic(pfm):
    wl = W.square_4x4_sweep()
    prob = pfm.Problem.from_workload(wl)
    prob.set_wave(3.0, 0.3)
    psi = torch.tensor(W.random_density(prob.n, 9), device="cuda")
    a = prob.matvec(psi).clone()
    b = prob.matvec(psi).clone()
    assert torch.equal(a, b)


@pytest.mark.parametrize("key,bpc", [("square_4x4", 0), ("square_8x8", 0), ("square_8x8", 4), ("hexagon_16x16", 0)])
def test_timed_apply_matches_overlapped_apply(pfm, key, bpc):
    """The overlapped apply (P2P on the side stream; with one column split
    per leaf the downward pass adds the far part into y after waiting for
    P2P, else a join kernel adds it) equals the in-order timed apply bit
    for bit."""
    wl = {"square_4x4": W.square_4x4_sweep, "square_8x8": W.square_8x8, "hexagon_16x16": W.hexagon_16x16}[key]()
    prob = pfm.Problem.from_workload(wl, p2p_blocks_per_cu=bpc, self_fft=False)
    prob.set_wave(2.0, 0.1)
    st = prob.stats()
    _say("overlapped vs in-order:", key, bpc, "split", st["p2p_split"], "circulant", st["n_near_circulant"],
         "stored", st["n_near_stored"])
    if key == "hexagon_16x16" or (key == "square_8x8" and bpc == 0):
        # one split per leaf and mostly circulant pairs: the fused join runs
        assert st["p2p_split"] == 1 and st["n_near_circulant"] > st["n_near_stored"]
    if key == "square_8x8" and bpc == 4:
        # 1024 workgroups for 848 leaves: two column splits, the join kernel
        assert st["p2p_split"] == 2
    psi = torch.tensor(W.random_density(prob.n, 10), device="cuda")
    a = prob.matvec(psi).clone()
    stages, tot, b = prob.matvec_timed(psi, reps=2)
    c = prob.matvec(psi).clone()
    assert torch.equal(a, b) and torch.equal(a, c)
    assert all(v >= 0 for v in stages.values()) and tot > 0


@pytest.mark.parametrize("key", ["square_4x4", "square_8x8", "hexagon_16x16"])
def test_self_fft_apply_timed_overlapped_and_tree(pfm, key):
    """With the fibres' own blocks applied by FFT (the default): the overlapped
    apply (FFT apply and P2P on the side stream, the downward pass adding the
    far part after the join) equals the in-order timed apply bit for bit, and
    differs from the apply with every pair in the tree by no more than the
    FMM truncation of the in-fibre far pairs (p = 24)."""
    wl = {"square_4x4": W.square_4x4_sweep, "square_8x8": W.square_8x8, "hexagon_16x16": W.hexagon_16x16}[key]()
    prob = pfm.Problem.from_workload(wl)
    prob.set_wave(2.0, 0.1)
    st = prob.stats()
    assert st["self_fft"] == 1 and st["n_m2l_int"] == 0 and st["p2p_split"] == 1
    psi = torch.tensor(W.random_density(prob.n, 10), device="cuda")
    a = prob.matvec(psi).clone()
    stages, tot, b = prob.matvec_timed(psi, reps=2)
    c = prob.matvec(psi).clone()
    assert torch.equal(a, b) and torch.equal(a, c)
    tree = pfm.Problem.from_workload(wl, self_fft=False)
    tree.set_wave(2.0, 0.1)
    t = tree.matvec(psi)
    d = float(torch.max(torch.abs(a - t)) / torch.max(torch.abs(t)))
    _say("own blocks by FFT vs tree:", key, d, "stages", stages)
    assert d < 1e-9


@pytest.mark.parametrize("key,n_spec", [("square_4x4", 16), ("hexagon_16x16", 256), ("square_8x8", 58)])
def test_spectral_roots_vs_tree_roots(pfm, key, n_spec):
    """The roots' moments by Fourier modes and, for the fibres with only
    root-to-root pairs, their far rows by a synthesis of the root's local
    expansion, against the same apply with P2M, M2M and the downward pass
    through every fibre's tree; they differ by the M2M/L2L truncation at
    p = 24 only.  On the square 8x8 block six fibres have neighbours close
    enough to keep their trees.  The in-order timed apply equals the fused
    one bit for bit, and the batched apply matches it."""
    wl = {"square_4x4": W.square_4x4_sweep, "hexagon_16x16": W.hexagon_16x16, "square_8x8": W.square_8x8}[key]()
    spec = pfm.Problem.from_workload(wl, max_batch=4)
    tree = pfm.Problem.from_workload(wl, spectral_roots=False)
    assert spec.stats()["spectral_roots"] == 1 and tree.stats()["spectral_roots"] == 0
    assert spec.stats()["n_spectral_fibres"] == n_spec
    spec.set_wave(2.0, 0.1)
    tree.set_wave(2.0, 0.1)
    psi = torch.tensor(W.random_density(spec.n, 13), device="cuda")
    a = spec.matvec(psi).clone()
    _, _, b = spec.matvec_timed(psi, reps=2)
    assert torch.equal(a, b)
    t = tree.matvec(psi)
    d = float(torch.max(torch.abs(a - t)) / torch.max(torch.abs(t)))
    steady = {s: spec.stage_timed(psi, s, reps=20) for s in ("p2m", "m2m", "m2l", "down_l2p")}
    _say("spectral roots vs tree roots:", key, d, "stages", steady)
    assert d < 1e-9
    th = [0.1, 0.3, -0.2]
    spec.set_batch(2.0, th)
    xs = torch.stack([torch.tensor(W.random_density(spec.n, 20 + i), device="cuda") for i in range(3)])
    yb = spec.matvec_batch(xs)
    for i, t_ in enumerate(th):
        spec.set_wave(2.0, t_)
        yi = spec.matvec(xs[i])
        e = float(torch.linalg.vector_norm(yb[i] - yi) / torch.linalg.vector_norm(yi))
        assert e < 1e-13, (i, e)


@pytest.mark.parametrize("key", ["square_8x8", "square_4x4"])
def test_m2l_matrix_cores_vs_vector_fullsize(pfm, key):
    """At the benchmark sizes, the M2L on the matrix cores against every
    entry on the vector ALU (the same sums, added in the same order; the
    products differ by rounding only): single angle and a batch of three.
    (The hexagon 16x16 block has no M2L entries: its fibres are separated
    and its lattice M2L is the grid convolution.)"""
    wl = {"square_4x4": W.square_4x4_sweep, "square_8x8": W.square_8x8}[key]()
    mf = pfm.Problem.from_workload(wl, max_batch=4)
    ve = pfm.Problem.from_workload(wl, max_batch=4, m2l_vector=True)
    st = mf.stats()
    _say("m2l mfma items", st["m2l_mfma_items"], "vector chunks", st["m2l_vector_chunks"],
         ve.stats()["m2l_vector_chunks"])
    assert st["m2l_mfma_items"] > 0
    psi = torch.tensor(W.random_density(mf.n, 31), device="cuda")
    for prob in (mf, ve):
        prob.set_wave(3.0, 0.2)
    a, b = mf.matvec(psi), ve.matvec(psi)
    d = float(torch.linalg.vector_norm(a - b) / torch.linalg.vector_norm(b))
    _say("single angle: rel diff", d)
    assert d < 1e-13
    th = [0.1, 0.3, -0.2]
    xs = torch.stack([torch.tensor(W.random_density(mf.n, 40 + i), device="cuda") for i in range(3)])
    for prob in (mf, ve):
        prob.set_batch(3.0, th)
    ya, yb = mf.matvec_batch(xs), ve.matvec_batch(xs)
    d = float(((ya - yb).norm(dim=1) / yb.norm(dim=1)).max())
    _say("batch of three: max rel diff", d)
    assert d < 1e-13


def test_row_windows_equal_cached_rows_square_8x8(pfm):
    """At the benchmark configuration the P2P row windows in LDS give the
    cache path's sums bit for bit."""
    wl = W.square_8x8()
    psi = torch.tensor(W.random_density(2 * wl.M * wl.n_elem, 12), device="cuda")
    ys, st = [], []
    for cached in (False, True):
        prob = pfm.Problem.from_workload(wl, p2p_cached_rows=cached, self_fft=False)
        prob.set_wave(3.338709677419355, 0.0)
        ys.append(prob.matvec(psi).clone())
        st.append(prob.stats())
        prob.close()
    _say("square 8x8 windows:", st[0]["p2p_window_leaves"], "of", st[0]["n_leaves"], "max", st[0]["p2p_window_max"])
    assert st[0]["p2p_window_leaves"] > st[0]["n_leaves"] // 2 and st[1]["p2p_window_leaves"] == 0
    assert torch.equal(ys[0], ys[1])


def test_gmres_noconv_and_wood_errors(pfm):
    wl = W.square_4x4_sweep()
    prob = pfm.Problem.from_workload(wl, max_iter=2, restart=2)
    prob.set_wave(3.0, 0.0)
    x, info = prob.solve()
    assert info["status"] == 4 and info["iters"] == 2
    assert np.isfinite(x.cpu().numpy()).all()
    with pytest.raises(pfm.PfmError) as e:
        prob.solve(raise_on_noconv=True)
    assert e.value.code == 4
    # k H (1 + sin 0) / (2 pi) = 1 exactly: a Wood anomaly of the 4-row block
    prob2 = pfm.Problem.from_workload(wl, wood_margin=1e-3)
    with pytest.raises(pfm.PfmError) as e:
        prob2.set_wave(2 * math.pi / 4, 0.0)
    assert e.value.code == 5
    with pytest.raises(ValueError):
        prob.matvec(torch.zeros(10, dtype=torch.complex128, device="cuda"))


def test_warm_start_from_solution_converges_immediately(pfm):
    wl = W.square_4x4_sweep()
    prob = pfm.Problem.from_workload(wl, tol=1e-10, restart=100)
    prob.set_wave(2.5, 0.2)
    x, info = prob.solve()
    assert info["status"] == 0
    x2, info2 = prob.solve(x0=x)
    assert info2["iters"] == 0 and info2["status"] == 0


def test_hexagon_16x16_mixed_solve(pfm):
    """Hexagon 16x16 block (131072 unknowns): the mixed-precision refined
    solution meets the FP64 residual 1e-8 (checked with the FP64 apply) and
    agrees with the FP64 GMRES solution to the accuracy the residual allows."""
    wl = W.hexagon_16x16()
    ka, th = wl.ka[0], wl.theta[0]
    _say("hexagon 16x16 mixed solve")
    p64 = pfm.Problem.from_workload(wl)
    p64.set_wave(ka, th)
    x64, i64 = p64.solve()
    _say("  fp64", i64)
    # complex64 stored blocks (self pairs stored too); p64 keeps the circulant rows
    pmx = pfm.Problem.from_workload(wl, precision=pfm.MIXED, store_self_blocks=True)
    pmx.set_wave(ka, th)
    xmx, imx = pmx.solve()
    _say("  mixed", imx)
    assert i64["status"] == 0 and imx["status"] == 0
    assert imx["matvecs_mixed"] > 0
    b = p64.rhs()
    r = b - p64.matvec(xmx)
    res = (torch.linalg.vector_norm(r) / torch.linalg.vector_norm(b)).item()
    dx = (torch.linalg.vector_norm(xmx - x64) / torch.linalg.vector_norm(x64)).item()
    _say("  fp64 residual of mixed solution", res, "difference to fp64 solution", dx)
    assert res < 1e-8
    assert dx < 1e-6


@pytest.mark.parametrize("key", ["hexagon_16x16", "square_12x12", "hexagon_13x11"])
def test_lattice_grid_m2l_equals_direct(pfm, key):
    """From 128 fibres up the root lattice M2L runs as a convolution over the
    fibre grid (zero-padded 2D DFTs); it equals the direct sum over every root
    pair to rounding.  Square and hexagonal grids, and an odd column count
    (the two hexagonal sublattices of different widths)."""
    wl = {"hexagon_16x16": W.hexagon_16x16(),
          "square_12x12": W.small_square(12, 12, 32, 0.3, 2.5, 0.3, lattice=W.SQUARE),
          "hexagon_13x11": W.small_square(13, 11, 32, 0.25, 2.0, 0.5, lattice=W.HEXAGON)}[key]
    ka, th = (2.0, math.pi / 6) if key == "hexagon_16x16" else (wl.ka[0], wl.theta[0])
    psi = torch.tensor(W.random_density(2 * wl.M * wl.n_elem, 14), device="cuda")
    ys, st = [], []
    for direct in (False, True):
        prob = pfm.Problem.from_workload(wl, p=24, leaf_max=16 if key != "hexagon_16x16" else 64,
                                         direct_lattice_m2l=direct)
        prob.set_wave(ka, th)
        ys.append(prob.matvec(psi).clone())
        st.append(prob.stats())
        prob.close()
    d = float(torch.max(torch.abs(ys[0] - ys[1])) / torch.max(torch.abs(ys[1])))
    _say("lattice grid vs direct:", key, st[0]["lattice_m2l_grid"], st[1]["lattice_m2l_grid"], d)
    assert st[0]["lattice_m2l_grid"] == 1 and st[1]["lattice_m2l_grid"] == 0
    assert d < 1e-12


def test_batched_apply_with_lattice_grid_m2l(pfm):
    """A batch of angles on a 144-fibre block (lattice M2L as a grid
    convolution, one set of transformed lattice rows per member) against the
    single-angle apply of each member and the direct lattice M2L."""
    wl = W.small_square(12, 12, 32, 0.3, 2.5, 0.3, lattice=W.SQUARE)
    th = [0.0, 0.4, 1.1]
    pb = pfm.Problem.from_workload(wl, p=24, leaf_max=16, max_batch=4)
    assert pb.stats()["lattice_m2l_grid"] == 1
    pb.set_batch(2.5, th)
    psi = torch.tensor(np.stack([W.random_density(pb.n, 60 + b) for b in range(3)]), device="cuda")
    yb = pb.matvec_batch(psi).cpu().numpy()
    single = pfm.Problem.from_workload(wl, p=24, leaf_max=16, direct_lattice_m2l=True)
    for b in range(3):
        single.set_wave(2.5, th[b])
        ys = single.matvec(psi[b].contiguous()).cpu().numpy()
        err = np.linalg.norm(yb[b] - ys) / np.linalg.norm(ys)
        _say("batched grid lattice vs single direct:", b, err)
        assert err < 1e-13


def test_mixed_apply_with_circulant_rows_hexagon(pfm):
    """The complex64 apply with the default near field (circulant self rows
    in FP64, only cross-fibre pairs stored and rounded to complex64; one
    column split per leaf, so the downward pass adds the far part after the
    P2P of the complex64 kernel) stays within the rounding of the stored
    blocks of the FP64 apply; on this block every near pair is a same-fibre
    pair, so the two applies agree exactly."""
    wl = W.hexagon_16x16()
    prob = pfm.Problem.from_workload(wl, precision=pfm.MIXED, self_fft=False)
    prob.set_wave(wl.ka[0], wl.theta[0])
    st = prob.stats()
    assert st["p2p_split"] == 1 and st["n_near_circulant"] > st["n_near_stored"]
    psi = torch.tensor(W.random_density(prob.n, 15), device="cuda")
    y64 = prob.matvec(psi).clone()
    y32 = prob.matvec_mixed(psi).clone()
    y32b = prob.matvec_mixed(psi).clone()
    d = float(torch.max(torch.abs(y32 - y64)) / torch.max(torch.abs(y64)))
    _say("hexagon mixed vs fp64 apply (circulant rows):", st["n_near_stored"], d)
    assert torch.equal(y32, y32b)
    assert d < 2e-6
    if st["n_near_stored"] == 0:
        assert d == 0.0
