"""GPU parity for the round-square scatterer of Sec. 4 (non-circular chords:
every near pair a stored block, the FMM through the tree at k and k1), and
the energy transmission coefficient of a band-gap configuration against the
oracle."""
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


def _rs(M_L, M_H, N, r, lattice=W.SQUARE):
    wl = W.small_square(M_L, M_H, N, r, lattice=lattice)
    wl.shape = W.ROUND_SQUARE
    return wl


CASES = {
    "rs1x1": (_rs(1, 1, 64, 0.07), 2.0, 0.4),
    "rs2x2": (_rs(2, 2, 64, 0.07), 3.0, 0.2),
    "rs_hex2x2": (_rs(2, 2, 64, 0.06, lattice=W.HEXAGON), 2.5, -0.3),
    # the band-gap block of Sec. 4 in miniature: a = 0.5, water in mercury
    "rs_water_mercury": (None, 4.0, 0.0),
}


def _workload(key):
    wl, ka, th = CASES[key]
    if wl is None:
        wl = W.bandgap_block("round_square_square", 0.35, n_elem=64, M_L=2, M_H=2)
    return wl, ka, th


@pytest.mark.parametrize("key", list(CASES))
def test_round_square_matvec_and_solve_vs_oracle(pfm, key):
    from oracle import system as sy
    wl, ka, th = _workload(key)
    pr = pfm.Problem.from_workload(wl, p=40, leaf_max=16, tol=1e-12, restart=100)
    pr.set_wave(ka, th)
    st = pr.stats()
    assert st["self_fft"] == 0 and st["n_near_circulant"] == 0 and st["n_near_stored"] > 0
    pb = sy.problem_from_workload(wl, ka, th)
    A = sy.dense_matrix(pb)
    B = sy.rhs(pb)
    psi = W.random_density(pr.n, 31)
    y = pr.matvec(torch.tensor(psi, device="cuda")).cpu().numpy()
    e_mv = np.linalg.norm(y - A @ psi) / np.linalg.norm(A @ psi)
    x, info = pr.solve()
    ref = np.linalg.solve(A, B)
    e_x = np.linalg.norm(x.cpu().numpy() - ref) / np.linalg.norm(ref)
    _say("round square", key, "matvec", e_mv, "solve", e_x, info["iters"])
    assert e_mv < 1e-10 and e_x < 1e-9


def test_round_square_rejects_precond_and_overlap(pfm):
    wl = _rs(1, 1, 64, 0.07)
    with pytest.raises(pfm.PfmError) as e:
        pfm.Problem.from_workload(wl, precond=True)
    assert e.value.code == 1
    with pytest.raises(pfm.PfmError) as e:
        pfm.Problem.from_workload(_rs(1, 1, 64, 0.13))       # 2 * 4 r > a
    assert e.value.code == 1


@pytest.mark.parametrize("case", ["circle_square", "circle_triangle", "round_square_square"])
def test_bandgap_etc_vs_oracle(pfm, case):
    """ETC (Sec. 4) of the library's solution against the oracle's, on a
    2 x 2 version of the band-gap blocks (water fibres in mercury, a = 0.5,
    64 elements per fibre, filling fraction 50 %), in and outside a gap."""
    from oracle import fields as fl
    from oracle import system as sy
    wl = W.bandgap_block(case, 0.5, n_elem=64, M_L=2, M_H=2)
    # the 2-row block has Wood anomalies at ka / (2 pi) = j / 2: stay clear
    for f in (0.4, 0.9):
        ka = 2 * math.pi * f
        pr = pfm.Problem.from_workload(wl, p=40, leaf_max=16, tol=1e-12, restart=100)
        pr.set_wave(ka, 0.0)
        x, info = pr.solve()
        R, T, etc, en = pr.fields(x, 6)
        pb = sy.problem_from_workload(wl, ka, 0.0)
        ref, _, _ = sy.solve(pb)
        etc_ref = fl.etc(pb, ref, n_orders=6)
        _say("ETC", case, f, etc, etc_ref, info["iters"])
        assert abs(etc - etc_ref) < 1e-8 * max(1.0, etc_ref)
