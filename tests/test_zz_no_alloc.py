"""pfm_matvec_static: the operator apply with its scratch in the library's
fixed device array (for callers that cannot allocate), against pfm_matvec.

Two calls in a row, the second on a smaller problem, so that the array holds
the first call's larger contents when the second runs; each result must equal
pfm_matvec's bit for bit (the same kernels in the same order), and no device
allocation may happen.  An apply whose scratch exceeds the array is rejected.
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
    sys.stdout.flush()


@pytest.fixture(scope="module")
def pfm():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1910_10863_amd import pfm as m
    m.lib()
    return m


def _pair(pfm, wl, ka, th, seed, **kw):
    pr = pfm.Problem.from_workload(wl, **kw)
    pr.set_wave(ka, th)
    psi = torch.tensor(W.random_density(pr.n, seed), device="cuda")
    return pr, psi


def test_static_apply_equals_the_workspace_apply(pfm):
    big = _pair(pfm, W.small_square(4, 2, 64, 0.45, 2.0, 0.3), 2.0, 0.3, 11, p=24, leaf_max=16)
    small = _pair(pfm, W.tiny(), 2.0, math.pi / 4, 12, p=16, leaf_max=32)
    hexg = _pair(pfm, W.small_square(16, 8, 16, 0.25, 2.0, 0.5, lattice=W.HEXAGON), 2.0, 0.5, 13, p=16,
                 leaf_max=8)
    assert hexg[0].stats()["lattice_m2l_grid"] == 1      # the grid-convolution spectra are in the array too
    for name, (pr, psi) in (("big", big), ("small", small), ("hex16x8", hexg), ("small again", small)):
        _say("static apply:", name, "n =", pr.n)
        n0 = pr.stats()["n_device_allocs"]
        ref = pr.matvec(psi)
        y = pr.matvec_static(psi)
        torch.cuda.synchronize()
        assert torch.equal(y, ref), float((y - ref).abs().max())
        # and the workspace apply after it is unchanged
        assert torch.equal(pr.matvec(psi), ref)
        assert pr.stats()["n_device_allocs"] == n0


def test_static_apply_against_dense_oracle(pfm):
    from oracle import system as sy
    wl, ka, th = W.tiny(), 2.0, math.pi / 4
    pr, psi = _pair(pfm, wl, ka, th, 14, p=40)
    y = pr.matvec_static(psi).cpu().numpy()
    A = sy.dense_matrix(sy.problem_from_workload(wl, ka, th))
    ref = A @ psi.cpu().numpy()
    err = np.linalg.norm(y - ref) / np.linalg.norm(ref)
    _say("static apply vs oracle:", err)
    assert err < 1e-12


def test_static_apply_rejects_scratch_beyond_the_array(pfm):
    # 256 fibres of 256 elements in leaves of 8, every pair in the tree:
    # about half a million M2L partial expansions, far above the array
    wl = W.small_square(16, 16, 256, 0.3, 2.0, 0.2)
    pr, psi = _pair(pfm, wl, 2.0, 0.2, 15, p=24, leaf_max=8, self_fft=False)
    with pytest.raises(pfm.PfmError) as e:
        pr.matvec_static(psi)
    assert e.value.code == 1 and "static array" in str(e.value)
    y = pr.matvec(psi)           # the handle stays usable
    assert torch.isfinite(y.abs()).all()


def test_static_apply_needs_a_wave(pfm):
    pr = pfm.Problem.from_workload(W.tiny(), p=16)
    with pytest.raises(pfm.PfmError) as e:
        pr.matvec_static(torch.zeros(pr.n, dtype=torch.complex128, device="cuda"))
    assert e.value.code == 7
