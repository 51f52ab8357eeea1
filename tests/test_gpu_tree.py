"""The quadtrees and interaction lists built by GPU kernels (Sec. 3.1)
against the host construction: every array of the plan bit for bit (eight
digests over the cells, element order, leaves, ancestor and upward lists,
fibre offsets and image ranges, M2L, interior M2L and near lists), the same
statistics, and bit-identical applies, on small blocks, blocks with close
fibres and images, non-circular fibres, deep trees and the full benchmark
blocks."""
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


# (workload, Problem keywords)
CASES = {
    "tiny_leaf32": (lambda: W.tiny(), dict(p=16, leaf_max=32)),
    "tiny_leaf1": (lambda: W.tiny(), dict(p=16, leaf_max=1)),
    "sq3x1_N96": (lambda: W.small_square(3, 1, 96, 0.25, radii=np.array([0.2, 0.3, 0.25])),
                  dict(p=24, leaf_max=16)),
    "sq2x2close": (lambda: W.small_square(2, 2, 64, 0.45), dict(p=16, leaf_max=16)),
    "sq4x2close_tree": (lambda: W.small_square(4, 2, 64, 0.45), dict(p=16, leaf_max=8, self_fft=False)),
    "hex3x4_leaf4": (lambda: W.small_square(3, 4, 128, 0.3, lattice=W.HEXAGON), dict(p=16, leaf_max=4)),
    "rs2x2": (lambda: _rs(2, 2, 64, 0.07), dict(p=24, leaf_max=16)),
    "rs_hex2x2": (lambda: _rs(2, 2, 64, 0.06, lattice=W.HEXAGON), dict(p=24, leaf_max=8)),
    "bandgap_rs": (lambda: W.bandgap_block("round_square_square", 0.5), dict(p=16, leaf_max=32)),
    "stored_blocks": (lambda: W.small_square(2, 3, 128, 0.4), dict(p=16, leaf_max=16, store_self_blocks=True)),
    "square_8x8_N512": (lambda: W.square_8x8(), dict()),
    "hexagon_16x16_N256": (lambda: W.hexagon_16x16(), dict()),
    "square_4x4_sweep": (lambda: W.square_4x4_sweep(), dict(leaf_max=32)),
}


@pytest.mark.parametrize("key", list(CASES))
def test_gpu_plan_equals_host_plan(pfm, key):
    make, kw = CASES[key]
    wl = make()
    _say(f"tree build {key}: M={wl.M} N={wl.n_elem} {kw}")
    dev = pfm.Problem.from_workload(wl, **kw)
    host = pfm.Problem.from_workload(wl, tree_on_host=True, **kw)
    sd, sh = dev.stats(), host.stats()
    assert sd["tree_on_device"] == 1 and sh["tree_on_device"] == 0
    for k in sd:
        if k not in ("tree_on_device",):
            assert sd[k] == sh[k], (k, sd[k], sh[k])
    dd, dh = dev.plan_digest(), host.plan_digest()
    names = ["cells", "levels/elements/leaves", "ancestors", "upward", "fibre offsets", "m2l", "m2l interior",
             "near"]
    bad = [names[i] for i in range(8) if dd[i] != dh[i]]
    assert not bad, bad
    # the same plan gives the same apply, bit for bit
    ka = wl.ka[len(wl.ka) // 2] if len(wl.ka) else 2.0
    th = wl.theta[0] if len(wl.theta) else 0.0
    dev.set_wave(ka, th)
    host.set_wave(ka, th)
    psi = torch.tensor(W.random_density(dev.n, 3), device="cuda")
    yd, yh = dev.matvec(psi), host.matvec(psi)
    torch.cuda.synchronize()
    assert torch.equal(yd, yh)
    _say(f"  cells {sd['n_cells']} leaves {sd['n_leaves']} depth {sd['depth']} m2l {sd['n_m2l_ext']} "
         f"near pairs {sd['n_near_pairs']}: identical")
    dev.close()
    host.close()


def test_gpu_tree_falls_back_beyond_its_limits(pfm):
    """More than 4096 elements per fibre: the host builds the plan, and the
    handle says so."""
    wl = W.small_square(1, 1, 8192, 0.3)
    pr = pfm.Problem.from_workload(wl, p=16, leaf_max=64, self_fft=False)
    assert pr.stats()["tree_on_device"] == 0
    pr.close()
