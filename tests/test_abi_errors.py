"""Argument validation of pfm_create runs before any device work, so it is
checked here without a GPU."""
import ctypes
import os

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
LIB = os.path.join(ROOT, "paper_1910_10863_amd", "libpfmbem.so")
pytestmark = pytest.mark.skipif(not os.path.exists(LIB), reason="library not built")


def _create(**over):
    from paper_1910_10863_amd import pfm
    L = pfm.lib()
    g = dict(lattice=0, a=1.0, M_L=2, M_H=2, n_elem=64, r0=0.3)
    m = dict(rho_fiber=13500.0, c_fiber=1450.0, rho_matrix=1000.0, c_matrix=1490.0, eta=0.0)
    o = dict(p=16, leaf_max=32, mac=0.65, g_far=4, restart=50, max_iter=100, tol=1e-8, wood_margin=0.0,
             precision=0, inner_tol=0.0, max_batch=0, use_graph=0, p2p_blocks_per_cu=0, p2p_unroll=0,
             store_self_blocks=0, p2p_cached_rows=0, direct_lattice_m2l=0, precond=0)
    for k, v in over.items():
        for d in (g, m, o):
            if k in d:
                d[k] = v
    geo = pfm.Geometry(g["lattice"], g["a"], g["M_L"], g["M_H"], g["n_elem"], None, g["r0"])
    mat = pfm.Material(**m)
    opt = pfm.Options(**o)
    h = ctypes.c_void_p()
    code = L.pfm_create(ctypes.byref(geo), ctypes.byref(mat), ctypes.byref(opt), ctypes.byref(h))
    msg = L.pfm_last_error(h).decode() if h else ""
    if h:
        L.pfm_destroy(h)
    return code, msg


@pytest.mark.parametrize("bad", [
    dict(p=10), dict(p=0), dict(leaf_max=0), dict(leaf_max=65), dict(mac=1.0), dict(mac=0.0),
    dict(n_elem=4), dict(M_L=0), dict(r0=0.5), dict(r0=-0.1), dict(lattice=2), dict(a=0.0),
    dict(g_far=0), dict(restart=0), dict(tol=0.0), dict(rho_fiber=-1.0), dict(precision=2), dict(max_batch=17), dict(use_graph=2),
    dict(p2p_blocks_per_cu=9), dict(p2p_unroll=3), dict(store_self_blocks=2), dict(p2p_cached_rows=2), dict(direct_lattice_m2l=2),
    dict(precond=2), dict(precond=1, n_elem=48), dict(precond=1, n_elem=1024),
])
def test_create_rejects_invalid_arguments(bad):
    code, msg = _create(**bad)
    assert code == 1, (bad, code, msg)
    assert "invalid argument" in msg


def test_null_arguments():
    from paper_1910_10863_amd import pfm
    L = pfm.lib()
    assert L.pfm_create(None, None, None, None) == 1
    assert L.pfm_matvec(None, None, None) == 1
    assert L.pfm_set_wave(None, 1.0, 0.0) == 1
    assert L.pfm_last_error(None) == b"null handle"
    assert L.pfm_set_batch(None, 1.0, 1, None) == 1
    assert L.pfm_matvec_batch(None, None, None) == 1
    assert L.pfm_rhs_batch(None, None) == 1
    assert L.pfm_solve_batch(None, None, None, 0, None) == 1
    assert L.pfm_sweep(None, 0, None, 1, None, None, None) == 1
    assert L.pfm_precond_apply(None, None, None, 1) == 1
