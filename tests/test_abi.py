"""The C-ABI library loads and exports every symbol that include/*.h declares.
No compute call is made here (no GPU needed)."""
import ctypes
import glob
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HDRS = sorted(glob.glob(os.path.join(ROOT, "include", "*.h")))
LIB = os.path.join(ROOT, "paper_1910_10863_amd", "libpfmbem.so")


def declared():
    names = set()
    for h in HDRS:
        txt = re.sub(r"/\*.*?\*/", "", open(h).read(), flags=re.S)
        names |= set(re.findall(r"\b(pfm_[a-z_0-9]+)\s*\(", txt))
    return sorted(names)


def test_header_declares_entry_points():
    names = declared()
    for must in ("pfm_create", "pfm_set_wave", "pfm_matvec", "pfm_solve", "pfm_fields", "pfm_destroy"):
        assert must in names


@pytest.mark.skipif(not os.path.exists(LIB), reason="library not built")
def test_library_exports_all_declared_symbols():
    L = ctypes.CDLL(LIB)
    missing = [n for n in declared() if not hasattr(L, n)]
    assert not missing, missing


@pytest.mark.skipif(not os.path.exists(LIB), reason="library not built")
def test_binding_lists_match_header():
    from paper_1910_10863_amd import pfm, warm
    assert sorted(pfm.EXPORTS + warm.EXPORTS) == declared()
