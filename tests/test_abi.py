"""The C-ABI library loads and exports every symbol that include/pfmbem.h declares.
No compute call is made here (no GPU needed)."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HDR = os.path.join(ROOT, "include", "pfmbem.h")
LIB = os.path.join(ROOT, "paper_1910_10863_amd", "libpfmbem.so")


def declared():
    txt = open(HDR).read()
    txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
    return sorted(set(re.findall(r"\b(pfm_[a-z_0-9]+)\s*\(", txt)))


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
    from paper_1910_10863_amd import pfm
    assert sorted(pfm.EXPORTS) == declared()
