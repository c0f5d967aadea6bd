"""The C-ABI library loads without a GPU and exports every function that
include/spectral.h declares (no compute calls here)."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "spectral.h")
LIB = os.path.join(ROOT, "paper_1708_07481_amd", "libspectral.so")


def _declared():
    src = open(HEADER).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(sc_[a-z0-9_]+)\s*\(", src)))


def test_header_declares_the_four_calls():
    names = _declared()
    for call in ("sc_graph_build", "sc_laplacian_csr", "sc_lobpcg_solve", "sc_kmeans_assign"):
        assert call in names


def test_library_exports_every_declared_symbol():
    if not os.path.exists(LIB):
        pytest.fail("libspectral.so is not built (python -m paper_1708_07481_amd.build)")
    lib = ctypes.CDLL(LIB)
    missing = [n for n in _declared() if not hasattr(lib, n)]
    assert not missing, missing
    lib.sc_version.restype = ctypes.c_int
    assert lib.sc_version() == 10000


def test_binding_declares_every_symbol():
    from paper_1708_07481_amd._lib import SIGNATURES
    assert sorted(SIGNATURES) == _declared()
