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


def _load():
    if not os.path.exists(LIB):
        pytest.fail("libspectral.so is not built (python -m paper_1708_07481_amd.build)")
    # through the binding, which loads torch (and its HIP runtime) first
    from paper_1708_07481_amd import _lib
    return _lib.lib()


def test_library_exports_every_declared_symbol():
    lib = _load()
    missing = [n for n in _declared() if not hasattr(lib, n)]
    assert not missing, missing
    assert lib.sc_version() == 10100


def test_one_hip_runtime_is_mapped():
    """The library resolves its HIP calls to the runtime torch loaded: one
    libamdhip64 in the process (no device call needed)."""
    lib = _load()
    cnt = ctypes.c_int()
    buf = ctypes.create_string_buffer(4096)
    assert lib.sc_runtime_info(None, ctypes.byref(cnt), buf, len(buf)) == 0
    assert cnt.value == 1
    import torch
    assert os.path.dirname(os.path.realpath(buf.value.decode())) == \
        os.path.realpath(os.path.join(os.path.dirname(torch.__file__), "lib"))


def test_binding_declares_every_symbol():
    from paper_1708_07481_amd._lib import SIGNATURES
    assert sorted(SIGNATURES) == _declared()


def test_binding_constants_match_the_header():
    """Every enumerator the binding names has the header's value."""
    from paper_1708_07481_amd import _lib
    src = re.sub(r"/\*.*?\*/", "", open(HEADER).read(), flags=re.S)
    consts = {n: int(v) for n, v in re.findall(r"\b(SC_[A-Z0-9_]+)\s*=\s*(-?\d+)", src)}
    named = [n for n in dir(_lib) if n.startswith("SC_") and isinstance(getattr(_lib, n), int)]
    assert len(named) >= 20
    for n in named:
        assert n in consts, n
        assert getattr(_lib, n) == consts[n], (n, getattr(_lib, n), consts[n])
