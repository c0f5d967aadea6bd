"""ctypes declarations of the C ABI in include/spectral.h (names unchanged).

Loading imports torch first so that the HIP runtime torch ships is the one
the library binds to (both carry the soname libamdhip64.so.7).  There is no
fallback: if libspectral.so is missing the import fails loudly.
"""
from __future__ import annotations

import ctypes as C
import os

import torch  # noqa: F401  (must be loaded before the HIP library)

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libspectral.so")

SC_OK, SC_E_INVAL, SC_E_NOMEM, SC_E_HIP, SC_E_BREAKDOWN, SC_E_NUMERIC, SC_E_UNSUPPORTED = \
    0, -1, -2, -3, -4, -5, -6
STATUS_NAMES = {0: "SC_OK", -1: "SC_E_INVAL", -2: "SC_E_NOMEM", -3: "SC_E_HIP",
                -4: "SC_E_BREAKDOWN", -5: "SC_E_NUMERIC", -6: "SC_E_UNSUPPORTED"}
SC_SYM_LOGICAL, SC_SYM_ALGEBRAIC = 0, 1
SC_PREC_FP64, SC_PREC_FP32, SC_PREC_FP32_BF16GRAM = 0, 1, 2

_p = C.c_void_p
_i64 = C.c_int64
_int = C.c_int
_dbl = C.c_double
_size = C.c_size_t


class sc_lobpcg_opts(C.Structure):
    _fields_ = [("k", _int), ("maxit", _int), ("tol", _dbl), ("prec", _int), ("ldx", _i64),
                ("lock_tol", _dbl), ("chol_tol", _dbl), ("diag", _p), ("op_norm", _dbl),
                ("k_conv", _int)]


class sc_lobpcg_info(C.Structure):
    _fields_ = [("iterations", _int), ("converged", _int), ("p_drops", _int),
                ("locked_cols", _int), ("max_relres", _dbl), ("w_drops", _int),
                ("gram_fallbacks", _int), ("restarts", _int)]


class sc_kmeans_opts(C.Structure):
    _fields_ = [("n_clusters", _int), ("restarts", _int), ("max_iter", _int),
                ("normalize_rows", _int), ("x_fp32", _int), ("scan", _int)]


SC_KM_SCAN_AUTO, SC_KM_SCAN_PRUNED, SC_KM_SCAN_FULL = 0, 1, 2
SC_RAND_NORMAL, SC_RAND_UNIFORM, SC_RAND_RAW = 0, 1, 2
SC_GATHER_FP32, SC_GATHER_FP16, SC_GATHER_BF16, SC_GATHER_FP32_LANE16 = 0, 1, 2, 3


SC_KIND_SPMM, SC_KIND_GRAM, SC_KIND_RR, SC_KIND_UPDATE, SC_KIND_CHOLQR, SC_KIND_RESIDUAL, \
    SC_KIND_GRAPH, SC_KIND_KMEANS, SC_KIND_GRAM_FP64ACC = range(9)
KIND_NAMES = ["spmm", "gram", "rayleigh_ritz", "block_update", "cholqr", "residual",
              "graph_build", "kmeans", "gram_fp64acc"]


# name -> (restype, argtypes); every function declared in include/spectral.h
SIGNATURES = {
    "sc_ctx_create": (_int, [_int, _p, C.POINTER(_p)]),
    "sc_ctx_destroy": (_int, [_p]),
    "sc_last_error": (C.c_char_p, [_p]),
    "sc_version": (_int, []),
    "sc_runtime_info": (_int, [C.POINTER(_int), C.POINTER(_int), C.c_char_p, _size]),
    "sc_graph_build_workspace": (_int, [_p, _i64, _i64, C.POINTER(_size)]),
    "sc_graph_build": (_int, [_p, _i64, _i64, _p, _p, _p, _int, _p, _p, _p, _p,
                              C.POINTER(_i64), C.POINTER(_i64), _p, _size]),
    "sc_laplacian_csr": (_int, [_p, _i64, _i64, _p, _p, _p, _p, _p, _p, _p]),
    "sc_laplacian_combinatorial": (_int, [_p, _i64, _i64, _p, _p, _p, _p, _p, _p]),
    "sc_spmm": (_int, [_p, _i64, _i64, _p, _p, _p, _int, _int, _p, _i64, _p, _i64]),
    "sc_spmm_diag": (_int, [_p, _i64, _i64, _p, _p, _p, _p, _int, _int, _p, _i64, _p, _i64]),
    "sc_lobpcg_workspace": (_int, [_p, _i64, _i64, C.POINTER(sc_lobpcg_opts), C.POINTER(_size)]),
    "sc_lobpcg_solve": (_int, [_p, _i64, _i64, _p, _p, _p, C.POINTER(sc_lobpcg_opts), _p, _p,
                               _p, _p, C.POINTER(sc_lobpcg_info), _p, _size]),
    "sc_lobpcg_begin": (_int, [_p, _i64, _i64, _p, _p, _p, C.POINTER(sc_lobpcg_opts), _p, _p,
                               _size, C.POINTER(_p), C.POINTER(_int)]),
    "sc_lobpcg_step": (_int, [_p, _p, C.POINTER(_int)]),
    "sc_lobpcg_step_async": (_int, [_p, _p]),
    "sc_lobpcg_step_poll": (_int, [_p, _p, C.POINTER(_int), C.POINTER(_int)]),
    "sc_lobpcg_end": (_int, [_p, _p, _p, _p, _p, C.POINTER(sc_lobpcg_info)]),
    "sc_kmeans_workspace": (_int, [_p, _i64, _int, C.POINTER(sc_kmeans_opts), C.POINTER(_size)]),
    "sc_kmeans_assign": (_int, [_p, _i64, _int, _p, _i64, C.POINTER(sc_kmeans_opts), _p, _p, _p,
                                _p, C.POINTER(_dbl), C.POINTER(C.c_uint64), C.POINTER(_int),
                                C.POINTER(_int), _p, _size]),
    "sc_kmeans_assign_static": (_int, [_p, _i64, _int, _p, _i64, C.POINTER(sc_kmeans_opts), _p,
                                       _p, _p, _p, C.POINTER(_dbl), C.POINTER(C.c_uint64),
                                       C.POINTER(_int), C.POINTER(_int)]),
    "sc_ctx_set_profiling": (_int, [_p, C.c_uint]),
    "sc_ctx_profile": (_int, [_p, _int, C.POINTER(_i64), C.POINTER(_dbl)]),
    "sc_ctx_profile_reset": (_int, [_p]),
    "sc_cpqr_workspace": (_int, [_p, _i64, _int, _int, C.POINTER(_size)]),
    "sc_cpqr_labels": (_int, [_p, _i64, _int, _p, _i64, _int, _p, _p, _p, _p, _size]),
    "sc_eigengap": (_int, [_p, _int, _p, _dbl, _p, _p]),
    "sc_warm_fill": (_int, [_p, _i64, _i64, _p, _p, _int, _p, _i64, _int]),
    "sc_symeig_workspace": (_int, [_p, _int, _int, C.POINTER(_size)]),
    "sc_symeig": (_int, [_p, _int, _int, _p, _p, _p, _p, _size]),
    "sc_randn": (_int, [_p, _i64, _int, _i64, C.c_uint64, C.c_uint64, _int, _p, _int]),
    "sc_spmm_ex": (_int, [_p, _i64, _i64, _p, _p, _p, _p, _int, _p, _i64, _p, _i64, _int, _p, _p,
                          _i64]),
    "sc_row_order_workspace": (_int, [_p, _i64, C.POINTER(_size)]),
    "sc_row_order": (_int, [_p, _i64, _p, _p, _p, _size]),
}

_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is missing: build it with "
                               "`python -m paper_1708_07481_amd.build` (no CPU fallback exists)")
        L = C.CDLL(LIB_PATH)
        for name, (res, args) in SIGNATURES.items():
            f = getattr(L, name, None)
            if f is None:
                continue          # calling it raises AttributeError
            f.restype = res
            f.argtypes = args
        _lib = L
    return _lib


class SpectralError(RuntimeError):
    def __init__(self, status: int, what: str, msg: str = ""):
        super().__init__(f"{what}: {STATUS_NAMES.get(status, status)} {msg}".strip())
        self.status = status
