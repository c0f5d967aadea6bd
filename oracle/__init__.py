"""Plain FP64 CPU oracle (test infrastructure).

The oracle is the reference the GPU library is checked against.  Only the
tests, ``__graft_entry__.smoke()`` and the CPU-baseline leg of ``bench.py`` may
import it; the product package never does.  It is a thin ctypes wrapper over
``oracle.c`` (plain C, FP64, built with gcc -O2 -ffp-contract=off) and shares
no code with the HIP library.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess
from dataclasses import dataclass

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")

OK, E_INVAL, E_NOMEM, E_BREAKDOWN, E_NUMERIC = 0, -1, -2, -4, -5


def build(force: bool = True) -> str:
    """Compile oracle.c into liboracle.so next to it."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp"
        cmd = ["gcc", "-O2", "-ffp-contract=off", "-fno-fast-math", "-fopenmp", "-fPIC",
               "-shared", "-std=c11", "-Wall", "-Wno-unused-function", "-o", tmp, _SRC, "-lm"]
        subprocess.run(cmd, check=True)
        os.replace(tmp, _LIB)
    return _LIB


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
            build(force=True)
        _lib = C.CDLL(_LIB)
        _declare(_lib)
    return _lib


_p = C.c_void_p
_i64 = C.c_int64
_int = C.c_int
_dbl = C.c_double


class LobpcgOpts(C.Structure):
    _fields_ = [("k", _int), ("maxit", _int), ("tol", _dbl), ("lock_tol", _dbl),
                ("chol_tol", _dbl), ("op_norm", _dbl), ("k_conv", _int)]


class LobpcgInfo(C.Structure):
    _fields_ = [("iterations", _int), ("converged", _int), ("p_drops", _int),
                ("locked_cols", _int), ("max_relres", _dbl), ("seconds_setup", _dbl),
                ("seconds_iters", _dbl)]


def _declare(L):
    L.orc_graph_build.restype = _int
    L.orc_graph_build.argtypes = [_i64, _i64, _p, _p, _p, _int, _p, _p, _p, _p, _p, _p]
    L.orc_laplacian.restype = _int
    L.orc_laplacian.argtypes = [_i64, _p, _p, _p, _p, _p, _p]
    L.orc_laplacian_combinatorial.restype = _int
    L.orc_laplacian_combinatorial.argtypes = [_i64, _p, _p, _p, _p]
    L.orc_spmm_rowmajor.restype = None
    L.orc_spmm_rowmajor.argtypes = [_i64, _p, _p, _p, _p, _int, _p, _i64, _p, _i64]
    L.orc_gram.restype = None
    L.orc_gram.argtypes = [_i64, _int, _p, _int, _p, _p, _int]
    L.orc_cholesky.restype = _int
    L.orc_cholesky.argtypes = [_int, _p, _p, _dbl]
    L.orc_symeig.restype = _int
    L.orc_symeig.argtypes = [_int, _p, _p, _p]
    L.orc_lobpcg.restype = _int
    L.orc_lobpcg.argtypes = [_i64, _p, _p, _p, _p, C.POINTER(LobpcgOpts), _p, _p, _p, _p, _p,
                             C.POINTER(LobpcgInfo)]
    L.orc_kmeans.restype = _int
    L.orc_kmeans.argtypes = [_i64, _int, _p, _i64, _int, _int, _int, _p, _p, _int, _p, _p,
                             _p, _p, _p, _p, _p]
    L.orc_cpqr_labels.restype = _int
    L.orc_cpqr_labels.argtypes = [_i64, _int, _p, _i64, _p, _p, _p]
    L.orc_eigengap.restype = _int
    L.orc_eigengap.argtypes = [_int, _p, _dbl, C.POINTER(_dbl)]
    L.orc_warm_fill.restype = None
    L.orc_warm_fill.argtypes = [_i64, _i64, _p, _p, _int, _p, _i64]
    L.orc_row_normalize.restype = None
    L.orc_row_normalize.argtypes = [_i64, _int, _p, _i64, _p]


def _ptr(a):
    return None if a is None else a.ctypes.data_as(C.c_void_p)


class OracleError(RuntimeError):
    def __init__(self, code, what):
        super().__init__(f"oracle {what} failed with status {code}")
        self.code = code


def _check(code, what):
    if code != OK:
        raise OracleError(code, what)


@dataclass
class CSR:
    n: int
    row_ptr: np.ndarray     # int64 [n+1]
    col: np.ndarray         # int32 [nnz]
    w: np.ndarray | None    # float64 [nnz] (None: unit weights)
    degree: np.ndarray      # float64 [n]
    self_loops: int = 0

    @property
    def nnz(self) -> int:
        return int(self.row_ptr[-1])


def graph_build(n, src, dst, w=None, algebraic=False) -> CSR:
    """Symmetrisation W + W' of a directed COO graph (Section II-A)."""
    src = np.ascontiguousarray(src, dtype=np.int32)
    dst = np.ascontiguousarray(dst, dtype=np.int32)
    m = src.shape[0]
    wv = None if w is None else np.ascontiguousarray(w, dtype=np.float64)
    row_ptr = np.zeros(n + 1, dtype=np.int64)
    col = np.zeros(max(2 * m, 1), dtype=np.int32)
    wsym = np.zeros(max(2 * m, 1), dtype=np.float64)
    deg = np.zeros(n, dtype=np.float64)
    nnz = np.zeros(1, dtype=np.int64)
    loops = np.zeros(1, dtype=np.int64)
    _check(lib().orc_graph_build(n, m, _ptr(src), _ptr(dst), _ptr(wv), int(bool(algebraic)),
                                 _ptr(row_ptr), _ptr(col), _ptr(wsym), _ptr(deg), _ptr(nnz),
                                 _ptr(loops)), "graph_build")
    z = int(nnz[0])
    return CSR(n, row_ptr, col[:z].copy(), wsym[:z].copy() if algebraic else None, deg,
               int(loops[0]))


def laplacian(g: CSR):
    """Off-diagonal values of L = I - D^-1/2 W D^-1/2 and D^-1/2."""
    val = np.zeros(max(g.nnz, 1), dtype=np.float64)
    dis = np.zeros(g.n, dtype=np.float64)
    _check(lib().orc_laplacian(g.n, _ptr(g.row_ptr), _ptr(g.col), _ptr(g.w), _ptr(g.degree),
                               _ptr(val), _ptr(dis)), "laplacian")
    return val[: g.nnz].copy(), dis


def laplacian_combinatorial(g: CSR):
    """L = D - W (Section II-A): off-diagonal values -w and the diagonal (degrees)."""
    val = np.zeros(max(g.nnz, 1), dtype=np.float64)
    _check(lib().orc_laplacian_combinatorial(g.n, _ptr(g.row_ptr), _ptr(g.col), _ptr(g.w),
                                             _ptr(val)), "laplacian_combinatorial")
    return val[: g.nnz].copy(), g.degree.copy()


def spmm(g: CSR, val, X, diag=None):
    """Y = L X for a row-major n x k block (same arithmetic as the definition);
    diag None: unit diagonal (normalised Laplacian)."""
    X = np.ascontiguousarray(X, dtype=np.float64)
    n, k = X.shape
    Y = np.empty_like(X)
    v = np.ascontiguousarray(val, dtype=np.float64)
    d = None if diag is None else np.ascontiguousarray(diag, dtype=np.float64)
    lib().orc_spmm_rowmajor(n, _ptr(g.row_ptr), _ptr(g.col), _ptr(v), _ptr(d), k, _ptr(X), k,
                            _ptr(Y), k)
    return Y


def dense_laplacian(g: CSR, val, diag=None) -> np.ndarray:
    """Dense L (tests only, small n)."""
    L = np.eye(g.n) if diag is None else np.diag(np.asarray(diag, dtype=np.float64))
    for i in range(g.n):
        for p in range(g.row_ptr[i], g.row_ptr[i + 1]):
            L[i, g.col[p]] += val[p]
    return L


def gram(A, B, sym=False):
    """A^T B with sequential fma sums over rows (A, B: n x ca, n x cb)."""
    A = np.asfortranarray(A, dtype=np.float64)
    B = np.asfortranarray(B, dtype=np.float64)
    G = np.zeros((A.shape[1], B.shape[1]))
    lib().orc_gram(A.shape[0], A.shape[1], _ptr(A), B.shape[1], _ptr(B), _ptr(G), int(sym))
    return G


def cholesky(G, tol=0.0):
    G = np.ascontiguousarray(G, dtype=np.float64)
    R = np.zeros_like(G)
    _check(lib().orc_cholesky(G.shape[0], _ptr(G), _ptr(R), tol), "cholesky")
    return R


def symeig(A):
    """Cyclic Jacobi eigendecomposition: ascending eigenvalues, eigenvectors in columns."""
    A = np.ascontiguousarray(A, dtype=np.float64)
    m = A.shape[0]
    w = np.zeros(m)
    V = np.zeros((m, m))
    _check(lib().orc_symeig(m, _ptr(A), _ptr(w), _ptr(V)), "symeig")
    return w, V


# default floors per precision (documented with the library)
LOCK_TOL = 1e-13
CHOL_TOL = 1e-14


@dataclass
class LobpcgResult:
    X: np.ndarray
    theta: np.ndarray
    relres_hist: np.ndarray
    theta_hist: np.ndarray
    iterations: int
    converged: bool
    p_drops: int
    locked_cols: int
    max_relres: float
    seconds_setup: float = 0.0     # wall time of the start-up (CholQR2, L X, first RR)
    seconds_iters: float = 0.0     # wall time of the iterations after it


def op_norm_bound(diag) -> float:
    """||L|| bound for the relative residual: 2 for the normalised Laplacian
    (diag None), 2 max_i d_i for L = D - W (Gershgorin)."""
    return 2.0 if diag is None else 2.0 * float(np.max(diag)) if len(diag) else 2.0


def lobpcg(g: CSR, val, X0, maxit, tol=0.0, lock_tol=LOCK_TOL, chol_tol=CHOL_TOL,
           diag=None, k_conv=0) -> LobpcgResult:
    """Smallest-k eigenpairs of L by block LOBPCG without preconditioning
    (diag None: the normalised Laplacian; else L = diag + offdiag(val))."""
    X0 = np.ascontiguousarray(X0, dtype=np.float64)
    n, k = X0.shape
    X = np.zeros_like(X0)
    theta = np.zeros(k)
    rh = np.zeros((maxit + 1, k))
    th = np.zeros((maxit + 1, k))
    o = LobpcgOpts(k, maxit, tol, lock_tol, chol_tol, op_norm_bound(diag), k_conv)
    info = LobpcgInfo()
    v = np.ascontiguousarray(val, dtype=np.float64)
    d = None if diag is None else np.ascontiguousarray(diag, dtype=np.float64)
    _check(lib().orc_lobpcg(n, _ptr(g.row_ptr), _ptr(g.col), _ptr(v), _ptr(d), C.byref(o),
                            _ptr(X0), _ptr(X), _ptr(theta), _ptr(rh), _ptr(th), C.byref(info)),
           "lobpcg")
    it = info.iterations
    return LobpcgResult(X, theta, rh[: it + 1].copy(), th[: it + 1].copy(), it,
                        bool(info.converged), info.p_drops, info.locked_cols, info.max_relres,
                        info.seconds_setup, info.seconds_iters)


def lobpcg_status(g: CSR, val, X0, maxit, tol=0.0, lock_tol=LOCK_TOL, chol_tol=CHOL_TOL) -> int:
    """Status code only (for the failure-path tests)."""
    X0 = np.ascontiguousarray(X0, dtype=np.float64)
    n, k = X0.shape
    o = LobpcgOpts(k, maxit, tol, lock_tol, chol_tol, 2.0)
    info = LobpcgInfo()
    X = np.zeros_like(X0)
    theta = np.zeros(k)
    v = np.ascontiguousarray(val, dtype=np.float64)
    return lib().orc_lobpcg(n, _ptr(g.row_ptr), _ptr(g.col), _ptr(v), None, C.byref(o),
                            _ptr(X0), _ptr(X), _ptr(theta), None, None, C.byref(info))


@dataclass
class KmeansResult:
    labels: np.ndarray
    centroids: np.ndarray
    inertia: float
    inertia_q: int
    best_restart: int
    lloyd_iters: int
    # wall seconds of normalisation, seedings (+ first assignment), Lloyd updates,
    # and the number of Lloyd updates, all restarts together
    timing: tuple = (0.0, 0.0, 0.0, 0)


def kmeans(X, n_clusters, draws=None, restarts=None, max_iter=100, normalize=True,
           init_centroids=None) -> KmeansResult:
    X = np.ascontiguousarray(X, dtype=np.float64)
    n, dim = X.shape
    if init_centroids is not None:
        restarts = 1
        init = np.ascontiguousarray(init_centroids, dtype=np.float64)
        dr = None
    else:
        dr = np.ascontiguousarray(draws, dtype=np.uint64)
        restarts = dr.shape[0] if restarts is None else restarts
        init = None
    labels = np.zeros(n, dtype=np.int32)
    cent = np.zeros((n_clusters, dim))
    inertia = np.zeros(1)
    iq = np.zeros(1, dtype=np.uint64)
    br = np.zeros(1, dtype=np.int32)
    li = np.zeros(1, dtype=np.int32)
    tm = np.zeros(4)
    _check(lib().orc_kmeans(n, dim, _ptr(X), dim, n_clusters, restarts, max_iter, _ptr(dr),
                            _ptr(init), int(bool(normalize)), _ptr(labels), _ptr(cent),
                            _ptr(inertia), _ptr(iq), _ptr(br), _ptr(li), _ptr(tm)), "kmeans")
    return KmeansResult(labels, cent, float(inertia[0]), int(iq[0]), int(br[0]), int(li[0]),
                        (float(tm[0]), float(tm[1]), float(tm[2]), int(tm[3])))


@dataclass
class CpqrResult:
    pivots: np.ndarray
    labels: np.ndarray
    Q: np.ndarray


def cpqr_labels(X) -> CpqrResult:
    """Labels by QR with column pivoting of X' (pivots, polar factor Q, argmax |X Q|)."""
    X = np.ascontiguousarray(X, dtype=np.float64)
    n, k = X.shape
    piv = np.zeros(k, dtype=np.int32)
    lab = np.zeros(n, dtype=np.int32)
    Q = np.zeros((k, k))
    _check(lib().orc_cpqr_labels(n, k, _ptr(X), k, _ptr(piv), _ptr(lab), _ptr(Q)), "cpqr_labels")
    return CpqrResult(piv, lab, Q)


def eigengap(theta, sig=10.0):
    """(count, ratio): clusters below the first increment more than sig times
    the mean of the increments before it (else below the largest)."""
    t = np.ascontiguousarray(theta, dtype=np.float64)
    r = C.c_double()
    c = lib().orc_eigengap(len(t), _ptr(t), sig, C.byref(r))
    return c, r.value


def warm_fill(g: CSR, n_old, X):
    """Start block for a stage that adds vertices: rows >= n_old become the mean
    of their old neighbours' rows (zero without one)."""
    X = np.array(X, dtype=np.float64, order="C", copy=True)
    n, k = X.shape
    lib().orc_warm_fill(n, n_old, _ptr(g.row_ptr), _ptr(g.col), k, _ptr(X), k)
    return X


def row_normalize(X):
    X = np.ascontiguousarray(X, dtype=np.float64)
    Y = np.zeros_like(X)
    lib().orc_row_normalize(X.shape[0], X.shape[1], _ptr(X), X.shape[1], _ptr(Y))
    return Y


def partition(n, src, dst, k, X0, maxit, tol, draws, max_iter=100):
    """Whole path on the CPU: graph, Laplacian, LOBPCG, k-means."""
    g = graph_build(n, src, dst)
    val, _ = laplacian(g)
    res = lobpcg(g, val, X0, maxit, tol)
    km = kmeans(res.X, k, draws, max_iter=max_iter)
    return g, val, res, km
