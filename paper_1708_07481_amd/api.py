"""Python entry points over the C ABI: argument marshalling only.

Every array is a torch tensor on the GPU (torch provides device memory and the
stream); every step of the computation runs in the HIP library.
"""
from __future__ import annotations

import ctypes as C
import sys
from dataclasses import dataclass

import torch

from . import _lib
from ._lib import (SC_PREC_FP32, SC_PREC_FP32_BF16GRAM, SC_PREC_FP64, SC_SYM_ALGEBRAIC,
                   SC_SYM_LOGICAL, SpectralError, lib)

PRECISIONS = {"fp64": SC_PREC_FP64, "fp32": SC_PREC_FP32, "fp32_bf16gram": SC_PREC_FP32_BF16GRAM}


def _ptr(t):
    return None if t is None else C.c_void_p(t.data_ptr())


class Context:
    """A library context bound to a device and to torch's current stream."""

    def __init__(self, device: int = 0, stream: torch.cuda.Stream | None = None):
        if not torch.cuda.is_available():
            raise RuntimeError("no GPU visible: the spectral library runs on the GPU only")
        self.device = device
        self.stream = stream if stream is not None else torch.cuda.current_stream(device)
        h = C.c_void_p()
        st = lib().sc_ctx_create(device, C.c_void_p(self.stream.cuda_stream), C.byref(h))
        if st != 0:
            raise SpectralError(st, "sc_ctx_create")
        self.handle = h

    def check(self, st: int, what: str):
        if st != 0:
            msg = lib().sc_last_error(self.handle)
            raise SpectralError(st, what, msg.decode() if msg else "")

    def workspace(self, nbytes: int) -> torch.Tensor:
        return torch.empty(max(int(nbytes), 256), dtype=torch.uint8, device=f"cuda:{self.device}")

    def set_profiling(self, kinds=()):
        mask = 0
        for k in kinds:
            mask |= 1 << (_lib.KIND_NAMES.index(k) if isinstance(k, str) else int(k))
        self.check(lib().sc_ctx_set_profiling(self.handle, mask), "sc_ctx_set_profiling")

    def profile(self) -> dict:
        out = {}
        for i, name in enumerate(_lib.KIND_NAMES):
            cnt = C.c_int64()
            ms = C.c_double()
            self.check(lib().sc_ctx_profile(self.handle, i, C.byref(cnt), C.byref(ms)),
                       "sc_ctx_profile")
            if cnt.value:
                out[name] = {"launches": cnt.value, "total_ms": ms.value,
                             "avg_ms": ms.value / cnt.value}
        return out

    def profile_reset(self):
        self.check(lib().sc_ctx_profile_reset(self.handle), "sc_ctx_profile_reset")

    def close(self):
        """Destroy the library context (synchronises its stream).  Programs
        call this before they exit: a context still open when the
        interpreter shuts down is left to the process exit, since the HIP
        runtime may already be going away then."""
        if getattr(self, "handle", None):
            lib().sc_ctx_destroy(self.handle)
            self.handle = None

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    def __del__(self, _finalizing=sys.is_finalizing):
        # module globals (sys, lib) may already be gone at interpreter exit
        if not getattr(self, "handle", None) or _finalizing():
            return
        try:
            self.close()
        except Exception:
            pass


def runtime_info() -> dict:
    """HIP runtime version, number of libamdhip64 copies mapped into the
    process and the path of the one the library calls."""
    v, cnt = C.c_int(), C.c_int()
    buf = C.create_string_buffer(4096)
    st = lib().sc_runtime_info(C.byref(v), C.byref(cnt), buf, len(buf))
    if st != 0:
        raise SpectralError(st, "sc_runtime_info")
    return {"hip_runtime_version": v.value, "hip_libs_mapped": cnt.value,
            "libamdhip64": buf.value.decode()}


@dataclass
class DeviceCSR:
    n: int
    nnz: int
    row_ptr: torch.Tensor   # int64 [n+1]
    col: torch.Tensor       # int32 [nnz]
    w_sym: torch.Tensor | None
    degree: torch.Tensor    # float64 [n]
    self_loops: int = 0


def graph_build(ctx: Context, n: int, src: torch.Tensor, dst: torch.Tensor,
                w: torch.Tensor | None = None, algebraic: bool = False,
                ws: torch.Tensor | None = None) -> DeviceCSR:
    dev = src.device
    m = int(src.numel())
    nb = C.c_size_t()
    ctx.check(lib().sc_graph_build_workspace(ctx.handle, n, m, C.byref(nb)), "sc_graph_build_workspace")
    if ws is None or ws.numel() < nb.value:
        ws = ctx.workspace(nb.value)
    row_ptr = torch.empty(n + 1, dtype=torch.int64, device=dev)
    col = torch.empty(max(2 * m, 1), dtype=torch.int32, device=dev)
    w_sym = torch.empty(max(2 * m, 1), dtype=torch.float64, device=dev) if algebraic else None
    degree = torch.empty(n, dtype=torch.float64, device=dev)
    nnz = C.c_int64()
    loops = C.c_int64()
    ctx.check(lib().sc_graph_build(ctx.handle, n, m, _ptr(src), _ptr(dst), _ptr(w),
                                   SC_SYM_ALGEBRAIC if algebraic else SC_SYM_LOGICAL,
                                   _ptr(row_ptr), _ptr(col), _ptr(w_sym), _ptr(degree),
                                   C.byref(nnz), C.byref(loops), _ptr(ws), nb.value),
              "sc_graph_build")
    z = nnz.value
    return DeviceCSR(n, z, row_ptr, col[:max(z, 1)], None if w_sym is None else w_sym[:max(z, 1)],
                     degree, loops.value)


def laplacian_csr(ctx: Context, g: DeviceCSR, fp64: bool = True, fp32: bool = False):
    dev = g.row_ptr.device
    val64 = torch.empty(max(g.nnz, 1), dtype=torch.float64, device=dev) if fp64 else None
    val32 = torch.empty(max(g.nnz, 1), dtype=torch.float32, device=dev) if fp32 else None
    dis = torch.empty(g.n, dtype=torch.float64, device=dev)
    ctx.check(lib().sc_laplacian_csr(ctx.handle, g.n, g.nnz, _ptr(g.row_ptr), _ptr(g.col),
                                     _ptr(g.w_sym), _ptr(g.degree), _ptr(val64), _ptr(val32),
                                     _ptr(dis)), "sc_laplacian_csr")
    return val64, val32, dis


def laplacian_combinatorial(ctx: Context, g: DeviceCSR, fp64: bool = True, fp32: bool = False):
    """L = D - W: off-diagonal values (FP64 and/or FP32) and the FP32 diagonal
    (the FP64 diagonal is g.degree itself)."""
    dev = g.row_ptr.device
    val64 = torch.empty(max(g.nnz, 1), dtype=torch.float64, device=dev) if fp64 else None
    val32 = torch.empty(max(g.nnz, 1), dtype=torch.float32, device=dev) if fp32 else None
    diag32 = torch.empty(g.n, dtype=torch.float32, device=dev) if fp32 else None
    ctx.check(lib().sc_laplacian_combinatorial(ctx.handle, g.n, g.nnz, _ptr(g.row_ptr),
                                               _ptr(g.w_sym), _ptr(g.degree), _ptr(val64),
                                               _ptr(val32), _ptr(diag32)),
              "sc_laplacian_combinatorial")
    return val64, val32, diag32


def spmm(ctx: Context, g: DeviceCSR, val: torch.Tensor, X: torch.Tensor,
         Y: torch.Tensor | None = None, diag: torch.Tensor | None = None) -> torch.Tensor:
    n, k = X.shape
    if Y is None:
        Y = torch.empty_like(X)
    fp64 = X.dtype == torch.float64
    if val.dtype != X.dtype or Y.dtype != X.dtype or (diag is not None and diag.dtype != X.dtype):
        raise TypeError("val, diag, X and Y must share one dtype")
    ctx.check(lib().sc_spmm_diag(ctx.handle, n, g.nnz, _ptr(g.row_ptr), _ptr(g.col), _ptr(val),
                                 _ptr(diag), int(fp64), k, _ptr(X), X.stride(0), _ptr(Y),
                                 Y.stride(0)), "sc_spmm_diag")
    return Y


def spmm_ex(ctx: Context, g: DeviceCSR, val: torch.Tensor, X: torch.Tensor,
            Y: torch.Tensor | None = None, Xg: torch.Tensor | None = None,
            order: torch.Tensor | None = None, diag: torch.Tensor | None = None,
            lane16: bool = False) -> torch.Tensor:
    """FP32 Y = L X with an optional 16-bit gather copy Xg (float16 or
    bfloat16) and an optional row order (int32 permutation); lane16 takes
    16-byte lane reads of the FP32 neighbour rows instead of 4-byte ones."""
    n, k = X.shape
    if X.dtype != torch.float32 or val.dtype != torch.float32:
        raise TypeError("spmm_ex takes FP32 X and values")
    if Y is None:
        Y = torch.empty_like(X)
    gather = _lib.SC_GATHER_FP32_LANE16 if lane16 else _lib.SC_GATHER_FP32
    if Xg is not None:
        gather = {torch.float16: _lib.SC_GATHER_FP16, torch.bfloat16: _lib.SC_GATHER_BF16}[Xg.dtype]
    ctx.check(lib().sc_spmm_ex(ctx.handle, n, g.nnz, _ptr(g.row_ptr), _ptr(g.col), _ptr(val),
                               _ptr(diag), k, _ptr(X), X.stride(0), _ptr(Xg),
                               Xg.stride(0) if Xg is not None else 0, gather, _ptr(order),
                               _ptr(Y), Y.stride(0)), "sc_spmm_ex")
    return Y


def row_order(ctx: Context, g: DeviceCSR) -> torch.Tensor:
    """The rows by descending length (stable), int32."""
    nb = C.c_size_t()
    ctx.check(lib().sc_row_order_workspace(ctx.handle, g.n, C.byref(nb)), "sc_row_order_workspace")
    ws = ctx.workspace(nb.value)
    order = torch.empty(g.n, dtype=torch.int32, device=g.row_ptr.device)
    ctx.check(lib().sc_row_order(ctx.handle, g.n, _ptr(g.row_ptr), _ptr(order), _ptr(ws), nb.value),
              "sc_row_order")
    return order


@dataclass
class LobpcgResult:
    X: torch.Tensor
    theta: torch.Tensor
    relres_hist: "list | None"
    iterations: int
    converged: bool
    p_drops: int
    locked_cols: int
    max_relres: float
    w_drops: int = 0
    gram_fallbacks: int = 0
    restarts: int = 0


def lobpcg_opts(k, maxit, tol, precision, ldx, lock_tol=0.0, chol_tol=0.0, diag=None,
                op_norm=0.0, k_conv=0):
    return _lib.sc_lobpcg_opts(k, maxit, tol, PRECISIONS[precision], ldx, lock_tol, chol_tol,
                               _ptr(diag), op_norm, k_conv)


def lobpcg_workspace(ctx: Context, n, nnz, opts) -> int:
    nb = C.c_size_t()
    ctx.check(lib().sc_lobpcg_workspace(ctx.handle, n, nnz, C.byref(opts), C.byref(nb)),
              "sc_lobpcg_workspace")
    return nb.value


def lobpcg_solve(ctx: Context, g: DeviceCSR, val: torch.Tensor, X0: torch.Tensor, maxit: int,
                 tol: float = 0.0, precision: str = "fp64", lock_tol: float = 0.0,
                 chol_tol: float = 0.0, history: bool = True, ws: torch.Tensor | None = None,
                 X_out: torch.Tensor | None = None, diag: torch.Tensor | None = None,
                 op_norm: float = 0.0, k_conv: int = 0) -> LobpcgResult:
    """diag None: the normalised Laplacian (unit diagonal, op_norm 2).  With a
    diagonal (L = D - W) and op_norm 0 the library bounds ||L|| by 2 max(diag)
    (Gershgorin)."""
    import numpy as np
    n, k = X0.shape
    if diag is not None and diag.dtype != X0.dtype:
        raise TypeError("diag must have X0's dtype")
    opts = lobpcg_opts(k, maxit, tol, precision, X0.stride(0), lock_tol, chol_tol, diag, op_norm,
                       k_conv)
    nb = lobpcg_workspace(ctx, n, g.nnz, opts)
    if ws is None or ws.numel() < nb:
        ws = ctx.workspace(nb)
    if X_out is None:
        X_out = torch.empty_like(X0)
    theta = torch.empty(k, dtype=torch.float64, device=X0.device)
    hist = np.zeros((maxit + 1) * k, dtype=np.float64) if history else None
    info = _lib.sc_lobpcg_info()
    ctx.check(lib().sc_lobpcg_solve(ctx.handle, n, g.nnz, _ptr(g.row_ptr), _ptr(g.col), _ptr(val),
                                    C.byref(opts), _ptr(X0), _ptr(X_out), _ptr(theta),
                                    None if hist is None else hist.ctypes.data_as(C.c_void_p),
                                    C.byref(info), _ptr(ws), nb), "sc_lobpcg_solve")
    it = info.iterations
    return LobpcgResult(X_out, theta, None if hist is None else hist.reshape(maxit + 1, k)[: it + 1],
                        it, bool(info.converged), info.p_drops, info.locked_cols, info.max_relres,
                        info.w_drops, info.gram_fallbacks, info.restarts)


def lobpcg_status(ctx: Context, g: DeviceCSR, val, X0, maxit, tol=0.0, precision="fp64") -> int:
    """Status code of a solve (for the failure-path tests)."""
    n, k = X0.shape
    opts = lobpcg_opts(k, maxit, tol, precision, X0.stride(0))
    nb = C.c_size_t()
    st = lib().sc_lobpcg_workspace(ctx.handle, n, g.nnz, C.byref(opts), C.byref(nb))
    if st != 0:
        return st
    ws = ctx.workspace(nb.value)
    X_out = torch.empty_like(X0)
    theta = torch.empty(max(k, 1), dtype=torch.float64, device=X0.device)
    info = _lib.sc_lobpcg_info()
    return lib().sc_lobpcg_solve(ctx.handle, n, g.nnz, _ptr(g.row_ptr), _ptr(g.col), _ptr(val),
                                 C.byref(opts), _ptr(X0), _ptr(X_out), _ptr(theta), None,
                                 C.byref(info), _ptr(ws), nb.value)


@dataclass
class KmeansResult:
    labels: torch.Tensor
    centroids: torch.Tensor
    inertia: float
    inertia_q: int
    best_restart: int
    lloyd_iterations: int = 0


def kmeans_assign(ctx: Context, X: torch.Tensor, n_clusters: int, draws: torch.Tensor | None,
                  restarts: int | None = None, max_iter: int = 100, normalize: bool = True,
                  init_centroids: torch.Tensor | None = None,
                  ws: torch.Tensor | None = None, scan: str = "auto") -> KmeansResult:
    n, dim = X.shape
    if init_centroids is not None:
        restarts = 1
    elif restarts is None:
        restarts = draws.shape[0]
    if X.dtype not in (torch.float64, torch.float32):
        raise TypeError("X must be float64 or float32")
    scan_mode = {"auto": _lib.SC_KM_SCAN_AUTO, "pruned": _lib.SC_KM_SCAN_PRUNED,
                 "full": _lib.SC_KM_SCAN_FULL}[scan]
    opts = _lib.sc_kmeans_opts(n_clusters, restarts, max_iter, int(bool(normalize)),
                               int(X.dtype == torch.float32), scan_mode)
    nb = C.c_size_t()
    ctx.check(lib().sc_kmeans_workspace(ctx.handle, n, dim, C.byref(opts), C.byref(nb)),
              "sc_kmeans_workspace")
    if ws is None or ws.numel() < nb.value:
        ws = ctx.workspace(nb.value)
    labels = torch.empty(n, dtype=torch.int32, device=X.device)
    cent = torch.empty((n_clusters, dim), dtype=torch.float64, device=X.device)
    inertia = C.c_double()
    iq = C.c_uint64()
    br = C.c_int()
    its = C.c_int()
    ctx.check(lib().sc_kmeans_assign(ctx.handle, n, dim, _ptr(X), X.stride(0), C.byref(opts),
                                     _ptr(draws), _ptr(init_centroids), _ptr(labels), _ptr(cent),
                                     C.byref(inertia), C.byref(iq), C.byref(br), C.byref(its),
                                     _ptr(ws), nb.value), "sc_kmeans_assign")
    return KmeansResult(labels, cent, inertia.value, iq.value, br.value, its.value)


@dataclass
class CpqrResult:
    pivots: torch.Tensor
    labels: torch.Tensor
    Q: torch.Tensor


def cpqr_labels(ctx: Context, X: torch.Tensor, ws: torch.Tensor | None = None) -> CpqrResult:
    """Labels by QR with column pivoting of X' (rows of X = vertices)."""
    n, k = X.shape
    if X.dtype not in (torch.float64, torch.float32) or X.stride(1) != 1:
        raise TypeError("X must be float64 or float32 with unit column stride")
    fp32 = int(X.dtype == torch.float32)
    nb = C.c_size_t()
    ctx.check(lib().sc_cpqr_workspace(ctx.handle, n, k, fp32, C.byref(nb)), "sc_cpqr_workspace")
    if ws is None or ws.numel() < nb.value:
        ws = ctx.workspace(nb.value)
    piv = torch.empty(k, dtype=torch.int32, device=X.device)
    lab = torch.empty(n, dtype=torch.int32, device=X.device)
    Q = torch.empty((k, k), dtype=torch.float64, device=X.device)
    ctx.check(lib().sc_cpqr_labels(ctx.handle, n, k, _ptr(X), X.stride(0), fp32, _ptr(piv),
                                   _ptr(lab), _ptr(Q), _ptr(ws), nb.value), "sc_cpqr_labels")
    return CpqrResult(piv, lab, Q)


def warm_fill(ctx: Context, g: DeviceCSR, X: torch.Tensor, n_old: int) -> torch.Tensor:
    """In place: rows >= n_old of the start block X become the mean of their
    old neighbours' rows (zero without one)."""
    n, k = X.shape
    if X.dtype not in (torch.float64, torch.float32) or X.stride(1) != 1:
        raise TypeError("X must be float64 or float32 with unit column stride")
    ctx.check(lib().sc_warm_fill(ctx.handle, n, n_old, _ptr(g.row_ptr), _ptr(g.col), k, _ptr(X),
                                 X.stride(0), int(X.dtype == torch.float32)), "sc_warm_fill")
    return X


def eigengap(ctx: Context, theta: torch.Tensor, sig: float = 10.0):
    """(count, ratio): number of Ritz values below the first increment more
    than sig times the mean of the ones before it (else below the largest),
    and that increment over the median one."""
    k = theta.numel()
    cnt = torch.empty(1, dtype=torch.int32, device=theta.device)
    ratio = torch.empty(1, dtype=torch.float64, device=theta.device)
    ctx.check(lib().sc_eigengap(ctx.handle, k, _ptr(theta), sig, _ptr(cnt), _ptr(ratio)),
              "sc_eigengap")
    return int(cnt.item()), float(ratio.item())


def randn(ctx: Context, rows: int, cols: int, seed: int, stream: int = 0,
          dist: str = "normal", dtype=torch.float64, out: torch.Tensor | None = None,
          device=None) -> torch.Tensor:
    """rows x cols block from the device Philox4x64-10 stream keyed (seed,
    stream): Gaussian (Box-Muller), uniform on [-1, 1), or the raw 64-bit
    words (dtype int64 holding the uint64 bits)."""
    code = {"normal": _lib.SC_RAND_NORMAL, "uniform": _lib.SC_RAND_UNIFORM,
            "raw": _lib.SC_RAND_RAW}[dist]
    if dist == "raw":
        dtype = torch.int64
    elif dtype not in (torch.float64, torch.float32):
        raise TypeError("dtype must be float64 or float32")
    if out is None:
        out = torch.empty((rows, cols), dtype=dtype,
                          device=device if device is not None else f"cuda:{ctx.device}")
    if out.shape != (rows, cols) or out.dtype != dtype or out.stride(1) != 1:
        raise TypeError("out must be a rows x cols block of dtype with unit column stride")
    prec = SC_PREC_FP64 if dtype in (torch.float64, torch.int64) else SC_PREC_FP32
    ctx.check(lib().sc_randn(ctx.handle, rows, cols, out.stride(0) if rows else cols,
                             seed & 0xFFFFFFFFFFFFFFFF, stream & 0xFFFFFFFFFFFFFFFF, code,
                             _ptr(out), prec), "sc_randn")
    return out


def symeig(ctx: Context, A: torch.Tensor, k: int, ws: torch.Tensor | None = None):
    m = A.shape[0]
    nb = C.c_size_t()
    ctx.check(lib().sc_symeig_workspace(ctx.handle, m, k, C.byref(nb)), "sc_symeig_workspace")
    if ws is None or ws.numel() < nb.value:
        ws = ctx.workspace(nb.value)
    w = torch.empty(k, dtype=torch.float64, device=A.device)
    V = torch.empty((m, k), dtype=torch.float64, device=A.device)
    ctx.check(lib().sc_symeig(ctx.handle, m, k, _ptr(A), _ptr(w), _ptr(V), _ptr(ws), nb.value),
              "sc_symeig")
    return w, V
