"""GPU parity: the FP64 dense eigensolver of the Rayleigh-Ritz step and the
whole LOBPCG solve against the oracle on the same X0 (Section II-B /
Section III).  Bar (FP64): Ritz values within max(1e-8 |theta|, 1e-12),
subspace sine ||X_g - X_o (X_o' X_g)||_2 <= 1e-6, same iteration count."""
import numpy as np
import pytest

from synth import dcsbm, gaussian_block
from tests import graphs
from tests.gpu_common import gpu_ctx, host, to_dev

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ctx():
    return gpu_ctx()


def _sine(Xg, Xo):
    return np.linalg.norm(Xg - Xo @ (Xo.T @ Xg), 2)


def _theta_ok(tg, to):
    return np.all(np.abs(tg - to) <= np.maximum(1e-8 * np.abs(to), 1e-12))


@pytest.mark.parametrize("m,k", [(1, 1), (2, 2), (5, 3), (24, 8), (60, 20), (132, 44),
                                 (300, 98), (480, 160), (700, 50), (1000, 20)])
def test_symeig_vs_numpy(ctx, m, k):
    from paper_1708_07481_amd import api
    rng = np.random.default_rng(m)
    A = rng.standard_normal((m, m))
    A = (A + A.T) / 2
    w, V = api.symeig(ctx, to_dev(A), k)
    w, V = host(w), host(V)
    ref = np.linalg.eigvalsh(A)[:k]
    scale = max(1.0, np.abs(ref).max())
    assert np.allclose(w, ref, atol=1e-12 * scale * max(1, m / 50), rtol=0)
    assert np.abs(V.T @ V - np.eye(k)).max() < 1e-11
    assert np.abs(A @ V - V * w).max() < 1e-11 * scale


def test_symeig_degenerate_and_split(ctx):
    from paper_1708_07481_amd import api
    rng = np.random.default_rng(7)
    # exactly repeated eigenvalues, and a block-diagonal matrix (split tridiagonal)
    Q = np.linalg.qr(rng.standard_normal((40, 40)))[0]
    lam = np.repeat([0.0, 0.5, 1.0, 1.5], 10)
    A = Q @ np.diag(lam) @ Q.T
    A = (A + A.T) / 2
    w, V = api.symeig(ctx, to_dev(A), 15)
    w, V = host(w), host(V)
    assert np.allclose(w, lam[:15], atol=1e-12)
    assert np.abs(V.T @ V - np.eye(15)).max() < 1e-11
    assert np.abs(A @ V - V * w).max() < 1e-11
    B = np.zeros((30, 30))
    B[:15, :15] = np.diag(np.arange(15.0))
    B[15:, 15:] = np.diag(np.arange(15.0))
    w, V = api.symeig(ctx, to_dev(B), 10)
    w, V = host(w), host(V)
    assert np.allclose(w, np.repeat(np.arange(5.0), 2), atol=1e-13)
    assert np.abs(V.T @ V - np.eye(10)).max() < 1e-12
    assert np.abs(B @ V - V * w).max() < 1e-12


def _graph_pair(orc, ctx, n, src, dst, fp32=False):
    from paper_1708_07481_amd import api
    go = orc.graph_build(n, src, dst)
    vo, _ = orc.laplacian(go)
    gd = api.graph_build(ctx, n, to_dev(src), to_dev(dst))
    v64, v32, _ = api.laplacian_csr(ctx, gd, True, fp32)
    return go, vo, gd, v64, v32


LOBPCG_CASES = [
    # name, graph maker, k, maxit, tol
    ("sbm1k-k8-20it", lambda: dcsbm(1000, 8, 20.0, 0.8, seed=1), 8, 20, 0.0),
    ("sbm1k-seed3", lambda: dcsbm(1000, 8, 20.0, 0.8, seed=3), 8, 20, 0.0),
    ("sbm5k-k19-tol", lambda: dcsbm(5000, 19, 40.0, 0.75, "dirichlet", 5.0, seed=2), 19, 30, 1e-2),
    ("sbm3k-k13-ragged", lambda: dcsbm(3001, 13, 30.0, 0.7, "dirichlet", 2.0, seed=4), 13, 12, 0.0),
    ("sbm2k-k1", lambda: dcsbm(2000, 4, 20.0, 0.8, seed=5), 1, 15, 0.0),
]


@pytest.mark.parametrize("name,make,k,maxit,tol", LOBPCG_CASES, ids=[c[0] for c in LOBPCG_CASES])
def test_lobpcg_fp64_parity(orc, ctx, name, make, k, maxit, tol):
    from paper_1708_07481_amd import api
    g0 = make()
    go, vo, gd, v64, _ = _graph_pair(orc, ctx, g0.n, g0.src, g0.dst)
    X0 = gaussian_block(g0.n, k, 11)
    ro = orc.lobpcg(go, vo, X0, maxit, tol)
    rg = api.lobpcg_solve(ctx, gd, v64, to_dev(X0), maxit, tol, "fp64")
    tg, Xg = host(rg.theta), host(rg.X)
    print(name, "iters", ro.iterations, rg.iterations, "relres", ro.max_relres, rg.max_relres,
          "pdrops", ro.p_drops, rg.p_drops)
    assert rg.iterations == ro.iterations
    assert _theta_ok(tg, ro.theta), np.abs(tg - ro.theta).max()
    assert _sine(Xg, ro.X) <= 1e-6
    assert np.allclose(Xg.T @ Xg, np.eye(k), atol=1e-10)
    # relative residual history follows the oracle's
    assert np.allclose(rg.relres_hist, ro.relres_hist, rtol=1e-5, atol=1e-12)


def test_lobpcg_fp64_sbm50k(orc, ctx):
    """Full 50K / 1M / 44 workload (Table I shape) to tolerance 1e-2."""
    from paper_1708_07481_amd import api
    g0 = dcsbm(50_000, 44, 40.0, 0.75, "dirichlet", 5.0, seed=1)
    go, vo, gd, v64, _ = _graph_pair(orc, ctx, g0.n, g0.src, g0.dst)
    X0 = gaussian_block(g0.n, 44, 1)
    ro = orc.lobpcg(go, vo, X0, 30, 1e-2)
    rg = api.lobpcg_solve(ctx, gd, v64, to_dev(X0), 30, 1e-2, "fp64")
    assert rg.converged and ro.converged and rg.iterations == ro.iterations
    assert _theta_ok(host(rg.theta), ro.theta)
    assert _sine(host(rg.X), ro.X) <= 1e-6


def test_lobpcg_cliques_exact_convergence(orc, ctx):
    """Disjoint cliques: residuals reach the machine-precision floor, columns
    lock, and the subspace is the span of the D^1/2-scaled indicators."""
    from paper_1708_07481_amd import api
    n, src, dst = graphs.cliques([12, 15, 18, 21])
    go, vo, gd, v64, _ = _graph_pair(orc, ctx, n, src, dst)
    X0 = gaussian_block(n, 4, 2)
    rg = api.lobpcg_solve(ctx, gd, v64, to_dev(X0), 50, 1e-12, "fp64")
    tg, Xg = host(rg.theta), host(rg.X)
    assert np.all(np.abs(tg) < 1e-12)
    ro = orc.lobpcg(go, vo, X0, 50, 1e-12)
    assert _sine(Xg, ro.X) < 1e-8


def test_lobpcg_fp32_against_fp64_oracle(orc, ctx):
    from paper_1708_07481_amd import api
    g0 = dcsbm(5000, 19, 40.0, 0.75, "dirichlet", 5.0, seed=2)
    go, vo, gd, v64, v32 = _graph_pair(orc, ctx, g0.n, g0.src, g0.dst, fp32=True)
    X0 = gaussian_block(g0.n, 19, 11)
    ro = orc.lobpcg(go, vo, X0, 30, 1e-2)
    for prec in ("fp32", "fp32_bf16gram"):
        rg = api.lobpcg_solve(ctx, gd, v32, to_dev(X0.astype(np.float32)), 30, 1e-2, prec)
        assert rg.converged, prec
        # FP32 multivectors: Ritz values to ~1e-5, subspace to ~1e-3 of the FP64 result
        assert np.max(np.abs(host(rg.theta) - ro.theta)) < 1e-4, prec
        assert _sine(host(rg.X).astype(np.float64), ro.X) < 5e-2, prec


def test_step_api_matches_solve(orc, ctx):
    from paper_1708_07481_amd import api
    import ctypes as C
    import torch
    from paper_1708_07481_amd._lib import lib, sc_lobpcg_info
    g0 = dcsbm(3000, 10, 24.0, 0.8, seed=6)
    go, vo, gd, v64, _ = _graph_pair(orc, ctx, g0.n, g0.src, g0.dst)
    X0 = to_dev(gaussian_block(g0.n, 10, 3))
    a = api.lobpcg_solve(ctx, gd, v64, X0, 15, 0.0, "fp64")
    opts = api.lobpcg_opts(10, 15, 0.0, "fp64", 10)
    nb = api.lobpcg_workspace(ctx, g0.n, gd.nnz, opts)
    ws = ctx.workspace(nb)
    state = C.c_void_p()
    done = C.c_int()
    p = lambda t: C.c_void_p(t.data_ptr())
    ctx.check(lib().sc_lobpcg_begin(ctx.handle, g0.n, gd.nnz, p(gd.row_ptr), p(gd.col), p(v64),
                                    C.byref(opts), p(X0), p(ws), nb, C.byref(state),
                                    C.byref(done)), "begin")
    steps = 0
    while not done.value:
        ctx.check(lib().sc_lobpcg_step(ctx.handle, state, C.byref(done)), "step")
        steps += 1
    X = torch.empty_like(X0)
    th = torch.empty(10, dtype=torch.float64, device="cuda")
    info = sc_lobpcg_info()
    ctx.check(lib().sc_lobpcg_end(ctx.handle, state, p(X), p(th), None, C.byref(info)), "end")
    assert steps == 15 and info.iterations == 15
    assert torch.equal(X, a.X) and torch.equal(th, a.theta)


def test_lobpcg_failure_paths(orc, ctx):
    from paper_1708_07481_amd import api
    from paper_1708_07481_amd._lib import (SC_E_BREAKDOWN, SC_E_INVAL, SC_E_NUMERIC,
                                           SC_E_UNSUPPORTED)
    g0 = dcsbm(900, 4, 16.0, 0.8, seed=5)
    go, vo, gd, v64, _ = _graph_pair(orc, ctx, g0.n, g0.src, g0.dst)
    X0 = gaussian_block(g0.n, 4, 1)
    bad = X0.copy()
    bad[:, 3] = 2.0 * bad[:, 0]
    assert api.lobpcg_status(ctx, gd, v64, to_dev(bad), 5) == SC_E_BREAKDOWN
    zero = X0.copy()
    zero[:, 2] = 0.0
    assert api.lobpcg_status(ctx, gd, v64, to_dev(zero), 5) == SC_E_BREAKDOWN
    nan = X0.copy()
    nan[3, 1] = np.nan
    assert api.lobpcg_status(ctx, gd, v64, to_dev(nan), 5) == SC_E_NUMERIC
    assert api.lobpcg_status(ctx, gd, v64, to_dev(gaussian_block(g0.n, 257, 1)), 5) == SC_E_UNSUPPORTED
    # 3k > n
    n, src, dst = graphs.cycle(11)
    _, _, gs, vs, _ = _graph_pair(orc, ctx, n, src, dst)
    assert api.lobpcg_status(ctx, gs, vs, to_dev(gaussian_block(n, 4, 1)), 5) == SC_E_INVAL
    r = api.lobpcg_solve(ctx, gd, v64, to_dev(X0), 0)
    ro = orc.lobpcg(go, vo, X0, 0)
    assert r.iterations == 0 and _theta_ok(host(r.theta), ro.theta)


def test_lobpcg_wider_block_leading_convergence(orc, ctx):
    """l = k + 3 columns, stopping on the first k (k_conv): same iterations,
    Ritz values and residual history as the oracle."""
    from paper_1708_07481_amd import api
    g0 = dcsbm(5000, 19, 40.0, 0.75, "dirichlet", 5.0, seed=2)
    go, vo, gd, v64, _ = _graph_pair(orc, ctx, g0.n, g0.src, g0.dst)
    X0 = gaussian_block(g0.n, 22, 5)
    ro = orc.lobpcg(go, vo, X0, 40, 1e-4, k_conv=19)
    rg = api.lobpcg_solve(ctx, gd, v64, to_dev(X0), 40, 1e-4, "fp64", k_conv=19)
    assert rg.converged and ro.converged and rg.iterations == ro.iterations
    assert abs(rg.max_relres - ro.max_relres) <= 1e-6 * ro.max_relres
    assert _theta_ok(host(rg.theta), ro.theta)
    assert np.allclose(rg.relres_hist, ro.relres_hist, rtol=1e-5, atol=1e-12)
    full = api.lobpcg_solve(ctx, gd, v64, to_dev(X0), 40, 1e-4, "fp64")
    assert rg.iterations <= full.iterations
