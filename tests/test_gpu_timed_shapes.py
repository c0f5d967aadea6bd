"""GPU parity at the benchmarked block width: k = 160 eigenvectors (a 480-wide
basis S = [X W P], Section II-B), 160 clusters in 160 dimensions with ten
k-means++ restarts (Section II-A), and soft locking (Section IV).

These are the kernel instantiations the 2M-vertex workload runs: the
three-tile FP32 Gram and row-GEMM shapes of a 480-wide basis, the
Rayleigh-Ritz chain at m = 480 (cooperative tridiagonalisation), the
ten-restart seeding pass over 160 FP32 coordinates and the 40-centre
assignment waves of K = 160.  The graphs are smaller (12K vertices) so
that the oracle finishes in under a minute.

Bars.  FP64: the C1 bar, Ritz values within max(1e-8 |theta|, 1e-12),
subspace sine <= 1e-6, the same iteration count and residual history.
FP32 and FP32 + BF16 Gram against the FP64 oracle, both run to relative
residual 1e-2 from the same start block.  Both Ritz values of pair j lie
above the eigenvalue and within |r_j|^2 / gap of it, |r_j| = 2 relres_j, so
they differ by at most that; with the gap taken as 0.1 and a floor for the
precision of the Ritz values themselves (2e-5 for FP32 Gram products, 5e-4
for BF16-rounded inputs, whose unit roundoff is 2^-9):
|dtheta_j| <= floor + 10 (2 max(relres_j))^2.  The subspace of the leading
columns converged to oracle relres <= 1e-4 within sine 2e-3 (FP32) and 5e-2
(BF16), and X'X = I within 1e-4 (FP32) and 4e-3 (BF16: the Rayleigh-Ritz
coefficients come from a basis Gram matrix of BF16-rounded inputs, whose
unit roundoff 2^-9 bounds how orthonormal S C can be).  k-means: labels, centroids, integer inertia and chosen restart
identical."""
import numpy as np
import pytest

from synth import dcsbm, gaussian_block, kmeans_draws
from tests.gpu_common import gpu_ctx, host, to_dev

pytestmark = pytest.mark.gpu

N, K = 12000, 160
MAXIT, TOL = 30, 1e-2


@pytest.fixture(scope="module")
def ctx():
    return gpu_ctx()


def _sine(Xg, Xo):
    return np.linalg.norm(Xg - Xo @ (Xo.T @ Xg), 2)


def _theta_ok(tg, to):
    return np.all(np.abs(tg - to) <= np.maximum(1e-8 * np.abs(to), 1e-12))


@pytest.fixture(scope="module")
def case160(orc, ctx):
    """12K-vertex degree-corrected SBM with 160 blocks (Dirichlet(2) sizes,
    mean degree 40, intra fraction 0.7: the 2M workload's generator), its
    CSR and Laplacian on both sides, and the oracle's FP64 solve to relative
    residual 1e-2 (ten iterations)."""
    from paper_1708_07481_amd import api
    g0 = dcsbm(N, K, 40.0, 0.7, "dirichlet", 2.0, seed=3)
    go = orc.graph_build(g0.n, g0.src, g0.dst)
    vo, _ = orc.laplacian(go)
    gd = api.graph_build(ctx, g0.n, to_dev(g0.src), to_dev(g0.dst))
    v64, v32, _ = api.laplacian_csr(ctx, gd, True, True)
    assert gd.nnz == go.nnz
    X0 = gaussian_block(N, K, 3)
    ro = orc.lobpcg(go, vo, X0, MAXIT, TOL)
    assert ro.converged and ro.iterations >= 5
    return g0, go, vo, gd, v64, v32, X0, ro


def test_lobpcg_fp64_parity_k160(case160, ctx):
    from paper_1708_07481_amd import api
    g0, go, vo, gd, v64, v32, X0, ro = case160
    rg = api.lobpcg_solve(ctx, gd, v64, to_dev(X0), MAXIT, TOL, "fp64")
    tg, Xg = host(rg.theta), host(rg.X)
    print("k160 fp64: iterations", rg.iterations, ro.iterations, "max |dtheta|",
          np.abs(tg - ro.theta).max(), "sine", _sine(Xg, ro.X), "pdrops", rg.p_drops, ro.p_drops)
    assert rg.converged and rg.iterations == ro.iterations
    assert rg.p_drops == ro.p_drops
    assert _theta_ok(tg, ro.theta), np.abs(tg - ro.theta).max()
    assert _sine(Xg, ro.X) <= 1e-6
    assert np.allclose(Xg.T @ Xg, np.eye(K), atol=1e-10)
    assert np.allclose(rg.relres_hist, ro.relres_hist, rtol=1e-5, atol=1e-12)


@pytest.mark.parametrize("prec,floor,sine_tol,orth_tol", [("fp32", 2e-5, 2e-3, 1e-4),
                                                          ("fp32_bf16gram", 5e-4, 5e-2, 4e-3)])
def test_lobpcg_reduced_precision_k160(case160, ctx, prec, floor, sine_tol, orth_tol):
    from paper_1708_07481_amd import api
    g0, go, vo, gd, v64, v32, X0, ro = case160
    rg = api.lobpcg_solve(ctx, gd, v32, to_dev(X0.astype(np.float32)), MAXIT, TOL, prec)
    tg = host(rg.theta)
    Xg = host(rg.X).astype(np.float64)
    rr = np.maximum(ro.relres_hist[-1], rg.relres_hist[-1])
    dth = np.abs(tg - ro.theta)
    bound = floor + 10.0 * (2.0 * rr) ** 2
    tight = ro.relres_hist[-1] <= 1e-4
    lead = int(np.argmin(tight)) if not tight.all() else K    # leading run of converged columns
    sine = _sine(Xg[:, :lead], ro.X[:, :lead]) if lead else 0.0
    print(f"k160 {prec}: iterations {rg.iterations} (oracle {ro.iterations}) restarts "
          f"{rg.restarts} fallbacks {rg.gram_fallbacks} w_drops {rg.w_drops}; max |dtheta| "
          f"{dth.max():.3e}, max |dtheta| / bound {np.max(dth / bound):.3f}; leading {lead} "
          f"columns sine {sine:.3e}")
    assert rg.converged
    assert np.all(dth <= bound), np.argmax(dth / bound)
    assert lead >= 100
    assert sine <= sine_tol
    assert np.abs(Xg.T @ Xg - np.eye(K)).max() < orth_tol


def test_lobpcg_fp32_soft_locking_k160(case160, ctx):
    """FP32 at the benchmarked width with soft locking at the tolerance
    (Section IV): columns at relres <= 1e-2 leave W, the active W columns are
    moved to the front of the W block and the products skip the rest.  The
    exact parity of that path with the oracle's locking is
    test_lobpcg_soft_locking_parity (FP64); here, at k = 160 in FP32: locking
    did take columns out of W before the last iteration, the solve converged
    in as many iterations as the oracle without locking, X'X = I, and every
    Ritz value lies within the first-order residual bound of the oracle's:
    both are within ||r_j|| = N relres_j (N = 2) of an eigenvalue, and a locked
    column stops near relres 1e-2, where the second-order bound of the
    unlocked test assumes a gap the end of the block does not have."""
    from paper_1708_07481_amd import api
    g0, go, vo, gd, v64, v32, X0, ro = case160
    rg = api.lobpcg_solve(ctx, gd, v32, to_dev(X0.astype(np.float32)), MAXIT, TOL, "fp32",
                          lock_tol=TOL)
    tg = host(rg.theta)
    Xg = host(rg.X).astype(np.float64)
    locked = (np.asarray(rg.relres_hist)[:, :K] <= TOL).sum(axis=1)
    dth = np.abs(tg - ro.theta)
    bound = 2e-5 + 2.0 * (np.asarray(rg.relres_hist)[-1, :K] + ro.relres_hist[-1])
    print(f"k160 fp32 soft locking: iterations {rg.iterations} (oracle {ro.iterations}), locked "
          f"per iteration {locked.tolist()}, max |dtheta| {dth.max():.3e}, max |dtheta| / bound "
          f"{np.max(dth / bound):.3f}")
    assert rg.converged and abs(rg.iterations - ro.iterations) <= 2
    assert np.any((locked[:-1] > 0) & (locked[:-1] < K))     # compacted iterations happened
    assert np.all(dth <= bound), np.argmax(dth / bound)
    assert np.abs(Xg.T @ Xg - np.eye(K)).max() < 1e-4


def test_kmeans_on_k160_eigenvectors(orc, ctx, case160):
    """The oracle's own 160-column eigenvector block, in FP32 as the FP32
    solver hands it over, read through a row stride wider than 160: ten
    restarts, 160 clusters; identical on both sides."""
    from paper_1708_07481_amd import api
    g0, go, vo, gd, v64, v32, X0, ro = case160
    X = ro.X.astype(np.float32)
    draws = kmeans_draws(10, K, 5)
    ko = orc.kmeans(X.astype(np.float64), K, draws, max_iter=100)
    big = np.zeros((N, K + 4), np.float32)
    big[:, :K] = X
    Xd = to_dev(big)[:, :K]
    for scan in ("pruned", "full"):
        kg = api.kmeans_assign(ctx, Xd, K, to_dev(draws.view(np.int64)), max_iter=100, scan=scan)
        print(f"k-means on eigenvectors ({scan}): lloyd {kg.lloyd_iterations} / {ko.lloyd_iters}, "
              f"best restart {kg.best_restart}")
        assert np.array_equal(host(kg.labels), ko.labels), scan
        assert np.array_equal(host(kg.centroids), ko.centroids), scan
        assert kg.inertia_q == ko.inertia_q and kg.best_restart == ko.best_restart, scan


@pytest.fixture(scope="module")
def km160(orc):
    """30011 points around 160 Gaussian centres in 160 dimensions (noise as
    large as the centres, so clusters overlap after normalisation), FP32."""
    rng = np.random.default_rng(160)
    n, dim = 30011, 160
    centers = rng.standard_normal((K, dim))
    X = (centers[rng.integers(0, K, n)] + rng.standard_normal((n, dim))).astype(np.float32)
    draws = kmeans_draws(10, K, 160)
    ko = orc.kmeans(X.astype(np.float64), K, draws, max_iter=100)
    return X, draws, ko


@pytest.mark.parametrize("scan", ["pruned", "full"])
def test_kmeans_bit_exact_k160_dim160(ctx, km160, scan):
    from paper_1708_07481_amd import api
    X, draws, ko = km160
    n, dim = X.shape
    big = np.zeros((n, dim + 8), np.float32)
    big[:, :dim] = X
    Xd = to_dev(big)[:, :dim]
    assert Xd.stride(0) == dim + 8
    kg = api.kmeans_assign(ctx, Xd, K, to_dev(draws.view(np.int64)), max_iter=100, scan=scan)
    print(f"k-means 160 x 160 ({scan}): lloyd {kg.lloyd_iterations} / {ko.lloyd_iters}")
    assert np.array_equal(host(kg.labels), ko.labels)
    assert np.array_equal(host(kg.centroids), ko.centroids)
    assert kg.inertia_q == ko.inertia_q and kg.best_restart == ko.best_restart
    assert abs(kg.inertia - ko.inertia) <= 1e-12 * max(1.0, abs(ko.inertia))


def test_lobpcg_soft_locking_parity(orc, ctx):
    """Soft locking at a real tolerance (Section IV): columns whose relative
    residual falls to 5e-3 leave W, the solve continues to 1e-4.  Same
    iterations, Ritz values and residual history (hence the same columns
    locked at every step) as the oracle."""
    from paper_1708_07481_amd import api
    g0 = dcsbm(5000, 19, 40.0, 0.75, "dirichlet", 5.0, seed=2)
    go = orc.graph_build(g0.n, g0.src, g0.dst)
    vo, _ = orc.laplacian(go)
    gd = api.graph_build(ctx, g0.n, to_dev(g0.src), to_dev(g0.dst))
    v64, _, _ = api.laplacian_csr(ctx, gd)
    X0 = gaussian_block(g0.n, 19, 7)
    ro = orc.lobpcg(go, vo, X0, 40, 1e-4, lock_tol=5e-3)
    rg = api.lobpcg_solve(ctx, gd, v64, to_dev(X0), 40, 1e-4, "fp64", lock_tol=5e-3)
    locked_hist = (ro.relres_hist <= 5e-3).sum(axis=1)
    print("soft locking: iterations", rg.iterations, ro.iterations, "locked per iteration",
          locked_hist.tolist(), "final", rg.locked_cols, ro.locked_cols)
    assert locked_hist.max() > 0 and locked_hist[1] < 19     # columns lock along the way
    assert rg.iterations == ro.iterations
    assert rg.converged == ro.converged
    assert rg.locked_cols == int((ro.relres_hist[-1] <= 5e-3).sum())
    assert _theta_ok(host(rg.theta), ro.theta)
    assert _sine(host(rg.X), ro.X) <= 1e-6
    assert np.allclose(rg.relres_hist, ro.relres_hist, rtol=1e-5, atol=1e-12)
