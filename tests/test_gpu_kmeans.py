"""GPU parity: k-means on the row-normalised eigenvectors against the oracle.
On the same input block the labels, centroids, integer inertia and chosen
restart must be identical (every distance, draw and centroid sum follows one
fixed order).  End to end (each side's own LOBPCG result), labels must agree
up to a permutation."""
import numpy as np
import pytest

from paper_1708_07481_amd.metrics import canonical_labels, partition_scores
from synth import dcsbm, gaussian_block, kmeans_draws
from tests.gpu_common import gpu_ctx, host, to_dev

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ctx():
    return gpu_ctx()


def _same(ko, kg):
    assert np.array_equal(host(kg.labels), ko.labels)
    assert np.array_equal(host(kg.centroids), ko.centroids)
    assert kg.inertia_q == ko.inertia_q and kg.best_restart == ko.best_restart
    assert abs(kg.inertia - ko.inertia) <= 1e-12 * max(1.0, abs(ko.inertia))


@pytest.mark.parametrize("n,dim,K,R,seed", [(10, 2, 3, 2, 0), (257, 5, 4, 3, 1),
                                            (1000, 8, 8, 10, 2), (3001, 19, 19, 4, 3),
                                            (20000, 44, 44, 3, 4)])
@pytest.mark.parametrize("scan", ["auto", "pruned"])
def test_kmeans_bit_exact_random(orc, ctx, n, dim, K, R, seed, scan):
    from paper_1708_07481_amd import api
    rng = np.random.default_rng(seed)
    centers = rng.standard_normal((K, dim))
    X = centers[rng.integers(0, K, n)] + 0.3 * rng.standard_normal((n, dim))
    draws = kmeans_draws(R, K, seed)
    ko = orc.kmeans(X, K, draws, max_iter=100)
    kg = api.kmeans_assign(ctx, to_dev(X), K, to_dev(draws.view(np.int64)), max_iter=100,
                           scan=scan)
    _same(ko, kg)


@pytest.mark.parametrize("n,dim,K,R,noise,seed", [(30000, 16, 24, 2, 1.0, 5),
                                                  (12000, 40, 40, 2, 0.6, 6)])
@pytest.mark.parametrize("scan", ["pruned", "full"])
def test_kmeans_bit_exact_overlapping(orc, ctx, n, dim, K, R, noise, seed, scan):
    """Overlapping clusters: many points cannot rule out more than a few
    centres, so the pruned scans hand a large share to the full scan, and
    waves mix narrow and wide points."""
    from paper_1708_07481_amd import api
    rng = np.random.default_rng(seed)
    centers = rng.standard_normal((K, dim))
    X = centers[rng.integers(0, K, n)] + noise * rng.standard_normal((n, dim))
    draws = kmeans_draws(R, K, seed)
    ko = orc.kmeans(X, K, draws, max_iter=100)
    kg = api.kmeans_assign(ctx, to_dev(X), K, to_dev(draws.view(np.int64)), max_iter=100,
                           scan=scan)
    _same(ko, kg)


@pytest.mark.parametrize("scan", ["pruned", "full"])
def test_kmeans_bit_exact_lattice_ties(orc, ctx, scan):
    """Integer points, no normalisation: many distances tie exactly, and a tie
    goes to the lowest centre index on both sides."""
    from paper_1708_07481_amd import api
    rng = np.random.default_rng(7)
    X = rng.integers(0, 3, (12000, 6)).astype(np.float64)
    draws = kmeans_draws(2, 10, 7)
    ko = orc.kmeans(X, 10, draws, max_iter=100, normalize=False)
    kg = api.kmeans_assign(ctx, to_dev(X), 10, to_dev(draws.view(np.int64)), max_iter=100,
                           normalize=False, scan=scan)
    _same(ko, kg)


@pytest.mark.parametrize("n,dim,K,R,seed,norm,scan", [(20000, 44, 44, 3, 11, True, "pruned"),
                                                      (20000, 44, 44, 3, 11, True, "full"),
                                                      (3001, 19, 19, 4, 12, False, "auto"),
                                                      (30000, 16, 24, 2, 13, True, "pruned"),
                                                      (5000, 7, 6, 3, 14, True, "auto")])
def test_kmeans_bit_exact_fp32_input(orc, ctx, n, dim, K, R, seed, norm, scan):
    """FP32 rows (the FP32 solver's eigenvector block) read through a row
    stride wider than dim.  The kernels form y = x / ||x|| from the FP32 values
    in registers; labels, centroids and inertia must equal the oracle's on the
    same values widened to FP64.  Zero rows, -0.0 entries and FP32 subnormals
    included."""
    from paper_1708_07481_amd import api
    rng = np.random.default_rng(seed)
    centers = rng.standard_normal((K, dim))
    X = (centers[rng.integers(0, K, n)] + 0.5 * rng.standard_normal((n, dim))).astype(np.float32)
    X[::97] = 0.0
    X[1::89, ::2] = -0.0
    X[2::113] = np.float32(1e-44) * np.sign(X[2::113])
    X[3::131, 0] = np.float32(3e-39)
    big = np.zeros((n, dim + 5), np.float32)
    big[:, :dim] = X
    Xd = to_dev(big)[:, :dim]
    assert Xd.stride(0) == dim + 5
    draws = kmeans_draws(R, K, seed)
    ko = orc.kmeans(X.astype(np.float64), K, draws, max_iter=100, normalize=norm)
    kg = api.kmeans_assign(ctx, Xd, K, to_dev(draws.view(np.int64)), max_iter=100,
                           normalize=norm, scan=scan)
    _same(ko, kg)


@pytest.mark.parametrize("R", [7, 12, 13, 20])
@pytest.mark.parametrize("fp32", [False, True])
def test_kmeans_bit_exact_restart_widths(orc, ctx, R, fp32):
    """Restart counts that take each seeding width (8, 12 and 16 restarts per
    pass over the points) and, at 20, two passes; the seeding's centre rows are
    strided by that width."""
    from paper_1708_07481_amd import api
    rng = np.random.default_rng(40 + R)
    n, dim, K = 3001, 12, 9
    centers = rng.standard_normal((K, dim))
    X = centers[rng.integers(0, K, n)] + 0.4 * rng.standard_normal((n, dim))
    if fp32:
        X = X.astype(np.float32)
    draws = kmeans_draws(R, K, R)
    ko = orc.kmeans(X.astype(np.float64), K, draws, max_iter=100)
    kg = api.kmeans_assign(ctx, to_dev(X), K, to_dev(draws.view(np.int64)), max_iter=100)
    _same(ko, kg)


def test_kmeans_edge_cases(orc, ctx):
    from paper_1708_07481_amd import api
    # zero rows, duplicate points, K == n, max_iter = 0, no normalisation
    X = np.array([[0.0, 0.0], [1.0, 0.0], [1.0, 0.0], [0.0, 2.0], [0.0, 0.0], [3.0, 3.0]])
    for K, R, it, norm in [(1, 1, 10, True), (6, 2, 10, False), (3, 4, 0, True), (2, 3, 5, False)]:
        draws = kmeans_draws(R, K, K + R)
        ko = orc.kmeans(X, K, draws, max_iter=it, normalize=norm)
        kg = api.kmeans_assign(ctx, to_dev(X), K, to_dev(draws.view(np.int64)), max_iter=it,
                               normalize=norm)
        _same(ko, kg)
    # given centroids, pure assignment
    C = np.array([[0.5, 0.0], [0.0, 1.0], [2.0, 2.0]])
    ko = orc.kmeans(X, 3, init_centroids=C, max_iter=0, normalize=False)
    kg = api.kmeans_assign(ctx, to_dev(X), 3, None, init_centroids=to_dev(C), max_iter=0,
                           normalize=False)
    assert np.array_equal(host(kg.labels), ko.labels)


def test_kmeans_on_oracle_eigenvectors(orc, ctx):
    """Same eigenvector block (the oracle's LOBPCG output) on both sides."""
    from paper_1708_07481_amd import api
    g0 = dcsbm(1000, 8, 20.0, 0.8, seed=1)
    go = orc.graph_build(g0.n, g0.src, g0.dst)
    vo, _ = orc.laplacian(go)
    ro = orc.lobpcg(go, vo, gaussian_block(g0.n, 8, 1), 20)
    draws = kmeans_draws(10, 8, 1)
    ko = orc.kmeans(ro.X, 8, draws)
    kg = api.kmeans_assign(ctx, to_dev(ro.X), 8, to_dev(draws.view(np.int64)))
    _same(ko, kg)
    assert partition_scores(g0.truth, ko.labels)["PM"] > 0.99


@pytest.mark.parametrize("n,B,dbar,f,sizes,alpha,k,maxit,tol", [
    (1000, 8, 20.0, 0.8, "equal", 1.0, 8, 20, 0.0),
    (5000, 19, 40.0, 0.75, "dirichlet", 5.0, 19, 30, 1e-2),
])
def test_end_to_end_labels(orc, ctx, n, B, dbar, f, sizes, alpha, k, maxit, tol):
    from paper_1708_07481_amd import api
    g0 = dcsbm(n, B, dbar, f, sizes, alpha, seed=1)
    X0 = gaussian_block(n, k, 1)
    draws = kmeans_draws(10, k, 1)
    go, vo, ro, ko = orc.partition(n, g0.src, g0.dst, k, X0, maxit, tol, draws)
    gd = api.graph_build(ctx, n, to_dev(g0.src), to_dev(g0.dst))
    v64, _, _ = api.laplacian_csr(ctx, gd)
    rg = api.lobpcg_solve(ctx, gd, v64, to_dev(X0), maxit, tol)
    kg = api.kmeans_assign(ctx, rg.X, k, to_dev(draws.view(np.int64)))
    lg = host(kg.labels)
    if not np.array_equal(canonical_labels(lg), canonical_labels(ko.labels)):
        # triage: labels may differ only where a point sits on a decision boundary
        Y = orc.row_normalize(ro.X)
        d = ((Y[:, None, :] - ko.centroids[None]) ** 2).sum(-1)
        d.sort(axis=1)
        margin = d[:, 1] - d[:, 0]
        bad = np.flatnonzero(canonical_labels(lg) != canonical_labels(ko.labels))
        pytest.fail(f"{bad.size} labels differ; smallest margins there {np.sort(margin[bad])[:5]}")
    assert partition_scores(g0.truth, lg)["PM"] > 0.98
