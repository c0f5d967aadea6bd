"""Pins of the oracle's LOBPCG (Section II-B / III: block LOBPCG without
preconditioning on the graph Laplacian, random Gaussian start) against the
dense symmetric eigendecomposition, the Rayleigh-Ritz characterisation of
each step, Cauchy interlacing, closed-form null spaces, SciPy's lobpcg and
numpy's eigh, plus the failure paths."""
import numpy as np
import pytest

from synth import dcsbm, gaussian_block
from tests import graphs


def _setup(orc, n, src, dst):
    g = orc.graph_build(n, src, dst)
    val, dis = orc.laplacian(g)
    return g, val, dis, orc.dense_laplacian(g, val)


def _orth(V):
    U, s, _ = np.linalg.svd(V, full_matrices=False)
    return U[:, s > 1e-10 * s[0]]


@pytest.fixture(scope="module")
def sbm_small(orc):
    gg = dcsbm(300, 4, 16.0, 0.8, seed=5)
    g, val, dis, L = _setup(orc, gg.n, gg.src, gg.dst)
    return gg, g, val, dis, L


def test_symeig_vs_numpy(orc):
    rng = np.random.default_rng(0)
    for m in (1, 2, 5, 24, 60):
        A = rng.standard_normal((m, m))
        A = A + A.T
        w, V = orc.symeig(A)
        assert np.allclose(w, np.linalg.eigvalsh(A), atol=1e-12 * max(1, np.abs(w).max()))
        assert np.allclose(V.T @ V, np.eye(m), atol=1e-13)
        assert np.allclose(A @ V, V * w, atol=1e-12 * max(1, np.abs(w).max()))
    # repeated eigenvalues
    Q = np.linalg.qr(rng.standard_normal((8, 8)))[0]
    A = Q @ np.diag([1, 1, 1, 2, 2, 3, 3, 3.0]) @ Q.T
    w, V = orc.symeig((A + A.T) / 2)
    assert np.allclose(w, [1, 1, 1, 2, 2, 3, 3, 3], atol=1e-13)


def test_cholesky(orc):
    rng = np.random.default_rng(1)
    B = rng.standard_normal((30, 12))
    G = B.T @ B
    R = orc.cholesky(G)
    assert np.allclose(np.triu(R), R) and np.allclose(R.T @ R, G, atol=1e-12)
    assert np.allclose(R, np.linalg.cholesky(G).T, atol=1e-12)
    with pytest.raises(orc.OracleError):
        orc.cholesky(np.array([[1.0, 2.0], [2.0, 1.0]]))
    with pytest.raises(orc.OracleError):  # singular
        orc.cholesky(np.ones((3, 3)))


def test_converges_to_dense_smallest(orc, sbm_small):
    gg, g, val, dis, L = sbm_small
    ev = np.linalg.eigvalsh(L)
    k = 4
    r = orc.lobpcg(g, val, gaussian_block(gg.n, k, 3), maxit=300, tol=1e-11)
    assert r.converged
    assert np.allclose(r.theta, ev[:k], atol=1e-9)
    # subspace equals the dense invariant subspace (gap at index k)
    w, V = np.linalg.eigh(L)
    Vk = V[:, :k]
    assert np.linalg.norm(r.X - Vk @ (Vk.T @ r.X), 2) < 1e-8


def test_iteration_invariants(orc, sbm_small):
    gg, g, val, dis, L = sbm_small
    ev = np.linalg.eigvalsh(L)
    k = 6
    r = orc.lobpcg(g, val, gaussian_block(gg.n, k, 4), maxit=15, tol=0.0)
    th = r.theta_hist
    # Rayleigh-Ritz over a growing span: Ritz values never increase (interlacing)
    assert np.all(np.diff(th, axis=0) <= 1e-12)
    # and never drop below the exact eigenvalues
    assert np.all(th >= ev[:k] - 1e-12)
    assert np.all((th >= -1e-12) & (th <= 2 + 1e-12))
    X = r.X
    assert np.allclose(X.T @ X, np.eye(k), atol=1e-12)
    assert np.allclose(X.T @ L @ X, np.diag(r.theta), atol=1e-12)
    R = L @ X - X * r.theta
    assert np.abs(X.T @ R).max() < 1e-12
    # the reported relative residual is ||L x - theta x|| / (2 ||x||)
    assert np.allclose(r.relres_hist[-1], np.linalg.norm(R, axis=0) / 2, rtol=1e-9, atol=1e-15)


def test_initial_rayleigh_ritz(orc, sbm_small):
    # maxit = 0: Ritz pairs of L on span(X0)
    gg, g, val, dis, L = sbm_small
    k = 5
    X0 = gaussian_block(gg.n, k, 9)
    r = orc.lobpcg(g, val, X0, maxit=0)
    Q = _orth(X0)
    assert r.iterations == 0
    assert np.allclose(r.theta, np.linalg.eigvalsh(Q.T @ L @ Q), atol=1e-13)
    assert np.linalg.norm(r.X - Q @ (Q.T @ r.X)) < 1e-12


def test_first_two_steps_are_rayleigh_ritz(orc, sbm_small):
    """Step 1 searches span{X0, L X0}; step 2 searches span{X1, R1, X0}
    (the implicit P direction spans X1 and the previous iterate)."""
    gg, g, val, dis, L = sbm_small
    k = 4
    X0 = gaussian_block(gg.n, k, 10)
    r1 = orc.lobpcg(g, val, X0, maxit=1)
    Q = _orth(np.hstack([X0, L @ X0]))
    assert np.allclose(r1.theta, np.linalg.eigvalsh(Q.T @ L @ Q)[:k], atol=1e-12)
    r2 = orc.lobpcg(g, val, X0, maxit=2)
    R1 = L @ r1.X - r1.X * r1.theta
    Q = _orth(np.hstack([r1.X, R1, X0]))
    assert Q.shape[1] == 3 * k
    assert np.allclose(r2.theta, np.linalg.eigvalsh(Q.T @ L @ Q)[:k], atol=1e-11)


def test_connected_graph_null_vector(orc):
    n, src, dst = graphs.random_multigraph(90, 700, 2, self_loops=False)
    g, val, dis, L = _setup(orc, n, src, dst)
    r = orc.lobpcg(g, val, gaussian_block(n, 3, 1), maxit=200, tol=1e-12)
    assert abs(r.theta[0]) < 1e-12
    u = np.sqrt(g.degree)
    u /= np.linalg.norm(u)
    x = r.X[:, 0]
    assert abs(abs(x @ u) - 1) < 1e-10


def test_disjoint_cliques_subspace(orc):
    sizes = [12, 15, 18, 21]
    n, src, dst = graphs.cliques(sizes)
    g, val, dis, L = _setup(orc, n, src, dst)
    k = 4
    r = orc.lobpcg(g, val, gaussian_block(n, k, 2), maxit=50, tol=1e-12)
    assert np.all(np.abs(r.theta) < 1e-12)
    ind = np.zeros((n, k))
    off = 0
    for b, s in enumerate(sizes):
        ind[off:off + s, b] = np.sqrt(g.degree[off:off + s])
        off += s
    Q = _orth(ind)
    assert np.linalg.norm(r.X - Q @ (Q.T @ r.X), 2) < 1e-10


def test_matches_scipy_lobpcg_at_convergence(orc, sbm_small):
    sp = pytest.importorskip("scipy.sparse")
    from scipy.sparse.linalg import lobpcg as scipy_lobpcg
    gg, g, val, dis, L = sbm_small
    k = 4
    X0 = gaussian_block(gg.n, k, 12)
    r = orc.lobpcg(g, val, X0, maxit=300, tol=1e-11)
    Ls = sp.csr_matrix(L)
    w, _ = scipy_lobpcg(Ls, X0.copy(), largest=False, tol=1e-10, maxiter=500)
    assert np.allclose(np.sort(w), r.theta, atol=1e-8)


def test_failure_paths(orc, sbm_small):
    gg, g, val, dis, L = sbm_small
    X0 = gaussian_block(gg.n, 4, 1)
    bad = X0.copy()
    bad[:, 3] = bad[:, 0] * 2.0            # rank deficient start
    assert orc.lobpcg_status(g, val, bad, 5) == orc.E_BREAKDOWN
    nan = X0.copy()
    nan[7, 1] = np.nan
    assert orc.lobpcg_status(g, val, nan, 5) == orc.E_NUMERIC
    big = gaussian_block(gg.n, gg.n // 3 + 1, 1)   # 3k > n
    assert orc.lobpcg_status(g, val, big, 5) == orc.E_INVAL


def test_sbm_recovers_blocks(orc):
    from paper_1708_07481_amd.metrics import partition_scores
    from synth import kmeans_draws
    gg = dcsbm(1000, 8, 20.0, 0.8, seed=1)
    g, val, dis, L = _setup(orc, gg.n, gg.src, gg.dst)
    r = orc.lobpcg(g, val, gaussian_block(gg.n, 8, 1), maxit=20)
    assert r.max_relres < 1e-2
    km = orc.kmeans(r.X, 8, kmeans_draws(10, 8, 1))
    assert partition_scores(gg.truth, km.labels)["PM"] > 0.99


def test_wider_block_converges_on_the_leading_columns(orc, sbm_small):
    """l = k + 2 columns with the convergence test on the first k (Section IV
    uses a block slightly wider than the clusters): the solve stops as soon as
    the k wanted pairs meet the tolerance, no later than the full test, and
    those k Ritz values are the dense ones."""
    gg, g, val, dis, L = sbm_small
    ev = np.linalg.eigvalsh(L)
    X0 = gaussian_block(gg.n, 6, 21)
    full = orc.lobpcg(g, val, X0, 300, 1e-9)
    lead = orc.lobpcg(g, val, X0, 300, 1e-9, k_conv=4)
    assert lead.converged and full.converged
    assert lead.iterations <= full.iterations
    assert np.all(lead.relres_hist[-1][:4] <= 1e-9)
    assert lead.max_relres == lead.relres_hist[-1][:4].max()
    assert np.allclose(lead.theta[:4], ev[:4], atol=1e-12)
    # identical iterates up to the earlier stop
    assert np.array_equal(lead.theta_hist, full.theta_hist[: lead.iterations + 1])
