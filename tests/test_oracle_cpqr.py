"""Pins of the oracle's labelling by QR with column pivoting (Section II-A;
Damle, Minden & Ying): LAPACK's pivoted QR (scipy.linalg.qr, pivoting=True)
picks the same pivots, the factor Q is SciPy's polar factor of the pivot block,
ideal block data are recovered exactly, labels do not change under a rotation
of the coordinates, a rank-deficient block is a breakdown, and on an SBM the
labels of the oracle's own eigenvectors recover the blocks."""
import numpy as np
import pytest

from paper_1708_07481_amd.metrics import canonical_labels, partition_scores
from synth import dcsbm, gaussian_block


def _rot(k, seed):
    return np.linalg.qr(np.random.default_rng(seed).standard_normal((k, k)))[0]


@pytest.mark.parametrize("n,k,seed", [(40, 3, 0), (500, 8, 1), (2000, 19, 2), (300, 44, 3)])
def test_pivots_match_lapack_qrcp(orc, n, k, seed):
    from scipy.linalg import qr
    X = np.random.default_rng(seed).standard_normal((n, k))
    r = orc.cpqr_labels(X)
    _, _, piv = qr(X.T, pivoting=True, mode="economic")
    assert np.array_equal(r.pivots, piv[:k].astype(np.int32))


@pytest.mark.parametrize("k,seed", [(4, 0), (12, 1), (30, 2)])
def test_factor_is_polar_of_pivot_block(orc, k, seed):
    from scipy.linalg import polar
    X = np.random.default_rng(seed).standard_normal((10 * k, k))
    r = orc.cpqr_labels(X)
    B = X[r.pivots]
    u, p = polar(B.T)
    assert np.allclose(r.Q, u, atol=1e-10)
    assert np.allclose(r.Q.T @ r.Q, np.eye(k), atol=1e-12)
    # labels are the argmax of |X Q| row by row
    assert np.array_equal(r.labels, np.abs(X @ u).argmax(1))


def test_ideal_blocks_recovered_and_rotation_invariant(orc):
    rng = np.random.default_rng(5)
    k, n = 7, 700
    truth = rng.integers(0, k, n)
    H = np.zeros((n, k))
    H[np.arange(n), truth] = 1.0 + 0.5 * rng.random(n)      # scaled indicators
    H += 0.05 * rng.standard_normal((n, k))
    for seed in (0, 1):
        X = H @ _rot(k, seed)
        r = orc.cpqr_labels(X)
        assert np.array_equal(canonical_labels(r.labels), canonical_labels(truth))
        assert len(set(truth[r.pivots])) == k                  # one pivot per cluster


def test_rank_deficient_is_breakdown(orc):
    """A dependent column leaves only rounding noise (about 1e-15 of ||x||^2)
    in the downdated residuals: below the rank floor (1e-10 of the first
    pivot's), a breakdown.  A small but real fifth direction passes."""
    rng = np.random.default_rng(0)
    for make in (lambda X: X[:, 0] + X[:, 1], lambda X: X[:, 0] - 2 * X[:, 2],
                 lambda X: 0.0 * X[:, 3]):
        X = rng.standard_normal((100, 5))
        X[:, 4] = make(X)
        with pytest.raises(orc.OracleError):
            orc.cpqr_labels(X)
    X = rng.standard_normal((100, 5))
    X[:, 4] = X[:, 0] + 1e-3 * X[:, 4]
    assert len(set(orc.cpqr_labels(X).pivots.tolist())) == 5


def test_sbm_eigenvectors_recover_blocks(orc):
    g0 = dcsbm(1000, 8, 20.0, 0.8, seed=1)
    g = orc.graph_build(g0.n, g0.src, g0.dst)
    val, _ = orc.laplacian(g)
    res = orc.lobpcg(g, val, gaussian_block(g0.n, 8, 1), 40, 1e-6)
    r = orc.cpqr_labels(res.X)
    assert partition_scores(g0.truth, r.labels)["PM"] > 0.97


def test_eigengap_hand_examples(orc):
    assert orc.eigengap([0.0, 0.1, 0.12, 0.9, 0.95])[0] == 3     # 0.78 > 10 * 0.06
    # the trivial eigenvalue's own increment is not a gap when a larger one follows
    assert orc.eigengap([0.0, 0.24, 0.245, 0.25, 0.26, 0.7])[0] == 5
    # no increment stands out: the largest one (first of equals)
    assert orc.eigengap([0.0, 0.5, 0.6, 1.0])[0] == 1
    assert orc.eigengap([0.0, 0.1, 0.2, 0.3])[0] == 1
    assert orc.eigengap([0.7])[0] == 1
    c, ratio = orc.eigengap([0.0, 0.01, 0.02, 0.03, 0.5, 0.52, 0.54])
    assert c == 4 and ratio > 20


def test_eigengap_counts_components_and_blocks(orc):
    from tests import graphs
    n, src, dst = graphs.cliques([9, 11, 14, 17, 20])
    g = orc.graph_build(n, src, dst)
    val, _ = orc.laplacian(g)
    ev = np.linalg.eigvalsh(orc.dense_laplacian(g, val))
    assert orc.eigengap(ev[:8])[0] == 5
    gg = dcsbm(400, 4, 24.0, 0.9, seed=2)
    g = orc.graph_build(gg.n, gg.src, gg.dst)
    val, _ = orc.laplacian(g)
    ev = np.linalg.eigvalsh(orc.dense_laplacian(g, val))
    assert orc.eigengap(ev[:7])[0] == 4
