"""Pins of the oracle's graph symmetrisation (Section II-A), normalised
Laplacian and SpMM against brute force, networkx, closed-form spectra
(Chung, Spectral Graph Theory, 1997) and invariants."""
import math

import numpy as np
import pytest

from tests import graphs


def _dense_w(n, src, dst, w=None, algebraic=False):
    W = np.zeros((n, n))
    for e, (a, b) in enumerate(zip(src, dst)):
        if a == b:
            continue
        x = 1.0 if w is None else w[e]
        if algebraic:
            W[a, b] += x
            W[b, a] += x
        else:
            W[a, b] = 1.0
            W[b, a] = 1.0
    return W


def _csr_dense(g, vals=None):
    D = np.zeros((g.n, g.n))
    for i in range(g.n):
        for p in range(g.row_ptr[i], g.row_ptr[i + 1]):
            D[i, g.col[p]] = 1.0 if vals is None else vals[p]
    return D


@pytest.mark.parametrize("seed", range(6))
def test_graph_build_matches_brute_force(orc, seed):
    n, src, dst = graphs.random_multigraph(17, 60, seed)
    g = orc.graph_build(n, src, dst)
    W = _dense_w(n, src, dst)
    assert np.array_equal(_csr_dense(g), W)
    assert np.array_equal(g.degree, W.sum(1))
    assert g.self_loops == int((src == dst).sum())
    for i in range(n):
        row = g.col[g.row_ptr[i]:g.row_ptr[i + 1]]
        assert np.all(np.diff(row) > 0), "columns strictly ascending, no duplicates"


@pytest.mark.parametrize("seed", range(4))
def test_graph_build_algebraic_sum(orc, seed):
    # dyadic weights: every order of summation is exact, so brute force is exact too
    n, src, dst = graphs.random_multigraph(13, 50, seed)
    w = np.random.default_rng(seed).integers(1, 9, src.shape[0]) / 8.0
    g = orc.graph_build(n, src, dst, w, algebraic=True)
    W = _dense_w(n, src, dst, w, algebraic=True)
    assert np.array_equal(_csr_dense(g, g.w), W)
    assert np.array_equal(g.degree, W.sum(1))


def test_graph_build_metamorphic(orc):
    n, src, dst = graphs.random_multigraph(40, 200, 7)
    g = orc.graph_build(n, src, dst)
    # reversing every edge and duplicating edges leave the symmetric CSR unchanged
    g2 = orc.graph_build(n, np.concatenate([dst, src]), np.concatenate([src, dst]))
    assert np.array_equal(g.row_ptr, g2.row_ptr) and np.array_equal(g.col, g2.col)
    assert np.array_equal(g.degree, g2.degree)


def test_graph_build_vs_networkx(orc):
    nx = pytest.importorskip("networkx")
    n, src, dst = graphs.random_multigraph(60, 400, 3, self_loops=False)
    G = nx.Graph()
    G.add_nodes_from(range(n))
    G.add_edges_from(zip(src.tolist(), dst.tolist()))
    A = nx.to_scipy_sparse_array(G, nodelist=range(n), format="csr")
    A.sort_indices()
    g = orc.graph_build(n, src, dst)
    assert np.array_equal(g.row_ptr, A.indptr.astype(np.int64))
    assert np.array_equal(g.col, A.indices.astype(np.int32))


def test_graph_build_rejects_bad_ids(orc):
    with pytest.raises(orc.OracleError) as e:
        orc.graph_build(4, np.array([0, 4], np.int32), np.array([1, 2], np.int32))
    assert e.value.code == orc.E_INVAL


def _spectrum(orc, n, src, dst):
    g = orc.graph_build(n, src, dst)
    val, dis = orc.laplacian(g)
    return np.sort(np.linalg.eigvalsh(orc.dense_laplacian(g, val))), g, val, dis


CLOSED_FORMS = [
    ("K7", graphs.complete(7), [0.0] + [7 / 6] * 6),
    ("C9", graphs.cycle(9), [1 - math.cos(2 * math.pi * j / 9) for j in range(9)]),
    ("P8", graphs.path(8), [1 - math.cos(math.pi * j / 7) for j in range(8)]),
    ("K3,5", graphs.bipartite(3, 5), [0.0] + [1.0] * 6 + [2.0]),
    ("star6", graphs.star(6), [0.0] + [1.0] * 4 + [2.0]),
    ("Q4", graphs.hypercube(4), sum(([2 * j / 4] * math.comb(4, j) for j in range(5)), [])),
    ("3 cliques", graphs.cliques([4, 5, 6]),
     [0.0] * 3 + [4 / 3] * 3 + [5 / 4] * 4 + [6 / 5] * 5),
]


@pytest.mark.parametrize("name,g,expected", CLOSED_FORMS, ids=[c[0] for c in CLOSED_FORMS])
def test_laplacian_closed_form_spectra(orc, name, g, expected):
    ev, *_ = _spectrum(orc, *g)
    assert np.allclose(ev, np.sort(expected), atol=1e-12)


@pytest.mark.parametrize("seed", range(4))
def test_laplacian_invariants(orc, seed):
    n, src, dst = graphs.random_multigraph(50, 300, seed)
    ev, g, val, dis = _spectrum(orc, n, src, dst)
    L = orc.dense_laplacian(g, val)
    # bitwise symmetric values (one rounded quotient per unordered pair)
    assert np.array_equal(L, L.T)
    # D^1/2 1 is in the kernel; spectrum in [0, 2]
    d12 = np.sqrt(g.degree)
    assert np.max(np.abs(L @ d12)) < 1e-13
    assert ev[0] > -1e-12 and ev[-1] < 2 + 1e-12
    assert np.array_equal(dis, np.where(g.degree > 0, 1.0 / np.sqrt(np.maximum(g.degree, 1)), 0.0))


def test_laplacian_vs_scipy_csgraph(orc):
    sp = pytest.importorskip("scipy.sparse")
    csgraph = pytest.importorskip("scipy.sparse.csgraph")
    n, src, dst = graphs.random_multigraph(80, 900, 11, self_loops=False)
    g = orc.graph_build(n, src, dst)
    assert np.all(g.degree > 0)
    val, _ = orc.laplacian(g)
    A = sp.csr_matrix((np.ones(g.nnz), g.col, g.row_ptr), shape=(n, n))
    Ls = csgraph.laplacian(A, normed=True).toarray()
    assert np.allclose(orc.dense_laplacian(g, val), Ls, atol=1e-15, rtol=0)


def test_isolated_vertex_convention(orc):
    # vertex 4 is isolated: L_44 = 1 (implicit unit diagonal), D^-1/2 entry 0
    n, src, dst = 5, np.array([0, 1, 2], np.int32), np.array([1, 2, 3], np.int32)
    ev, g, val, dis = _spectrum(orc, n, src, dst)
    L = orc.dense_laplacian(g, val)
    assert L[4, 4] == 1.0 and dis[4] == 0.0 and np.count_nonzero(L[4]) == 1
    assert np.sum(np.abs(ev) < 1e-12) == 1


@pytest.mark.parametrize("seed", range(3))
def test_spmm_matches_dense(orc, seed):
    n, src, dst = graphs.random_multigraph(70, 500, seed)
    g = orc.graph_build(n, src, dst)
    val, _ = orc.laplacian(g)
    X = np.random.default_rng(seed).standard_normal((n, 9))
    Y = orc.spmm(g, val, X)
    assert np.allclose(Y, orc.dense_laplacian(g, val) @ X, atol=1e-13, rtol=0)
