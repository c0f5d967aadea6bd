"""Pins of the oracle's graph Laplacian L = D - W (Section II-A introduces it;
Section III applies it matrix-free as diag(L) X - W X) and of LOBPCG on it.

- closed-form spectra of D - W for complete, cycle, path, star, complete
  bipartite and hypercube graphs (textbook results, e.g. Chung / Brouwer &
  Haemers), against the dense matrix the oracle's values assemble;
- exact invariants: L 1 = 0 (integer arithmetic for unit weights), symmetry,
  the algebraic (weight-summing) symmetrisation against a brute-force dense W;
- SpMM with the diagonal against the dense product;
- LOBPCG: converged Ritz values equal numpy's smallest eigenvalues, disjoint
  cliques give the constant-on-each-clique null space, Ritz values interlace
  and never drop below the exact ones, and the relative residual is scaled by
  the Gershgorin bound 2 max d."""
from math import comb

import numpy as np
import pytest

from synth import dcsbm, gaussian_block
from tests import graphs


def _lap(orc, n, src, dst, w=None, algebraic=False):
    g = orc.graph_build(n, src, dst, w, algebraic)
    val, diag = orc.laplacian_combinatorial(g)
    return g, val, diag, orc.dense_laplacian(g, val, diag)


def _orth(V):
    U, s, _ = np.linalg.svd(V, full_matrices=False)
    return U[:, s > 1e-10 * s[0]]


CASES = [
    ("K7", graphs.complete(7), [0.0] + [7.0] * 6),
    ("C9", graphs.cycle(9), [2 - 2 * np.cos(2 * np.pi * j / 9) for j in range(9)]),
    ("P8", graphs.path(8), [2 - 2 * np.cos(np.pi * j / 8) for j in range(8)]),
    ("star6", graphs.star(6), [0.0] + [1.0] * 4 + [6.0]),
    ("K3,5", graphs.bipartite(3, 5), [0.0] + [3.0] * 4 + [5.0] * 2 + [8.0]),
    ("Q4", graphs.hypercube(4), sum(([2.0 * i] * comb(4, i) for i in range(5)), [])),
]


@pytest.mark.parametrize("name,g,expected", CASES, ids=[c[0] for c in CASES])
def test_combinatorial_closed_form_spectra(orc, name, g, expected):
    _, _, _, L = _lap(orc, *g)
    assert np.allclose(np.linalg.eigvalsh(L), np.sort(expected), atol=1e-12)


@pytest.mark.parametrize("seed", [0, 1, 2])
def test_combinatorial_invariants(orc, seed):
    n, src, dst = graphs.random_multigraph(60, 400, seed)
    g, val, diag, L = _lap(orc, n, src, dst)
    assert np.all(val == -1.0)
    assert np.array_equal(diag, g.degree)
    assert np.array_equal(L, L.T)
    # L 1 = 0 exactly: integer degrees minus integer neighbour counts
    Y = orc.spmm(g, val, np.ones((n, 3)), diag)
    assert np.all(Y == 0.0)
    ev = np.linalg.eigvalsh(L)
    assert ev[0] > -1e-12 and ev[-1] <= 2 * diag.max() + 1e-9


def test_combinatorial_algebraic_weights(orc):
    """Weighted directed edges: W = A + A' summed, L = diag(W 1) - W."""
    rng = np.random.default_rng(4)
    n, m = 40, 300
    src = rng.integers(0, n, m).astype(np.int32)
    dst = rng.integers(0, n, m).astype(np.int32)
    w = rng.integers(1, 5, m).astype(np.float64)
    g, val, diag, L = _lap(orc, n, src, dst, w, algebraic=True)
    W = np.zeros((n, n))
    for s, d, x in zip(src, dst, w):
        if s != d:
            W[s, d] += x
            W[d, s] += x
    assert np.array_equal(L, np.diag(W.sum(1)) - W)


@pytest.mark.parametrize("seed", [0, 1])
def test_combinatorial_spmm_matches_dense(orc, seed):
    gg = dcsbm(200, 4, 12.0, 0.8, seed=seed + 20)
    g, val, diag, L = _lap(orc, gg.n, gg.src, gg.dst)
    X = np.random.default_rng(seed).standard_normal((gg.n, 7))
    Y = orc.spmm(g, val, X, diag)
    assert np.allclose(Y, L @ X, rtol=1e-13, atol=1e-12)


@pytest.fixture(scope="module")
def sbm_comb(orc):
    gg = dcsbm(300, 4, 16.0, 0.8, seed=5)
    g, val, diag, L = _lap(orc, gg.n, gg.src, gg.dst)
    return gg, g, val, diag, L


def test_combinatorial_lobpcg_converges_to_dense(orc, sbm_comb):
    gg, g, val, diag, L = sbm_comb
    ev, V = np.linalg.eigh(L)
    k = 4
    r = orc.lobpcg(g, val, gaussian_block(gg.n, k, 3), maxit=600, tol=1e-12, diag=diag)
    assert r.converged
    assert np.allclose(r.theta, ev[:k], atol=1e-8 * ev[-1])
    Vk = V[:, :k]
    assert np.linalg.norm(r.X - Vk @ (Vk.T @ r.X), 2) < 1e-6


def test_combinatorial_lobpcg_invariants(orc, sbm_comb):
    gg, g, val, diag, L = sbm_comb
    ev = np.linalg.eigvalsh(L)
    k = 5
    r = orc.lobpcg(g, val, gaussian_block(gg.n, k, 4), maxit=12, tol=0.0, diag=diag)
    th = r.theta_hist
    assert np.all(np.diff(th, axis=0) <= 1e-9)
    assert np.all(th >= ev[:k] - 1e-9)
    X = r.X
    assert np.allclose(X.T @ X, np.eye(k), atol=1e-12)
    assert np.allclose(X.T @ L @ X, np.diag(r.theta), atol=1e-9)
    R = L @ X - X * r.theta
    bound = 2 * diag.max()
    assert np.allclose(r.relres_hist[-1], np.linalg.norm(R, axis=0) / bound, rtol=1e-9, atol=1e-15)


def test_combinatorial_disjoint_cliques(orc):
    sizes = [10, 13, 17]
    n, src, dst = graphs.cliques(sizes)
    g, val, diag, L = _lap(orc, n, src, dst)
    k = 3
    r = orc.lobpcg(g, val, gaussian_block(n, k, 2), maxit=80, tol=1e-13, diag=diag)
    assert np.all(np.abs(r.theta) < 1e-10)
    ind = np.zeros((n, k))
    off = 0
    for b, s in enumerate(sizes):
        ind[off:off + s, b] = 1.0               # D - W: constant on each component
        off += s
    Q = _orth(ind)
    assert np.linalg.norm(r.X - Q @ (Q.T @ r.X), 2) < 1e-9


def test_normalised_default_unchanged(orc, sbm_comb):
    """diag=None keeps the normalised operator and the bound 2."""
    gg = sbm_comb[0]
    g = orc.graph_build(gg.n, gg.src, gg.dst)
    val, _ = orc.laplacian(g)
    X0 = gaussian_block(gg.n, 3, 6)
    a = orc.lobpcg(g, val, X0, maxit=5)
    L = orc.dense_laplacian(g, val)
    R = L @ a.X - a.X * a.theta
    assert np.allclose(a.relres_hist[-1], np.linalg.norm(R, axis=0) / 2, rtol=1e-9, atol=1e-15)
