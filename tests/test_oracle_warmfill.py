"""Pins of the warm-start fill-in for stages that add vertices (Section III:
the previous stage's eigenvectors start the next solve; the rows of new
vertices must be filled in): exact interpolation of linear data along a path,
constant blocks preserved exactly, rows without an old neighbour left zero,
old rows untouched, and on a snowball stream a better start than zero rows
(a smaller Rayleigh quotient residual after one CholQR)."""
import numpy as np

from synth import dcsbm, gaussian_block
from synth import snowball_stages
from tests import graphs


def test_linear_data_on_a_path_is_interpolated_exactly(orc):
    # path 0-1-2-...-9, old vertices 0..5 carry x = (i, 2i, -i); new 6..9
    n, src, dst = graphs.path(10)
    # relabel so that old vertices are 0, 2, 4, 6, 8 -> ids 0..4 and new ones 5..9
    old = [0, 2, 4, 6, 8]
    new = [1, 3, 5, 7, 9]
    idmap = np.empty(10, dtype=np.int32)
    idmap[old] = np.arange(5)
    idmap[new] = 5 + np.arange(5)
    g = orc.graph_build(10, idmap[src], idmap[dst])
    X = np.zeros((10, 3))
    pos = np.empty(10)
    pos[idmap] = np.arange(10, dtype=float)
    X[:5] = np.stack([pos[:5], 2 * pos[:5], -pos[:5]], 1)
    Y = orc.warm_fill(g, 5, X)
    assert np.array_equal(Y[:5], X[:5])
    # interior new vertices sit between two old ones: the mean is exact
    for i in range(5, 9):
        assert np.array_equal(Y[i], [pos[i], 2 * pos[i], -pos[i]])
    # vertex 9 (last on the path) has one old neighbour, 8
    assert np.array_equal(Y[9], [8.0, 16.0, -8.0])


def test_constant_rows_and_isolated_new_vertices(orc):
    n, src, dst = graphs.random_multigraph(200, 900, 1, self_loops=False)
    src = np.concatenate([src, [150]]).astype(np.int32)       # 199 stays without old neighbour
    dst = np.concatenate([dst, [151]]).astype(np.int32)
    keep = (src != 199) & (dst != 199)
    g = orc.graph_build(n, src[keep], dst[keep])
    X = np.zeros((n, 4))
    X[:150] = [0.25, -1.5, 3.0, 0.0]
    Y = orc.warm_fill(g, 150, X)
    has_old = np.array([np.any(g.col[g.row_ptr[i]:g.row_ptr[i + 1]] < 150) for i in range(n)])
    assert np.all(Y[150:][has_old[150:]] == [0.25, -1.5, 3.0, 0.0])
    assert np.all(Y[150:][~has_old[150:]] == 0.0)
    assert not has_old[199]


def test_fill_improves_the_start_of_a_snowball_stage(orc):
    g0 = dcsbm(3000, 8, 20.0, 0.85, seed=3)
    stages, _ = snowball_stages(g0, 10, seed=1)
    (n1, s1, d1), (n2, s2, d2) = stages[5], stages[6]
    g1 = orc.graph_build(n1, s1, d1)
    v1, _ = orc.laplacian(g1)
    X1 = orc.lobpcg(g1, v1, gaussian_block(n1, 8, 1), 60, 1e-8).X
    g2 = orc.graph_build(n2, s2, d2)
    v2, _ = orc.laplacian(g2)
    zero = np.zeros((n2, 8))
    zero[:n1] = X1
    fill = orc.warm_fill(g2, n1, zero)
    r0 = orc.lobpcg(g2, v2, zero, 0)
    rf = orc.lobpcg(g2, v2, fill, 0)
    assert rf.max_relres < r0.max_relres
    assert np.sum(rf.theta) < np.sum(r0.theta)
