"""Pins of the oracle's row normalisation + k-means++ / Lloyd labelling
(Section II-A: labels from the approximate eigenvectors, k-means++ as the
classic choice) against hand-derived seeding draws, brute-force optimal
partitions, scikit-learn and orthogonal invariance."""
import itertools

import numpy as np
import pytest

from paper_1708_07481_amd.metrics import canonical_labels


def _blobs(n_per, centers, spread, seed):
    rng = np.random.default_rng(seed)
    pts = [c + spread * rng.standard_normal((n_per, len(c))) for c in centers]
    return np.vstack(pts), np.repeat(np.arange(len(centers)), n_per)


DIAMOND = np.array([[1.0, 0.0], [0.0, 1.0], [-1.0, 0.0], [0.0, -1.0]])


def test_seeding_hand_example(orc):
    """Four unit vectors.  n = 4, max ||y||^2 = 1 so the weight shift is
    61 - 2 - 3 = 56.  u0 = 0 picks y0; D2 = [0, 2, 4, 2] gives weights
    [0, 2^57, 2^58, 2^57], prefix [0, 2^57, 3*2^57, 2^59], T = 2^59 and
    t = floor(u1 * T / 2^64) = u1 >> 5.  The second centre is the first i
    with prefix_i > t."""
    for u1, pick in [(1 << 63, 2), (1 << 62, 2), ((1 << 62) - 1, 1), (0, 1),
                     ((1 << 64) - 1, 3), (3 << 62, 3), ((3 << 62) - 1, 2)]:
        draws = np.array([[0, u1]], dtype=np.uint64)
        km = orc.kmeans(DIAMOND, 2, draws, max_iter=0)
        assert np.array_equal(km.centroids[1], DIAMOND[pick]), (u1, pick)
    # Lloyd from centres y0, y2: y1 and y3 are equidistant -> ties to cluster 0;
    # update gives c0 = (1/3, 0), c1 = (-1, 0); nothing moves afterwards.
    km = orc.kmeans(DIAMOND, 2, np.array([[0, 1 << 63]], dtype=np.uint64), max_iter=10)
    assert km.labels.tolist() == [0, 0, 1, 0]
    assert np.array_equal(km.centroids, [[1 / 3, 0.0], [-1.0, 0.0]])
    assert km.lloyd_iters == 1
    # inertia: (2/3)^2 + (1/3)^2+1 + 0 + (1/3)^2+1
    assert abs(km.inertia - (4 / 9 + 2 * (10 / 9))) < 1e-15


def test_row_normalize(orc):
    X = np.array([[3.0, 4.0], [0.0, 0.0], [-1e-150, 1e-150], [2.0, 0.0], [1e-200, 1e-200]])
    Y = orc.row_normalize(X)
    assert np.array_equal(Y[0], [0.6, 0.8])
    assert np.array_equal(Y[1], [0.0, 0.0])
    assert np.array_equal(Y[3], [1.0, 0.0])
    assert np.allclose(np.linalg.norm(Y[[0, 2, 3]], axis=1), 1.0, atol=1e-15)
    # the sum of squares underflows to zero: the row counts as a zero row
    assert np.array_equal(Y[4], [0.0, 0.0])


@pytest.mark.parametrize("seed", range(4))
def test_brute_force_optimum(orc, seed):
    rng = np.random.default_rng(seed)
    K = 3
    centers = rng.standard_normal((K, 3)) * 5
    X, _ = _blobs(3, centers, 0.2, seed)
    n = X.shape[0]
    best = np.inf
    for lab in itertools.product(range(K), repeat=n):
        lab = np.array(lab)
        if len(set(lab.tolist())) < K:
            continue
        s = sum(((X[lab == j] - X[lab == j].mean(0)) ** 2).sum() for j in range(K))
        best = min(best, s)
    draws = np.random.default_rng(seed + 100).integers(0, 2**63, (10, K), dtype=np.uint64) * 2
    km = orc.kmeans(X, K, draws, normalize=False)
    assert abs(km.inertia - best) < 1e-9 * max(1.0, best)


def test_matches_sklearn_on_separated_blobs(orc):
    skc = pytest.importorskip("sklearn.cluster")
    rng = np.random.default_rng(3)
    centers = rng.standard_normal((6, 5)) * 8
    X, truth = _blobs(40, centers, 0.3, 3)
    draws = rng.integers(0, 2**63, (10, 6), dtype=np.uint64) * 2
    km = orc.kmeans(X, 6, draws, normalize=False)
    ref = skc.KMeans(6, n_init=10, random_state=0).fit(X)
    assert np.array_equal(canonical_labels(km.labels), canonical_labels(ref.labels_))
    assert np.array_equal(canonical_labels(km.labels), canonical_labels(truth))


def test_orthogonal_invariance(orc):
    rng = np.random.default_rng(4)
    centers = rng.standard_normal((5, 7)) * 6
    X, _ = _blobs(30, centers, 0.2, 4)
    Q = np.linalg.qr(rng.standard_normal((7, 7)))[0]
    draws = rng.integers(0, 2**63, (5, 5), dtype=np.uint64) * 2
    a = orc.kmeans(X, 5, draws)
    b = orc.kmeans(X @ Q, 5, draws)
    assert np.array_equal(canonical_labels(a.labels), canonical_labels(b.labels))


def test_restart_choice_is_least_integer_inertia(orc):
    rng = np.random.default_rng(5)
    X = rng.standard_normal((200, 4))
    draws = rng.integers(0, 2**63, (6, 5), dtype=np.uint64) * 2
    full = orc.kmeans(X, 5, draws)
    qs = [orc.kmeans(X, 5, draws[r:r + 1]).inertia_q for r in range(6)]
    assert full.inertia_q == min(qs) and full.best_restart == int(np.argmin(qs))


def test_pure_assignment_with_given_centroids(orc):
    rng = np.random.default_rng(6)
    X = rng.standard_normal((100, 3))
    C = rng.standard_normal((4, 3))
    km = orc.kmeans(X, 4, init_centroids=C, max_iter=0, normalize=False)
    d = ((X[:, None, :] - C[None]) ** 2).sum(-1)
    assert np.array_equal(km.labels, np.argmin(d, axis=1))


@pytest.mark.parametrize("sizes", [(1000, 257, 256), (255, 513, 1)])
def test_centroid_is_exact_mean_of_large_clusters(orc, sizes):
    """Centroids are member means.  Coordinates are multiples of 2^-10 below
    2^4, so every partial sum is exact whatever the order: the centroid must
    equal the exact rational mean rounded once (by the division).  A member
    dropped, added twice or counted in the wrong cluster changes the result."""
    from fractions import Fraction
    rng = np.random.default_rng(7)
    centres = np.array([[100.0, 0.0, 0.0], [0.0, 100.0, 0.0], [0.0, 0.0, 100.0]])
    pts, truth = [], []
    for j, s in enumerate(sizes):
        off = rng.integers(-8192, 8192, size=(s, 3)) / 1024.0
        pts.append(centres[j] + off)
        truth += [j] * s
    X = np.concatenate(pts)
    perm = rng.permutation(X.shape[0])
    X, truth = X[perm], np.array(truth)[perm]
    r = orc.kmeans(X, 3, init_centroids=centres, max_iter=1, normalize=False)
    assert np.array_equal(r.labels, truth)
    for j in range(3):
        mem = X[truth == j]
        for d in range(3):
            exact = sum(Fraction(float(v)) for v in mem[:, d]) / len(mem)
            assert r.centroids[j, d] == float(exact), (j, d)


def _rn(q):
    """Round an exact rational to the nearest double (ties to even)."""
    from fractions import Fraction
    return float(Fraction(q))


def test_centroid_sum_is_one_ordered_chain(orc):
    """Each centroid coordinate is one FP64 chain from 0.0 over the members
    in ascending vertex order, then divided by the count.  The chain is
    replayed here with exact rationals, every addition rounded to the nearest
    double, on coordinates that are not dyadic, so the rounding of every step
    shows.  The data are chosen so that the replay tells the orders apart: a
    sum in blocks of 256 members, a descending order and the exactly rounded
    mean each differ from the ordered chain in some coordinate, and the
    oracle must equal the ordered chain in every coordinate.  Its distance to
    the exact mean stays within the chain's error bound."""
    from fractions import Fraction
    rng = np.random.default_rng(17)
    sizes = (700, 513, 300)
    dim = 4
    centres = np.zeros((3, dim))
    centres[:, :3] = 1e7 * np.eye(3)
    pts, truth = [], []
    for j, s in enumerate(sizes):
        pts.append(centres[j] + rng.standard_normal((s, dim)) * np.array([3.0, 1e-3, 7e5, 0.1]))
        truth += [j] * s
    X = np.concatenate(pts)
    perm = rng.permutation(X.shape[0])
    X, truth = X[perm], np.array(truth)[perm]
    r = orc.kmeans(X, 3, init_centroids=centres, max_iter=1, normalize=False)
    assert np.array_equal(r.labels, truth)

    def chain(vals):
        s = 0.0
        for v in vals:
            s = _rn(Fraction(s) + Fraction(float(v)))
        return s

    diffs = {"blocked": 0, "descending": 0, "exact": 0}
    eps = 2.0 ** -53
    for j in range(3):
        mem = X[truth == j]          # ascending vertex order (a boolean mask keeps order)
        cnt = len(mem)
        for d in range(dim):
            col = mem[:, d]
            seq = chain(col)
            want = _rn(Fraction(seq) / cnt)
            assert r.centroids[j, d] == want, (j, d, r.centroids[j, d], want)
            blocks = [chain(col[b:b + 256]) for b in range(0, cnt, 256)]
            diffs["blocked"] += _rn(Fraction(chain(blocks)) / cnt) != want
            diffs["descending"] += _rn(Fraction(chain(col[::-1])) / cnt) != want
            exact = sum(Fraction(float(v)) for v in col) / cnt
            diffs["exact"] += _rn(exact) != want
            # |fl(chain) - sum| <= (cnt - 1) eps sum|y| (+ the division's half ulp)
            bound = (cnt - 1) * eps * float(np.abs(col).sum()) / cnt + abs(want) * eps
            assert abs(Fraction(want) - exact) <= Fraction(bound) * 1.01, (j, d)
    assert all(v > 0 for v in diffs.values()), diffs
