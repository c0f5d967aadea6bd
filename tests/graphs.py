"""Small named graphs (directed COO, one direction per edge) for closed-form pins."""
import itertools

import numpy as np


def _coo(edges, n):
    e = np.array(list(edges), dtype=np.int64).reshape(-1, 2)
    return n, e[:, 0].astype(np.int32), e[:, 1].astype(np.int32)


def complete(n):
    return _coo(itertools.combinations(range(n), 2), n)


def cycle(n):
    return _coo(((i, (i + 1) % n) for i in range(n)), n)


def path(n):
    return _coo(((i, i + 1) for i in range(n - 1)), n)


def bipartite(a, b):
    return _coo(((i, a + j) for i in range(a) for j in range(b)), a + b)


def star(n):
    return bipartite(1, n - 1)


def hypercube(d):
    n = 1 << d
    return _coo(((i, i ^ (1 << b)) for i in range(n) for b in range(d) if i < i ^ (1 << b)), n)


def cliques(sizes):
    edges, off = [], 0
    for s in sizes:
        edges += [(off + i, off + j) for i, j in itertools.combinations(range(s), 2)]
        off += s
    return _coo(edges, off)


def random_multigraph(n, m, seed, self_loops=True):
    rng = np.random.default_rng(seed)
    src = rng.integers(0, n, m).astype(np.int32)
    dst = rng.integers(0, n, m).astype(np.int32)
    if not self_loops:
        keep = src != dst
        src, dst = src[keep], dst[keep]
    return n, src, dst
