"""Degree-corrected stochastic block model (Karrer & Newman 2011) generator.

The paper evaluates on the stochastic-block-partition challenge graphs with
known truth partitions (Section III).  Those files are not available here, so
seeded synthetic graphs of the same family and the same shapes (vertices /
edges / blocks of Table I) stand in for them.  The recipe:

1. block sizes: near-equal (floor(N/B), +1 for the first N mod B blocks) or
   proportions p ~ Dirichlet(alpha 1_B) turned into sizes by largest-remainder
   rounding on top of a floor of 2 vertices per block;
2. vertex -> block through a seeded random permutation (ids carry no locality);
3. degree propensities theta_i: power law with exponent 2.5 truncated to
   [1, 50], drawn by inverse CDF;
4. m* = round(N * dbar / 2) target undirected edges.  Block r receives
   Poisson(f m* S_r / S) intra-block edges whose endpoints are drawn
   proportionally to theta inside r (S_r = sum of theta over r); the
   Poisson((1-f) m*) inter-block edges draw both endpoints proportionally to
   theta over all vertices and redraw pairs that fall in one block;
5. self loops are dropped, unordered duplicates are merged (unit weights) and
   the graph is emitted as a directed COO list, one direction per edge, which
   the symmetrisation of Section II-A turns back into an undirected graph.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np

THETA_MAX = 50.0
THETA_EXPONENT = 2.5


def _rng(seed: int, stream: int = 0) -> np.random.Generator:
    # Philox4x32-10 keyed by the seed; `stream` separates independent uses.
    return np.random.Generator(np.random.Philox(key=[int(seed) & 0xFFFFFFFFFFFFFFFF,
                                                     int(stream)]))


@dataclass
class SBMGraph:
    n: int
    src: np.ndarray          # int32 [m], one direction per undirected edge
    dst: np.ndarray          # int32 [m]
    truth: np.ndarray        # int32 [n], generating block of every vertex
    n_blocks: int
    theta: np.ndarray = field(repr=False, default=None)

    @property
    def m(self) -> int:
        return int(self.src.shape[0])


def block_sizes(n: int, n_blocks: int, kind: str = "equal", alpha: float = 1.0,
                seed: int = 0) -> np.ndarray:
    """Block sizes summing to n (step 1 of the recipe)."""
    if kind == "equal":
        sizes = np.full(n_blocks, n // n_blocks, dtype=np.int64)
        sizes[: n % n_blocks] += 1
        return sizes
    if kind != "dirichlet":
        raise ValueError(f"unknown block size kind {kind!r}")
    if n < 2 * n_blocks:
        raise ValueError("need at least 2 vertices per block")
    p = _rng(seed, 1).dirichlet(np.full(n_blocks, float(alpha)))
    free = n - 2 * n_blocks
    raw = free * p
    base = np.floor(raw).astype(np.int64)
    rem = free - int(base.sum())
    order = np.argsort(-(raw - base), kind="stable")
    base[order[:rem]] += 1
    return base + 2


def _theta(n: int, rng: np.random.Generator) -> np.ndarray:
    a = THETA_EXPONENT - 1.0
    u = rng.random(n)
    return (1.0 - u * (1.0 - THETA_MAX ** (-a))) ** (-1.0 / a)


def dcsbm(n: int, n_blocks: int, mean_degree: float, intra_fraction: float,
          sizes: str = "equal", alpha: float = 1.0, seed: int = 1) -> SBMGraph:
    """Draw one degree-corrected SBM graph (steps 1-5 of the module recipe)."""
    rng = _rng(seed, 0)
    bs = block_sizes(n, n_blocks, sizes, alpha, seed)
    perm = rng.permutation(n)
    truth = np.empty(n, dtype=np.int32)
    starts = np.concatenate([[0], np.cumsum(bs)])
    for r in range(n_blocks):
        truth[perm[starts[r]:starts[r + 1]]] = r
    theta = _theta(n, rng)

    m_target = int(round(n * mean_degree / 2.0))
    th_perm = theta[perm]
    cum = np.cumsum(th_perm)
    cum_before = np.concatenate([[0.0], cum])[starts[:-1]]
    s_r = np.add.reduceat(th_perm, starts[:-1])
    s_tot = float(th_perm.sum())

    def draw_intra(blk):
        ends = []
        for _ in range(2):
            t = cum_before[blk] + rng.random(blk.shape[0]) * s_r[blk]
            idx = np.searchsorted(cum, t, side="right")
            idx = np.clip(idx, starts[blk], starts[blk + 1] - 1)
            ends.append(perm[idx].astype(np.int64))
        return ends

    def draw_inter(cnt):
        eu = np.empty(0, dtype=np.int64)
        ev = np.empty(0, dtype=np.int64)
        while eu.shape[0] < cnt:
            need = cnt - eu.shape[0]
            t1 = rng.random(need) * s_tot
            t2 = rng.random(need) * s_tot
            a = perm[np.minimum(np.searchsorted(cum, t1, side="right"), n - 1)]
            b = perm[np.minimum(np.searchsorted(cum, t2, side="right"), n - 1)]
            keep = truth[a] != truth[b]
            eu = np.concatenate([eu, a[keep]])
            ev = np.concatenate([ev, b[keep]])
        return eu, ev

    # Target counts: Poisson(f m* S_r / S) intra edges per block r and
    # Poisson((1-f) m*) inter-block edges.  Self loops and repeated pairs are
    # discarded and redrawn (a few top-up rounds), so the emitted graph has
    # close to m* distinct edges and the requested mean degree.
    want = np.append(rng.poisson(intra_fraction * m_target * s_r / s_tot),
                     rng.poisson((1.0 - intra_fraction) * m_target)).astype(np.int64)
    cap = starts[1:] - starts[:-1]
    want[:-1] = np.minimum(want[:-1], cap * (cap - 1) // 4)
    have = np.zeros(n_blocks + 1, dtype=np.int64)
    keys = np.empty(0, dtype=np.int64)          # sorted keys of accepted edges
    parts_u, parts_v = [], []
    for _ in range(12):
        deficit = want - have
        if deficit.sum() <= 1e-4 * m_target:
            break
        blk = np.repeat(np.arange(n_blocks), deficit[:-1])
        iu, iv = draw_intra(blk)
        eu, ev = draw_inter(int(deficit[-1]))
        u = np.concatenate([iu, eu])
        v = np.concatenate([iv, ev])
        keep = u != v
        u, v = u[keep], v[keep]
        key = np.minimum(u, v) * n + np.maximum(u, v)
        pos = np.searchsorted(keys, key)
        fresh = (pos >= keys.shape[0]) | (keys[np.minimum(pos, max(keys.shape[0] - 1, 0))] != key) \
            if keys.shape[0] else np.ones(key.shape[0], dtype=bool)
        u, v, key = u[fresh], v[fresh], key[fresh]
        _, first = np.unique(key, return_index=True)
        first.sort()
        u, v, key = u[first], v[first], key[first]
        # accept at most the remaining target of each category, in draw order
        cat = np.where(truth[u] == truth[v], truth[u], n_blocks)
        order = np.argsort(cat, kind="stable")
        cnt = np.bincount(cat, minlength=n_blocks + 1)
        cstart = np.concatenate([[0], np.cumsum(cnt)[:-1]])
        rank = np.empty_like(order)
        rank[order] = np.arange(order.shape[0]) - np.repeat(cstart, cnt)
        ok = rank < deficit[cat]
        u, v, key, cat = u[ok], v[ok], key[ok], cat[ok]
        have += np.bincount(cat, minlength=n_blocks + 1)
        parts_u.append(u)
        parts_v.append(v)
        keys = np.sort(np.concatenate([keys, key]), kind="stable")
    u = np.concatenate(parts_u) if parts_u else np.empty(0, dtype=np.int64)
    v = np.concatenate(parts_v) if parts_v else np.empty(0, dtype=np.int64)
    first = np.arange(u.shape[0])
    return SBMGraph(n=n, src=u[first].astype(np.int32), dst=v[first].astype(np.int32),
                    truth=truth, n_blocks=n_blocks, theta=theta)


def gaussian_block(n: int, k: int, seed: int) -> np.ndarray:
    """n x k block of i.i.d. N(0,1) entries, float64, row-major (Section III)."""
    return _rng(seed, 2).standard_normal((n, k))


def kmeans_draws(restarts: int, n_clusters: int, seed: int) -> np.ndarray:
    """Uniform 64-bit words consumed by k-means++ seeding: [restarts, n_clusters]."""
    bg = np.random.Philox(key=[int(seed) & 0xFFFFFFFFFFFFFFFF, 3])
    return bg.random_raw(restarts * n_clusters).astype(np.uint64).reshape(restarts, n_clusters)


def emerging_stages(g: SBMGraph, stages: int = 10, seed: int = 0):
    """Emerging-edge stream: a seeded permutation of the edge list; stage s
    (1-based) holds the first ceil(s m / stages) edges.  All n vertices exist
    from the first stage.  Returns a list of (n, src, dst)."""
    order = _rng(seed, 4).permutation(g.m)
    src, dst = g.src[order], g.dst[order]
    out = []
    for s in range(1, stages + 1):
        c = int(math.ceil(s * g.m / stages))
        out.append((g.n, src[:c].copy(), dst[:c].copy()))
    return out, g.truth.copy()


def snowball_stages(g: SBMGraph, stages: int = 10, seed: int = 0, n_sources: int | None = None):
    """Snowball stream: vertices are revealed in multi-source breadth-first
    order (FIFO, neighbours in ascending id) from seeded random sources; when
    the frontier empties, a seeded unvisited vertex restarts the search.
    Vertices are renumbered in reveal order, so the vertices of earlier stages
    keep their ids and come first (Section III, snowball warm start).  Stage s
    is the subgraph induced by the first ceil(s n / stages) revealed vertices.
    Returns (list of (n_s, src, dst), truth in the new numbering)."""
    rng = _rng(seed, 5)
    n = g.n
    a = np.concatenate([g.src, g.dst]).astype(np.int64)
    b = np.concatenate([g.dst, g.src]).astype(np.int64)
    o = np.lexsort((b, a))
    a, b = a[o], b[o]
    ptr = np.zeros(n + 1, dtype=np.int64)
    np.add.at(ptr, a + 1, 1)
    ptr = np.cumsum(ptr)
    visited = np.zeros(n, dtype=bool)
    order = []
    n_src = n_sources if n_sources is not None else g.n_blocks
    frontier = rng.choice(n, size=min(n_src, n), replace=False).astype(np.int64)
    visited[frontier] = True
    order.append(frontier)
    seen = frontier.shape[0]
    while seen < n:
        if frontier.shape[0] == 0:
            unv = np.flatnonzero(~visited)
            frontier = np.array([unv[rng.integers(unv.shape[0])]], dtype=np.int64)
            visited[frontier] = True
            order.append(frontier)
            seen += 1
            continue
        lens = ptr[frontier + 1] - ptr[frontier]
        idx = np.repeat(ptr[frontier] - np.concatenate([[0], np.cumsum(lens)[:-1]]), lens) \
            + np.arange(int(lens.sum()))
        nb = b[idx]
        nb = nb[~visited[nb]]
        _, first = np.unique(nb, return_index=True)
        first.sort()
        nxt = nb[first]
        visited[nxt] = True
        order.append(nxt)
        seen += nxt.shape[0]
        frontier = nxt
    reveal = np.concatenate(order)
    new_id = np.empty(n, dtype=np.int64)
    new_id[reveal] = np.arange(n)
    su, sv = new_id[g.src], new_id[g.dst]
    out = []
    for s in range(1, stages + 1):
        ns = int(math.ceil(s * n / stages))
        keep = (su < ns) & (sv < ns)
        out.append((ns, su[keep].astype(np.int32), sv[keep].astype(np.int32)))
    truth = np.empty(n, dtype=np.int32)
    truth[new_id] = g.truth
    return out, truth
