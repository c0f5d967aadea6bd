"""Host evaluation metrics (Section IV: PM / PR / PP) and the seeded input
generators (synthetic stand-ins for the challenge graphs of Section III)."""
import hashlib
import json
import math
import os

import numpy as np
import pytest

from paper_1708_07481_amd.metrics import canonical_labels, partition_scores
from synth import (block_sizes, dcsbm, emerging_stages, gaussian_block, kmeans_draws,
                   snowball_stages)
from synth.configs import CONFIGS

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def test_metrics_hand_example():
    s = partition_scores([0, 0, 1, 1], [0, 1, 1, 1])
    assert s["PM"] == 0.75
    assert s["PR"] == pytest.approx(1 / 2)
    assert s["PP"] == pytest.approx(1 / 3)


def test_metrics_permutation_invariant_and_perfect():
    t = np.array([0, 0, 1, 1, 2, 2, 2])
    f = np.array([5, 5, 3, 3, 9, 9, 9])
    assert partition_scores(t, f) == {"PM": 1.0, "PR": 1.0, "PP": 1.0}
    assert np.array_equal(canonical_labels(f), canonical_labels(t))


def test_metrics_pm_brute_force():
    import itertools
    rng = np.random.default_rng(0)
    t = rng.integers(0, 4, 30)
    f = rng.integers(0, 4, 30)
    best = max(sum(int(np.sum((t == a) & (f == p[a]))) for a in range(4))
               for p in itertools.permutations(range(4)))
    assert partition_scores(t, f)["PM"] == best / 30


def test_table1_shapes():
    """The configurations follow the vertex / edge / cluster counts of Table I."""
    with open(os.path.join(GOLDEN, "table1_shapes.json")) as fh:
        tab = json.load(fh)["columns"]
    by_n = {c["n"]: c for c in CONFIGS.values()}
    for col in tab:
        if col["vertices"] not in by_n:
            continue
        c = by_n[col["vertices"]]
        assert c["k"] == col["clusters"] == c["blocks"]
        assert abs(c["n"] * c["mean_degree"] / 2 - col["edges"]) <= 0.03 * col["edges"]


def test_block_sizes():
    s = block_sizes(1000, 8)
    assert s.sum() == 1000 and s.max() - s.min() <= 1
    d = block_sizes(50_000, 44, "dirichlet", 5.0, seed=1)
    assert d.sum() == 50_000 and d.min() >= 2
    d1 = block_sizes(5000, 98, "dirichlet", 1.0, seed=2)
    assert d1.sum() == 5000 and d1.min() >= 2


def test_dcsbm_properties():
    g = dcsbm(5000, 19, 40.0, 0.75, "dirichlet", 5.0, seed=3)
    assert np.all(g.src != g.dst)
    key = np.minimum(g.src, g.dst).astype(np.int64) * g.n + np.maximum(g.src, g.dst)
    assert np.unique(key).size == g.m
    assert abs(g.m - 5000 * 20) < 0.01 * 5000 * 20
    intra = np.mean(g.truth[g.src] == g.truth[g.dst])
    assert abs(intra - 0.75) < 0.01
    deg = np.bincount(np.concatenate([g.src, g.dst]), minlength=g.n)
    assert abs(deg.mean() - 40.0) < 0.5
    assert np.all((g.theta >= 1.0) & (g.theta <= 50.0))
    assert set(np.unique(g.truth)) == set(range(19))


def test_dcsbm_deterministic():
    a = dcsbm(2000, 8, 20.0, 0.8, seed=7)
    b = dcsbm(2000, 8, 20.0, 0.8, seed=7)
    c = dcsbm(2000, 8, 20.0, 0.8, seed=8)
    h = lambda g: hashlib.sha256(g.src.tobytes() + g.dst.tobytes() + g.truth.tobytes()).hexdigest()
    assert h(a) == h(b) and h(a) != h(c)
    assert np.array_equal(gaussian_block(50, 3, 1), gaussian_block(50, 3, 1))
    assert kmeans_draws(10, 8, 1).dtype == np.uint64 and kmeans_draws(10, 8, 1).shape == (10, 8)


def test_emerging_stages_nested():
    g = dcsbm(3000, 10, 20.0, 0.8, seed=2)
    st, truth = emerging_stages(g, 10, seed=1)
    assert len(st) == 10 and st[-1][1].shape[0] == g.m
    for s in range(10):
        n, src, dst = st[s]
        assert n == g.n and src.shape[0] == math.ceil((s + 1) * g.m / 10)
        if s:
            assert np.array_equal(src[: st[s - 1][1].shape[0]], st[s - 1][1])


def test_snowball_stages_keep_old_ids():
    g = dcsbm(3000, 10, 20.0, 0.8, seed=2)
    st, truth = snowball_stages(g, 10, seed=1)
    assert [s[0] for s in st] == [math.ceil((i + 1) * 3000 / 10) for i in range(10)]
    prev = None
    for ns, src, dst in st:
        assert src.max(initial=-1) < ns and dst.max(initial=-1) < ns
        e = set(zip(src.tolist(), dst.tolist()))
        if prev is not None:
            assert prev <= e     # induced subgraphs grow; old vertices keep their ids
        prev = e
    assert st[-1][1].shape[0] == g.m
    assert np.array_equal(np.sort(np.bincount(truth)), np.sort(np.bincount(g.truth)))
