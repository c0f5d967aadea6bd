"""Partition quality against a known truth (Section IV): optimal partition
matching (PM), pairwise recall (PR) and pairwise precision (PP).

The paper names the three measures without defining them; the readings used
here, from the contingency table N[a, b] = #{i : truth_i = a, found_i = b}:
  PM = max over one-to-one block matchings of sum N[a, match(a)] / n
       (Hungarian assignment, Kuhn 1955),
  PR = sum C(N[a,b], 2) / sum_a C(rowsum_a, 2)   (truth pairs kept together),
  PP = sum C(N[a,b], 2) / sum_b C(colsum_b, 2)   (found pairs that are true).
Host-side evaluation only; not part of the GPU path.
"""
from __future__ import annotations

import numpy as np


def contingency(truth, found) -> np.ndarray:
    truth = np.asarray(truth, dtype=np.int64)
    found = np.asarray(found, dtype=np.int64)
    if truth.shape != found.shape:
        raise ValueError("truth and found must have the same length")
    _, t = np.unique(truth, return_inverse=True)
    _, f = np.unique(found, return_inverse=True)
    M = np.zeros((t.max() + 1 if t.size else 0, f.max() + 1 if f.size else 0), dtype=np.int64)
    np.add.at(M, (t, f), 1)
    return M


def _pairs(x):
    x = np.asarray(x, dtype=np.float64)
    return (x * (x - 1.0) / 2.0).sum()


def partition_scores(truth, found) -> dict:
    from scipy.optimize import linear_sum_assignment
    M = contingency(truth, found)
    n = int(M.sum())
    if n == 0:
        return {"PM": 1.0, "PR": 1.0, "PP": 1.0}
    r, c = linear_sum_assignment(-M)
    pm = float(M[r, c].sum()) / n
    same = _pairs(M)
    tp = _pairs(M.sum(axis=1))
    fp = _pairs(M.sum(axis=0))
    pr = float(same / tp) if tp > 0 else 1.0
    pp = float(same / fp) if fp > 0 else 1.0
    return {"PM": pm, "PR": pr, "PP": pp}


def canonical_labels(labels) -> np.ndarray:
    """Relabel clusters by first occurrence in vertex order (label-permutation
    invariant form used to compare two labelings for equality)."""
    labels = np.asarray(labels)
    _, first = np.unique(labels, return_index=True)
    order = np.argsort(first, kind="stable")
    uniq = np.unique(labels)
    remap = {int(uniq[o]): i for i, o in enumerate(order)}
    return np.array([remap[int(x)] for x in labels], dtype=np.int32) if labels.size < 4096 \
        else np.vectorize(remap.get, otypes=[np.int32])(labels)
