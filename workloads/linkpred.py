"""Synthetic link-prediction and graph-reconstruction harness (Sec. 5.2).

The paper's evaluation removes a share of the edges, embeds the remaining
graph, and scores node pairs by the inner product of u's context vector and
v's content vector (for undirected graphs the larger of both directions);
link prediction reports the area under the ROC curve and the average
precision over the removed edges plus as many unconnected pairs, and graph
reconstruction the precision@K of the top-K scored pairs of a pair set.

This module holds the seeded splits and the metrics only (no arithmetic of
the method): the scores come from the library (damf_score_pairs) or, in the
tests, from the oracle.  The metrics follow their textbook definitions:

- AUC: the probability that a random positive pair scores above a random
  negative one, ties counting one half (the Mann-Whitney statistic).
- AP: the mean over the positives of the precision among the pairs scored at
  least as high as that positive (pairs sorted by descending score, ties
  broken by a stable order).
- precision@K: the share of edges among the K highest-scored pairs.
"""
from __future__ import annotations

import numpy as np


def holdout_split(src, dst, frac, seed, directed=True):
    """Split an edge list into (kept, removed) by a seeded permutation; the
    removed share is round(frac * m) edges.  Undirected lists hold each edge
    once, so the split keeps both orientations together."""
    src = np.asarray(src)
    dst = np.asarray(dst)
    rng = np.random.default_rng(seed)
    perm = rng.permutation(len(src))
    k = int(round(frac * len(src)))
    rem, keep = perm[:k], perm[k:]
    return (src[keep], dst[keep]), (src[rem], dst[rem])


def negative_pairs(n, count, edge_keys, seed, directed=True):
    """`count` node pairs (u, v), u != v, that are not edges of the full graph
    (edge_keys: a set of u * n + v keys; undirected graphs list both
    orientations), drawn uniformly with rejection."""
    rng = np.random.default_rng(seed)
    us, vs = [], []
    need = count
    while need > 0:
        u = rng.integers(0, n, 2 * need + 16)
        v = rng.integers(0, n, 2 * need + 16)
        ok = u != v
        keys = u.astype(np.int64) * n + v
        ok &= ~np.isin(keys, edge_keys)
        u, v = u[ok][:need], v[ok][:need]
        us.append(u)
        vs.append(v)
        need -= len(u)
    return np.concatenate(us).astype(np.int32), np.concatenate(vs).astype(np.int32)


def edge_keys(src, dst, n, directed=True):
    """Sorted unique int64 keys u * n + v of an edge list (both orientations
    when undirected)."""
    s = np.asarray(src, dtype=np.int64)
    t = np.asarray(dst, dtype=np.int64)
    k = s * n + t
    if not directed:
        k = np.concatenate([k, t * n + s])
    return np.unique(k)


def auc(pos, neg):
    """Area under the ROC curve: P(score_pos > score_neg) + P(tie) / 2, from the
    average ranks of all scores (the Mann-Whitney U statistic over |pos| |neg|)."""
    from scipy.stats import rankdata
    pos = np.asarray(pos, dtype=np.float64)
    neg = np.asarray(neg, dtype=np.float64)
    ranks = rankdata(np.concatenate([pos, neg]))  # 1-based, ties averaged
    r_pos = ranks[:len(pos)].sum()
    return float((r_pos - len(pos) * (len(pos) + 1) / 2.0) / (len(pos) * len(neg)))


def average_precision(pos, neg):
    """Mean over positives of the precision at the positive's position in the
    descending score order (a stable sort: positives first among equal
    scores, the order in which they were given)."""
    scores = np.concatenate([np.asarray(pos, np.float64), np.asarray(neg, np.float64)])
    labels = np.concatenate([np.ones(len(pos)), np.zeros(len(neg))])
    order = np.argsort(-scores, kind="mergesort")
    lab = labels[order]
    hits = np.cumsum(lab)
    prec = hits / np.arange(1, len(lab) + 1)
    return float(prec[lab == 1].mean())


def precision_at_k(scores, is_edge, ks):
    """precision@K for each K in ks: share of edges among the K highest scores."""
    order = np.argsort(-np.asarray(scores, np.float64), kind="mergesort")
    hit = np.cumsum(np.asarray(is_edge, np.float64)[order])
    return {int(k): float(hit[min(k, len(hit)) - 1] / min(k, len(hit))) for k in ks}
