"""The link-prediction harness's metrics and splits (CPU): AUC and AP against
brute force over all pairs and against scikit-learn, precision@K by hand."""
import numpy as np
import pytest

from workloads import linkpred as lp


def test_auc_is_pairwise_probability():
    rng = np.random.default_rng(0)
    pos = rng.integers(0, 5, 40).astype(float)  # many ties
    neg = rng.integers(0, 4, 55).astype(float)
    brute = np.mean([(p > q) + 0.5 * (p == q) for p in pos for q in neg])
    assert abs(lp.auc(pos, neg) - brute) <= 1e-12


def test_auc_ap_match_sklearn():
    skm = pytest.importorskip("sklearn.metrics")
    rng = np.random.default_rng(1)
    pos = rng.normal(1.0, 1.0, 500)
    neg = rng.normal(0.0, 1.0, 700)
    y = np.r_[np.ones(500), np.zeros(700)]
    sc = np.r_[pos, neg]
    assert abs(lp.auc(pos, neg) - skm.roc_auc_score(y, sc)) <= 1e-12
    assert abs(lp.average_precision(pos, neg) - skm.average_precision_score(y, sc)) <= 1e-12


def test_ap_brute_force_and_extremes():
    pos, neg = np.array([0.9, 0.4, 0.7]), np.array([0.8, 0.1])
    # descending: 0.9(+) 0.8(-) 0.7(+) 0.4(+) 0.1(-): precisions 1, 2/3, 3/4
    assert abs(lp.average_precision(pos, neg) - (1 + 2 / 3 + 3 / 4) / 3) <= 1e-12
    assert lp.average_precision([2.0, 3.0], [0.0, 1.0]) == 1.0
    assert lp.auc([2.0, 3.0], [0.0, 1.0]) == 1.0 and lp.auc([0.0], [1.0]) == 0.0


def test_precision_at_k():
    sc = np.array([0.5, 0.9, 0.1, 0.7, 0.3])
    ed = np.array([1, 0, 1, 1, 0])
    p = lp.precision_at_k(sc, ed, [1, 2, 3, 5])
    assert p == {1: 0.0, 2: 0.5, 3: 2 / 3, 5: 0.6}


def test_split_and_negatives():
    rng = np.random.default_rng(2)
    n = 200
    s, t = rng.integers(0, n, 1000), rng.integers(0, n, 1000)
    (ks, kt), (rs, rt) = lp.holdout_split(s, t, 0.3, seed=3)
    assert len(rs) == 300 and len(ks) == 700
    assert sorted(zip(np.r_[ks, rs], np.r_[kt, rt])) == sorted(zip(s, t))
    keys = lp.edge_keys(s, t, n)
    u, v = lp.negative_pairs(n, 500, keys, seed=4)
    assert len(u) == 500 and np.all(u != v)
    assert not np.isin(u.astype(np.int64) * n + v, keys).any()
    keys_u = lp.edge_keys(s, t, n, directed=False)
    assert np.isin(t.astype(np.int64) * n + s, keys_u).all()
