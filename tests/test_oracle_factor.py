"""Pins for the oracle's t-SVD, randomized t-SVD and sketch generator."""
import os

import numpy as np
import scipy.sparse as sp

from oracle.factor import rademacher_sketch, splitmix64, tsvd_exact, tsvd_randomized
from workloads import block_graph

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def test_splitmix64_known_answers():
    vals = [int(line, 16) for line in open(os.path.join(GOLDEN, "splitmix64_seed0.txt"))
            if line.strip() and not line.startswith("#")]
    g = 0x9E3779B97F4A7C15
    got = [int(splitmix64(np.uint64((i * g) % 2**64))) for i in range(3)]
    assert got == vals


def test_sketch_is_balanced_rademacher():
    om = rademacher_sketch(4000, 50, seed=3)
    assert set(np.unique(om)) == {-1.0, 1.0}
    assert abs(om.mean()) < 0.01
    # columns nearly orthogonal: |<w_i, w_j>| / n ~ 1/sqrt(n)
    G = om.T @ om / om.shape[0]
    assert np.abs(G - np.eye(50)).max() < 0.08
    assert not np.array_equal(om, rademacher_sketch(4000, 50, seed=4))


def test_tsvd_exact_eckart_young():
    rng = np.random.default_rng(0)
    A = (rng.random((30, 25)) < 0.3).astype(float)
    d = 7
    U, s, V = tsvd_exact(A, d)
    full = np.linalg.svd(A, compute_uv=False)
    assert np.all(np.diff(s) <= 0)
    assert np.allclose(U.T @ U, np.eye(d), atol=1e-12)
    assert np.allclose(V.T @ V, np.eye(d), atol=1e-12)
    err = np.linalg.norm(A - U @ np.diag(s) @ V.T)
    assert np.isclose(err, np.sqrt((full[d:] ** 2).sum()), rtol=1e-10)


def test_randomized_exact_on_low_rank():
    n, blocks, d = 300, 6, 8
    s_, t_ = block_graph(n, blocks, seed=5)
    A = sp.csr_matrix((np.ones(len(s_)), (s_, t_)), shape=(n, n))
    U, s, V = tsvd_randomized(A, d, oversample=4, power_iters=2, seed=9)
    assert np.allclose(U @ np.diag(s) @ V.T, A.toarray(), atol=1e-10)
    ref = np.linalg.svd(A.toarray(), compute_uv=False)[:d]
    assert np.allclose(s, ref, atol=1e-10)


def test_randomized_close_to_exact_with_gap():
    rng = np.random.default_rng(1)
    n, d = 200, 5
    # strong rank-5 signal plus weak noise: large gap after sigma_5
    L = rng.standard_normal((n, d)) @ np.diag([40, 30, 25, 20, 15]) @ rng.standard_normal((d, n)) / np.sqrt(n)
    A = L + 0.01 * rng.standard_normal((n, n))
    U, s, V = tsvd_randomized(A, d, oversample=10, power_iters=2, seed=2)
    Ue, se, Ve = tsvd_exact(A, d)
    assert np.allclose(s, se, rtol=1e-8)
    assert np.linalg.norm(U @ np.diag(s) @ V.T - Ue @ np.diag(se) @ Ve.T) < 1e-6 * se[0]
