"""Pins for the oracle's space-projection update (Theorem 2 and Algorithm 1)."""
import numpy as np
import pytest

from oracle.factor import tsvd_exact
from oracle.graph import EdgeSet
from oracle.model import DAMFOracle
from oracle.update import chunk, chunk_update, residual_factor, update_one_edge_xform
from workloads import block_graph, er_undirected


def _tsvd_product(M, d):
    U, s, V = tsvd_exact(M, d)
    return U @ np.diag(s) @ V.T, s


def test_proposition1_residual_norm():
    rng = np.random.default_rng(0)
    n, d = 50, 8
    U, _ = np.linalg.qr(rng.standard_normal((n, d)))
    x = rng.standard_normal(n)
    W = U.T @ x
    T, R = residual_factor(np.array([[x @ x - W @ W]]), np.array([[x @ x]]), 1e-12)
    explicit = np.linalg.norm(x - U @ (U.T @ x))
    assert np.isclose(R[0, 0], explicit, rtol=1e-12)
    assert np.isclose(T[0, 0], 1.0 / explicit, rtol=1e-12)


def test_residual_factor_block_is_orthonormal_and_exact():
    rng = np.random.default_rng(1)
    n, d, k = 60, 6, 5
    U, _ = np.linalg.qr(rng.standard_normal((n, d)))
    B = rng.standard_normal((n, k))
    B[:, 4] = B[:, 0] - 2 * B[:, 1]          # rank-deficient block
    W = U.T @ B
    T, R = residual_factor(B.T @ B - W.T @ W, B.T @ B, 1e-10)
    assert R.shape == (4, 5)
    M = B - U @ W
    Q = M @ T
    assert np.allclose(Q.T @ Q, np.eye(4), atol=1e-10)
    assert np.allclose(Q @ R, M, atol=1e-9)


@pytest.mark.parametrize("seed", range(5))
@pytest.mark.parametrize("directed", [True, False])
def test_theorem2_every_chunk(seed, directed):
    """Each chunk gives the exact rank-d t-SVD of (current factorisation + chunk)."""
    rng = np.random.default_rng(seed)
    n, d = 40, 6
    g = EdgeSet(n, directed, rng.integers(0, n, 120), rng.integers(0, n, 120))
    U, s, V = tsvd_exact(g.dense(), d)
    for _ in range(4):
        k = 8
        net = g.apply(rng.integers(0, n, k), rng.integers(0, n, k), rng.choice([-1, 1], k))
        for S1, S2, D in chunk(net, directed, r=3, r_max=6):
            cur = U @ np.diag(s) @ V.T
            dA = np.zeros((n, n))
            dA[np.ix_(S1, S2)] = D
            ref, sref = _tsvd_product(cur + dA, d)
            full = np.linalg.svd(cur + dA, compute_uv=False)
            U, s, V, _ = chunk_update(U, s, V, S1, S2, D, tau=1e-12)
            if full[d - 1] - full[d] > 1e-6:
                assert np.allclose(s, sref, atol=1e-10)
                assert np.allclose(U @ np.diag(s) @ V.T, ref, atol=1e-9)
            assert np.allclose(U.T @ U, np.eye(d), atol=1e-10)
            assert np.allclose(V.T @ V, np.eye(d), atol=1e-10)


def test_row_corrections_only_on_touched_rows():
    """Lemma 1: dU = B T_B E[d:] has nonzero rows only where B does."""
    rng = np.random.default_rng(3)
    n, d = 50, 5
    g = EdgeSet(n, True, rng.integers(0, n, 150), rng.integers(0, n, 150))
    U, s, V = tsvd_exact(g.dense(), d)
    net = g.apply(rng.integers(0, n, 6), rng.integers(0, n, 6), np.ones(6, dtype=np.int8))
    for S1, S2, D in chunk(net, True, r=8, r_max=8):
        U2, s2, V2, info = chunk_update(U, s, V, S1, S2, D, tau=1e-12)
        dU = U2 - U @ info["FU"]
        dV = V2 - V @ info["FV"]
        rows_u = set(np.nonzero(np.abs(dU).max(axis=1) > 1e-13)[0].tolist())
        rows_v = set(np.nonzero(np.abs(dV).max(axis=1) > 1e-13)[0].tolist())
        assert rows_u <= set(S1.tolist())
        assert rows_v <= set(S2.tolist())
        U, s, V = U2, s2, V2


@pytest.mark.parametrize("seed", range(4))
def test_xform_algorithm1_matches_uform(seed):
    """Algorithm 1 as printed (X-form, one edge) and the U-form give the same embedding product."""
    rng = np.random.default_rng(seed)
    n, d = 30, 5
    g = EdgeSet(n, True, rng.integers(0, n, 90), rng.integers(0, n, 90))
    U, s, V = tsvd_exact(g.dense(), d)
    X, Y = U * np.sqrt(s), V * np.sqrt(s)
    for _ in range(6):
        u, v = rng.integers(0, n, 2)
        b = np.zeros(n); b[u] = 1.0
        c = np.zeros(n); c[v] = 1.0
        X, Y, s_x = update_one_edge_xform(X, Y, s, b, c)
        U, s, V, _ = chunk_update(U, s, V, np.array([u]), np.array([v]), np.array([[1.0]]), tau=1e-14)
        assert np.allclose(s_x, s, rtol=1e-12)
        assert np.allclose(X @ Y.T, (U * s) @ V.T, atol=1e-10)
        # X = U Sigma^(1/2) column by column, up to sign
        Xu = U * np.sqrt(s)
        sign = np.sign((X * Xu).sum(axis=0))
        assert np.allclose(X, Xu * sign, atol=1e-9)


def test_exact_when_d_at_least_n():
    """With d = n the t-SVD keeps everything, so X Y^T equals A after every batch."""
    rng = np.random.default_rng(11)
    n = 16
    s0, t0 = rng.integers(0, n, 50), rng.integers(0, n, 50)
    o = DAMFOracle(n, n, True, r=4, r_max=8, tau=1e-12).init_exact(s0, t0)
    for _ in range(10):
        k = 6
        o.update(rng.integers(0, n, k), rng.integers(0, n, k), rng.choice([-1, 1], k))
        assert np.allclose(o.X() @ o.Y().T, o.graph.dense(), atol=1e-10)


def test_exact_when_rank_stays_below_d():
    """rank(A_t) <= d at every step (block graph plus few edits) => X Y^T == A_t."""
    n, blocks, d = 60, 3, 10
    s0, t0 = block_graph(n, blocks, seed=2)
    o = DAMFOracle(n, d, True, r=4, r_max=8, tau=1e-10).init_exact(s0, t0)
    rng = np.random.default_rng(4)
    for _ in range(3):
        k = 2                      # each batch raises rank by at most 2
        o.update(rng.integers(0, n, k), rng.integers(0, n, k), np.ones(k, dtype=np.int8))
        A = o.graph.dense()
        assert np.linalg.matrix_rank(A) <= d
        assert np.allclose(o.X() @ o.Y().T, A, atol=1e-9)


def test_undirected_c1_like_runs_and_stays_orthonormal():
    src, dst = er_undirected(300, 2000, seed=1)
    o = DAMFOracle(300, 12, False, r=8, r_max=16, tau=1e-6).init_exact(src[:1800], dst[:1800])
    for b in range(20):
        lo = 1800 + 10 * b
        o.update(src[lo:lo + 10], dst[lo:lo + 10], np.ones(10, dtype=np.int8))
    assert np.abs(o.U.T @ o.U - np.eye(12)).max() < 1e-10
    assert np.abs(o.V.T @ o.V - np.eye(12)).max() < 1e-10
    assert np.all(np.diff(o.s) <= 1e-12)
