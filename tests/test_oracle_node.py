"""Pins of the node-change oracle (Theorem 1, Sec. 4.2) against dense linear algebra.

Theorem 1 states that the column step returns a rank-d t-SVD of [A~, B] where
A~ = U Sigma V^T is the current factorisation: each pin compares with
numpy's dense SVD of that matrix, truncated to d.
"""
import numpy as np
import pytest

from oracle import node, update


def _tsvd(A, d):
    U, s, Vt = np.linalg.svd(A)
    return U[:, :d], s[:d], Vt[:d].T


def _factors(n, d, seed, zero_rows=()):
    """Orthonormal U, V (rows in zero_rows exactly 0) and decreasing s."""
    rng = np.random.default_rng(seed)
    def basis():
        M = rng.standard_normal((n, d))
        M[list(zero_rows)] = 0.0
        return np.linalg.qr(M)[0]
    s = np.sort(rng.uniform(1.0, 6.0, d))[::-1].copy()
    return basis(), s, basis()


def _lowrank(U, s, V):
    return (U * s) @ V.T


def _close(U2, s2, V2, ref, d, tol=1e-10):
    Ur, sr, Vr = _tsvd(ref, d)
    assert np.abs(s2 - sr).max() <= tol * sr[0]
    assert np.abs(_lowrank(U2, s2, V2) - _lowrank(Ur, sr, Vr)).max() <= tol * sr[0]
    assert np.abs(U2.T @ U2 - np.eye(d)).max() <= 1e-10
    assert np.abs(V2.T @ V2 - np.eye(d)).max() <= 1e-10


def test_column_step_is_tsvd_of_extended_matrix():
    n, d, new = 30, 5, 17
    U, s, V = _factors(n, d, 1, zero_rows=[new])
    b = np.zeros(n)
    b[[2, 5, 9, 22, 29]] = 1.0
    U2, s2, V2, info = node.add_column(U, s, V, b, new)
    A = _lowrank(U, s, V)
    A[:, new] += b
    assert info["rb"] > 0
    _close(U2, s2, V2, A, d)


def test_row_step_is_tsvd_of_extended_matrix():
    n, d, new = 30, 5, 4
    U, s, V = _factors(n, d, 2, zero_rows=[new])
    c = np.zeros(n)
    c[[0, 4, 11, 12]] = 1.0  # includes the self-loop column
    U2, s2, V2, _ = node.add_row(U, s, V, c, new)
    A = _lowrank(U, s, V)
    A[new, :] += c
    _close(U2, s2, V2, A, d)


def test_node_event_is_column_then_row():
    n, d, new = 40, 6, 33
    U, s, V = _factors(n, d, 3, zero_rows=[new])
    ins, outs = [1, 7, 8, 30, 33], [2, 3, 19]
    U2, s2, V2, info = node.node_event(U, s, V, new, ins, outs)
    A = _lowrank(U, s, V)
    A[[1, 7, 8, 30], new] += 1.0               # column step, self-loop excluded
    Uc, sc, Vc = _tsvd(A, d)
    A1 = _lowrank(Uc, sc, Vc)
    A1[new, [2, 3, 19, 33]] += 1.0             # row step, with the self-loop
    _close(U2, s2, V2, A1, d)
    assert info["steps"] == [("column", 4), ("row", 4)]


def test_column_step_equals_edge_update_with_unit_column():
    # Theorem 1 is Theorem 2 with C = e_new when the new column of V is zero
    n, d, new = 25, 4, 3
    U, s, V = _factors(n, d, 4, zero_rows=[new])
    nb = np.array([0, 6, 13, 20])
    b = np.zeros(n)
    b[nb] = 1.0
    U2, s2, V2, _ = node.add_column(U, s, V, b, new)
    U3, s3, V3, _ = update.chunk_update(U, s, V, nb, np.array([new]), np.ones((4, 1)), 1e-12)
    assert np.abs(s2 - s3).max() <= 1e-12 * s2[0]
    assert np.abs(_lowrank(U2, s2, V2) - _lowrank(U3, s3, V3)).max() <= 1e-11


def test_paper_xform_procedure_agrees():
    n, d, new = 25, 4, 9
    U, s, V = _factors(n, d, 5, zero_rows=[new])
    b = np.zeros(n)
    b[[1, 2, 24]] = 1.0
    X, Y = U * np.sqrt(s), V * np.sqrt(s)
    X2, Y2, s2 = node.update_node_xform(X, Y, s, b, new)
    U3, s3, V3, _ = node.add_column(U, s, V, b, new)
    assert np.abs(s2 - s3).max() <= 1e-12 * s2[0]
    assert np.abs(X2 @ Y2.T - _lowrank(U3, s3, V3)).max() <= 1e-11


def test_column_inside_span_drops_residual():
    n, d, new = 20, 4, 0
    U, s, V = _factors(n, d, 6, zero_rows=[new])
    b = U @ np.array([2.0, -1.0, 0.5, 0.0])  # b[new] = 0 since U[new] = 0
    U2, s2, V2, info = node.add_column(U, s, V, b, new)
    assert info["rb"] == 0.0 and info["core"] == (d, d + 1)
    A = _lowrank(U, s, V)
    A[:, new] += b
    _close(U2, s2, V2, A, d)


def test_long_column_in_pieces_is_sequential_truncation():
    n, d, new, r_max = 40, 5, 39, 3
    U, s, V = _factors(n, d, 7, zero_rows=[new])
    ins = [0, 4, 9, 15, 16, 22, 30]
    U2, s2, V2, info = node.node_event(U, s, V, new, ins, [], r_max=r_max)
    assert info["steps"] == [("column", 3), ("column", 3), ("column", 1)]
    A = _lowrank(U, s, V)
    for piece in ([0, 4, 9], [15, 16, 22], [30]):
        A[piece, new] += 1.0
        Ut, st, Vt = _tsvd(A, d)
        A = _lowrank(Ut, st, Vt)
    assert np.abs(_lowrank(U2, s2, V2) - A).max() <= 1e-10 * s2[0]


def test_exact_when_rank_stays_within_d():
    # a graph of rank 3 represented exactly at d = 6; the new node's column
    # repeats an existing column and its row repeats an existing row, so the
    # rank grows by at most 2 and X Y^T reproduces A exactly
    n, d, new = 24, 6, 20
    A = np.zeros((n, n))
    A[0:5, 10:15] = 1.0
    A[5:9, 15:18] = 1.0
    A[9:11, 0:3] = 1.0
    U, s, V = _tsvd(A, d)
    U[np.abs(U) < 1e-15] = 0.0
    ins = [5, 6, 7, 8]          # the column pattern of 15..17
    outs = [0, 1, 2]            # the row pattern of 9, 10
    U2, s2, V2, _ = node.node_event(U, s, V, new, ins, outs)
    A[ins, new] = 1.0
    A[new, outs] = 1.0
    assert np.abs(_lowrank(U2, s2, V2) - A).max() <= 1e-10


def test_model_add_node_edits_graph_and_factors():
    from oracle.model import DAMFOracle
    rng = np.random.default_rng(8)
    n, d = 30, 6
    s0 = rng.integers(0, 25, 120)
    t0 = rng.integers(0, 25, 120)
    for directed in (True, False):
        orc = DAMFOracle(n, d, directed, alpha=1.0, r=4, r_max=4, tau=1e-12).init_exact(s0, t0)
        A = orc.graph.dense()
        U, s, V = orc.U.copy(), orc.s.copy(), orc.V.copy()
        info = orc.add_node(27, [1, 2, 3, 4, 5, 27], [6, 7] if directed else ())
        A2 = orc.graph.dense()
        expect = A.copy()
        expect[[1, 2, 3, 4, 5], 27] = 1.0
        expect[27, 27] = 1.0
        if directed:
            expect[27, [6, 7]] = 1.0
        else:
            expect[27, [1, 2, 3, 4, 5]] = 1.0
        assert np.array_equal(A2, expect)
        # the same steps by hand: column of 5 in pieces (4, 1), then the row
        from oracle import node as nd
        U2, s2, V2, _ = nd.node_event(U, s, V, 27, [1, 2, 3, 4, 5, 27],
                                      [6, 7] if directed else [1, 2, 3, 4, 5], 1e-12, 4)
        assert np.abs(_lowrank(U2, s2, V2) - _lowrank(orc.U, orc.s, orc.V)).max() <= 1e-12
        assert info["steps"][0] == ("column", 4)
        with pytest.raises(ValueError):
            orc.add_node(27, [0], [])
