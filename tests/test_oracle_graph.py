"""Pins for the oracle's graph semantics against dense brute force."""
import numpy as np
import pytest

from oracle.graph import EdgeSet
from oracle.update import chunk, edit_units


def _brute(n, directed, init, ops):
    A = np.zeros((n, n), dtype=np.int64)
    for u, v in zip(*init):
        A[u, v] = 1
        if not directed:
            A[v, u] = 1
    A0 = A.copy()
    for u, v, o in zip(*ops):
        val = 1 if o == 1 else 0
        A[u, v] = val
        if not directed:
            A[v, u] = val
    diff = A - A0
    net = [(int(u), int(v), int(diff[u, v])) for u, v in zip(*np.nonzero(diff))]
    return A, sorted(net)


@pytest.mark.parametrize("directed", [True, False])
@pytest.mark.parametrize("seed", range(6))
def test_apply_matches_dense_bruteforce(directed, seed):
    rng = np.random.default_rng(seed)
    n = 9
    m0 = 20
    init = (rng.integers(0, n, m0), rng.integers(0, n, m0))   # duplicates and loops allowed
    k = 40
    ops = (rng.integers(0, n, k), rng.integers(0, n, k), rng.choice([-1, 1], k))
    g = EdgeSet(n, directed, *init)
    net = g.apply(*ops)
    A, net_ref = _brute(n, directed, init, ops)
    assert net == net_ref
    assert np.array_equal(g.dense(), A.astype(np.float64))
    indptr, idx = g.csr()
    assert indptr.dtype == np.int64 and idx.dtype == np.int32
    for u in range(n):
        row = idx[indptr[u]:indptr[u + 1]]
        assert np.array_equal(row, np.nonzero(A[u])[0])
    indptr_t, idx_t = g.csr(transpose=True)
    for v in range(n):
        assert np.array_equal(idx_t[indptr_t[v]:indptr_t[v + 1]], np.nonzero(A[:, v])[0])
    assert np.array_equal(g.out_degree(), A.sum(axis=1))


def test_noop_edits():
    g = EdgeSet(4, True, [0], [1])
    assert g.apply([0, 2], [1, 3], [1, -1]) == []        # insert present, delete absent
    assert g.apply([0, 0], [1, 1], [-1, 1]) == []        # delete then re-insert
    assert g.apply([2, 2], [3, 3], [1, -1]) == []        # insert then delete
    assert g.apply([3], [3], [1]) == [(3, 3, 1)]         # self-loop is a legal entry
    g2 = EdgeSet(4, False)
    assert g2.apply([2], [2], [1]) == [(2, 2, 1)]        # undirected loop stored once
    assert g2.apply([3], [1], [1]) == [(1, 3, 1), (3, 1, 1)]


@pytest.mark.parametrize("directed", [True, False])
@pytest.mark.parametrize("r,r_max", [(2, 4), (3, 3), (4, 8), (32, 64)])
def test_chunk_partition(directed, r, r_max):
    rng = np.random.default_rng(7)
    n = 40
    g = EdgeSet(n, directed)
    net = g.apply(rng.integers(0, n, 60), rng.integers(0, n, 60), np.ones(60, dtype=np.int8))
    units = edit_units(net, directed)
    chunks = chunk(net, directed, r, r_max)
    # the chunks cover the net change exactly, in order
    total = np.zeros((n, n))
    for S1, S2, D in chunks:
        assert list(S1) == sorted(set(S1)) and list(S2) == sorted(set(S2))
        assert min(len(S1), len(S2)) <= r and max(len(S1), len(S2)) <= r_max
        total[np.ix_(S1, S2)] += D
    ref = np.zeros((n, n))
    for u, v, dl in net:
        ref[u, v] += dl
    assert np.array_equal(total, ref)
    # greedy maximality: the first unit of each chunk would not have fit the previous one
    pos = 0
    for c, (S1, S2, D) in enumerate(chunks):
        cnt = int(np.count_nonzero(D))
        taken = 0
        start = pos
        while taken < cnt:
            taken += len(units[pos])
            pos += 1
        assert taken == cnt
        if c > 0:
            prevS1, prevS2, _ = chunks[c - 1]
            rows = set(prevS1) | {e[0] for e in units[start]}
            cols = set(prevS2) | {e[1] for e in units[start]}
            assert not (min(len(rows), len(cols)) <= r and max(len(rows), len(cols)) <= r_max)
    assert pos == len(units)
