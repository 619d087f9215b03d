"""Pins for the oracle's PPR (definition, closed forms, push invariant)."""
import numpy as np
import pytest
import scipy.sparse as sp

from oracle.model import DAMFOracle
from oracle.ppr import PushState, ppr_dense_inverse, ppr_series


def _csr(n, src, dst):
    return sp.csr_matrix((np.ones(len(src)), (src, dst)), shape=(n, n))


def test_series_matches_dense_inverse():
    rng = np.random.default_rng(0)
    n = 25
    A = _csr(n, rng.integers(0, n, 70), rng.integers(0, n, 70))
    A.data[:] = 1.0
    X = rng.standard_normal((n, 4))
    for alpha in (0.15, 0.3, 0.9):
        assert np.allclose(ppr_series(A, X, alpha), ppr_dense_inverse(A, X, alpha), atol=1e-12)


def test_row_sums_one_without_dangling():
    n = 30
    src = np.arange(n)
    dst = (np.arange(n) * 7 + 3) % n
    A = _csr(n, np.concatenate([src, src]), np.concatenate([dst, (dst + 1) % n]))
    Z = ppr_series(A, np.ones((n, 1)), 0.15)
    assert np.allclose(Z, 1.0, atol=1e-13)


@pytest.mark.parametrize("L", [3, 5, 8])
def test_directed_cycle_closed_form(L):
    """On a directed L-cycle, (I - (1-a)P)^-1 = sum_{i<L} (1-a)^i P^i / (1 - (1-a)^L)."""
    a = 0.15
    A = _csr(L, np.arange(L), (np.arange(L) + 1) % L)
    X = np.eye(L)
    Z = ppr_series(A, X, a)
    ref = np.zeros((L, L))
    for u in range(L):
        for i in range(L):
            ref[u, (u + i) % L] += a * (1 - a) ** i
    ref /= 1 - (1 - a) ** L
    assert np.allclose(Z, ref, atol=1e-13)


def test_complete_graph_closed_form():
    """K_n without loops: P = (J - I)/(n-1); on x orthogonal to 1, Pi x = a/(1 + (1-a)/(n-1)) x."""
    n, a = 12, 0.3
    s, t = np.nonzero(1 - np.eye(n))
    A = _csr(n, s, t)
    rng = np.random.default_rng(2)
    x = rng.standard_normal((n, 1))
    x -= x.mean()
    Z = ppr_series(A, x, a)
    assert np.allclose(Z, a / (1 + (1 - a) / (n - 1)) * x, atol=1e-13)


def test_dangling_rows_are_zero_in_p():
    n, a = 4, 0.2
    A = _csr(n, [0, 1], [1, 2])       # nodes 2, 3 have no out-edges
    X = np.eye(n)
    Z = ppr_series(A, X, a)
    assert np.allclose(Z[2], a * X[2]) and np.allclose(Z[3], a * X[3])
    assert np.isclose(Z[1, 2], a * (1 - a))
    assert np.isclose(Z[0, 2], a * (1 - a) ** 2)


def test_alpha_one_is_identity():
    """The ablation alpha = 1 gives no enhancement: PPR(X) = X."""
    rng = np.random.default_rng(3)
    n = 20
    A = _csr(n, rng.integers(0, n, 60), rng.integers(0, n, 60))
    X = rng.standard_normal((n, 3))
    assert np.allclose(ppr_series(A, X, 1.0), X)
    o = DAMFOracle(n, 3, True, alpha=1.0).init_exact(rng.integers(0, n, 60), rng.integers(0, n, 60))
    assert np.allclose(o.Z(), o.X())


def test_push_bound_and_dynamic_changes():
    """Push keeps |Z - PPR(X)| <= eps through structure and signal changes."""
    rng = np.random.default_rng(4)
    n, d, a, eps = 60, 3, 0.15, 1e-6
    src, dst = rng.integers(0, n, 240), rng.integers(0, n, 240)
    A = _csr(n, src, dst)
    A.data[:] = 1.0
    X = rng.standard_normal((n, d))
    st = PushState(A, X, a, eps)
    assert np.abs(st.R).max() <= eps
    assert np.abs(st.Z - ppr_series(A, X, a)).max() <= eps
    for _ in range(5):
        A2 = A.tolil()
        for _ in range(6):
            u, v = rng.integers(0, n, 2)
            A2[u, v] = 1.0 - A2[u, v]
        A2 = A2.tocsr()
        A2.eliminate_zeros()
        st.change_structure(A2)
        rows = rng.choice(n, 4, replace=False)
        st.change_signal(rows, rng.standard_normal((4, d)))
        # the invariant holds exactly before pushing
        Pi_R = ppr_series(A2, st.R, a)
        assert np.allclose(st.Z + Pi_R, ppr_series(A2, st.X, a), atol=1e-11)
        st.push_all()
        assert np.abs(st.R).max() <= eps
        assert np.abs(st.Z - ppr_series(A2, st.X, a)).max() <= eps
        A = A2
