"""Pins for the oracle's flush and re-orthogonalisation (Sec. 4.1)."""
import numpy as np
import scipy.sparse as sp

from oracle.ppr import ppr_series
from oracle.reorth import flush, reorthogonalize


def _drifted(n, d, seed, drift=1e-3):
    rng = np.random.default_rng(seed)
    U, _ = np.linalg.qr(rng.standard_normal((n, d)))
    V, _ = np.linalg.qr(rng.standard_normal((n, d)))
    U = U @ (np.eye(d) + drift * rng.standard_normal((d, d))) + drift * rng.standard_normal((n, d)) / np.sqrt(n)
    V = V @ (np.eye(d) + drift * rng.standard_normal((d, d)))
    s = np.sort(rng.uniform(1.0, 20.0, d))[::-1].copy()
    return U, s, V


def test_reorth_is_the_tsvd_of_the_product():
    n, d = 40, 6
    U, s, V = _drifted(n, d, 0)
    M = U @ np.diag(s) @ V.T
    U2, s2, V2 = reorthogonalize(U, s, V)
    Ud, sd, Vdt = np.linalg.svd(M)  # dense SVD of the n x n product
    assert np.allclose(s2, sd[:d], rtol=0, atol=1e-12 * sd[0])
    assert np.allclose(sd[d:], 0.0, atol=1e-12 * sd[0])
    assert np.allclose(U2 @ np.diag(s2) @ V2.T, M, atol=1e-12 * sd[0])
    assert np.allclose(U2.T @ U2, np.eye(d), atol=1e-13)
    assert np.allclose(V2.T @ V2, np.eye(d), atol=1e-13)
    # left and right singular subspaces (distinct singular values: each vector up to sign)
    for j in range(d):
        assert abs(abs(U2[:, j] @ Ud[:, j]) - 1.0) < 1e-10
        assert abs(abs(V2[:, j] @ Vdt[j]) - 1.0) < 1e-10


def test_reorth_of_orthonormal_factors_is_identity_up_to_sign():
    rng = np.random.default_rng(1)
    n, d = 50, 5
    U, _ = np.linalg.qr(rng.standard_normal((n, d)))
    V, _ = np.linalg.qr(rng.standard_normal((n, d)))
    s = np.array([9.0, 7.0, 4.0, 2.0, 0.5])
    U2, s2, V2 = reorthogonalize(U, s, V)
    assert np.allclose(s2, s, atol=1e-13)
    sign = np.sign(np.sum(U2 * U, axis=0))
    assert np.allclose(U2 * sign, U, atol=1e-12)
    assert np.allclose(V2 * sign, V, atol=1e-12)


def test_reorth_rank_deficient_keeps_product_and_orthonormality():
    n, d = 30, 6
    U, s, V = _drifted(n, d, 2)
    s[4:] = 0.0
    U2, s2, V2 = reorthogonalize(U, s, V)
    assert np.allclose(U2 @ np.diag(s2) @ V2.T, U @ np.diag(s) @ V.T, atol=1e-12 * s[0])
    assert np.allclose(s2[4:], 0.0, atol=1e-12 * s[0])
    assert np.allclose(U2.T @ U2, np.eye(d), atol=1e-12)
    assert np.allclose(V2.T @ V2, np.eye(d), atol=1e-12)


def test_flush_matches_the_lazy_form_and_ppr_linearity():
    """Flushing P into U_b keeps U = U_b P; PPR(U_b P) = PPR(U_b) P, so Z_b and R take P too."""
    rng = np.random.default_rng(3)
    n, d, alpha = 25, 4, 0.2
    A = sp.random(n, n, density=0.2, random_state=4, data_rvs=lambda k: np.ones(k)).tocsr()
    Ub = rng.standard_normal((n, d))
    P = np.eye(d) + 0.3 * rng.standard_normal((d, d))
    U = flush(Ub, P)
    assert np.allclose(U @ np.linalg.inv(P), Ub, atol=1e-12)
    assert np.allclose(ppr_series(A, U, alpha), ppr_series(A, Ub, alpha) @ P, atol=1e-12)
