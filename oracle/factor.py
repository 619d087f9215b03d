"""Initial factorisation (oracle).

Sec. 4.1: the embedding is the rank-d truncated SVD of A, X = U Sigma^(1/2),
Y = V Sigma^(1/2).  Appendix A (Algorithm 3) initialises DAMF from a t-SVD of
the initial graph, computed by the randomized method of Halko, Martinsson and
Tropp that the paper cites for an O(n d^2 + m d) cost.  The paper gives no
oversampling p, power-iteration count q or test-matrix distribution; this
oracle uses a Rademacher test matrix drawn from SplitMix64 (so the GPU can
draw the identical matrix) with a QR after every product with A or A^T.
"""
from __future__ import annotations

import numpy as np

_GOLDEN = np.uint64(0x9E3779B97F4A7C15)
_M1 = np.uint64(0xBF58476D1CE4E5B9)
_M2 = np.uint64(0x94D049BB133111EB)


def splitmix64(x):
    """SplitMix64 output for state increments ``x`` (Steele, Lea and Flood, OOPSLA 2014).

    Returns mix(x + golden) for each uint64 ``x``: the value SplitMix64 yields
    when its state before the call is ``x``.
    """
    with np.errstate(over="ignore"):
        z = np.asarray(x, dtype=np.uint64) + _GOLDEN
        z = (z ^ (z >> np.uint64(30))) * _M1
        z = (z ^ (z >> np.uint64(27))) * _M2
        return z ^ (z >> np.uint64(31))


def rademacher_sketch(n, l, seed):
    """Omega[i, j] = +1 or -1 from the top bit of splitmix64((seed << 40) ^ (i * l + j))."""
    i = np.arange(n, dtype=np.uint64)[:, None]
    j = np.arange(l, dtype=np.uint64)[None, :]
    ctr = (np.uint64(seed) << np.uint64(40)) ^ (i * np.uint64(l) + j)
    top = splitmix64(ctr) >> np.uint64(63)
    return 1.0 - 2.0 * top.astype(np.float64)


def tsvd_exact(A, d):
    """Rank-d t-SVD of a dense matrix, singular values descending (Sec. 4.1)."""
    U, s, Vt = np.linalg.svd(np.asarray(A, dtype=np.float64), full_matrices=False)
    if d > len(s):
        raise ValueError("d exceeds the matrix rank bound")
    return U[:, :d].copy(), s[:d].copy(), Vt[:d, :].T.copy()


def _qr_q(M):
    q, _ = np.linalg.qr(M, mode="reduced")
    return q


def tsvd_randomized(A, d, oversample, power_iters, seed, full_spectrum=False):
    """Randomized rank-d t-SVD of a (sparse or dense) A, in the order the GPU follows.

    Y = A Omega, Q = qr(Y); q times: Q = qr(A^T Q), Q = qr(A Q);
    B^T = A^T Q = Q2 R2; svd(R2^T) = Ut S Vt;  U = Q Ut[:, :d], V = Q2 Vt^T[:, :d].
    Then A ~ Q Q^T A = Q B = (Q Ut) S (Q2 Vt^T)^T.
    With full_spectrum, also returns all d + p singular values of R2^T (the
    gap after the d-th one decides how well the truncation is determined).
    """
    n = A.shape[0]
    l = d + oversample
    omega = rademacher_sketch(A.shape[1], l, seed)
    Q = _qr_q(A @ omega)
    for _ in range(power_iters):
        Q = _qr_q(A.T @ Q)
        Q = _qr_q(A @ Q)
    Bt = A.T @ Q
    Q2, R2 = np.linalg.qr(Bt, mode="reduced")
    Ut, s, Vth = np.linalg.svd(R2.T)
    U = Q @ Ut[:, :d]
    V = Q2 @ Vth.T[:, :d]
    assert U.shape == (n, d)
    if full_spectrum:
        return U, s[:d].copy(), V, s.copy()
    return U, s[:d].copy(), V
