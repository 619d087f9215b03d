"""Personalized PageRank enhancement (oracle).

Sec. 4.4 defines the enhancement of a graph signal X (n x d) as

    PPR(X) = sum_{i >= 0} alpha (1 - alpha)^i (D^-1 A)^i X,

with D the diagonal out-degree matrix, truncated to an error tolerance eps.
A node without out-edges has a zero row in D^-1 A (reading: the paper does not
say).  ``ppr_series`` evaluates the series by its partial sums until the tail
is below 1e-15 relative; it is the definition the tests compare against.

The paper delegates the dynamic maintenance to InstantGNN, which is not
reproduced here.  ``PushState`` is the residual-push scheme that the library
uses, derived from the definition alone: with Pi = alpha (I - (1-alpha) P)^-1
(P = D^-1 A) it keeps the invariant  PPR(X) = Z + Pi R.  Pushing node v
moves alpha R[v] into Z[v] and (1 - alpha) A[u, v] / deg(u) R[v] into R[u] for
every in-neighbour u, which keeps the invariant because
Pi = alpha I + (1 - alpha) Pi P.  Since Pi >= 0 with row sums <= 1, stopping
once max |R| <= eps gives |Z - PPR(X)| <= eps entrywise.
"""
from __future__ import annotations

import math
from collections import deque

import numpy as np
import scipy.sparse as sp


def transition(A):
    """P = D^-1 A as scipy CSR (zero rows for nodes without out-edges)."""
    A = sp.csr_matrix(A, dtype=np.float64)
    deg = np.asarray(A.sum(axis=1)).ravel()
    inv = np.zeros_like(deg)
    nz = deg > 0
    inv[nz] = 1.0 / deg[nz]
    return sp.diags(inv) @ A


def series_terms(alpha, rel=1e-15):
    """Number of terms after which (1 - alpha)^T <= rel."""
    if alpha >= 1.0:
        return 1
    return int(math.ceil(math.log(rel) / math.log(1.0 - alpha)))


def ppr_series(A, X, alpha):
    """PPR(X) by partial sums of the series: Z_T = sum_{i < T} alpha (1-alpha)^i P^i X."""
    P = transition(A)
    X = np.asarray(X, dtype=np.float64)
    term = alpha * X.copy()
    Z = term.copy()
    for _ in range(series_terms(alpha) - 1):
        term = (1.0 - alpha) * (P @ term)
        Z += term
    return Z


def ppr_dense_inverse(A, X, alpha):
    """PPR(X) = alpha (I - (1 - alpha) P)^-1 X by a dense solve (tiny graphs)."""
    P = transition(A).toarray()
    n = P.shape[0]
    return alpha * np.linalg.solve(np.eye(n) - (1.0 - alpha) * P, np.asarray(X, dtype=np.float64))


class PushState:
    """Residual-push maintenance of Z ~ PPR(X) under signal and structure changes."""

    def __init__(self, A, X, alpha, eps):
        self.alpha = float(alpha)
        self.eps = float(eps)
        self.A = sp.csr_matrix(A, dtype=np.float64)
        self.X = np.asarray(X, dtype=np.float64).copy()
        self.Z = np.zeros_like(self.X)
        self.R = self.X.copy()
        self.pushes = 0
        self.push_all()

    def _deg(self):
        return np.asarray(self.A.sum(axis=1)).ravel()

    def push_all(self):
        """Push nodes (FIFO) until max |R| <= eps."""
        a = self.alpha
        AT = self.A.T.tocsr()
        deg = self._deg()
        q = deque(np.nonzero(np.abs(self.R).max(axis=1) > self.eps)[0].tolist())
        queued = set(q)
        while q:
            v = q.popleft()
            queued.discard(v)
            rv = self.R[v].copy()
            if np.abs(rv).max() <= self.eps:
                continue
            self.R[v] = 0.0
            self.Z[v] += a * rv
            self.pushes += 1
            for u in AT.indices[AT.indptr[v]:AT.indptr[v + 1]].tolist():
                self.R[u] += (1.0 - a) * rv / deg[u]
                if u not in queued and np.abs(self.R[u]).max() > self.eps:
                    q.append(u)
                    queued.add(u)

    def change_signal(self, rows, dX):
        """X[rows] += dX: PPR is linear, so R[rows] += dX restores the invariant."""
        rows = np.asarray(rows)
        np.add.at(self.X, rows, dX)
        np.add.at(self.R, rows, dX)

    def change_structure(self, A_new):
        """Replace A, adjusting R on rows whose out-neighbourhood changed.

        From the invariant, R = X - (Z - (1 - alpha) P Z) / alpha for the old P;
        keeping Z and X, the new residual is R + ((1 - alpha) / alpha) (P' Z - P Z).
        """
        a = self.alpha
        A_new = sp.csr_matrix(A_new, dtype=np.float64)
        P_old = transition(self.A)
        P_new = transition(A_new)
        diff = (P_new - P_old).tocsr()
        rows = np.nonzero(np.diff(diff.indptr))[0]
        if len(rows):
            delta = (diff[rows] @ self.Z) * ((1.0 - a) / a)
            self.R[rows] += delta
        self.A = A_new
