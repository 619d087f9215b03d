"""Flush of the lazy projections and re-orthogonalisation (oracle).

TEST INFRASTRUCTURE ONLY (see ``oracle/__init__.py``).

Sec. 4.1 (the lazy update equation) stores each factor as a base matrix times
a d x d projection, U = U_b P_U; a flush multiplies the projection in and
resets it to I.  Z_b and the push residual R are in U_b's coordinates
(PPR(U_b P) = PPR(U_b) P, PPR acting on the left), so they take the same
right factor.

Re-orthogonalisation replaces a factorisation U diag(s) V^T whose U, V have
drifted from orthonormal by the rank-d t-SVD of the same product (Sec. 4.1's
t-SVD embedding equation): QR of U and V, then the SVD of the small core
R_U diag(s) R_V^T.  The product is unchanged, so the truncation the update
performs next sees the same matrix.
"""
from __future__ import annotations

import numpy as np


def flush(Mb, P):
    """M_b P: the base matrix with its projection multiplied in (Sec. 4.1)."""
    return np.asarray(Mb, dtype=np.float64) @ np.asarray(P, dtype=np.float64)


def reorthogonalize(U, s, V):
    """(U', s', V') with orthonormal U', V', s' descending and U' diag(s') V'^T = U diag(s) V^T.

    U = Q_U R_U, V = Q_V R_V (Householder QR); R_U diag(s) R_V^T = Ut S Vt^T
    (dense SVD); U' = Q_U Ut, V' = Q_V Vt, s' = S.  Singular vectors of a
    zero singular value are whatever the SVD returns (orthonormal, otherwise
    arbitrary).
    """
    U = np.asarray(U, dtype=np.float64)
    V = np.asarray(V, dtype=np.float64)
    s = np.asarray(s, dtype=np.float64)
    QU, RU = np.linalg.qr(U, mode="reduced")
    QV, RV = np.linalg.qr(V, mode="reduced")
    core = RU @ np.diag(s) @ RV.T
    Ut, S, Vth = np.linalg.svd(core)
    return QU @ Ut, S, QV @ Vth.T
