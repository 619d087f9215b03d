"""Space-projection update for node change (oracle; test infrastructure only).

Sec. 4.2 adds a node as one new column and one new row of the adjacency
matrix, in two steps (the node-change equation): A' = [A, B1] (the new
node's in-edges from the existing nodes), then A_t = [A'^T, B2]^T (its
out-edges, over all columns including its own).  Theorem 1 updates a rank-d
factorisation A~ = U Sigma V^T by the column step:

  W_B = U^T B, R_B = ||(I - U U^T) B||, Q_B = (I - U U^T) B / R_B,
  M = [[Sigma, W_B], [0, R_B]]  ((d+1) x (d+1)),  E Theta H^T = t-SVD(M, d),
  U' = [U, Q_B] E = U (E[:d] - R_B^-1 W_B E[d:]) + R_B^-1 B E[d:],
  V' = [[V, 0], [0, 1]] H  (the new column's row of V' is H[d:]),
  Sigma' = Theta.

The row step is the same with the roles of U and V exchanged (Algorithm 2,
node branch, calls UpdateEmbeddingN with X and Y swapped).

Storage reading: the library keeps a fixed node range, so a node that joins
is a slot whose row and column of A are empty.  Its rows of U and V are then
zero (to rounding) and [V; 0] is V itself; ``add_column`` takes the slot's
index ``new`` and assumes V[new] = 0, which the caller checks.

Like ``update.py`` this works in the U-form (X = U Sigma^(1/2) applied at
query).  ``update_node_xform`` follows Algorithm 1's UpdateEmbeddingN as
printed (W_B's Sigma exponent read as -1/2) for cross-checking.

Reading for long lists: the library's chunk kernels take at most r_max rows
of B per step.  A column (row) with more than r_max entries is applied as
consecutive rank-1 pieces of at most r_max entries: the first is Theorem 1's
column (row) step; each later piece finds the column (row) already present and
is Theorem 2's edge update with C = e_new (B = e_new).  With at most r_max
entries per side the event is exactly Theorem 1's two steps.
"""
from __future__ import annotations

import numpy as np

from . import update


def _residual(U, b, tau):
    """W_B = U^T b and the residual norm R_B (Theorem 1, the normalisation of
    (I - U U^T) B); R_B is taken as 0 when R_B^2 <= tau * max(1, ||b||^2)."""
    wb = U.T @ b
    r2 = float(b @ b - wb @ wb)
    thr = tau * max(1.0, float(b @ b))
    return wb, (np.sqrt(r2) if r2 > thr else 0.0)


def add_column(U, s, V, b, new, tau=1e-12):
    """Theorem 1's column step: [A~, b] with b (n-vector, b[new] = 0) as column `new`.

    Returns (U', s', V', info).  With R_B = 0 (b inside span(U)) the residual
    direction is dropped and M is the d x (d+1) block [Sigma, W_B].
    """
    n, d = U.shape
    b = np.asarray(b, dtype=np.float64)
    wb, rb = _residual(U, b, tau)
    rows = d + (1 if rb > 0 else 0)
    M = np.zeros((rows, d + 1))
    M[:d, :d] = np.diag(s)
    M[:d, d] = wb
    if rb > 0:
        M[d, d] = rb
    E, th, Ht = np.linalg.svd(M)
    H = Ht.T
    Etop = E[:d, :d]
    Ebot = E[d:, :d]           # 1 x d, or 0 x d when R_B = 0
    Htop, Hbot = H[:d, :d], H[d:, :d]
    if rb > 0:
        F = Etop - np.outer(wb, Ebot[0]) / rb
        U2 = U @ F + np.outer(b, Ebot[0]) / rb
    else:
        U2 = U @ Etop
    V2 = V @ Htop
    V2[new, :] += Hbot[0]
    return U2, th[:d].copy(), V2, dict(rb=rb, core=M.shape, theta_all=th)


def add_row(U, s, V, c, new, tau=1e-12):
    """The row step: [A~; c^T] with c (n-vector over all columns) as row `new`
    (U[new] = 0): the column step with U and V exchanged."""
    V2, s2, U2, info = add_column(V, s, U, c, new, tau)
    return U2, s2, V2, info


def _indicator(n, idx):
    v = np.zeros(n)
    v[np.asarray(idx, dtype=np.int64)] = 1.0
    return v


def _pieces(idx, r_max):
    idx = np.asarray(sorted(set(int(i) for i in idx)), dtype=np.int64)
    if r_max is None or len(idx) <= r_max:
        return [idx] if len(idx) else []
    return [idx[i:i + r_max] for i in range(0, len(idx), r_max)]


def node_event(U, s, V, new, in_nbrs, out_nbrs, tau=1e-12, r_max=None):
    """Node `new` (no edges yet) joins with in-edges (v, new), v in in_nbrs, and
    out-edges (new, w), w in out_nbrs: the column step (in-edges without a
    self-loop), then the row step (out-edges, with the self-loop (new, new)
    when either list names `new`).  Returns (U', s', V', info).
    """
    n = U.shape[0]
    ins = sorted(set(int(v) for v in in_nbrs) - {new})
    outs = set(int(w) for w in out_nbrs)
    if new in set(int(v) for v in in_nbrs):
        outs.add(new)
    outs = sorted(outs)
    steps = []
    # Theorem 1 needs the new column's (row's) entries of V (U) to be zero; a
    # slot whose old basis rows are not (a kept zero singular value may put
    # weight anywhere) takes Theorem 2 with C = e_new (B = e_new) instead
    for j, piece in enumerate(_pieces(ins, r_max)):
        if j == 0 and np.abs(V[new]).max() <= 1e-12:
            U, s, V, inf = add_column(U, s, V, _indicator(n, piece), new, tau)
        else:
            D = np.ones((len(piece), 1))
            U, s, V, inf = update.chunk_update(U, s, V, piece, np.array([new]), D, tau)
        steps.append(("column", len(piece)))
    for j, piece in enumerate(_pieces(outs, r_max)):
        if j == 0 and np.abs(U[new]).max() <= 1e-12:
            U, s, V, inf = add_row(U, s, V, _indicator(n, piece), new, tau)
        else:
            D = np.ones((1, len(piece)))
            U, s, V, inf = update.chunk_update(U, s, V, np.array([new]), piece, D, tau)
        steps.append(("row", len(piece)))
    return U, s, V, dict(steps=steps, in_edges=ins, out_edges=outs)


def update_node_xform(X, Y, s, b, new):
    """Algorithm 1, UpdateEmbeddingN, as printed, for one column b in the X-form
    (P_X = P_Y = I, all s > 0, nonzero residual; W_B with Sigma^(-1/2)).

    Returns (X2, Y2, s2) with the new column's row of Y2 at `new`.
    """
    d = X.shape[1]
    isq = 1.0 / np.sqrt(s)
    WB = (b @ X) * isq
    RB = np.sqrt(b @ b - WB @ WB)
    M = np.zeros((d + 1, d + 1))
    M[:d, :d] = np.diag(s)
    M[:d, d] = WB
    M[d, d] = RB
    E, s2, Ht = np.linalg.svd(M)
    H = Ht.T
    E, s2, H = E[:, :d], s2[:d], H[:, :d]
    sq2 = np.sqrt(s2)
    F = (isq[:, None] * (E[:d] - np.outer(WB, E[d:]) / RB)) * sq2[None, :]
    G = (isq[:, None] * H[:d]) * sq2[None, :]
    dX = np.outer(b, E[d:] * sq2) / RB
    dY = np.zeros_like(Y)
    dY[new] = H[d:][0] * sq2
    return X @ F + dX, Y @ G + dY, s2
