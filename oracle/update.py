"""Space-projection update for edge changes (oracle).

Theorem 2 (Sec. 4.3) and Algorithm 1 (UpdateEmbeddingE) update a rank-d
factorisation A~ = U Sigma V^T by one rank-1 change B C^T in three steps:

  Step 1, Orthogonalization: W_B = U^T B, W_C = V^T C, and the norms R_B, R_C of
          the parts of B, C outside span(U), span(V) (Proposition 1);
  Step 2, Rediagonalization: the rank-d t-SVD E Theta H^T of the core
          [[Sigma, 0], [0, 0]] + [W_B; R_B][W_C; R_C]^T;
  Step 3, Space rotation: F, G and the sparse row corrections dX, dY, applied
          through the lazy base space (Sec. 4.1, the lazy update equation).

This oracle keeps U and V explicitly (no lazy projection) and works in the
U-form: the rotation of U is F_U = E[:d] - W_B T_B E[d:] and the row
correction is dU = B T_B E[d:].  The paper's X-form F equals
Sigma_1^(-1/2) F_U Sigma_2^(1/2) (compare the F and dX formulas of Theorem 2),
so both describe the same factorisation; the U-form stays defined when some
singular value is zero.  ``update_one_edge_xform`` follows Algorithm 1 as
printed (with the Sigma exponent of W_B read as -1/2) for cross-checking.

A batch generalises B, C from n x 1 to n x k, as in Zha and Simon's block
update, which the paper cites: the residual of B outside span(U) is factored
through the eigen-decomposition of its k x k Gram matrix (Proposition 1 is the
k = 1 case), and directions whose Gram eigenvalue is below ``tau`` are dropped.
A batch is cut into chunks of bounded rank before it is applied (``chunk``).
"""
from __future__ import annotations

import numpy as np


# --------------------------------------------------------------------------
# chunking of a batch's net change


def edit_units(net, directed):
    """Group the net change into edit units.

    Directed: every (u, v, delta) entry is a unit.  Undirected: the entries
    (u, v, delta) and (v, u, delta) with u < v form one unit; a self-loop is a
    unit of one entry.  Units come in ascending (min, max) order.
    """
    if directed:
        return [[e] for e in net]
    units = []
    for (u, v, dl) in net:
        if u < v:
            units.append([(u, v, dl), (v, u, dl)])
        elif u == v:
            units.append([(u, v, dl)])
    units.sort(key=lambda un: (un[0][0], un[0][1]))
    return units


def chunk(net, directed, r, r_max):
    """Greedy partition of the net change into chunks of bounded size.

    Units are taken in order; a unit joins the current chunk while the chunk's
    distinct rows S1 and columns S2 satisfy min(|S1|, |S2|) <= r and
    max(|S1|, |S2|) <= r_max, otherwise it starts a new chunk.  Each chunk is
    returned as (S1 sorted, S2 sorted, D) with D = dA[S1, S2] in {-1, 0, +1}.
    """
    chunks = []
    cur, S1, S2 = [], set(), set()
    for unit in edit_units(net, directed):
        rows = S1 | {e[0] for e in unit}
        cols = S2 | {e[1] for e in unit}
        if cur and not (min(len(rows), len(cols)) <= r and max(len(rows), len(cols)) <= r_max):
            chunks.append(_close(cur, S1, S2))
            cur, S1, S2 = [], set(), set()
            rows = {e[0] for e in unit}
            cols = {e[1] for e in unit}
        cur.extend(unit)
        S1, S2 = rows, cols
    if cur:
        chunks.append(_close(cur, S1, S2))
    return chunks


def _close(entries, S1, S2):
    s1 = sorted(S1)
    s2 = sorted(S2)
    ri = {u: i for i, u in enumerate(s1)}
    ci = {v: j for j, v in enumerate(s2)}
    D = np.zeros((len(s1), len(s2)), dtype=np.float64)
    for (u, v, dl) in entries:
        D[ri[u], ci[v]] += dl
    return np.array(s1, dtype=np.int64), np.array(s2, dtype=np.int64), D


# --------------------------------------------------------------------------
# one chunk


def residual_factor(G, BtB, tau):
    """Factor the residual Gram matrix G = B^T B - W_B^T W_B (Proposition 1, k columns).

    G = Z Lambda Z^T; keep eigenvalues above tau * max(1, max diag(B^T B)).
    Returns T = Z+ Lambda+^(-1/2) (k x rho) and R = Lambda+^(1/2) Z+^T (rho x k),
    so (I - U U^T) B T has orthonormal columns and (I - U U^T) B ~ ((I - U U^T) B T) R.
    For k = 1 this is R_B = sqrt(||B||^2 - ||W_B||^2).
    """
    G = 0.5 * (G + G.T)
    lam, Z = np.linalg.eigh(G)
    lam = np.maximum(lam, 0.0)
    thr = tau * max(1.0, float(np.max(np.diag(BtB))) if BtB.size else 1.0)
    keep = lam > thr
    lam_k = lam[keep]
    Zk = Z[:, keep]
    T = Zk / np.sqrt(lam_k)[None, :]
    R = (Zk * np.sqrt(lam_k)[None, :]).T
    return T, R


def chunk_update(U, s, V, S1, S2, D, tau):
    """Apply one chunk dA = I[:, S1] D I[:, S2]^T to U diag(s) V^T (explicit U-form).

    Returns (U', s', V', info); U and V are not modified in place.
    """
    n, d = U.shape
    s1, s2 = len(S1), len(S2)
    if s1 <= s2:
        # B = I[:, S1]           C = I[:, S2] D^T
        WB = U[S1, :].T.copy()
        WC = V[S2, :].T @ D.T
        BtB = np.eye(s1)
        CtC = D @ D.T
    else:
        # B = I[:, S1] D         C = I[:, S2]
        WB = U[S1, :].T @ D
        WC = V[S2, :].T.copy()
        BtB = D.T @ D
        CtC = np.eye(s2)
    # Step 1: orthogonalization
    TB, RB = residual_factor(BtB - WB.T @ WB, BtB, tau)
    TC, RC = residual_factor(CtC - WC.T @ WC, CtC, tau)
    rb, rc = RB.shape[0], RC.shape[0]
    # Step 2: rediagonalization of the core
    K = np.zeros((d + rb, d + rc))
    K[:d, :d] = np.diag(s)
    K += np.vstack([WB, RB]) @ np.vstack([WC, RC]).T
    E, th, Ht = np.linalg.svd(K)
    H = Ht.T
    Etop, Ebot = E[:d, :d], E[d:, :d]
    Htop, Hbot = H[:d, :d], H[d:, :d]
    # Step 3: space rotation and row corrections
    YB = TB @ Ebot            # k x d
    YC = TC @ Hbot
    FU = Etop - WB @ YB
    FV = Htop - WC @ YC
    if s1 <= s2:
        dU_rows = YB                  # B YB = I[:, S1] YB
        dV_rows = D.T @ YC            # C YC = I[:, S2] D^T YC
    else:
        dU_rows = D @ YB              # B YB = I[:, S1] D YB
        dV_rows = YC
    U2 = U @ FU
    U2[S1, :] += dU_rows
    V2 = V @ FV
    V2[S2, :] += dV_rows
    info = dict(rho_b=rb, rho_c=rc, core=K.shape, FU=FU, FV=FV,
                dU_rows=dU_rows, dV_rows=dV_rows, theta_all=th)
    return U2, th[:d].copy(), V2, info


def update_one_edge_xform(X, Y, s, b, c):
    """Algorithm 1, UpdateEmbeddingE, for one change b c^T in the paper's X-form.

    X = U Sigma^(1/2), Y = V Sigma^(1/2), P_X = P_Y = I (explicit embeddings);
    the Sigma exponent in the W_B and W_C lines is read as -1/2, the value
    Step 1 derives from U = X_b P_X Sigma^(-1/2).  Needs all s > 0 and a
    nonzero residual.  Returns (X2, Y2, s2).
    """
    d = X.shape[1]
    isq = 1.0 / np.sqrt(s)
    WB = (b @ X) * isq              # (B^T X P_X Sigma^(-1/2))^T
    WC = (c @ Y) * isq
    RB = np.sqrt(b @ b - WB @ WB)   # Proposition 1
    RC = np.sqrt(c @ c - WC @ WC)
    M = np.zeros((d + 1, d + 1))
    M[:d, :d] = np.diag(s)
    M += np.concatenate([WB, [RB]])[:, None] * np.concatenate([WC, [RC]])[None, :]
    E, s2, Ht = np.linalg.svd(M)
    H = Ht.T
    E, s2, H = E[:, :d], s2[:d], H[:, :d]
    sq2 = np.sqrt(s2)
    F = (isq[:, None] * (E[:d] - np.outer(WB, E[d:]) / RB)) * sq2[None, :]
    G = (isq[:, None] * (H[:d] - np.outer(WC, H[d:]) / RC)) * sq2[None, :]
    dX = np.outer(b, E[d:] * sq2) / RB
    dY = np.outer(c, H[d:] * sq2) / RC
    return X @ F + dX, Y @ G + dY, s2
