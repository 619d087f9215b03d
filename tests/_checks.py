"""Comparison helpers for GPU-vs-oracle parity (plain numpy, float64)."""
import numpy as np


def product_rel_err(X1, Y1, X2, Y2):
    """||X1 Y1^T - X2 Y2^T||_F / ||X2 Y2^T||_F through d x d Gram traces (any n)."""
    X1, Y1, X2, Y2 = (np.asarray(a, dtype=np.float64) for a in (X1, Y1, X2, Y2))
    a = np.trace((X1.T @ X1) @ (Y1.T @ Y1))
    b = np.trace((X1.T @ X2) @ (Y2.T @ Y1))
    c = np.trace((X2.T @ X2) @ (Y2.T @ Y2))
    return float(np.sqrt(max(a - 2 * b + c, 0.0)) / np.sqrt(c))


def orth_err(M):
    """max |M^T M - I| for the column-orthonormal factor M."""
    M = np.asarray(M, dtype=np.float64)
    return float(np.abs(M.T @ M - np.eye(M.shape[1])).max())


def unit_factor(Xq, s):
    """U = X Sigma^(-1/2) from a queried embedding (columns with s > 0)."""
    return np.asarray(Xq, dtype=np.float64) / np.sqrt(np.maximum(s, 1e-300))[None, :]


def subspace_sines(M_gpu, U_orc):
    """sin of the largest principal angle between span(M_gpu[:, :j]) and
    span(U_orc[:, :j]) for j = 1..d.

    U_orc has orthonormal columns (FP64 oracle).  M_gpu is first
    orthonormalised in FP64 (QR keeps the span of every leading block), so the
    FP32 non-orthogonality of the GPU basis does not enter.  With Q = qr(M_gpu),
    sin_j = ||Q_j - U_j U_j^T Q_j||_2, evaluated for all j from C = U^T Q and
    W = Q - U C:  Q_j^T (I - U_j U_j^T) Q_j = W_j^T W_j + C[j:, :j]^T C[j:, :j].
    """
    Q, _ = np.linalg.qr(np.asarray(M_gpu, dtype=np.float64))
    U = np.asarray(U_orc, dtype=np.float64)
    d = Q.shape[1]
    C = U.T @ Q  # d x d
    W = Q - U @ C  # part of Q outside span(U[:, :d]), n x d
    G = W.T @ W
    out = np.empty(d)
    for j in range(1, d + 1):
        Cj = C[j:, :j]
        H = G[:j, :j] + Cj.T @ Cj
        out[j - 1] = np.sqrt(max(np.linalg.eigvalsh(H)[-1], 0.0))
    return out


def relative_gaps(s_full, d):
    """g_j = (sigma_j - sigma_{j+1}) / sigma_1 for j = 1..d (needs d + 1 values;
    the last gap is taken as sigma_d / sigma_1 when only d are given)."""
    s = np.asarray(s_full, dtype=np.float64)
    nxt = np.append(s[1:d + 1], 0.0)[:d] if len(s) > d else np.append(s[1:d], 0.0)
    return (s[:d] - nxt) / s[0]


def gap_scaled_ratio(sines, gaps, tol=1e-5):
    """max_j sin_j * g_j / tol over j with g_j > 0; <= 1 means every leading
    subspace meets the gap-scaled bar sin_j <= tol / g_j (Wedin's bound)."""
    g = np.asarray(gaps)
    ok = g > 0
    return float(np.max(np.asarray(sines)[ok] * g[ok]) / tol) if ok.any() else 0.0


def row_product_errs(X1, Y1, X2, Y2, rows, floor=1e-2):
    """Per-row relative error of X Y^T rows:
    ||X1[i] Y1^T - X2[i] Y2^T|| / ||X2[i] Y2^T|| for i in rows, through d x d
    Grams (any n).  Rows whose reference norm is below `floor` times the median
    reference row norm are skipped (isolated or near-isolated nodes)."""
    X1, Y1, X2, Y2 = (np.asarray(a, dtype=np.float64) for a in (X1, Y1, X2, Y2))
    G11, G12, G22 = Y1.T @ Y1, Y1.T @ Y2, Y2.T @ Y2
    a, b = X1[rows], X2[rows]
    num = np.einsum("ij,jk,ik->i", a, G11, a) - 2 * np.einsum("ij,jk,ik->i", a, G12, b) \
        + np.einsum("ij,jk,ik->i", b, G22, b)
    den = np.einsum("ij,jk,ik->i", b, G22, b)
    keep = den > (floor ** 2) * np.median(den)
    return np.sqrt(np.maximum(num[keep], 0.0) / den[keep])


def recon_err2(A, X, Y):
    """Reconstruction error ||A - X Y^T||_F^2 = ||A||_F^2 - 2 tr(X^T A Y)
    + tr((X^T X)(Y^T Y)): one sparse product, any n.  A is scipy sparse."""
    X = np.asarray(X, dtype=np.float64)
    Y = np.asarray(Y, dtype=np.float64)
    nnz = float(A.multiply(A).sum())
    return nnz - 2.0 * float(np.sum(X * (A @ Y))) + float(np.trace((X.T @ X) @ (Y.T @ Y)))
