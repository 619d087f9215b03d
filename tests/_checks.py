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
