"""Accuracy measures of the paper's Figure 1: deviation from orthonormality
||I - Q^T Q||_2 and relative backward error ||A - QR||_2 / ||A||_2.

Both are evaluated in float64 with row-chunked products whose chunk partials
are summed pairwise, so that the evaluation error (about log2(#chunks) * u
plus chunk * u relative to each chunk's share) stays far below 1e-13 even for
m = 2^21 rows; plain recursive summation over m terms would not.
"""
from __future__ import annotations

import numpy as np


def _chunked_gram(X: np.ndarray, chunk: int) -> np.ndarray:
    parts = [X[i:i + chunk].T @ X[i:i + chunk] for i in range(0, X.shape[0], chunk)]
    return np.sum(np.stack(parts), axis=0)


def orthogonality(Q: np.ndarray, chunk: int = 4096) -> float:
    Q = np.asarray(Q, dtype=np.float64)
    n = Q.shape[1]
    E = np.eye(n) - _chunked_gram(Q, chunk)
    E = 0.5 * (E + E.T)
    return float(np.max(np.abs(np.linalg.eigvalsh(E))))


def residual(A: np.ndarray, Q: np.ndarray, R: np.ndarray, norm_a: float | None = None,
             chunk: int = 1 << 15) -> float:
    """||A - QR||_2 / ||A||_2 (2-norms via the n x n Gram of the residual)."""
    A = np.asarray(A, dtype=np.float64)
    Q = np.asarray(Q, dtype=np.float64)
    R = np.asarray(R, dtype=np.float64)
    n = A.shape[1]
    parts = []
    for i in range(0, A.shape[0], chunk):
        E = A[i:i + chunk] - Q[i:i + chunk] @ R
        parts.append(E.T @ E)
    EtE = np.sum(np.stack(parts), axis=0)
    en = float(np.sqrt(max(np.max(np.linalg.eigvalsh(0.5 * (EtE + EtE.T))), 0.0)))
    if norm_a is None:
        norm_a = float(np.sqrt(np.max(np.linalg.eigvalsh(_chunked_gram(A, 4096)))))
    return en / norm_a


def rel_diff(X: np.ndarray, Y: np.ndarray) -> float:
    """||X - Y||_F / ||Y||_F."""
    return float(np.linalg.norm(np.asarray(X) - np.asarray(Y)) / np.linalg.norm(Y))
