"""Stage 2 and Stage 3 of Algorithm 2 in float64: the preconditioned matrix
A1 = A Rs^{-1}, Cholesky-QR of it (Algorithm 1: Gram matrix, Cholesky,
triangular solve) and the product R = R2 Rs.

The triangular solves are substitutions (the paper forbids forming Rs^{-1}
explicitly, Section "Algorithm Description"): column j of X = A R^{-1} is
x_j = (a_j - X[:, :j] R[:j, j]) / r_jj.
"""
from __future__ import annotations

import numpy as np


class CholeskyBreakdown(Exception):
    def __init__(self, index: int):
        super().__init__(f"Cholesky breakdown at pivot {index}")
        self.index = index


def trsm_right_upper(A: np.ndarray, R: np.ndarray) -> np.ndarray:
    """X = A R^{-1} for upper-triangular R, by forward substitution."""
    A = np.asarray(A, dtype=np.float64)
    m, n = A.shape
    X = np.empty((m, n), dtype=np.float64, order="F")
    for j in range(n):
        acc = A[:, j].copy()
        if j:
            acc -= X[:, :j] @ R[:j, j]
        X[:, j] = acc / R[j, j]
    return X


def gram(B: np.ndarray, chunk: int = 1 << 14) -> np.ndarray:
    """G = B^T B, summing row-chunk products pairwise."""
    B = np.asarray(B, dtype=np.float64)
    parts = [B[i:i + chunk].T @ B[i:i + chunk] for i in range(0, B.shape[0], chunk)]
    G = np.sum(np.stack(parts), axis=0)
    return 0.5 * (G + G.T)


def cholesky_upper(G: np.ndarray) -> np.ndarray:
    """Upper R with G = R^T R (textbook row-by-row); raises CholeskyBreakdown(j)
    when pivot j is not positive or not finite."""
    G = np.asarray(G, dtype=np.float64)
    n = G.shape[0]
    R = np.zeros((n, n), dtype=np.float64)
    for j in range(n):
        piv = G[j, j] - R[:j, j] @ R[:j, j]
        if not np.isfinite(piv) or piv <= 0:
            raise CholeskyBreakdown(j)
        R[j, j] = np.sqrt(piv)
        if j + 1 < n:
            R[j, j + 1:] = (G[j, j + 1:] - R[:j, j] @ R[:j, j + 1:]) / R[j, j]
    return R


def upper_inverse(R: np.ndarray) -> np.ndarray:
    """X = R^{-1} for upper-triangular R: column j solves R x = e_j by back
    substitution, x_i = (e_j[i] - R[i, i+1:j+1] x[i+1:j+1]) / r_ii for
    i = j, ..., 0 (rows below j are zero). Algorithm 1 forms Q = B Rc^{-1};
    with kappa(Rc) = kappa(B) small this inverse may be applied as a
    product (Rs, which can be ill conditioned, is only ever solved with)."""
    R = np.asarray(R, dtype=np.float64)
    n = R.shape[0]
    X = np.zeros((n, n), dtype=np.float64)
    for j in range(n):
        x = np.zeros(j + 1)
        for i in range(j, -1, -1):
            rhs = (1.0 if i == j else 0.0) - R[i, i + 1:j + 1] @ x[i + 1:j + 1]
            x[i] = rhs / R[i, i]
        X[:j + 1, j] = x
    return X


def form_q(B: np.ndarray, X: np.ndarray) -> np.ndarray:
    """Q = B X for upper-triangular X (the plain product)."""
    return np.asarray(B, dtype=np.float64) @ np.triu(np.asarray(X, dtype=np.float64))


def trmm_upper(R2: np.ndarray, Rs: np.ndarray) -> np.ndarray:
    """R = R2 Rs (product of upper-triangular factors, Stage 3)."""
    return np.triu(np.asarray(R2) @ np.asarray(Rs))


def cholqr(A: np.ndarray):
    """Algorithm 1 (CholQR) on A itself: G = A^T A, G = R^T R, Q = A R^{-1}
    by substitution. Raises CholeskyBreakdown when the Gram matrix is not
    numerically positive definite."""
    R = cholesky_upper(gram(A))
    return trsm_right_upper(A, R), R


def cholqr2(A: np.ndarray):
    """CholQR2: Algorithm 1 applied twice, R = R2 R1 (the paper's stability
    baseline in Section "Numerical Stability", which breaks down once the
    Gram matrix of A loses positive definiteness, kappa(A) past about 1e8)."""
    Q1, R1 = cholqr(A)
    Q, R2 = cholqr(Q1)
    return Q, trmm_upper(R2, R1)
