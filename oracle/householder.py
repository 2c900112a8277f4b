"""Textbook Householder thin QR (Golub and Van Loan, Section 5.2; the
blocked geqrf the paper cites in its background section and uses as its
stable reference), unblocked, column by column.

Reflector convention (as LAPACK's larfg): for x = [alpha; x2] with
sigma = ||x2||, if sigma == 0 no reflection is applied (tau = 0, beta =
alpha); otherwise beta = -sign(alpha) * sqrt(alpha^2 + sigma^2),
tau = (beta - alpha) / beta, v = [1; x2 / (alpha - beta)], and
H = I - tau v v^T maps x to beta e1.

After the loop the factors are sign-normalized so that diag(R) >= 0, which
makes the thin QR of a full-rank matrix unique.
"""
from __future__ import annotations

import numpy as np


def householder_qr(A: np.ndarray, dtype=np.float64, want_q: bool = True):
    """Return (Q, R) (Q is None when want_q is False), computed in `dtype`."""
    X = np.array(A, dtype=dtype, copy=True)
    m, n = X.shape
    if m < n:
        raise ValueError("need m >= n")
    taus = np.zeros(n, dtype=dtype)
    for j in range(n):
        alpha = X[j, j]
        x2 = X[j + 1:, j]
        sigma = np.linalg.norm(x2) if x2.size else dtype(0)
        if sigma == 0:
            taus[j] = 0
            continue
        beta = -np.copysign(np.hypot(alpha, sigma), alpha).astype(dtype)
        tau = dtype((beta - alpha) / beta)
        v = np.empty(m - j, dtype=dtype)
        v[0] = 1
        v[1:] = x2 / dtype(alpha - beta)
        if j + 1 < n:
            w = v @ X[j:, j + 1:]
            X[j:, j + 1:] -= tau * np.outer(v, w)
        X[j, j] = beta
        X[j + 1:, j] = v[1:]
        taus[j] = tau
    R = np.triu(X[:n, :])
    Q = None
    if want_q:
        Q = np.zeros((m, n), dtype=dtype)
        Q[np.arange(n), np.arange(n)] = 1
        for j in range(n - 1, -1, -1):
            if taus[j] == 0:
                continue
            v = np.empty(m - j, dtype=dtype)
            v[0] = 1
            v[1:] = X[j + 1:, j]
            w = v @ Q[j:, j:]
            Q[j:, j:] -= taus[j] * np.outer(v, w)
    d = np.sign(np.diag(R))
    d[d == 0] = 1
    R = R * d[:, None]
    if Q is not None:
        Q = Q * d[None, :]
    return Q, R


def householder_r(A: np.ndarray, dtype=np.float64) -> np.ndarray:
    return householder_qr(A, dtype=dtype, want_q=False)[1]
