"""Condition estimate of an upper-triangular factor, used to pick the sketch
precision (Section "Adaptive Precision Selection": only a coarse regime
kappa < 1e4 / < 1e8 / otherwise is needed; the paper leaves the estimator
open and names cheap options).

This project uses incremental condition estimation (ICE; C. Bischof, "Incremental
condition estimation", SIAM J. Matrix Anal. Appl. 11(2), 1990) on L = R^T:
keep a unit vector x with ||L_j x|| = est_j for the leading j x j block; when
row [w^T, gamma] is appended, the unit vector [s x; c] gives

  ||L_{j+1} [s x; c]||^2 = [s c] M [s c]^T,
  M = [[est_j^2 + alpha^2, alpha*gamma], [alpha*gamma, gamma^2]],  alpha = w^T x,

so est_{j+1}^2 is the largest (for sigma_max) or smallest (for sigma_min)
eigenvalue of the 2 x 2 matrix M and (s, c) its eigenvector. The estimate
of sigma_max is a lower bound and the estimate of sigma_min an upper bound,
so kappa_hat = est_max / est_min never exceeds kappa_2(R).
"""
from __future__ import annotations

import numpy as np


def _ice(R: np.ndarray, largest: bool) -> float:
    R = np.asarray(R, dtype=np.float64)
    n = R.shape[0]
    est = abs(R[0, 0])
    x = np.ones(1)
    for j in range(1, n):
        alpha = float(R[:j, j] @ x)
        gamma = float(R[j, j])
        M = np.array([[est * est + alpha * alpha, alpha * gamma],
                      [alpha * gamma, gamma * gamma]])
        lam, vec = np.linalg.eigh(M)  # ascending
        idx = 1 if largest else 0
        s, c = vec[0, idx], vec[1, idx]
        x = np.concatenate([s * x, [c]])
        est = float(np.sqrt(max(lam[idx], 0.0)))
    return est


def sigma_max_est(R: np.ndarray) -> float:
    return _ice(R, largest=True)


def sigma_min_est(R: np.ndarray) -> float:
    return _ice(R, largest=False)


def kappa_est(R: np.ndarray) -> float:
    smin = sigma_min_est(R)
    smax = sigma_max_est(R)
    if not np.isfinite(smin) or not np.isfinite(smax):
        return float("inf")
    if smin == 0.0:
        return float("inf")
    return smax / smin
