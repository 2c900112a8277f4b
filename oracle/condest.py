"""Condition estimate of an upper-triangular factor, used to pick the sketch
precision (Section "Adaptive Precision Selection": only a coarse regime
kappa < 1e4 / < 1e8 / otherwise is needed; the paper leaves the estimator
open and names cheap options).

This project uses incremental condition estimation (ICE; C. Bischof,
"Incremental condition estimation", SIAM J. Matrix Anal. Appl. 11(2), 1990)
on L = R^T: keep a unit vector x with ||L_j x|| = est_j for the leading
j x j block; when row [w^T, gamma] is appended, the unit vector [s x; c]
gives

  ||L_{j+1} [s x; c]||^2 = [s c] M [s c]^T,
  M = [[est_j^2 + alpha^2, alpha*gamma], [alpha*gamma, gamma^2]],  alpha = w^T x,

so est_{j+1}^2 is the largest (for sigma_max) or smallest (for sigma_min)
eigenvalue of the 2 x 2 matrix M and (s, c) its eigenvector. The estimate
of sigma_max is a lower bound and the estimate of sigma_min an upper bound,
so kappa_hat = est_max / est_min never exceeds kappa_2(R).

The 2 x 2 eigenpair is written out (M scaled by rho^2, rho the largest of
est, |alpha|, |gamma|, to keep squares in range):
  lam_max = (A + C)/2 + sqrt(((A - C)/2)^2 + B^2),
  lam_min = det(M) / lam_max = (est * gamma)^2 / lam_max   (no cancellation),
  eigenvector: whichever of (lam - C, B) and (B, lam - A) has the larger
  norm, normalized; if both vanish (M a multiple of I): (0, 1) for the
  largest and (1, 0) for the smallest.
"""
from __future__ import annotations

import math

import numpy as np


def ice_step(est: float, alpha: float, gamma: float, largest: bool):
    """One ICE update; returns (s, c, est_new)."""
    rho = max(est, abs(alpha), abs(gamma))
    if rho == 0.0:
        return 1.0, 0.0, 0.0
    e, a, g = est / rho, alpha / rho, gamma / rho
    A = e * e + a * a
    B = a * g
    C = g * g
    hd = 0.5 * (A - C)
    lmax = 0.5 * (A + C) + math.sqrt(hd * hd + B * B)
    if largest:
        lam = lmax
    else:
        lam = (e * g) * (e * g) / lmax if lmax > 0 else 0.0
    v1 = (lam - C, B)
    v2 = (B, lam - A)
    n1 = v1[0] * v1[0] + v1[1] * v1[1]
    n2 = v2[0] * v2[0] + v2[1] * v2[1]
    if n1 == 0.0 and n2 == 0.0:
        s, c = (0.0, 1.0) if largest else (1.0, 0.0)
    elif n1 >= n2:
        nn = math.sqrt(n1)
        s, c = v1[0] / nn, v1[1] / nn
    else:
        nn = math.sqrt(n2)
        s, c = v2[0] / nn, v2[1] / nn
    return s, c, math.sqrt(max(lam, 0.0)) * rho


def _ice(R: np.ndarray, largest: bool) -> float:
    R = np.asarray(R, dtype=np.float64)
    n = R.shape[0]
    est = abs(float(R[0, 0]))
    x = np.ones(1)
    for j in range(1, n):
        alpha = float(R[:j, j] @ x)
        gamma = float(R[j, j])
        s, c, est = ice_step(est, alpha, gamma, largest)
        x = np.concatenate([s * x, [c]])
    return est


def sigma_max_est(R: np.ndarray) -> float:
    return _ice(R, largest=True)


def sigma_min_est(R: np.ndarray) -> float:
    return _ice(R, largest=False)


def kappa_est(R: np.ndarray) -> float:
    smin = sigma_min_est(R)
    smax = sigma_max_est(R)
    if not np.isfinite(smin) or not np.isfinite(smax) or smin == 0.0:
        return float("inf")
    return smax / smin


# ---- posterior estimate of kappa_2(Rc) -------------------------------------
# The posterior check of the adaptive policy (Section "Adaptive Precision
# Selection": a result whose orthogonality is lost is detected and the
# factorization rerun one precision higher) needs kappa_2(Rc) = kappa_2(B)
# without forming Q^T Q. ICE alone can underestimate it several-fold on the
# well-conditioned factors met there, so the estimate also runs a few steps
# of the power method (Golub and Van Loan, Section 8.2) on Rc^T Rc and on
# X^T X with X = Rc^{-1} (which the factorization forms anyway), each started
# from the normalized all-ones vector. Every quantity is a lower bound of
# its exact counterpart, and so is their maximum.
POWER_STEPS = 12


def power_norm(M: np.ndarray, steps: int = POWER_STEPS) -> float:
    """||M x|| after `steps` normalized applications of M^T M to x0 =
    ones/sqrt(n): a lower bound on sigma_max(M)."""
    M = np.asarray(M, dtype=np.float64)
    n = M.shape[1]
    x = np.full(n, 1.0 / np.sqrt(n))
    for _ in range(steps):
        z = M.T @ (M @ x)
        nz = float(np.linalg.norm(z))
        if not np.isfinite(nz) or nz == 0.0:
            return nz
        x = z / nz
    return float(np.linalg.norm(M @ x))


def kappa_posterior(Rc: np.ndarray, X: np.ndarray) -> float:
    """max(ICE(Rc), power_norm(Rc) * power_norm(X)), X = Rc^{-1}."""
    k_ice = kappa_est(Rc)
    k_pow = power_norm(Rc) * power_norm(X)
    if not np.isfinite(k_ice) or not np.isfinite(k_pow):
        return float("inf")
    return max(k_ice, k_pow)
