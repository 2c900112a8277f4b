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


# ---- the two other estimators the paper names (Section "Adaptive Precision
# Selection"), kept for comparison with ICE ----------------------------------

def _rademacher_column(seed: int, col: int, n: int) -> np.ndarray:
    """+-1 entries from the counter-based generator (stream 3, one counter
    per entry), for the estimator's random starting and replacement columns."""
    from . import rng
    return np.array([1.0 if (rng.h(seed, 3, col * n + i) >> 63) == 0 else -1.0 for i in range(n)])


def onenorm_est(apply, apply_t, n: int, t: int = 2, itmax: int = 5, seed: int = 0) -> float:
    """Block 1-norm estimate of ||B||_1 (Higham and Tisseur, "A block
    algorithm for matrix 1-norm estimation", SIAM J. Matrix Anal. Appl. 21,
    2000, Algorithm 2.4), B given by products apply(X) = B X and
    apply_t(X) = B^T X with n x t blocks. A lower bound on ||B||_1.

    Steps, as the algorithm states them: start from X with first column
    ones/n and the others random +-1/n (parallel columns replaced); repeat
    Y = B X, est = the largest column 1-norm of Y; stop when est stops
    growing (keeping the previous one), after itmax steps, or when every
    column of S = sign(Y) is parallel to one of the previous S; otherwise
    replace columns of S parallel to another column of S or of the previous
    S by random +-1 columns, form Z = B^T S, h_i = max_j |Z_ij|; stop if the
    best index already gave the largest h (from the second step on); take
    the t indices of largest h not used before as unit vectors for X (stop
    if all of the t largest were used before)."""
    if n == 1:
        return float(abs(apply(np.ones((1, 1)))[0, 0]))
    t = min(t, n)
    tries = 16  # random draws for one column before the last one is kept (small n may have no other choice)
    rcol = [0]

    def fresh():
        c = _rademacher_column(seed, rcol[0], n)
        rcol[0] += 1
        return c

    def parallel(a, b):
        return abs(float(a @ b)) == n

    X = np.ones((n, t))
    for j in range(1, t):
        for _ in range(tries):
            c = fresh()
            if not any(parallel(c, X[:, i]) for i in range(j)):
                break
        X[:, j] = c
    X /= n
    est_old = 0.0
    S_old = np.zeros((n, t))
    ind_hist = []
    ind_best = 0
    est = 0.0
    for k in range(1, itmax + 2):
        Y = apply(X)
        norms = np.abs(Y).sum(axis=0)
        est = float(norms.max())
        if est > est_old or k == 2:
            ind_best_col = int(np.argmax(norms))
            if k >= 2:
                ind_best = ind_cur[ind_best_col]
        if k >= 2 and est <= est_old:
            est = est_old
            break
        est_old = est
        if k > itmax:
            break
        S = np.where(Y >= 0, 1.0, -1.0)
        if k > 1 and all(any(parallel(S[:, j], S_old[:, i]) for i in range(t)) for j in range(t)):
            break
        for j in range(t):
            for _ in range(tries):
                if not (any(parallel(S[:, j], S[:, i]) for i in range(j)) or
                        (k > 1 and any(parallel(S[:, j], S_old[:, i]) for i in range(t)))):
                    break
                S[:, j] = fresh()
        S_old = S.copy()
        Z = apply_t(S)
        h = np.abs(Z).max(axis=1)
        if k >= 2 and h.max() == h[ind_best]:
            break
        order = np.argsort(-h, kind="stable")
        if t > 1 and all(i in ind_hist for i in order[:t]):
            break
        ind_cur = [int(i) for i in order if i not in ind_hist][:t]
        if len(ind_cur) < t:
            break
        X = np.zeros((n, t))
        for j, i in enumerate(ind_cur):
            X[i, j] = 1.0
        ind_hist += ind_cur
    return est


def kappa_1norm_tri(R: np.ndarray, seed: int = 0) -> float:
    """kappa_1(R) = ||R||_1 ||R^{-1}||_1 for upper-triangular R, the inverse's
    norm estimated by onenorm_est with triangular solves."""
    import scipy.linalg
    R = np.triu(np.asarray(R, dtype=np.float64))
    n = R.shape[0]
    inv = onenorm_est(lambda X: scipy.linalg.solve_triangular(R, X, lower=False),
                      lambda X: scipy.linalg.solve_triangular(R, X, lower=False, trans="T"), n, seed=seed)
    return float(np.abs(R).sum(axis=0).max()) * inv


def kappa_bound_gram(Rg: np.ndarray, seed: int = 0) -> float:
    """The paper's classification bound kappa_2(A)^2 <= n ||A^T A||_1
    ||(A^T A)^{-1}||_1, with A^T A = Rg^T Rg (its Cholesky factor) and the
    inverse's norm estimated by onenorm_est; returns the square root."""
    import scipy.linalg
    Rg = np.triu(np.asarray(Rg, dtype=np.float64))
    n = Rg.shape[0]
    G = Rg.T @ Rg

    def solve(X):
        return scipy.linalg.solve_triangular(Rg, scipy.linalg.solve_triangular(Rg, X, lower=False, trans="T"),
                                             lower=False)
    inv = onenorm_est(solve, solve, n, seed=seed)
    return float(np.sqrt(n * np.abs(G).sum(axis=0).max() * inv))


def cholqr_probe(q: float, u: float = 2.0 ** -53) -> float:
    """The CholQR probe's lower bound kappa_2(A) >= sqrt(q / (u (1 + q))),
    q = ||I - Q^T Q||_2 of one CholQR (Algorithm 1) pass on A."""
    return float(np.sqrt(q / (u * (1.0 + q))))


def sym_power_norm(E: np.ndarray, steps: int = POWER_STEPS) -> float:
    """||E x|| after `steps` normalized applications of the symmetric E to
    x0 = ones/sqrt(n): a lower bound on ||E||_2."""
    E = np.asarray(E, dtype=np.float64)
    x = np.full(E.shape[0], 1.0 / np.sqrt(E.shape[0]))
    for _ in range(steps):
        z = E @ x
        x = z / np.linalg.norm(z)
    return float(np.linalg.norm(E @ x))


def probe_kappa(A: np.ndarray, exact: bool = True) -> float:
    """The CholQR probe on A: one pass of Algorithm 1, q = ||I - Q^T Q||_2
    of its Q (exact, or by sym_power_norm as the GPU estimates it), the bound
    above; +inf when the pass breaks down (kappa(A) beyond about u^(-1/2),
    the double regime)."""
    from . import cholqr as CQ, metrics as MT
    try:
        Q, _ = CQ.cholqr(A)
    except CQ.CholeskyBreakdown:
        return float("inf")
    if exact:
        return cholqr_probe(MT.orthogonality(Q))
    E = np.eye(Q.shape[1]) - CQ.gram(Q)
    return cholqr_probe(sym_power_norm(E))
