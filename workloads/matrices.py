"""Seeded generators for matrices with known structure (inputs only).

All generators use numpy's PCG64 bit generator seeded by an integer, so the
same (shape, seed) always yields the same array on any machine.
"""
from __future__ import annotations

import numpy as np


def _rng(seed: int) -> np.random.Generator:
    return np.random.Generator(np.random.PCG64(int(seed)))


def _orthonormal_columns(rng: np.random.Generator, m: int, n: int) -> np.ndarray:
    """Q factor of an m x n Gaussian matrix, columns sign-fixed (diag(R) > 0)."""
    g = rng.standard_normal((m, n))
    q, r = np.linalg.qr(g, mode="reduced")
    d = np.sign(np.diag(r))
    d[d == 0] = 1.0
    return q * d[None, :]


def singular_values(n: int, kappa: float) -> np.ndarray:
    """Geometric singular values sigma_i = kappa**(-i/(n-1)), i = 0..n-1.

    sigma_0 = 1 and sigma_{n-1} = 1/kappa, so kappa_2 = kappa exactly.
    """
    if n == 1:
        return np.ones(1)
    i = np.arange(n, dtype=np.float64)
    return np.power(float(kappa), -i / (n - 1))


def test_matrix_factors(m: int, n: int, kappa: float, seed: int):
    """Return (U, sigma, V) with U m x n and V n x n orthonormal, seeded."""
    rng = _rng(seed)
    u = _orthonormal_columns(rng, m, n)
    v = _orthonormal_columns(rng, n, n)
    return u, singular_values(n, kappa), v


def test_matrix(m: int, n: int, kappa: float, seed: int, order: str = "F") -> np.ndarray:
    """A = U diag(sigma) V^T in float64 (column-major by default)."""
    u, s, v = test_matrix_factors(m, n, kappa, seed)
    a = (u * s[None, :]) @ v.T
    return np.asarray(a, order=order)


def gaussian(m: int, n: int, seed: int, dtype=np.float64, order: str = "F") -> np.ndarray:
    """Plain standard-normal matrix."""
    return np.asarray(_rng(seed).standard_normal((m, n)).astype(dtype), order=order)


def upper_triangular(n: int, kappa: float, seed: int) -> np.ndarray:
    """Upper-triangular n x n matrix with positive diagonal and kappa_2 ~ kappa.

    Built as the R factor of U diag(sigma) V^T for a small square U, so its
    singular values are exactly the geometric sigma (up to rounding).
    """
    rng = _rng(seed)
    u = _orthonormal_columns(rng, n, n)
    v = _orthonormal_columns(rng, n, n)
    s = singular_values(n, kappa)
    x = (u * s[None, :]) @ v.T
    _, r = np.linalg.qr(x)
    d = np.sign(np.diag(r))
    d[d == 0] = 1.0
    return np.asfortranarray(np.triu(r * d[:, None]))


def spd_matrix(n: int, kappa: float, seed: int) -> np.ndarray:
    """Symmetric positive-definite n x n matrix with eigenvalues 1 .. 1/kappa."""
    rng = _rng(seed)
    v = _orthonormal_columns(rng, n, n)
    lam = singular_values(n, kappa)
    g = (v * lam[None, :]) @ v.T
    g = 0.5 * (g + g.T)
    return np.asfortranarray(g)


def instance_mix(count: int, seed: int, m_range=(4096, 131072), n_choices=(8, 16, 32, 64),
                 log_kappa_range=(2.0, 12.0)):
    """Draw (m, n, kappa) triples for a batch of uneven instances."""
    rng = _rng(seed)
    ms = rng.integers(m_range[0], m_range[1] + 1, size=count)
    ns = rng.choice(np.asarray(n_choices), size=count)
    ks = np.power(10.0, rng.uniform(log_kappa_range[0], log_kappa_range[1], size=count))
    return [(int(a), int(b), float(c)) for a, b, c in zip(ms, ns, ks)]


def rising_kappas(calls: int, lo_exp: float = 2.0, hi_exp: float = 14.0) -> np.ndarray:
    """kappa_k = 10^(lo + (hi - lo) k / (calls - 1)), k = 0..calls-1: the
    slowly worsening conditioning of a repeated-QR loop (block Krylov or
    power steps), with the same U and V and only sigma changing per call."""
    if calls == 1:
        return np.array([10.0 ** lo_exp])
    return 10.0 ** (lo_exp + (hi_exp - lo_exp) * np.arange(calls) / (calls - 1))


def device_test_matrix(m: int, n: int, kappa: float, seed: int, device="cuda"):
    """A = U diag(sigma) V^T drawn on the device, the family of test_matrix:
    U from the QR of an m x n Gaussian drawn with torch's seeded generator on
    the device, V orthonormal from a host Gaussian, sigma geometric from 1 to
    1/kappa. Column-major float64 tensor. For large batches where building
    every U on the host would take minutes."""
    import torch

    gen = torch.Generator(device=device)
    gen.manual_seed(int(seed))
    g = torch.randn(m, n, generator=gen, device=device, dtype=torch.float64)
    u, _ = torch.linalg.qr(g)
    v = _orthonormal_columns(_rng(seed), n, n)
    w = torch.from_numpy(np.ascontiguousarray(singular_values(n, kappa)[:, None] * v.T)).to(device)  # diag(sigma) V^T
    a = torch.empty((n, m), device=device, dtype=torch.float64).t()  # column-major
    torch.mm(u, w, out=a)
    return a


def paper_sweep_matrix(m: int, n: int, kappa: float, seed: int, order: str = "F") -> np.ndarray:
    """The stability sweep's matrices: A = U diag(sigma) V^T with U (m x n),
    V (n x n) the sign-fixed Q factors of matrices with entries uniform on
    [-1, 1], and sigma_i = kappa^(1/2 - i/(n-1)) (so sigma_max = kappa^(1/2),
    sigma_min = kappa^(-1/2), kappa_2 = kappa), as the paper builds them."""
    rng = _rng(seed)
    def q_of_uniform(r, c):
        q, rr = np.linalg.qr(rng.uniform(-1.0, 1.0, (r, c)), mode="reduced")
        d = np.sign(np.diag(rr))
        d[d == 0] = 1.0
        return q * d[None, :]
    u = q_of_uniform(m, n)
    v = q_of_uniform(n, n)
    i = np.arange(n, dtype=np.float64)
    sig = np.power(float(kappa), 0.5 - i / max(n - 1, 1))
    return np.asarray((u * sig[None, :]) @ v.T, order=order)
