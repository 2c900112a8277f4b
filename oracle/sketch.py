"""The SRTT sketch Y = S F D A of Algorithm 2, Stage 1 (DiagMult, transform,
Select), with the transform F read as an orthonormal DCT-II along the m rows.

Definition used here (a reading: the paper takes the real part of selected
real-FFT bins; this project uses the DCT-II, a real cosine transform with m
distinct rows):

  Y[i, j] = gamma_k * sum_t c(k, t) * at[t, j],   k = S[i]
  c(k, t) = cos(pi * (2t+1) * k / (2m))          (DCT-II kernel)
  gamma_0 = sqrt(1/s),  gamma_k = sqrt(2/s) for k > 0

i.e. Y = sqrt(m/s) * DCT-II_ortho(D A)[S, :], which makes E[Omega^T Omega] = I.
The phase (2t+1)k is reduced modulo 4m in exact integer arithmetic before
the cosine is taken.

Precision p (Algorithm 2, Stage 1 runs in p): for FP32/FP16/BF16 the signed
matrix at = fl_p(D A) (block-prescaled cast, see precision.py) and the
coefficients fl_p(c(k, t)) are rounded to p, their products are summed
exactly (float64 here; the GPU sums in float32, the paper's FP32
accumulation), gamma is applied after the sum, and Y is rounded to float32.
For FP64 nothing is rounded to a lower precision.
"""
from __future__ import annotations

import numpy as np

from . import precision as P


def phase(k: np.ndarray, t: np.ndarray, m: int) -> np.ndarray:
    """((2t+1) k) mod 4m for every (k, t) pair, exact in int64."""
    k = np.asarray(k, dtype=np.int64)
    t = np.asarray(t, dtype=np.int64)
    return ((2 * t[None, :] + 1) * k[:, None]) % (4 * m)


def coefficients(k: np.ndarray, t: np.ndarray, m: int) -> np.ndarray:
    """c(k, t) = cos(pi * phase / (2m)) in float64."""
    return np.cos(np.pi * phase(k, t, m).astype(np.float64) / (2.0 * m))


def rfft_phase(k: np.ndarray, t: np.ndarray, m: int) -> np.ndarray:
    """4 k t mod 4m: the phase of cos(2 pi k t / m) = cos(pi * phase / (2m)),
    exact in int64."""
    k = np.asarray(k, dtype=np.int64)
    t = np.asarray(t, dtype=np.int64)
    return ((4 * t[None, :]) % (4 * m) * k[:, None]) % (4 * m)


def rfft_coefficients(k: np.ndarray, t: np.ndarray, m: int) -> np.ndarray:
    """Re exp(-2 pi i k t / m) = cos(2 pi k t / m) in float64."""
    return np.cos(np.pi * rfft_phase(k, t, m).astype(np.float64) / (2.0 * m))


def gammas(S: np.ndarray, s: int) -> np.ndarray:
    S = np.asarray(S)
    return np.where(S == 0, np.sqrt(1.0 / s), np.sqrt(2.0 / s))


def signed_cast(A: np.ndarray, d: np.ndarray, prec: int) -> np.ndarray:
    """at = fl_p(D A): exact sign flip, then the block-prescaled cast."""
    at = np.asarray(A, dtype=np.float64) * d[:, None]
    return P.cast_blockscaled(at, prec)


def sketch(A: np.ndarray, S: np.ndarray, d: np.ndarray, prec: int, chunk: int = 1 << 15,
           s_total: int | None = None) -> np.ndarray:
    """Y (s x n) per the definition above; float64 array (FP32-valued unless FP64).
    s_total: the sketch size the gammas refer to when S holds only some of
    the sampled rows (default: len(S))."""
    A = np.asarray(A, dtype=np.float64)
    m, n = A.shape
    S = np.asarray(S, dtype=np.int64)
    s = S.shape[0]
    at = signed_cast(A, d, prec)
    y = np.zeros((s, n), dtype=np.float64)
    for t0 in range(0, m, chunk):
        t = np.arange(t0, min(m, t0 + chunk), dtype=np.int64)
        c = coefficients(S, t, m)
        if prec != P.FP64:
            c = P.round_to(c, prec)
        y += c @ at[t0:t0 + t.shape[0]]
    y *= gammas(S, s if s_total is None else s_total)[:, None]
    if prec != P.FP64:
        y = P.to_f32(y)
    return y


def sketch_abs_bound(A: np.ndarray, S: np.ndarray, d: np.ndarray, prec: int, chunk: int = 1 << 15,
                     s_total: int | None = None) -> np.ndarray:
    """gamma_k * sum_t |c(k,t)| |at[t,j]|: the scale against which rounding
    errors of the sketch are measured (elementwise)."""
    A = np.asarray(A, dtype=np.float64)
    m, n = A.shape
    S = np.asarray(S, dtype=np.int64)
    at = np.abs(signed_cast(A, d, prec))
    y = np.zeros((S.shape[0], n), dtype=np.float64)
    for t0 in range(0, m, chunk):
        t = np.arange(t0, min(m, t0 + chunk), dtype=np.int64)
        y += np.abs(coefficients(S, t, m)) @ at[t0:t0 + t.shape[0]]
    return y * gammas(S, S.shape[0] if s_total is None else s_total)[:, None]


def sketch_rfft(A: np.ndarray, S: np.ndarray, d: np.ndarray, prec: int, chunk: int = 1 << 15,
                s_total: int | None = None) -> np.ndarray:
    """The paper's operator (Algorithm 2, FFT and Select): the real parts of
    the DFT bins S (0 <= k <= m/2) of fl_p(D A), scaled by sqrt(c/m):
      Y[i, j] = sqrt(c/m) * sum_t cos(2 pi k_i t / m) * at[t, j].
    Precision rules as in sketch(): coefficients and data rounded to p, the
    products summed exactly here (float32 on the GPU), the scale applied
    after the sum, Y rounded to float32 for p != FP64."""
    A = np.asarray(A, dtype=np.float64)
    m, n = A.shape
    S = np.asarray(S, dtype=np.int64)
    c_total = S.shape[0] if s_total is None else s_total
    at = signed_cast(A, d, prec)
    y = np.zeros((S.shape[0], n), dtype=np.float64)
    for t0 in range(0, m, chunk):
        t = np.arange(t0, min(m, t0 + chunk), dtype=np.int64)
        c = rfft_coefficients(S, t, m)
        if prec != P.FP64:
            c = P.round_to(c, prec)
        y += c @ at[t0:t0 + t.shape[0]]
    y *= np.sqrt(c_total / m)
    if prec != P.FP64:
        y = P.to_f32(y)
    return y


def sketch_rfft_abs_bound(A: np.ndarray, S: np.ndarray, d: np.ndarray, prec: int, chunk: int = 1 << 15,
                          s_total: int | None = None) -> np.ndarray:
    """sqrt(c/m) sum_t |cos(2 pi k t / m)| |at[t, j]|, the error scale of
    sketch_rfft (elementwise)."""
    A = np.asarray(A, dtype=np.float64)
    m, n = A.shape
    S = np.asarray(S, dtype=np.int64)
    at = np.abs(signed_cast(A, d, prec))
    y = np.zeros((S.shape[0], n), dtype=np.float64)
    for t0 in range(0, m, chunk):
        t = np.arange(t0, min(m, t0 + chunk), dtype=np.int64)
        y += np.abs(rfft_coefficients(S, t, m)) @ at[t0:t0 + t.shape[0]]
    return y * np.sqrt((S.shape[0] if s_total is None else s_total) / m)
