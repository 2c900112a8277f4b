"""Rounding to the sketch precision p (Algorithm 2, Stage 1, DiagMult step:
the sign-flipped matrix is cast to precision p) and the block prescale.

Readings fixed by this project (the paper leaves them open):
  * rounding is round-to-nearest-even;
  * half and bfloat16 are reached in two steps, float64 -> float32 -> p,
    which is how the hardware converts;
  * before the cast, each aligned block of BLOCK_ROWS rows of each column is
    multiplied by a power of two 2^e chosen from the block's largest
    magnitude mu (mu*2^e in [2^14, 2^15), e clamped to [-100, 100], e = 0
    when mu is 0 or not finite), and the rounded value is multiplied back by
    2^-e. Scaling by a power of two commutes with rounding whenever no
    value leaves the normal range, so this equals the plain cast for
    well-scaled inputs and keeps half precision usable for matrices whose
    entries are far from 1 (half has only 5 exponent bits). The same rule
    applies to FP32 and BF16 sketches; FP64 sketches are not rounded.
"""
from __future__ import annotations

import numpy as np

FP64, FP32, FP16, BF16 = 1, 2, 3, 4
NAMES = {FP64: "fp64", FP32: "fp32", FP16: "fp16", BF16: "bf16"}
UNIT_ROUNDOFF = {FP64: 2.0 ** -53, FP32: 2.0 ** -24, FP16: 2.0 ** -11, BF16: 2.0 ** -8}
BLOCK_ROWS = 64
SCALE_TARGET_EXP = 15  # mu * 2^e lies in [2^(T-1), 2^T)
SCALE_CLAMP = 100


def to_f32(x: np.ndarray) -> np.ndarray:
    return np.asarray(x, dtype=np.float64).astype(np.float32).astype(np.float64)


def to_f16(x: np.ndarray) -> np.ndarray:
    return np.asarray(x, dtype=np.float64).astype(np.float32).astype(np.float16).astype(np.float64)


def to_bf16(x: np.ndarray) -> np.ndarray:
    """float64 -> float32 (RNE) -> bfloat16 (RNE on the top 16 bits)."""
    f = np.ascontiguousarray(np.asarray(x, dtype=np.float64).astype(np.float32))
    b = f.view(np.uint32).astype(np.uint64)
    lsb = (b >> np.uint64(16)) & np.uint64(1)
    b = (b + np.uint64(0x7FFF) + lsb) >> np.uint64(16) << np.uint64(16)
    out = (b & np.uint64(0xFFFFFFFF)).astype(np.uint32).view(np.float32)
    return out.astype(np.float64).reshape(np.shape(x))


def round_to(x: np.ndarray, prec: int) -> np.ndarray:
    if prec == FP64:
        return np.asarray(x, dtype=np.float64)
    if prec == FP32:
        return to_f32(x)
    if prec == FP16:
        return to_f16(x)
    if prec == BF16:
        return to_bf16(x)
    raise ValueError(f"unknown precision {prec}")


def block_exponent(mu: float) -> int:
    """Power-of-two exponent e with mu*2^e in [2^14, 2^15) (clamped)."""
    if not np.isfinite(mu) or mu == 0.0:
        return 0
    _, e_mu = np.frexp(mu)  # mu = f * 2^e_mu, f in [0.5, 1)
    e = SCALE_TARGET_EXP - int(e_mu)
    return max(-SCALE_CLAMP, min(SCALE_CLAMP, e))


def block_exponents(x: np.ndarray) -> np.ndarray:
    """Exponents e[b, j] for every aligned BLOCK_ROWS-row block b and column j."""
    m, n = x.shape
    nb = (m + BLOCK_ROWS - 1) // BLOCK_ROWS
    e = np.zeros((nb, n), dtype=np.int64)
    for b in range(nb):
        blk = np.abs(x[b * BLOCK_ROWS:(b + 1) * BLOCK_ROWS, :])
        mu = blk.max(axis=0)
        for j in range(n):
            e[b, j] = block_exponent(float(mu[j]))
    return e


def cast_blockscaled(x: np.ndarray, prec: int) -> np.ndarray:
    """fl_p of x with the block power-of-two prescale; returned in float64."""
    x = np.asarray(x, dtype=np.float64)
    if prec == FP64:
        return x.copy()
    m, n = x.shape
    e = block_exponents(x)
    out = np.empty_like(x)
    for b in range(e.shape[0]):
        rows = slice(b * BLOCK_ROWS, min(m, (b + 1) * BLOCK_ROWS))
        sc = np.ldexp(1.0, e[b])            # exact powers of two
        out[rows] = np.ldexp(round_to(x[rows] * sc[None, :], prec), -e[b][None, :])
    return out
