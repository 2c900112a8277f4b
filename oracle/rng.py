"""Random draws of Algorithm 2, Stage 1, first step: the Rademacher diagonal
D and the row sample S (Section "Our Mixed-Precision Algorithm", Algorithm 2).

The paper does not state its generator. This project fixes one, counter
based, so that the CPU oracle and the GPU library (two independent
implementations) draw bit-identical D and S from the same seed:

  mix64(z)        SplitMix64 output finalizer (Steele, Lea and Flood, 2014):
                  z ^= z>>30; z *= 0xBF58476D1CE4E5B9; z ^= z>>27;
                  z *= 0x94D049BB133111EB; z ^= z>>31   (all mod 2^64)
  key(seed, st)   mix64(seed XOR st*0xD1B54A32D192ED03)
  h(seed, st, i)  mix64(key(seed, st) + (i+1)*0x9E3779B97F4A7C15)
                  i.e. the (i+1)-th SplitMix64 output from state key.

  stream 0: sign d_t = -1 if the top bit of h(seed,0,t) is set, else +1.
  stream 1: S by Floyd's algorithm (Bentley and Floyd, 1987): for
            j = m-s .. m-1, r = floor(h(seed,1,j) * (j+1) / 2^64) (a number
            in [0, j]); insert r unless already present, else insert j.
            S is returned sorted ascending: a uniformly random s-subset of
            {0, ..., m-1} (the DCT-II has m distinct rows, so every row,
            including row 0, may be drawn).
  stream 2: per-instance seeds of a batch: seed_i = h(base, 2, i).
"""
from __future__ import annotations

import numpy as np

MASK = (1 << 64) - 1
GOLDEN = 0x9E3779B97F4A7C15
STREAM_MUL = 0xD1B54A32D192ED03
M1 = 0xBF58476D1CE4E5B9
M2 = 0x94D049BB133111EB


def mix64(z: int) -> int:
    z &= MASK
    z ^= z >> 30
    z = (z * M1) & MASK
    z ^= z >> 27
    z = (z * M2) & MASK
    z ^= z >> 31
    return z


def key(seed: int, stream: int) -> int:
    return mix64((seed & MASK) ^ ((stream * STREAM_MUL) & MASK))


def h(seed: int, stream: int, i: int) -> int:
    return mix64(key(seed, stream) + ((i + 1) * GOLDEN))


def _mix64_array(z: np.ndarray) -> np.ndarray:
    z = z.astype(np.uint64, copy=True)
    with np.errstate(over="ignore"):
        z ^= z >> np.uint64(30)
        z *= np.uint64(M1)
        z ^= z >> np.uint64(27)
        z *= np.uint64(M2)
        z ^= z >> np.uint64(31)
    return z


def h_array(seed: int, stream: int, idx: np.ndarray) -> np.ndarray:
    k = np.uint64(key(seed, stream))
    i1 = idx.astype(np.uint64) + np.uint64(1)
    with np.errstate(over="ignore"):
        z = k + i1 * np.uint64(GOLDEN)
    return _mix64_array(z)


def signs(seed: int, m: int) -> np.ndarray:
    """Rademacher diagonal d in {+1,-1}^m as float64."""
    hv = h_array(seed, 0, np.arange(m, dtype=np.uint64))
    top = (hv >> np.uint64(63)).astype(np.int64)
    return (1 - 2 * top).astype(np.float64)


def sample_rows(seed: int, m: int, s: int) -> np.ndarray:
    """Floyd's uniform s-subset of range(m), sorted ascending, as int64."""
    if not (0 < s <= m):
        raise ValueError("need 0 < s <= m")
    chosen = set()
    for j in range(m - s, m):
        r = (h(seed, 1, j) * (j + 1)) >> 64
        if r in chosen:
            chosen.add(j)
        else:
            chosen.add(r)
    return np.array(sorted(chosen), dtype=np.int64)


def instance_seed(base: int, i: int) -> int:
    return h(base, 2, i)
