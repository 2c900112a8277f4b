"""Pins of the oracle's rounding to the sketch precision."""
import os
import struct

import numpy as np
import pytest

from oracle import precision as P
from conftest import GOLDEN


def _cases():
    out = []
    for line in open(os.path.join(GOLDEN, "ieee_rounding.txt")):
        if line.startswith("#") or not line.strip():
            continue
        f, a, b = line.split()
        out.append((f, float.fromhex(a), float("inf") if b == "inf" else float.fromhex(b)))
    return out


@pytest.mark.parametrize("fmt,x,want", _cases())
def test_rounding_fixtures(fmt, x, want):
    fn = {"fp16": P.to_f16, "bf16": P.to_bf16, "fp32": P.to_f32}[fmt]
    with np.errstate(over="ignore"):
        got = float(fn(np.array([x]))[0])
    assert got == want


def _bf16_bruteforce(x32):
    """Nearest bfloat16 by comparing the two bracketing candidates exactly."""
    b = struct.unpack("<I", struct.pack("<f", x32))[0]
    lo = b & 0xFFFF0000
    hi = lo + 0x10000
    flo = struct.unpack("<f", struct.pack("<I", lo))[0]
    fhi = struct.unpack("<f", struct.pack("<I", hi & 0xFFFFFFFF))[0]
    dlo, dhi = abs(float(x32) - flo), abs(fhi - float(x32))
    if dlo < dhi:
        return flo
    if dhi < dlo:
        return fhi
    return flo if ((lo >> 16) & 1) == 0 else fhi


def test_bf16_matches_bruteforce_nearest_even():
    rng = np.random.default_rng(1)
    x = rng.standard_normal(5000) * np.exp2(rng.integers(-30, 30, 5000))
    got = P.to_bf16(x)
    for xi, gi in zip(x, got):
        assert gi == _bf16_bruteforce(np.float32(xi))


def test_block_exponent_targets_window():
    for mu in [1e-300, 3e-5, 0.7, 1.0, 65504.0, 1e300]:
        e = P.block_exponent(mu)
        if -P.SCALE_CLAMP < e < P.SCALE_CLAMP:
            assert 2.0 ** 14 <= mu * 2.0 ** e < 2.0 ** 15
    assert P.block_exponent(0.0) == 0
    assert P.block_exponent(float("nan")) == 0


@pytest.mark.parametrize("prec", [P.FP32, P.FP16, P.BF16])
def test_blockscaled_cast_relative_error(prec):
    rng = np.random.default_rng(2)
    x = rng.standard_normal((300, 5)) * np.exp2(rng.integers(-40, 40, (1, 5)))
    y = P.cast_blockscaled(x, prec)
    assert np.all(np.abs(y - x) <= P.UNIT_ROUNDOFF[prec] * np.abs(x) * (1 + 1e-12) + 2.0 ** -40 * np.abs(x).max(axis=0))


@pytest.mark.parametrize("prec", [P.FP32, P.FP16, P.BF16])
def test_blockscaled_cast_equals_plain_cast_in_normal_range(prec):
    rng = np.random.default_rng(3)
    x = rng.uniform(0.5, 2.0, (200, 4)) * rng.choice([-1, 1], (200, 4))
    assert np.array_equal(P.cast_blockscaled(x, prec), P.round_to(x, prec))


@pytest.mark.parametrize("prec", [P.FP32, P.FP16, P.BF16])
def test_blockscaled_cast_commutes_with_power_of_two(prec):
    rng = np.random.default_rng(4)
    x = rng.standard_normal((130, 3)) * 1e-6
    for k in [-20, 7, 33]:
        assert np.array_equal(P.cast_blockscaled(x * 2.0 ** k, prec), P.cast_blockscaled(x, prec) * 2.0 ** k)


def test_fp16_plain_cast_would_lose_small_entries():
    # the reason for the prescale: 1e-7 underflows to a subnormal in binary16
    x = np.full((64, 1), 1.2345e-7)
    assert abs(P.to_f16(x)[0, 0] - 1.2345e-7) > 1e-2 * 1.2345e-7
    assert abs(P.cast_blockscaled(x, P.FP16)[0, 0] - 1.2345e-7) <= 2 ** -11 * 1.2345e-7
