"""Pins of the oracle's DCT-II sketch (Algorithm 2, Stage 1, transform and
Select steps, with the DCT-II reading of the transform)."""
import numpy as np
import pytest
import scipy.fft

from oracle import sketch as SK, precision as P, rng
import workloads as W


def test_fp64_sketch_matches_scipy_dct():
    m, n, s = 1000, 7, 40
    A = W.gaussian(m, n, 1)
    S = rng.sample_rows(5, m, s)
    d = rng.signs(5, m)
    Y = SK.sketch(A, S, d, P.FP64)
    ref = np.sqrt(m / s) * scipy.fft.dct(d[:, None] * A, type=2, norm="ortho", axis=0)[S, :]
    assert np.max(np.abs(Y - ref)) <= 1e-13 * np.max(np.abs(ref))


def test_dct_matrix_is_orthogonal_when_all_rows_sampled():
    # s = m: gamma_k * c(k, t) is the orthonormal DCT-II matrix (brute force)
    m = 48
    k = np.arange(m)
    C = SK.coefficients(k, np.arange(m), m) * SK.gammas(k, m)[:, None]
    assert np.max(np.abs(C @ C.T - np.eye(m))) < 1e-13
    assert np.max(np.abs(C.T @ C - np.eye(m))) < 1e-13


def test_all_rows_sketch_preserves_gram():
    m, n = 64, 5
    A = W.gaussian(m, n, 2)
    S = rng.sample_rows(1, m, m)
    Y = SK.sketch(A, S, rng.signs(1, m), P.FP64)
    assert np.allclose(Y.T @ Y, A.T @ A, rtol=0, atol=1e-12 * np.abs(A.T @ A).max())


def test_phase_is_exact_for_large_m():
    m = 1 << 21
    k = np.array([m - 1, 12345, 0])
    t = np.array([m - 1, 0, 777])
    ph = SK.phase(k, t, m)
    for i, kk in enumerate(k):
        for j, tt in enumerate(t):
            assert ph[i, j] == ((2 * int(tt) + 1) * int(kk)) % (4 * m)


def test_coefficient_symmetry():
    # c(k, m-1-t) = (-1)^k c(k, t): the DCT-II kernel's reflection symmetry
    m = 1 << 12
    k = np.array([1, 2, 777, 4095])
    t = np.arange(0, m, 97)
    c1 = SK.coefficients(k, t, m)
    c2 = SK.coefficients(k, m - 1 - t, m)
    sign = np.where(k % 2 == 0, 1.0, -1.0)[:, None]
    assert np.max(np.abs(c2 - sign * c1)) < 1e-15


@pytest.mark.parametrize("prec", [P.FP32, P.FP16, P.BF16])
def test_low_precision_sketch_is_close_to_exact(prec):
    m, n, s = 2048, 6, 24
    A = W.gaussian(m, n, 3)
    S = rng.sample_rows(9, m, s)
    d = rng.signs(9, m)
    Y = SK.sketch(A, S, d, prec)
    Y64 = SK.sketch(A, S, d, P.FP64)
    bound = SK.sketch_abs_bound(A, S, d, P.FP64)
    u = P.UNIT_ROUNDOFF[prec]
    # coefficient and input rounding (2u), float32 output rounding
    assert np.all(np.abs(Y - Y64) <= (2.0 * u + u * u) * bound + 2.0 ** -24 * np.abs(Y64) + 1e-300)
    assert np.max(np.abs(Y - Y64)) > 0


def test_low_precision_sketch_uses_rounded_inputs():
    # an FP16 sketch only sees fl16(DA): entries k/64 (|k| < 1024) are exact
    # in binary16, and a relative perturbation of 2^-20 (far below half an
    # ulp, 2^-11) rounds back to them, so Y is unchanged
    m, n, s = 256, 3, 8
    A = np.asfortranarray(np.clip(np.round(W.gaussian(m, n, 4) * 64), -1000, 1000) / 64)
    S = rng.sample_rows(2, m, s)
    d = rng.signs(2, m)
    Y1 = SK.sketch(A, S, d, P.FP16)
    Y2 = SK.sketch(A * (1 + 2.0 ** -20), S, d, P.FP16)
    assert np.array_equal(Y1, Y2)


def _coefficient_cases():
    import os
    from conftest import GOLDEN
    out = {}
    for line in open(os.path.join(GOLDEN, "sketch_coefficients.txt")):
        if line.startswith("#") or not line.strip():
            continue
        fmt, i, j, y = line.split()
        out.setdefault(fmt, {})[(int(i), int(j))] = float.fromhex(y)
    return out


@pytest.mark.parametrize("fmt,prec", [("fp16", P.FP16), ("bf16", P.BF16), ("fp32", P.FP32)])
def test_sketch_of_unit_vectors_matches_hand_derived_values(fmt, prec):
    """Algorithm 2, Stage 1 in precision p: the cosine coefficients are
    rounded to p (unit-vector columns expose fl_p(c) directly) and the
    float32-accumulated Y is a float32 value (column 8's exact sum needs 31
    bits). Values: tests/golden/sketch_coefficients.txt, derived from 60-digit
    cosines and the formats' spacing, not from this oracle."""
    want = _coefficient_cases()[fmt]
    m = 8
    A = np.zeros((m, 9))
    A[np.arange(m), np.arange(m)] = 1.0
    A[0, 8], A[1, 8] = 1.0, 2.0 ** -20
    d = np.array([1, 1, 1, -1, 1, 1, -1, 1], dtype=np.float64)
    Y = SK.sketch(A, np.array([1, 2]), d, prec)
    for (i, j), y in want.items():
        assert Y[i, j] == y, (fmt, i, j, Y[i, j].hex(), y.hex())


def test_rfft_sketch_matches_numpy_rfft():
    """The paper's operator: sqrt(c/m) Re(rfft(D A))[S] (numpy's DFT,
    exp(-2 pi i k t / m) summed over t), bins from {0..m/2}, odd and even m."""
    for m in [1000, 1001]:
        n, c = 7, 21
        A = W.gaussian(m, n, 11)
        S = rng.sample_rows(3, m // 2 + 1, c)
        d = rng.signs(3, m)
        Y = SK.sketch_rfft(A, S, d, P.FP64)
        ref = np.sqrt(c / m) * np.real(np.fft.rfft(d[:, None] * A, axis=0))[S, :]
        assert np.max(np.abs(Y - ref)) <= 1e-12 * np.max(np.abs(ref))


def test_rfft_phase_is_exact_for_large_m():
    m = (1 << 21) + 5
    k = np.array([m // 2, 12345, 1])
    t = np.array([m - 1, 0, 777])
    ph = SK.rfft_phase(k, t, m)
    for i, kk in enumerate(k):
        for j, tt in enumerate(t):
            assert ph[i, j] == (4 * int(tt) * int(kk)) % (4 * m)


@pytest.mark.parametrize("prec", [P.FP32, P.FP16, P.BF16])
def test_low_precision_rfft_sketch_rounds_coefficients(prec):
    # k = 0 gives cos = 1 at every t (exact in every format): Y is
    # sqrt(c/m) times the column sums of fl_p(D A), rounded to float32
    m, n = 512, 3
    A = W.gaussian(m, n, 12)
    d = rng.signs(4, m)
    S = np.array([0, 5, 9])
    Y = SK.sketch_rfft(A, S, d, prec)
    at = SK.signed_cast(A, d, prec)
    assert np.array_equal(Y[0], P.to_f32(np.sqrt(3 / m) * at.sum(axis=0)))
