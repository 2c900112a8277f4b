"""The largest shapes the library accepts, in the launch configuration the
bench uses: m just below 2^28 (the row limit of the exact integer DCT phase,
4m < 2^32) with a ragged last tile, and the largest sketch (s = 2048 for
n <= 16). Checked on properties and on cheap exact references: with
A = U (Sigma V^T) and Sigma V^T = Qt Rt, R = Rt and Q = U Qt."""
import numpy as np
import pytest

import workloads as W
from oracle import householder as HH, metrics as MT, mrcqr as OM, rng
from gpu_common import require_gpu, to_dev, to_host, progress, torch

pytestmark = pytest.mark.gpu
U64 = 2.0 ** -53
M_MAX = (1 << 28) - 1001


@pytest.fixture(scope="module")
def M():
    return require_gpu()


@pytest.fixture(scope="module")
def tallest():
    n, kappa = 2, 1e3
    progress(f"building A at m={M_MAX}, n={n}")
    U, sig, V = W.test_matrix_factors(M_MAX, n, kappa, 41)
    A = np.asfortranarray((U * sig[None, :]) @ V.T)
    Qt, Rt = HH.householder_qr(sig[:, None] * V.T)
    return A, U, Qt, Rt, kappa


@pytest.mark.parametrize("prec", ["fp16", "fp64"])
def test_max_rows_factor(M, tallest, prec):
    A, U, Qt, Rt, kappa = tallest
    m, n = A.shape
    progress(f"max rows factor {prec}")
    Ad = to_dev(A)
    Q, R, info = M.factor(Ad, prec, seed=8)
    del Ad
    assert info.status == 0, info
    Qh, Rh = to_host(Q), to_host(R)
    del Q
    assert MT.orthogonality(Qh) <= 1e-13
    assert MT.residual(A, Qh, Rh, 1.0) <= 1e-13
    tol = 50 * n * U64 * kappa
    assert MT.rel_diff(Rh, Rt) <= tol
    rows = np.concatenate([[0, 1, m - 2, m - 1], np.random.default_rng(2).choice(m, 508, replace=False)])
    assert np.max(np.abs(Qh[rows] - U[rows] @ Qt)) <= tol


def test_max_rows_draw(M):
    m, s, seed = M_MAX, 2048, 12
    progress("max rows draw")
    assert np.array_equal(to_host(M.draw(seed, m, s)), rng.sample_rows(seed, m, s))


@pytest.mark.parametrize("prec", ["fp32", "fp16", "auto"])
def test_max_sketch_rows(M, prec):
    m, n, s, kappa = 100003, 16, 2048, 1e3
    progress(f"max sketch rows {prec}")
    A = W.test_matrix(m, n, kappa, 43)
    Q, R, info = M.factor(to_dev(A), prec, seed=6, s=s)
    assert info.status == 0, info
    Qh, Rh = to_host(Q), to_host(R)
    Qr, Rr = OM.reference_qr(A)
    tol = 50 * n * U64 * kappa
    assert MT.rel_diff(Rh, Rr) <= tol
    assert np.max(np.abs(Qh - Qr)) <= tol
    with pytest.raises(Exception):
        M.factor(to_dev(A), prec, seed=6, s=s + 1)
