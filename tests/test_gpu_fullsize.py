"""Full-size checks at m = 2^20, n = 128, s = 256 (the headline shape) in the
launch configuration the bench times, on properties and sampled outputs:
A = U (Sigma V^T) and Sigma V^T = Qt Rt give R = Rt and Q = U Qt exactly,
so R and sampled rows of Q have a cheap reference."""
import numpy as np
import pytest

import workloads as W
from oracle import cholqr as CQ, householder as HH, metrics as MT, mrcqr as OM, precision as P, rng, sketch as SK
from gpu_common import require_gpu, to_dev, to_host, progress, torch

U32 = 2.0 ** -24
# same bounds as the small-size sketch parity test
SKETCH_TOL = {P.FP64: 2e-12, P.FP32: 200 * U32, P.FP16: 2e-5, P.BF16: 1.6e-4}

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def M():
    return require_gpu()


@pytest.fixture(scope="module")
def big():
    m, n, kappa = 1 << 20, 128, 1e4
    U, sig, V = W.test_matrix_factors(m, n, kappa, 11)
    A = np.asfortranarray((U * sig[None, :]) @ V.T)
    Qt, Rt = HH.householder_qr((sig[:, None] * V.T))
    return A, U, Qt, Rt, kappa


@pytest.mark.parametrize("prec", ["fp16", "fp64"])
def test_headline_shape(M, big, prec):
    A, U, Qt, Rt, kappa = big
    m, n = A.shape
    progress(f"full size {prec}")
    Q, R, info = M.factor(to_dev(A), prec, seed=3)
    assert info.status == 0, info
    Qh, Rh = to_host(Q), to_host(R)
    assert MT.orthogonality(Qh) <= 1e-13
    assert MT.residual(A, Qh, Rh, 1.0) <= 1e-13
    tol = 50 * n * 2.0 ** -53 * kappa
    assert MT.rel_diff(Rh, Rt) <= tol
    rows = np.random.default_rng(0).choice(m, 512, replace=False)
    assert np.max(np.abs(Qh[rows] - U[rows] @ Qt)) <= tol


@pytest.mark.parametrize("prec,name", [(P.FP16, "fp16"), (P.BF16, "bf16"), (P.FP32, "fp32"), (P.FP64, "fp64")])
def test_headline_sketch_all_rows(M, big, prec, name):
    """Full-size sketch in the bench's launch configuration: all s = 256
    sampled rows against the oracle, elementwise, in every precision (each
    row chunk holds 64 panels, so the coefficient re-seeding every 8 panels
    of the half-width sketches is exercised throughout)."""
    A = big[0]
    m, n = A.shape
    s, seed = 2 * n, 5
    progress(f"full size sketch {name}")
    S = rng.sample_rows(seed, m, s)
    assert np.array_equal(to_host(M.draw(seed, m, s)), S)
    Y = to_host(M.sketch(to_dev(A), torch.from_numpy(S.astype(np.int32)).cuda(), seed, name))
    d = rng.signs(seed, m)
    Yo = SK.sketch(A, S, d, prec, s_total=s)
    bound = SK.sketch_abs_bound(A, S, d, prec, s_total=s)
    tol = SKETCH_TOL[prec] * bound + (U32 * np.abs(Yo) if prec != P.FP64 else 0)
    err = np.abs(Y - Yo)
    assert np.all(err <= tol), (np.unravel_index(np.argmax(err - tol), err.shape), float(np.max(err / bound)))


def test_headline_shape_auto(M, big):
    """AUTO at the headline shape (kappa = 1e4, the edge of the half regime)
    lands where the oracle's AUTO lands on the same seed, with the same
    escalations and estimates."""
    A, U, Qt, Rt, kappa = big
    progress("full size auto")
    Q, R, info = M.factor(to_dev(A), "auto", seed=4)
    assert info.status == 0, info
    Qh, Rh = to_host(Q), to_host(R)
    assert MT.orthogonality(Qh) <= 1e-13
    assert MT.residual(A, Qh, Rh, 1.0) <= 1e-13
    progress("full size auto: oracle")
    o = OM.factor(A, OM.AUTO, seed=4)
    assert (info.status, info.precision_used, info.escalations) == (o.status, o.precision_used, o.escalations), o
    # the two float32 sketch QRs round differently (about n u32 kappa apart)
    assert abs(info.kappa_rs_est - o.kappa_rs) <= 1e-3 * o.kappa_rs
    assert info.precision == "fp16", info


def test_headline_solve_and_form_q_sampled_rows(M, big):
    """B = A R^{-1} and Q = B X at the full size in the bench's launch
    configuration; 512 sampled rows (first and last included) against the
    oracle's substitution and product."""
    A = big[0]
    m, n = A.shape
    progress("full size trsm + form_q")
    R = W.upper_triangular(n, 1e4, 31)
    X = W.upper_triangular(n, 30.0, 32)
    B = M.trsm(to_dev(A), to_dev(R))
    Q = M.form_q(B, to_dev(X))
    rows = np.concatenate([[0, m - 1], np.random.default_rng(1).choice(np.arange(1, m - 1), 510, replace=False)])
    ridx = torch.from_numpy(rows).cuda()
    Bh, Qh = to_host(B[ridx]), to_host(Q[ridx])
    Bo = CQ.trsm_right_upper(A[rows], R)
    assert np.linalg.norm(Bh - Bo) / np.linalg.norm(Bo) <= 10 * n * 2.0 ** -53 * 1e4
    assert np.all(np.abs(Qh - CQ.form_q(Bh, X)) <= 2 * n * 2.0 ** -53 * (np.abs(Bh) @ np.abs(X)))
