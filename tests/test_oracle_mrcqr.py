"""Pins of the oracle's full MRCQR (Algorithm 2) against facts fixed by the
mathematics: uniqueness of the thin QR, the construction's singular values,
Theorem 1, and the paper's stated precision regimes."""
import json
import os

import numpy as np
import pytest

from oracle import mrcqr as M, precision as P, metrics as MT, householder as HH
from oracle import condest as CE
import workloads as W
from conftest import GOLDEN

CLAIMS = json.load(open(os.path.join(GOLDEN, "paper_claims.json")))
m, n = 4096, 32


@pytest.fixture(scope="module")
def mats():
    return {k: W.test_matrix(m, n, k, 21) for k in [1e2, 1e4, 1e8, 1e12, 1e16]}


@pytest.mark.parametrize("kappa", [1e2, 1e4, 1e8])
def test_fp64_matches_unique_householder_qr(mats, kappa):
    A = mats[kappa]
    r = M.factor(A, P.FP64, seed=1)
    Qh, Rh = M.reference_qr(A)
    tol = 50 * n * 2.0 ** -53 * kappa
    assert MT.rel_diff(r.R, Rh) < tol
    assert np.max(np.abs(r.Q - Qh)) < tol


@pytest.mark.parametrize("kappa", [1e2, 1e4, 1e8, 1e12, 1e16])
def test_fp64_sketch_orthogonality_and_residual(mats, kappa):
    A = mats[kappa]
    r = M.factor(A, P.FP64, seed=2)
    assert r.status == M.STATUS_OK
    assert MT.orthogonality(r.Q) < CLAIMS["orthogonality_fp64_sketch_all_kappa"] * 4
    assert MT.residual(A, r.Q, r.R, 1.0) < CLAIMS["target_residual"]


@pytest.mark.parametrize("prec,kappa", [(P.FP16, 1e2), (P.FP16, 1e4), (P.FP32, 1e4), (P.FP32, 1e8),
                                        (P.BF16, 1e2)])
def test_low_precision_inside_regime(mats, prec, kappa):
    A = mats[kappa]
    r = M.factor(A, prec, seed=3)
    assert r.status == M.STATUS_OK
    assert MT.orthogonality(r.Q) < CLAIMS["target_orthogonality"]
    assert MT.residual(A, r.Q, r.R, 1.0) < CLAIMS["target_residual"]


@pytest.mark.parametrize("prec,kappa", [(P.FP16, 1e8), (P.FP32, 1e12)])
def test_low_precision_outside_regime_degrades_and_is_flagged(mats, prec, kappa):
    A = mats[kappa]
    r = M.factor(A, prec, seed=4)
    if r.Q is None:
        assert r.status in (M.STATUS_CHOL_BREAKDOWN, M.STATUS_SKETCH_SINGULAR)
        return
    assert MT.orthogonality(r.Q) > 1e-12
    assert r.status == M.STATUS_POSTERIOR_WARN
    assert MT.residual(A, r.Q, r.R, 1.0) < 1e-13  # still backward stable


def test_singular_values_of_r_are_the_constructed_ones(mats):
    A = mats[1e4]
    r = M.factor(A, P.FP16, seed=5)
    sv = np.linalg.svd(r.R, compute_uv=False)
    sig = W.singular_values(n, 1e4)
    assert np.max(np.abs(sv - sig)) < 100 * n * 2.0 ** -53


def test_kappa_one_gives_identity_r():
    U, _, _ = W.test_matrix_factors(2048, 16, 1.0, 6)
    r = M.factor(U, P.FP32, seed=7)
    assert np.max(np.abs(r.R - np.eye(16))) < 1e-14
    assert np.max(np.abs(r.Q - U)) < 1e-14


@pytest.mark.parametrize("prec", [P.FP64, P.FP32])
def test_power_of_two_scaling_is_exact(mats, prec):
    A = mats[1e4]
    r1 = M.factor(A, prec, seed=8)
    r2 = M.factor(A * 2.0 ** 37, prec, seed=8)
    assert np.array_equal(r2.R, r1.R * 2.0 ** 37)
    assert np.array_equal(r2.Q, r1.Q)


def test_seed_and_precision_invariance(mats):
    A = mats[1e4]
    Rs = [M.factor(A, p, seed=sd).R for p, sd in [(P.FP64, 1), (P.FP64, 99), (P.FP16, 5), (P.FP32, 6)]]
    for R in Rs[1:]:
        assert MT.rel_diff(R, Rs[0]) < 1e-11


def _cond(X):
    sv = np.linalg.svd(X, compute_uv=False)
    return sv[0] / sv[-1]


def _theorem1_terms(A, prec):
    _, _, _, Rs = M.stage1(A, P.FP64, 9, 2 * n)
    _, _, _, Rh = M.stage1(A, prec, 9, 2 * n)
    k_rs = _cond(Rs)
    eps = np.linalg.norm(Rh - Rs, 2) / np.linalg.norm(Rs, 2)
    k_hat = _cond(np.linalg.solve(Rh.T, A.T).T)
    k_one = _cond(np.linalg.solve(Rs.T, A.T).T)
    return eps * k_rs, k_hat, k_one


@pytest.mark.parametrize("prec,kappa", [(P.FP16, 1e2), (P.FP16, 1e3), (P.FP32, 1e4), (P.FP32, 1e6),
                                        (P.BF16, 1e2)])
def test_theorem1_bound_holds(prec, kappa):
    # Theorem 1: with E = Rs_hat - Rs and eps = ||E|| / ||Rs||, if eps*kappa(Rs) < 1
    # then kappa(A Rs_hat^-1) <= kappa(A Rs^-1) (1 + eps k) / (1 - eps k).
    A = W.test_matrix(m, n, kappa, 21)
    ek, k_hat, k_one = _theorem1_terms(A, prec)
    assert ek < 1
    assert k_hat <= k_one * (1 + ek) / (1 - ek) * (1 + 1e-6)
    assert k_hat < 50


def test_theorem1_is_sufficient_not_necessary_at_fp16_edge(mats):
    # at the paper's FP16 regime bound (1e4) the hypothesis eps*kappa < 1 fails,
    # yet the preconditioned matrix stays well conditioned
    ek, k_hat, _ = _theorem1_terms(mats[1e4], P.FP16)
    assert ek > 1
    assert k_hat < 50


def test_preconditioned_matrix_is_well_conditioned(mats):
    A = mats[1e12]
    _, _, _, Rs = M.stage1(A, P.FP64, 10, 2 * n)
    sv = np.linalg.svd(np.linalg.solve(Rs.T, A.T).T, compute_uv=False)
    assert sv[0] / sv[-1] < 20  # about (1 + sqrt(1/2)) / (1 - sqrt(1/2)) = 5.8 for s = 2n


def test_all_rows_sketch_gives_exact_r():
    # s = m: the sketch operator is orthogonal, so Rs = R(A) and R2 = I
    A = W.test_matrix(256, 8, 1e6, 11)
    r = M.factor(A, P.FP64, seed=12, s=256, keep=True)
    _, Rh = HH.householder_qr(A)
    assert MT.rel_diff(r.intermediates["Rs"], Rh) < 1e-9
    assert np.max(np.abs(r.intermediates["Rc"] - np.eye(8))) < 1e-9


@pytest.mark.parametrize("kappa,expect", [(1e2, P.FP16), (1e8, P.FP32), (1e16, P.FP64)])
def test_auto_policy_lands_in_the_papers_regime(mats, kappa, expect):
    A = mats[kappa]
    r = M.factor(A, M.AUTO, seed=13)
    assert r.status == M.STATUS_OK
    assert r.precision_used == expect
    assert MT.orthogonality(r.Q) < CLAIMS["target_orthogonality"]


def test_zero_column_gives_singular_sketch():
    A = W.gaussian(512, 6, 14)
    A[:, 3] = 0.0
    for prec in [P.FP64, P.FP16]:
        r = M.factor(A, prec, seed=15)
        assert r.status == M.STATUS_SKETCH_SINGULAR and r.Q is None


def test_numerically_rank_deficient_input_still_backward_stable():
    # a duplicated column leaves Rs with a pivot at rounding level; the result
    # is a backward-stable QR with orthonormal Q (as Householder QR would give)
    A = W.gaussian(512, 6, 14)
    A[:, 5] = A[:, 2]
    r = M.factor(A, P.FP64, seed=15)
    assert r.kappa_rs > 1e14
    if r.Q is not None:
        assert MT.orthogonality(r.Q) < 1e-13
        assert MT.residual(A, r.Q, r.R) < 1e-14


def test_ice_estimate_tracks_kappa_of_sketch_factor(mats):
    for kappa in [1e2, 1e4, 1e8]:
        _, _, _, Rs = M.stage1(mats[kappa], P.FP64, 16, 2 * n)
        k = CE.kappa_est(Rs)
        assert kappa / 20 < k <= kappa * 1.01


@pytest.mark.parametrize("start", [P.FP32, P.FP64])
def test_auto_started_higher_never_goes_below_its_start(mats, start):
    """Repeated calls start AUTO from the precision the previous call
    accepted: started at p on an easy matrix, it stays at p with no
    escalation and reproduces the factorization forced to p exactly (the
    AUTO branch against the fixed-precision branch)."""
    A = mats[1e2]
    r = M.factor(A, M.AUTO, seed=13, start=start)
    f = M.factor(A, start, seed=13)
    assert (r.status, r.precision_used, r.escalations) == (M.STATUS_OK, start, 0)
    assert np.array_equal(r.Q, f.Q) and np.array_equal(r.R, f.R)


def test_auto_escalation_from_a_carried_start_matches_a_fresh_one(mats):
    """Started at FP16 on a kappa = 1e8 matrix AUTO escalates to FP32; started
    at FP32 it lands there directly with the same result."""
    A = mats[1e8]
    a = M.factor(A, M.AUTO, seed=13)
    b = M.factor(A, M.AUTO, seed=13, start=P.FP32)
    assert a.precision_used == b.precision_used == P.FP32
    assert a.escalations == 1 and b.escalations == 0
    assert np.array_equal(a.Q, b.Q) and np.array_equal(a.R, b.R)


def _lapack_r(Y, dtype):
    import scipy.linalg
    R = scipy.linalg.qr(np.asarray(Y, dtype=dtype), mode="r")[0][: Y.shape[1]]
    d = np.sign(np.diag(R))
    d[d == 0] = 1
    return np.triu(R * d[:, None]).astype(np.float64)


@pytest.mark.parametrize("prec,kappa", [(P.FP16, 1e2), (P.FP16, 1e4), (P.BF16, 1e2), (P.FP32, 1e4),
                                        (P.FP32, 1e8)])
def test_sketch_qr_runs_in_single_precision(mats, prec, kappa):
    """Section "Algorithm Description": the sketch QR of a half, bfloat16 or
    single sketch is a single-precision QR (no half QR exists). Rs is then a
    float32 value before its promotion, and agrees with float32 LAPACK
    (sgeqrf, through scipy) within c n u32 kappa."""
    _, _, Y, Rs = M.stage1(mats[kappa], prec, 17, 2 * n)
    assert np.array_equal(Rs.astype(np.float32).astype(np.float64), Rs)
    Rl = _lapack_r(Y, np.float32)
    k = np.linalg.cond(Y)
    assert MT.rel_diff(Rs, Rl) <= 20 * n * 2.0 ** -24 * k


def test_fp64_sketch_qr_runs_in_double_precision(mats):
    _, _, Y, Rs = M.stage1(mats[1e8], P.FP64, 17, 2 * n)
    assert not np.array_equal(Rs.astype(np.float32).astype(np.float64), Rs)
    assert MT.rel_diff(Rs, _lapack_r(Y, np.float64)) <= 20 * n * 2.0 ** -53 * 1e8


def test_posterior_bound_keeps_orthogonality_within_target():
    """The posterior bound tau_c on kappa(Rc) = kappa(A Rs^-1): Cholesky-QR
    loses orthogonality like kappa^2 u, so tau_c^2 u must stay below the
    paper's 1e-13 target."""
    assert M.TAU_POSTERIOR ** 2 * 2.0 ** -53 <= CLAIMS["target_orthogonality"]


@pytest.mark.parametrize("s,seed", [(17, 0), (18, 26)])
def test_posterior_check_reruns_up_the_ladder(s, seed):
    """A sketch with barely more rows than columns leaves kappa(Rc) between
    tau_c = 20 and 30 at every precision (the draw, not the precision, is
    the cause): AUTO reruns at FP32, then at FP64, and reports the posterior
    warning (Section "Adaptive Precision Selection": rerun at the next
    higher level)."""
    A = W.test_matrix(2048, 16, 1e2, 3)
    r = M.factor(A, M.AUTO, seed, s=s)
    assert 20.0 < r.kappa_rc < 30.0
    assert (r.status, r.precision_used, r.escalations) == (M.STATUS_POSTERIOR_WARN, P.FP64, 2)
    f = M.factor(A, P.FP16, seed, s=s)
    assert f.status == M.STATUS_POSTERIOR_WARN and 20.0 < f.kappa_rc < 30.0


def test_accepted_results_meet_the_target_and_estimate_is_tight():
    """Every result the policy accepts (status 0) meets ||I - Q^T Q|| <= 1e-13,
    including sketches barely taller than n where kappa(Rc) is large, and the
    posterior estimate is within a factor 0.6 of kappa_2(Rc)."""
    m_, n_ = 2048, 16
    accepted = 0
    for kappa in [1e2, 1e4, 1e8]:
        A = W.test_matrix(m_, n_, kappa, 3)
        for s in [17, 20, 32]:
            for prec in [P.FP16, P.FP32, P.FP64]:
                for seed in range(6):
                    r = M.factor(A, prec, seed, s=s, keep=True)
                    if "Rc" not in r.intermediates:
                        continue
                    sv = np.linalg.svd(r.intermediates["Rc"], compute_uv=False)
                    assert r.kappa_rc >= 0.6 * sv[0] / sv[-1]
                    if r.status == M.STATUS_OK:
                        accepted += 1
                        assert MT.orthogonality(r.Q) <= CLAIMS["target_orthogonality"]
    assert accepted > 50


@pytest.mark.parametrize("prec,kappa", [(P.FP64, 1e8), (P.FP32, 1e6), (P.FP16, 1e3)])
def test_rfft_sketch_gives_the_unique_qr(mats, prec, kappa):
    """With the paper's operator (real DFT bins, c = 3n) the factorization is
    the same unique thin QR."""
    A = mats[kappa] if kappa in mats else W.test_matrix(m, n, kappa, 21)
    r = M.factor(A, prec, seed=31, transform=M.RFFT)
    assert r.status == M.STATUS_OK
    Qh, Rh = M.reference_qr(A)
    assert MT.rel_diff(r.R, Rh) < 50 * n * 2.0 ** -53 * kappa
    assert MT.orthogonality(r.Q) < CLAIMS["target_orthogonality"]
