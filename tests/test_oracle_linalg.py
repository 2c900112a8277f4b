"""Pins of the oracle's Householder QR, Cholesky-QR pieces, ICE and metrics."""
import mpmath
import numpy as np
import pytest
import scipy.linalg

from oracle import householder as HH, cholqr as CQ, condest as CE, metrics as MT
import workloads as W


def _lapack_qr(A):
    q, r = np.linalg.qr(A)
    d = np.sign(np.diag(r))
    d[d == 0] = 1
    return q * d[None, :], r * d[:, None]


@pytest.mark.parametrize("m,n", [(50, 7), (300, 32), (64, 64)])
def test_householder_matches_lapack(m, n):
    A = W.test_matrix(m, n, 1e3, m + n)
    Q, R = HH.householder_qr(A)
    Ql, Rl = _lapack_qr(A)
    assert np.max(np.abs(R - Rl)) < 1e-12 * np.abs(Rl).max()
    assert np.max(np.abs(Q - Ql)) < 1e-10
    assert np.all(np.diag(R) > 0)
    assert MT.orthogonality(Q) < 1e-14


def test_householder_matches_mpmath_gram_schmidt_tiny():
    mpmath.mp.dps = 50
    A = W.gaussian(9, 4, 11)
    M = mpmath.matrix(A.tolist())
    # modified Gram-Schmidt in 50 digits = exact thin QR (diag(R) > 0)
    m, n = A.shape
    Q = [[M[i, j] for i in range(m)] for j in range(n)]
    R = mpmath.matrix(n, n)
    for j in range(n):
        for k in range(j):
            R[k, j] = mpmath.fsum(Q[k][i] * Q[j][i] for i in range(m))
            Q[j] = [Q[j][i] - R[k, j] * Q[k][i] for i in range(m)]
        R[j, j] = mpmath.sqrt(mpmath.fsum(x * x for x in Q[j]))
        Q[j] = [x / R[j, j] for x in Q[j]]
    Rx = np.array([[float(R[i, j]) for j in range(n)] for i in range(n)])
    Qx = np.array([[float(Q[j][i]) for j in range(n)] for i in range(m)])
    Qh, Rh = HH.householder_qr(A)
    assert np.max(np.abs(Rh - Rx)) < 1e-14 * np.abs(Rx).max()
    assert np.max(np.abs(Qh - Qx)) < 1e-14


def test_householder_float32_within_backward_bound():
    A = W.test_matrix(200, 16, 1e2, 3)
    _, R32 = HH.householder_qr(A.astype(np.float32), dtype=np.float32)
    _, R64 = HH.householder_qr(A.astype(np.float32).astype(np.float64))
    assert R32.dtype == np.float32
    rel = np.linalg.norm(R32 - R64) / np.linalg.norm(R64)
    assert rel < 50 * 16 * 2.0 ** -24 * 1e2


def test_householder_zero_column_below_diagonal():
    A = np.zeros((6, 3))
    A[0, 0], A[1, 1], A[2, 2] = -2.0, 3.0, -1.0
    Q, R = HH.householder_qr(A)
    assert np.allclose(R, np.diag([2.0, 3.0, 1.0]))
    assert np.allclose(Q @ R, A)


def test_trsm_matches_scipy():
    A = W.gaussian(500, 20, 5)
    R = W.upper_triangular(20, 1e6, 6)
    X = CQ.trsm_right_upper(A, R)
    ref = scipy.linalg.solve_triangular(R, A.T, trans="T", lower=False).T
    assert np.max(np.abs(X - ref)) < 1e-9 * np.abs(ref).max()
    assert np.max(np.abs(X @ R - A)) < 1e-12 * np.abs(A).max() * 20


def test_upper_inverse_closed_forms():
    # 2 x 2 with dyadic entries: [[a, b], [0, c]]^{-1} = [[1/a, -b/(ac)], [0, 1/c]] exactly
    X = CQ.upper_inverse(np.array([[2.0, 3.0], [0.0, 4.0]]))
    assert np.array_equal(X, np.array([[0.5, -0.375], [0.0, 0.25]]))
    # unit upper bidiagonal with -1 above the diagonal: the inverse is the
    # all-ones upper triangle (x_i = x_{i+1} for every column), exactly
    n = 9
    R = np.eye(n) - np.eye(n, k=1)
    assert np.array_equal(CQ.upper_inverse(R), np.triu(np.ones((n, n))))
    # a diagonal matrix inverts entrywise
    d = np.array([2.0, -4.0, 0.5, 8.0])
    assert np.array_equal(CQ.upper_inverse(np.diag(d)), np.diag(1.0 / d))


def test_upper_inverse_matches_scipy():
    R = W.upper_triangular(40, 1e6, 9)
    X = CQ.upper_inverse(R)
    ref = scipy.linalg.solve_triangular(R, np.eye(40), lower=False)
    assert np.max(np.abs(X - ref)) <= 1e-9 * np.abs(ref).max()
    assert np.array_equal(np.tril(X, -1), np.zeros((40, 40)))
    assert np.max(np.abs(R @ X - np.eye(40))) <= 1e-9


def test_form_q_is_orthogonal_with_inverse_of_cholesky_factor():
    # Algorithm 1 with the inverse applied as a product: for a
    # well-conditioned B the result is orthonormal to working accuracy and
    # agrees with the substitution Q = B Rc^{-1}
    B = W.test_matrix(4000, 24, 10.0, 11)
    Rc = CQ.cholesky_upper(CQ.gram(B))
    Q = CQ.form_q(B, CQ.upper_inverse(Rc))
    assert MT.orthogonality(Q) <= 1e-14
    assert np.max(np.abs(Q - CQ.trsm_right_upper(B, Rc))) <= 1e-14
    # only the upper triangle of X is used
    X = CQ.upper_inverse(Rc)
    assert np.array_equal(CQ.form_q(B, X + np.tril(np.ones_like(X), -1)), Q)


def test_cholesky_matches_numpy():
    G = W.spd_matrix(40, 1e6, 7)
    R = CQ.cholesky_upper(G)
    L = np.linalg.cholesky(G)
    assert np.max(np.abs(R - L.T)) < 1e-12 * np.abs(L).max() * 1e3
    assert np.allclose(np.triu(R), R)


@pytest.mark.parametrize("j", [0, 3, 7])
def test_cholesky_breakdown_index(j):
    G = np.eye(8)
    G[j, j] = -1.0
    with pytest.raises(CQ.CholeskyBreakdown) as e:
        CQ.cholesky_upper(G)
    assert e.value.index == j


def test_cholesky_breakdown_on_exactly_singular_gram():
    # [[4,2,0],[2,1,0],[0,0,1]]: r00 = 2, r01 = 1, second pivot 1 - 1 = 0 exactly
    G = np.array([[4.0, 2.0, 0.0], [2.0, 1.0, 0.0], [0.0, 0.0, 1.0]])
    with pytest.raises(CQ.CholeskyBreakdown) as e:
        CQ.cholesky_upper(G)
    assert e.value.index == 1
    # indefinite: second pivot 1 - 4 = -3
    with pytest.raises(CQ.CholeskyBreakdown) as e:
        CQ.cholesky_upper(np.array([[1.0, 2.0], [2.0, 1.0]]))
    assert e.value.index == 1


def test_trmm_upper():
    R1 = W.upper_triangular(10, 10, 1)
    R2 = W.upper_triangular(10, 10, 2)
    assert np.allclose(CQ.trmm_upper(R1, R2), R1 @ R2)


def test_ice_exact_for_two_by_two_and_diagonal():
    R = np.array([[3.0, -1.5], [0.0, 0.25]])
    sv = np.linalg.svd(R, compute_uv=False)
    assert abs(CE.sigma_max_est(R) - sv[0]) < 1e-14 * sv[0]
    assert abs(CE.sigma_min_est(R) - sv[1]) < 1e-13 * sv[1]
    D = np.diag([5.0, 1e-3, 2.0, 7.0])
    assert abs(CE.kappa_est(D) - 7.0 / 1e-3) < 1e-9


@pytest.mark.parametrize("kappa", [1e2, 1e6, 1e12])
def test_ice_brackets_and_is_close(kappa):
    R = W.upper_triangular(64, kappa, 9)
    sv = np.linalg.svd(R, compute_uv=False)
    smax, smin = CE.sigma_max_est(R), CE.sigma_min_est(R)
    assert smax <= sv[0] * (1 + 1e-12) and smin >= sv[-1] * (1 - 1e-9)
    k = CE.kappa_est(R)
    assert kappa / 30 < k <= (sv[0] / sv[-1]) * (1 + 1e-9)


def test_ice_singular():
    R = np.triu(np.ones((4, 4)))
    R[2, 2] = 0.0
    R[2, 3] = 0.0
    R[3, 3] = 0.0
    assert CE.kappa_est(R) == float("inf") or CE.kappa_est(R) > 1e15


def test_orthogonality_metric_vs_mpmath():
    mpmath.mp.dps = 40
    Q, _ = np.linalg.qr(W.gaussian(30, 3, 12))
    Q[0, 0] += 1e-12
    Qm = mpmath.matrix(Q.tolist())
    E = mpmath.eye(3) - Qm.T * Qm
    ev = mpmath.eigsy(0.5 * (E + E.T))[0]
    ref = max(abs(float(v)) for v in ev)
    assert abs(MT.orthogonality(Q, chunk=7) - ref) < 1e-15


def test_orthogonality_accurate_for_long_columns():
    m = 1 << 19
    u, _, _ = W.test_matrix_factors(m, 4, 1.0, 13)
    assert MT.orthogonality(u) < 5e-15


def test_residual_metric():
    A = W.test_matrix(100, 5, 10.0, 14)
    Q, R = np.linalg.qr(A)
    assert MT.residual(A, Q, R) < 1e-14
    assert abs(MT.residual(A, Q, R * 1.001) - 1e-3 * np.linalg.norm(R, 2) / np.linalg.norm(A, 2)) < 1e-6


def _ice_mpmath(R, largest):
    """ICE with the 2x2 eigenproblem solved by mpmath in 60 digits."""
    mpmath.mp.dps = 60
    n = R.shape[0]
    est = mpmath.mpf(abs(R[0, 0]))
    x = [mpmath.mpf(1)]
    for j in range(1, n):
        alpha = mpmath.fsum(mpmath.mpf(R[i, j]) * x[i] for i in range(j))
        gamma = mpmath.mpf(R[j, j])
        M = mpmath.matrix([[est ** 2 + alpha ** 2, alpha * gamma], [alpha * gamma, gamma ** 2]])
        ev, Q = mpmath.eigsy(M)
        idx = (1 if ev[1] > ev[0] else 0) if largest else (0 if ev[0] < ev[1] else 1)
        s, c = Q[0, idx], Q[1, idx]
        x = [s * xi for xi in x] + [c]
        est = mpmath.sqrt(max(ev[idx], 0))
    return float(est)


@pytest.mark.parametrize("kappa", [1e3, 1e16])
def test_ice_closed_form_matches_high_precision(kappa):
    R = W.upper_triangular(24, kappa, 17)
    for largest in (True, False):
        want = _ice_mpmath(R, largest)
        got = CE._ice(R, largest)
        assert abs(got - want) <= 1e-10 * want


def test_ice_step_eigenpair_definition():
    for est, a, g in [(1.0, 0.3, 2.0), (1e-9, 1.0, 1e-9), (2.0, 0.0, 2.0), (0.5, -3.0, 0.25)]:
        M = np.array([[est * est + a * a, a * g], [a * g, g * g]])
        for largest in (True, False):
            s, c, e2 = CE.ice_step(est, a, g, largest)
            lam = e2 * e2
            v = np.array([s, c])
            assert abs(np.hypot(s, c) - 1) < 1e-15
            assert np.linalg.norm(M @ v - lam * v) <= 1e-14 * max(1.0, np.abs(M).max())


def test_power_norm_exact_on_diagonal_and_rank_one():
    # diagonal: the iteration converges to the largest entry (ratio of the
    # two largest (1/3)^24 after 12 steps); rank one u v^T: exact after one step
    D = np.diag([1.0, 3.0, 0.5, 0.25])
    assert abs(CE.power_norm(D) - 3.0) < 1e-9
    u, v = np.array([1.0, -2.0, 0.5]), np.array([0.3, 0.4, 1.2])
    assert abs(CE.power_norm(np.outer(u, v)) - np.linalg.norm(u) * np.linalg.norm(v)) < 1e-12


@pytest.mark.parametrize("kappa", [2.0, 10.0, 1e3, 1e8])
def test_posterior_estimate_is_a_tight_lower_bound(kappa):
    for seed in range(6):
        R = W.upper_triangular(24, kappa, 40 + seed)
        X = np.linalg.inv(R)
        sv = np.linalg.svd(R, compute_uv=False)
        k2 = sv[0] / sv[-1]
        est = CE.kappa_posterior(R, X)
        assert CE.kappa_est(R) <= est <= k2 * (1 + 1e-10)
        assert est >= 0.6 * k2


def test_cholqr_matches_householder_on_well_conditioned_input():
    A = W.test_matrix(3000, 12, 1e3, 70)
    Q, R = CQ.cholqr2(A)
    Qh, Rh = HH.householder_qr(A)
    assert MT.rel_diff(R, Rh) < 50 * 12 * 2.0 ** -53 * 1e3
    assert np.max(np.abs(Q - Qh)) < 50 * 12 * 2.0 ** -53 * 1e3
    assert MT.orthogonality(Q) < 1e-14


def test_cholqr_single_pass_loses_orthogonality_like_kappa_squared():
    # one pass of Algorithm 1 leaves I - Q^T Q ~ kappa^2 u; the second pass
    # brings it back to ~u (the reason CholQR2 exists)
    A = W.test_matrix(4000, 10, 1e5, 71)
    Q1, _ = CQ.cholqr(A)
    Q2, _ = CQ.cholqr2(A)
    o1, o2 = MT.orthogonality(Q1), MT.orthogonality(Q2)
    assert 1e-9 < o1 < 1e-3
    assert o2 < 1e-14


def test_cholqr2_breaks_down_on_a_numerically_singular_gram():
    # sigma_min^2 / sigma_max^2 = 1e-24 is below the float64 resolution of
    # the Gram matrix: a pivot of the Cholesky factorization is not positive
    A = W.paper_sweep_matrix(2000, 20, 1e12, 72)
    with pytest.raises(CQ.CholeskyBreakdown):
        CQ.cholqr2(A)
    B = W.gaussian(500, 6, 73)
    B[:, 4] = 0.0  # exactly rank deficient: row and pivot 4 of the Gram are zero
    with pytest.raises(CQ.CholeskyBreakdown) as e:
        CQ.cholqr(B)
    assert e.value.index == 4


def test_paper_sweep_matrix_has_the_stated_spectrum():
    A = W.paper_sweep_matrix(4096, 50, 1e10, 74)
    sv = np.linalg.svd(A, compute_uv=False)
    assert abs(sv[0] / 1e5 - 1) < 1e-12 and abs(sv[-1] / 1e-5 - 1) < 1e-5


def test_block_onenorm_estimator_is_exact_on_diagonals_and_a_lower_bound():
    d = np.array([0.5, -7.0, 2.0, 3.0, -1.0])
    D = np.diag(d)
    est = CE.onenorm_est(lambda X: D @ X, lambda X: D.T @ X, 5)
    assert est == 7.0
    import scipy.linalg
    for kappa in [10.0, 1e4, 1e9]:
        for sd in range(8):
            R = W.upper_triangular(30, kappa, 200 + sd)
            Ri = np.linalg.inv(R)
            exact = np.abs(Ri).sum(axis=0).max()
            est = CE.onenorm_est(lambda X: scipy.linalg.solve_triangular(R, X),
                                 lambda X: scipy.linalg.solve_triangular(R, X, trans="T"), 30, seed=sd)
            assert exact / 3 <= est <= exact * (1 + 1e-10)


def test_estimators_bracket_the_condition_number():
    """kappa_1(R) lies in [kappa_2(R)/n, n kappa_2(R)] (norm equivalence) and
    the Gram bound sqrt(n kappa_1(A^T A)) is at least kappa_2(A) when the
    inverse's norm is estimated exactly; the CholQR probe is a lower bound."""
    import scipy.linalg
    m_, n_ = 4096, 20
    for kappa in [1e2, 1e5]:
        A = W.test_matrix(m_, n_, kappa, 300)
        R = CQ.cholesky_upper(A.T @ A)
        k1 = CE.kappa_1norm_tri(R)
        k2 = kappa
        assert k2 / n_ <= k1 <= n_ * k2 * (1 + 1e-6)
        kb = CE.kappa_bound_gram(R)
        assert kb >= 0.5 * k2
        kp = CE.probe_kappa(A)
        assert kp <= k2 * (1 + 1e-6)
    assert CE.probe_kappa(W.paper_sweep_matrix(m_, n_, 1e12, 301)) == float("inf")


def test_probe_power_estimate_is_below_the_exact_one():
    A = W.test_matrix(4096, 16, 1e5, 302)
    assert CE.probe_kappa(A, exact=False) <= CE.probe_kappa(A, exact=True) * (1 + 1e-9)
