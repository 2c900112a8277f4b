"""Column counts 128 < n <= 512 (the column-panel path): each step against
the oracle, the whole factorization against the unique thin QR in every
precision and with AUTO, and full-size runs at m = 2^20.

The reference QR of A = U (Sigma V^T) is R = Rt, Q = U Qt with Sigma V^T =
Qt Rt (an n x n Householder QR), exact up to the rounding of A."""
import numpy as np
import pytest

import workloads as W
from oracle import cholqr as CQ, condest as CE, householder as HH, metrics as MT, mrcqr as OM, precision as P
from oracle import rng, sketch as SK
from gpu_common import require_gpu, to_dev, to_host, progress, torch, _chunked_gram_dev

pytestmark = pytest.mark.gpu
U64 = 2.0 ** -53


@pytest.fixture(scope="module")
def M():
    return require_gpu()


_REF = {}


def _problem(m, n, kappa, seed):
    key = (m, n, kappa, seed)
    if key not in _REF:
        U, sig, V = W.test_matrix_factors(m, n, kappa, seed)
        A = np.asfortranarray((U * sig[None, :]) @ V.T)
        Qt, Rt = HH.householder_qr(sig[:, None] * V.T)
        _REF[key] = (A, U, Qt, Rt)
    return _REF[key]


U32 = 2.0 ** -24
SKETCH_TOL = {P.FP64: 2e-12, P.FP32: 200 * U32, P.FP16: 2e-5, P.BF16: 1.6e-4}


# m = 2^14 gives 256 row chunks, so the sketch-row blocks (s / 256 of them)
# that share rows of A run on one XCD (the remapped grid); m = 5003 keeps
# the plain grid
@pytest.mark.parametrize("prec", [P.FP64, P.FP32, P.FP16, P.BF16])
@pytest.mark.parametrize("m,n", [(16384, 512), (16384, 256), (5003, 300)])
def test_wide_sketch_matches_definition(M, prec, m, n):
    s, seed = 2 * n, 3 + n
    progress(f"wide sketch {P.NAMES[prec]} m={m} n={n} s={s}")
    A = W.test_matrix(m, n, 1e4, 2)
    S = rng.sample_rows(seed, m, s)
    d = rng.signs(seed, m)
    Y = to_host(M.sketch(to_dev(A), torch.from_numpy(S.astype(np.int32)).cuda(), seed, P.NAMES[prec]))
    Yo = SK.sketch(A, S, d, prec)
    bound = SK.sketch_abs_bound(A, S, d, prec)
    err = np.abs(Y - Yo) - (SKETCH_TOL[prec] * bound + (U32 * np.abs(Yo) if prec != P.FP64 else 0))
    assert np.max(err) <= 0, f"max excess {np.max(err):.3e}"


# the paper's real-DFT operator at n > 128 (c = 3n = 768 bins from
# {0..m/2}, three sketch-row blocks; m = 2^14 takes the remapped grid)
@pytest.mark.parametrize("prec", [P.FP64, P.FP16])
@pytest.mark.parametrize("m,n", [(16384, 256), (5003, 200)])
def test_wide_rfft_sketch_matches_definition(M, prec, m, n):
    c, seed = 3 * n, 9 + n
    progress(f"wide rfft sketch {P.NAMES[prec]} m={m} n={n} c={c}")
    A = W.test_matrix(m, n, 1e4, 6)
    S = rng.sample_rows(seed, m // 2 + 1, c)
    d = rng.signs(seed, m)
    Y = to_host(M.sketch(to_dev(A), torch.from_numpy(S.astype(np.int32)).cuda(), seed, P.NAMES[prec],
                         transform="rfft"))
    Yo = SK.sketch_rfft(A, S, d, prec)
    bound = SK.sketch_rfft_abs_bound(A, S, d, prec)
    err = np.abs(Y - Yo) - (SKETCH_TOL[prec] * bound + (U32 * np.abs(Yo) if prec != P.FP64 else 0))
    assert np.max(err) <= 0, f"max excess {np.max(err):.3e}"


@pytest.mark.parametrize("prec", ["fp16", "fp64", "auto"])
def test_wide_rfft_factor_matches_unique_qr(M, prec):
    m, n, kappa = 4099, 256, 1e3
    A, U, Qt, Rt = _problem(m, n, kappa, 50 + n)
    progress(f"wide rfft factor {prec}")
    plan = M.Plan(m, n, transform="rfft")
    Q, R = M.empty_colmajor(m, n), M.empty_colmajor(n, n)
    plan.execute(to_dev(A), Q, R, prec, seed=3)
    torch.cuda.synchronize()
    info = plan.last_info()
    o = OM.factor(A, {"fp16": P.FP16, "fp64": P.FP64, "auto": OM.AUTO}[prec], 3, transform=OM.RFFT)
    assert (info.status, info.precision_used, info.escalations) == (o.status, o.precision_used, o.escalations)
    assert info.status == 0, info
    Qh, Rh = to_host(Q), to_host(R)
    assert MT.orthogonality(Qh) <= 1e-13 and MT.residual(A, Qh, Rh, 1.0) <= 1e-13
    assert MT.rel_diff(Rh, Rt) <= 50 * n * U64 * kappa


@pytest.mark.parametrize("m,n,kappa", [(3001, 256, 1e6), (1200, 200, 1e4), (5003, 512, 1e8)])
def test_wide_trsm_matches_substitution(M, m, n, kappa):
    progress(f"wide trsm m={m} n={n} kappa={kappa:g}")
    A = W.gaussian(m, n, 31)
    R = W.upper_triangular(n, kappa, 32 + n)
    X = to_host(M.trsm(to_dev(A), to_dev(R)))
    Xo = CQ.trsm_right_upper(A, R)
    assert np.linalg.norm(X - Xo) / np.linalg.norm(Xo) <= 10 * n * U64 * kappa
    res = np.abs(X @ R - A)
    assert np.max(res) <= 4 * n * U64 * np.max(np.abs(X) @ np.abs(R))


@pytest.mark.parametrize("m,n", [(3001, 256), (1000, 200), (4099, 512)])
def test_wide_gram_matches_definition(M, m, n):
    progress(f"wide gram m={m} n={n}")
    B = W.gaussian(m, n, 33)
    G = to_host(M.gram(to_dev(B)))
    Go = B.T @ B
    bound = np.abs(B).T @ np.abs(B)
    chain = 1 + min(m, 4096) / 4 + 512
    assert np.all(np.abs(G - Go) <= 2 * chain * U64 * bound)
    assert np.array_equal(G, G.T)


@pytest.mark.parametrize("n,kappa", [(256, 1e4), (512, 1e8), (300, 10.0)])
def test_wide_small_steps(M, n, kappa):
    """X = R^{-1}, R2 R1 and the posterior power estimate for n > 128."""
    progress(f"wide small steps n={n}")
    R = W.upper_triangular(n, kappa, 40 + n)
    R2 = W.upper_triangular(n, 10.0, 41 + n)
    X = to_host(M.tri_inverse(to_dev(R)))
    Xo = CQ.upper_inverse(R)
    assert np.linalg.norm(X - Xo) / np.linalg.norm(Xo) <= 10 * n * U64 * kappa
    assert np.all(np.tril(X, -1) == 0)
    P2 = to_host(M.trmm(to_dev(R2), to_dev(R)))
    assert np.max(np.abs(P2 - CQ.trmm_upper(R2, R))) <= 4 * n * U64 * np.max(np.abs(R2) @ np.abs(R))
    k = float(to_host(M.posterior_kappa(to_dev(R2), to_dev(CQ.upper_inverse(R2))))[0])
    ko = CE.power_norm(R2) * CE.power_norm(CQ.upper_inverse(R2))
    assert abs(k - ko) <= 1e-10 * ko


@pytest.mark.parametrize("m,n", [(3001, 256), (2000, 512)])
def test_wide_form_q(M, m, n):
    progress(f"wide form_q m={m} n={n}")
    B = W.gaussian(m, n, 35)
    Rc = W.upper_triangular(n, 10.0, 36)
    X = CQ.upper_inverse(Rc)
    Q = to_host(M.form_q(to_dev(B), to_dev(X)))
    Qo = B @ X
    assert np.max(np.abs(Q - Qo)) <= 4 * n * U64 * np.max(np.abs(B) @ np.abs(X))


# kappa inside every precision's regime, so that each returns the unique QR
@pytest.mark.parametrize("m,n", [(2301, 256), (4099, 512), (1500, 200)])
@pytest.mark.parametrize("prec", ["fp64", "fp32", "fp16", "auto"])
def test_wide_factor_matches_unique_qr(M, m, n, prec):
    kappa = 1e3
    A, U, Qt, Rt = _problem(m, n, kappa, 50 + n)
    progress(f"wide factor m={m} n={n} {prec}")
    Q, R, info = M.factor(to_dev(A), prec, seed=7)
    assert info.status == 0, info
    Qh, Rh = to_host(Q), to_host(R)
    assert MT.orthogonality(Qh) <= 1e-13
    assert MT.residual(A, Qh, Rh, 1.0) <= 1e-13
    tol = 50 * n * U64 * kappa
    assert MT.rel_diff(Rh, Rt) <= tol
    assert np.max(np.abs(Qh - U @ Qt)) <= tol
    assert np.all(np.tril(Rh, -1) == 0) and np.all(np.diag(Rh) > 0)
    if prec == "auto":
        assert info.precision == "fp16" and info.escalations == 0


# edges of the column-panel path: n just above 128, ragged last panels
# (n = 129, 300, 511), the sketch as tall as A (s = 2n = m), few row chunks
@pytest.mark.parametrize("m,n", [(258, 129), (600, 300), (1100, 511), (5000, 129)])
@pytest.mark.parametrize("prec", ["fp64", "fp16"])
def test_wide_edge_shapes(M, m, n, prec):
    kappa = 1e2
    A, U, Qt, Rt = _problem(m, n, kappa, 60 + n)
    progress(f"wide edge m={m} n={n} {prec}")
    Q, R, info = M.factor(to_dev(A), prec, seed=5)
    assert info.status == 0, info
    Qh, Rh = to_host(Q), to_host(R)
    assert MT.orthogonality(Qh) <= 1e-13
    assert MT.residual(A, Qh, Rh, 1.0) <= 1e-13
    assert MT.rel_diff(Rh, Rt) <= 50 * n * U64 * kappa
    assert np.all(np.tril(Rh, -1) == 0) and np.all(np.diag(Rh) > 0)


def test_wide_auto_escalates_like_the_oracle(M):
    """kappa = 1e6 at n = 256: the FP16 attempt's condition estimate on the
    blocked Householder factor crosses 1e4 and AUTO lands on FP32, as the
    oracle's AUTO does on the same matrix and seed."""
    m, n, kappa = 2048, 256, 1e6
    A, U, Qt, Rt = _problem(m, n, kappa, 77)
    Q, R, info = M.factor(to_dev(A), "auto", seed=9)
    o = OM.factor(A, OM.AUTO, seed=9)
    progress(f"wide auto: gpu {info.precision} esc {info.escalations}, oracle {P.NAMES[o.precision_used]} "
             f"esc {o.escalations}")
    assert info.status == 0 and o.status == 0
    assert info.precision == P.NAMES[o.precision_used]
    assert info.precision == "fp32"
    Qh, Rh = to_host(Q), to_host(R)
    assert MT.orthogonality(Qh) <= 1e-13
    assert MT.rel_diff(Rh, Rt) <= 50 * n * U64 * kappa


@pytest.mark.parametrize("s,seed", [(201, 0), (204, 2)])
def test_wide_posterior_rerun_ladder_matches_oracle(M, s, seed):
    """n = 200 with a sketch barely taller than n: kappa(Rc) stays above the
    posterior bound at every precision, so AUTO reruns the column-panel pass
    at FP32, then FP64, and reports the posterior warning, as the oracle
    does."""
    A = W.test_matrix(2048, 200, 1e2, 3)
    progress(f"wide posterior ladder s={s} seed={seed}")
    Q, R, info = M.factor(to_dev(A), "auto", seed=seed, s=s)
    o = OM.factor(A, OM.AUTO, seed, s=s)
    assert (info.status, info.precision, info.escalations) == (o.status, "fp64", 2), (info, o.status)
    assert abs(info.kappa_rc_est - o.kappa_rc) <= 1e-4 * o.kappa_rc
    assert MT.residual(A, to_host(Q), to_host(R), 1.0) <= 1e-13


def test_wide_fp64_sketch_factor_and_estimate_match_the_oracle(M):
    """FP64 sketch at n = 512, kappa = 1e12: the blocked Householder factor's
    condition estimate (ICE on Rs, kappa_rs_est) against the oracle's ICE on
    its own float64 sketch factor, and the unique QR."""
    m, n, kappa = 4099, 512, 1e12
    A, U, Qt, Rt = _problem(m, n, kappa, 78)
    Q, R, info = M.factor(to_dev(A), "auto", seed=4)
    assert info.status == 0 and info.precision == "fp64", info
    Rs = OM.stage1(A, P.FP64, 4, 2 * n)[3]
    k_oracle = CE.kappa_est(Rs)
    progress(f"wide fp64: kappa_rs_est {info.kappa_rs_est:.4g} oracle {k_oracle:.4g}")
    assert abs(info.kappa_rs_est - k_oracle) <= 1e-3 * k_oracle
    Qh, Rh = to_host(Q), to_host(R)
    assert MT.orthogonality(Qh) <= 1e-13
    assert MT.residual(A, Qh, Rh, 1.0) <= 1e-13
    assert MT.rel_diff(Rh, Rt) <= 50 * n * U64 * kappa


@pytest.mark.parametrize("n", [256, 512])
@pytest.mark.parametrize("prec", ["fp16", "fp64"])
def test_wide_full_size(M, n, prec):
    """m = 2^20: orthogonality and backward error on the GPU (chunked float64
    Gram of Q and of A - QR), R against the n x n reference."""
    m, kappa = 1 << 20, 1e3
    progress(f"wide full size n={n} {prec}")
    U, sig, V = W.test_matrix_factors(m, n, kappa, 90 + n)
    Ud = to_dev(U)
    SV = sig[:, None] * V.T
    # (SV^T U^T)^T: the column-major product U SV on the device
    Ad = (to_dev(SV).t() @ Ud.t()).t()
    Qt, Rt = HH.householder_qr(SV)
    Q, R, info = M.factor(Ad, prec, seed=6)
    assert info.status == 0, info
    Gq = _chunked_gram_dev(Q)
    orth = float(np.max(np.abs(np.linalg.eigvalsh(np.eye(n) - Gq))))
    E = Ad - Q @ R
    res = float(np.sqrt(np.max(np.linalg.eigvalsh(_chunked_gram_dev(E)))))
    progress(f"wide full size n={n} {prec}: orth {orth:.2e} res {res:.2e}")
    assert orth <= 1e-13 and res <= 1e-13
    assert MT.rel_diff(to_host(R), Rt) <= 50 * n * U64 * kappa
