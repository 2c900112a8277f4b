"""GPU parity of each step of the path against the CPU oracle on the same
seeded inputs (Algorithm 2 stages; element by element with tolerances
derived from the arithmetic of each step)."""
import numpy as np
import pytest

import workloads as W
from oracle import rng, sketch as SK, precision as P, householder as HH, cholqr as CQ, condest as CE
from gpu_common import require_gpu, to_dev, to_host, progress, torch

pytestmark = pytest.mark.gpu
U32 = 2.0 ** -24
U64 = 2.0 ** -53


@pytest.fixture(scope="module")
def M():
    return require_gpu()


@pytest.mark.parametrize("seed,m,s", [(0, 4096, 64), (7, 5000, 48), (123, 1 << 20, 256), (5, 300, 300),
                                      (9, 100, 64), (11, 1 << 21, 2048), (3, 17, 1)])
def test_draw_bit_exact(M, seed, m, s):
    progress(f"draw seed={seed} m={m} s={s}")
    S, D = M.draw(seed, m, s, signs=True)
    torch.cuda.synchronize()
    assert np.array_equal(to_host(S).astype(np.int64), rng.sample_rows(seed, m, s))
    assert np.array_equal(to_host(D).astype(np.float64), rng.signs(seed, m))


SKETCH_TOL = {P.FP64: 2e-12, P.FP32: 200 * U32, P.FP16: 2e-5, P.BF16: 1.6e-4}
NAMES = {P.FP64: "fp64", P.FP32: "fp32", P.FP16: "fp16", P.BF16: "bf16"}


@pytest.mark.parametrize("prec", [P.FP64, P.FP32, P.FP16, P.BF16])
@pytest.mark.parametrize("m,n,s,kind", [(4096, 32, 64, "test"), (5003, 20, 48, "gauss"),
                                        (70001, 128, 256, "test"), (200, 130 // 2, 130, "gauss")])
def test_sketch_matches_definition(M, prec, m, n, s, kind):
    progress(f"sketch {NAMES[prec]} m={m} n={n} s={s}")
    seed = 31 + m
    A = W.test_matrix(m, n, 1e4, 1) if kind == "test" else W.gaussian(m, n, 2) * 1e-3
    S = rng.sample_rows(seed, m, s)
    d = rng.signs(seed, m)
    Ydev = M.sketch(to_dev(A), torch.from_numpy(S.astype(np.int32)).cuda(), seed, NAMES[prec])
    Y = to_host(Ydev)
    Yo = SK.sketch(A, S, d, prec)
    bound = SK.sketch_abs_bound(A, S, d, prec)
    err = np.abs(Y - Yo) - (SKETCH_TOL[prec] * bound + (U32 * np.abs(Yo) if prec != P.FP64 else 0))
    assert np.max(err) <= 0, f"max excess {np.max(err):.3e}, max rel {np.max(np.abs(Y - Yo) / bound):.3e}"
    if prec != P.FP64:
        assert np.array_equal(Y, Y.astype(np.float32).astype(np.float64))  # float32 values


@pytest.mark.parametrize("prec", [P.FP64, P.FP32, P.FP16, P.BF16])
@pytest.mark.parametrize("m,n,c", [(4096, 32, 96), (5003, 20, 60), (70001, 128, 384), (1 << 20, 64, 192),
                                   (401, 50, 150)])
def test_rfft_sketch_matches_definition(M, prec, m, n, c):
    """The paper's operator (real parts of DFT bins from {0..m/2}, scale
    sqrt(c/m)) on the same MFMA contraction, element by element."""
    progress(f"rfft sketch {NAMES[prec]} m={m} n={n} c={c}")
    seed = 77 + m
    A = W.test_matrix(m, n, 1e4, 5)
    S = rng.sample_rows(seed, m // 2 + 1, c)
    assert np.array_equal(to_host(M.draw(seed, m // 2 + 1, c)).astype(np.int64), S)
    d = rng.signs(seed, m)
    Y = to_host(M.sketch(to_dev(A), torch.from_numpy(S.astype(np.int32)).cuda(), seed, NAMES[prec], transform="rfft"))
    Yo = SK.sketch_rfft(A, S, d, prec)
    bound = SK.sketch_rfft_abs_bound(A, S, d, prec)
    err = np.abs(Y - Yo) - (SKETCH_TOL[prec] * bound + (U32 * np.abs(Yo) if prec != P.FP64 else 0))
    assert np.max(err) <= 0, f"max excess {np.max(err):.3e}, max rel {np.max(np.abs(Y - Yo) / bound):.3e}"


def test_sketch_rows_and_columns_are_independent(M):
    # permuting nothing but checking that each output column only sees its own input column
    m, n, s = 3000, 40, 80
    A = W.gaussian(m, n, 3)
    A[:, 17] = 0.0
    S = rng.sample_rows(2, m, s)
    Y = to_host(M.sketch(to_dev(A), torch.from_numpy(S.astype(np.int32)).cuda(), 2, "fp64"))
    assert np.all(Y[:, 17] == 0.0)


@pytest.mark.parametrize("qrp", ["fp64", "fp32"])
@pytest.mark.parametrize("s,n,kappa", [(64, 32, 1e3), (256, 128, 1e3), (48, 20, 1e2), (16, 8, 10.0),
                                       (130, 100, 1e2), (256, 128, 1e8), (100, 50, 1e4), (200, 64, 1e6),
                                       (300, 40, 1e2), (512, 64, 1e3), (250, 128, 1e4), (1024, 32, 1e3),
                                       (2048, 16, 1e5), (1, 1, 1.0)])
def test_sketch_qr_matches_householder(M, qrp, s, n, kappa):
    progress(f"sketch_qr {qrp} s={s} n={n} kappa={kappa:g}")
    Yh = W.test_matrix(s, n, kappa, 4 + n)
    if qrp == "fp32":
        Yh = Yh.astype(np.float32).astype(np.float64)
    Rs, kap = M.sketch_qr(to_dev(Yh), qrp)
    torch.cuda.synchronize()
    R = to_host(Rs)
    u = U64 if qrp == "fp64" else U32
    assert np.all(np.tril(R, -1) == 0) and np.all(np.diag(R) > 0)
    if qrp == "fp32":
        # the QR runs in single precision (Section "Algorithm Description")
        assert np.array_equal(R, R.astype(np.float32).astype(np.float64))
    # backward stability, independent of kappa: R^T R = (Y + dY)^T (Y + dY)
    ny = np.linalg.norm(Yh, 2)
    assert np.linalg.norm(R.T @ R - Yh.T @ Yh, 2) <= 40 * n * u * ny * ny
    if qrp == "fp32" and kappa > 1e6:
        return  # the forward error n u32 kappa says nothing at kappa = 1e8
    _, Ro = HH.householder_qr(Yh)
    assert np.linalg.norm(R - Ro) / np.linalg.norm(Ro) <= 20 * n * u * kappa
    ko = CE.kappa_est(Ro)
    assert abs(float(to_host(kap)[0]) - ko) <= max(1e-6, 40 * n * u * kappa) * ko


@pytest.mark.parametrize("n,kappa", [(8, 1e2), (24, 1e6), (64, 1e12), (128, 1e3), (128, 1e16)])
def test_condest_matches_oracle_ice(M, n, kappa):
    R = W.upper_triangular(n, kappa, 40 + n)
    k = float(to_host(M.condest(to_dev(R)))[0])
    assert abs(k - CE.kappa_est(R)) <= 1e-9 * CE.kappa_est(R)


@pytest.mark.parametrize("n,kappa", [(8, 3.0), (16, 40.0), (50, 1e3), (128, 25.0), (128, 1e8)])
def test_posterior_power_estimate_matches_oracle(M, n, kappa):
    """Power-step part of the posterior estimate (12 steps on R^T R and
    X^T X from the normalized all-ones vector) against the oracle's."""
    R = W.upper_triangular(n, kappa, 60 + n)
    X = M.tri_inverse(to_dev(R))
    k = float(to_host(M.posterior_kappa(to_dev(R), X))[0])
    ko = CE.power_norm(R) * CE.power_norm(to_host(X))
    assert abs(k - ko) <= 1e-10 * ko
    assert k <= np.linalg.cond(R) * (1 + 1e-10)


@pytest.mark.parametrize("m,n,kappa", [(1000, 8, 1e2), (1000, 20, 1e6), (4096, 32, 1e8), (777, 50, 1e4),
                                       (5000, 64, 1e10), (70001, 100, 1e6), (4097, 128, 1e12), (1, 1, 1.0)])
def test_trsm_matches_substitution(M, m, n, kappa):
    progress(f"trsm m={m} n={n} kappa={kappa:g}")
    A = W.gaussian(m, n, 5)
    R = W.upper_triangular(n, kappa, 6 + n)
    X = to_host(M.trsm(to_dev(A), to_dev(R)))
    Xo = CQ.trsm_right_upper(A, R)
    # forward error of a backward-stable solve: ~ n u kappa; backward error ~ n u
    assert np.linalg.norm(X - Xo) / np.linalg.norm(Xo) <= 10 * n * U64 * kappa
    res = np.abs(X @ R - A)
    assert np.max(res) <= 4 * n * U64 * np.max(np.abs(X) @ np.abs(R))


@pytest.mark.parametrize("m,n", [(1000, 8), (4096, 32), (70001, 100), (33333, 128), (64, 64), (5, 3)])
def test_gram_matches_definition(M, m, n):
    progress(f"gram m={m} n={n}")
    B = W.gaussian(m, n, 7)
    G = to_host(M.gram(to_dev(B)))
    Go = B.T @ B
    bound = np.abs(B).T @ np.abs(B)
    # per-chunk sequential MFMA accumulation plus a sequential sum of chunk partials
    chain = 1 + min(m, 4096) / 4 + 512
    assert np.all(np.abs(G - Go) <= 2 * chain * U64 * bound)
    assert np.array_equal(G, G.T)


@pytest.mark.parametrize("n,kappa", [(8, 1e2), (32, 1e6), (100, 1e4), (128, 1e8), (1, 1.0)])
def test_cholesky_matches_oracle(M, n, kappa):
    G = W.spd_matrix(n, kappa, 8 + n)
    Rc, fail, kap = M.cholesky(to_dev(G))
    torch.cuda.synchronize()
    R = to_host(Rc)
    Ro = CQ.cholesky_upper(G)
    assert int(to_host(fail)[0]) == -1
    assert np.linalg.norm(R - Ro) / np.linalg.norm(Ro) <= 10 * n * U64 * kappa
    assert abs(float(to_host(kap)[0]) - CE.kappa_est(Ro)) <= 1e-6 * CE.kappa_est(Ro)


@pytest.mark.parametrize("j", [0, 1, 5])
def test_cholesky_breakdown_index(M, j):
    G = np.eye(8)
    G[j, j] = -1.0
    if j == 1:
        G = np.array([[4.0, 2.0], [2.0, 1.0]])
    Rc, fail, _ = M.cholesky(to_dev(G))
    torch.cuda.synchronize()
    assert int(to_host(fail)[0]) == j
    assert np.all(to_host(Rc) == 0)


@pytest.mark.parametrize("n,kappa", [(1, 1.0), (7, 10.0), (16, 1e2), (33, 30.0), (64, 1e3), (100, 10.0),
                                     (128, 30.0), (128, 1e4)])
def test_tri_inverse_matches_substitution(M, n, kappa):
    progress(f"tri_inverse n={n} kappa={kappa:g}")
    R = W.upper_triangular(n, kappa, 20 + n)
    Rg = R + np.tril(np.full((n, n), np.nan), -1)  # only the upper triangle may be read
    X = to_host(M.tri_inverse(to_dev(Rg)))
    Xo = CQ.upper_inverse(R)
    assert np.array_equal(np.tril(X, -1), np.zeros((n, n)))
    # componentwise forward error of a triangular inverse: ~ n u |X| |R| |X|
    bound = np.abs(Xo) @ np.abs(R) @ np.abs(Xo)
    assert np.all(np.abs(X - Xo) <= 8 * n * U64 * bound)


@pytest.mark.parametrize("m,n,pad", [(1, 1, 0), (5, 3, 0), (100, 16, 0), (129, 7, 3), (1000, 33, 0),
                                     (4096 + 37, 64, 0), (50000, 100, 0), (70001, 128, 0), (1 << 16, 128, 0),
                                     (20000, 128, 5), (300, 48, 0)])
def test_form_q_matches_product(M, m, n, pad):
    progress(f"form_q m={m} n={n} pad={pad}")
    B = W.gaussian(m, n, 12)
    X = W.upper_triangular(n, 30.0, 13 + n)
    Xg = X + np.tril(np.full((n, n), np.nan), -1)  # only the upper triangle may be read
    Bd = to_dev(np.vstack([B, np.full((pad, n), np.nan)]))[:m] if pad else to_dev(B)
    Qd = M.form_q(Bd, to_dev(Xg))
    Q = to_host(Qd)
    Qo = CQ.form_q(B, X)
    # any summation order: |Q - B X| <= n u |B| |X|
    assert np.all(np.abs(Q - Qo) <= 2 * n * U64 * (np.abs(B) @ np.abs(X)))


@pytest.mark.parametrize("n", [1, 7, 64, 100, 128])
def test_trmm_matches_product(M, n):
    R2 = W.upper_triangular(n, 10.0, 9)
    R1 = W.upper_triangular(n, 1e5, 10)
    R = to_host(M.trmm(to_dev(R2), to_dev(R1)))
    Ro = CQ.trmm_upper(R2, R1)
    assert np.all(np.abs(R - Ro) <= 2 * n * U64 * (np.abs(R2) @ np.abs(R1)))
