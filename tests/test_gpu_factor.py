"""GPU parity of the whole factorization (Algorithm 2) against the unique
thin QR with diag(R) > 0, the paper's accuracy targets, and the library's
determinism and status reporting."""
import json
import os

import numpy as np
import pytest

import workloads as W
from oracle import householder as HH, metrics as MT, mrcqr as OM, precision as P
from gpu_common import require_gpu, to_dev, to_host, progress, torch
from conftest import GOLDEN

pytestmark = pytest.mark.gpu
CLAIMS = json.load(open(os.path.join(GOLDEN, "paper_claims.json")))
U64 = 2.0 ** -53


@pytest.fixture(scope="module")
def M():
    return require_gpu()


def _check_against_reference(A, Q, R, kappa, n):
    Qh, Rh = HH.householder_qr(A)
    tol = 50 * n * U64 * kappa
    assert MT.rel_diff(R, Rh) <= tol
    assert np.max(np.abs(Q - Qh)) <= tol
    assert np.all(np.tril(R, -1) == 0) and np.all(np.diag(R) > 0)


@pytest.mark.parametrize("prec", ["fp64", "fp32", "fp16", "bf16", "auto"])
def test_config1_matches_unique_qr(M, prec):
    # m=4096, n=32, kappa=1e4, s=64 (sigma log-spaced 1 -> 1e-4)
    m, n, kappa = 4096, 32, 1e4
    progress(f"factor config1 {prec}")
    A = W.test_matrix(m, n, kappa, 101)
    if prec == "bf16":
        kappa_ok = 1e2
        A = W.test_matrix(m, n, kappa_ok, 101)
        kappa = kappa_ok
    Q, R, info = M.factor(to_dev(A), prec, seed=5)
    Q, R = to_host(Q), to_host(R)
    assert info.status == 0, info
    assert MT.orthogonality(Q) <= CLAIMS["target_orthogonality"]
    assert MT.residual(A, Q, R, 1.0) <= CLAIMS["target_residual"]
    _check_against_reference(A, Q, R, kappa, n)
    if prec == "auto":
        assert info.precision == "fp16" and info.escalations == 0


@pytest.mark.parametrize("kappa", [1e2, 1e8, 1e12, 1e16])
def test_fp64_sketch_orthogonal_for_all_kappa(M, kappa):
    m, n = 1 << 16, 64
    progress(f"factor fp64 kappa={kappa:g}")
    A = W.test_matrix(m, n, kappa, 202)
    Q, R, info = M.factor(to_dev(A), "fp64", seed=3)
    Q, R = to_host(Q), to_host(R)
    assert info.status == 0, info
    assert MT.orthogonality(Q) <= CLAIMS["orthogonality_fp64_sketch_all_kappa"] * 4
    assert MT.residual(A, Q, R, 1.0) <= CLAIMS["target_residual"]
    if kappa <= 1e10:
        _check_against_reference(A, Q, R, kappa, n)


@pytest.mark.parametrize("prec,kappa,ok", [("fp16", 1e4, True), ("fp32", 1e8, True), ("fp16", 1e8, False),
                                           ("fp32", 1e12, False)])
def test_precision_regimes(M, prec, kappa, ok):
    m, n = 1 << 15, 64
    progress(f"regime {prec} kappa={kappa:g}")
    A = W.test_matrix(m, n, kappa, 303)
    Q, R, info = M.factor(to_dev(A), prec, seed=9)
    if ok:
        assert info.status == 0, info
        assert MT.orthogonality(to_host(Q)) <= CLAIMS["target_orthogonality"]
    else:
        assert info.status in (3, 7), info  # breakdown or posterior warning
        if info.status == 7:
            assert MT.orthogonality(to_host(Q)) > 1e-12
            assert MT.residual(A, to_host(Q), to_host(R), 1.0) <= 1e-13


@pytest.mark.parametrize("kappa,expect", [(1e2, "fp16"), (1e6, "fp32"), (1e10, "fp64"), (1e16, "fp64")])
def test_auto_lands_in_regime(M, kappa, expect):
    m, n = 1 << 15, 64
    progress(f"auto kappa={kappa:g}")
    A = W.test_matrix(m, n, kappa, 404)
    Q, R, info = M.factor(to_dev(A), "auto", seed=11)
    assert info.status == 0, info
    assert info.precision == expect, info
    o = OM.factor(A, OM.AUTO, seed=11)
    assert P.NAMES[o.precision_used] == expect
    assert MT.orthogonality(to_host(Q)) <= CLAIMS["target_orthogonality"]


def test_deterministic_bitwise(M):
    A = to_dev(W.test_matrix(20000, 48, 1e6, 505))
    Q1, R1, _ = M.factor(A, "fp16", seed=1)
    Q2, R2, _ = M.factor(A, "fp16", seed=1)
    assert torch.equal(Q1, Q2) and torch.equal(R1, R2)


def test_seed_invariance(M):
    A = W.test_matrix(20000, 48, 1e6, 606)
    _, R1, _ = M.factor(to_dev(A), "fp32", seed=1)
    _, R2, _ = M.factor(to_dev(A), "fp32", seed=987654321)
    assert MT.rel_diff(to_host(R1), to_host(R2)) <= 1e-9


def test_power_of_two_scaling_exact(M):
    A = W.test_matrix(8192, 32, 1e3, 707)
    Q1, R1, _ = M.factor(to_dev(A), "fp64", seed=2)
    Q2, R2, _ = M.factor(to_dev(A * 2.0 ** 40), "fp64", seed=2)
    assert torch.equal(Q1, Q2) and torch.equal(R1 * 2.0 ** 40, R2)


@pytest.mark.parametrize("m,n,s", [(129, 7, 20), (1000, 1, 2), (3000, 100, 250), (64, 64, 64), (50000, 96, 192)])
def test_ragged_shapes(M, m, n, s):
    progress(f"ragged m={m} n={n} s={s}")
    A = W.test_matrix(m, n, 1e3, 808 + n)
    Q, R, info = M.factor(to_dev(A), "fp32", seed=4, s=s)
    assert info.status == 0, info
    _check_against_reference(A, to_host(Q), to_host(R), 1e3, n)


def test_zero_column_reports_singular_sketch(M):
    A = W.gaussian(4096, 16, 9)
    A[:, 5] = 0.0
    _, _, info = M.factor(to_dev(A), "fp64", seed=1)
    assert info.status == 4


@pytest.mark.parametrize("bad", [np.nan, np.inf])
@pytest.mark.parametrize("prec", ["fp16", "fp64", "auto"])
def test_nonfinite_input_is_reported(M, bad, prec):
    A = W.gaussian(4096, 16, 10)
    A[100, 3] = bad
    _, _, info = M.factor(to_dev(A), prec, seed=1)
    assert info.status == M.ERR_NONFINITE, info
    if prec == "auto":  # escalated through every precision before reporting
        assert info.precision == "fp64" and info.escalations == 2, info


def test_out_of_range_input_escalates_to_a_wider_sketch(M):
    """Entries near 2^118 leave binary16's range even after the block
    prescale (the exponent shift is clamped at 100, so they stay near 2^18 >
    65504): the FP16 sketch is not finite, AUTO escalates, and FP32 (8
    exponent bits) forms it."""
    A = W.test_matrix(4096, 16, 1e2, 11) * 2.0 ** 124
    _, _, info = M.factor(to_dev(A), "fp16", seed=1)
    assert info.status == M.ERR_NONFINITE, info
    Q, R, info = M.factor(to_dev(A), "auto", seed=1)
    assert info.status == 0 and info.precision == "fp32" and info.escalations == 1, info
    assert MT.orthogonality(to_host(Q)) <= 1e-13


@pytest.mark.parametrize("s,seed", [(17, 0), (18, 26)])
def test_posterior_rerun_ladder_matches_oracle(M, s, seed):
    """A sketch barely taller than n leaves kappa(Rc) above the posterior
    bound at every precision: AUTO reruns at FP32, then FP64, and reports the
    posterior warning, as the oracle does (same decision, same estimate)."""
    A = W.test_matrix(2048, 16, 1e2, 3)
    progress(f"posterior ladder s={s} seed={seed}")
    Q, R, info = M.factor(to_dev(A), "auto", seed=seed, s=s)
    o = OM.factor(A, OM.AUTO, seed, s=s)
    assert (info.status, P.NAMES[info.precision_used], info.escalations) == (o.status, "fp64", 2), (info, o.status)
    assert abs(info.kappa_rc_est - o.kappa_rc) <= 1e-6 * o.kappa_rc
    assert MT.residual(A, to_host(Q), to_host(R), 1.0) <= 1e-13


def test_concurrent_streams_same_shape(M):
    """Calls of one shape from two streams share the cached workspace; the
    library orders them on the device, so each result is bitwise that of a
    call made alone."""
    mats = [to_dev(W.test_matrix(30000, 48, 1e5, 1200 + i)) for i in range(4)]
    ref = [M.factor(a, "auto", seed=7) for a in mats]
    streams = [torch.cuda.Stream(), torch.cuda.Stream()]
    for st in streams:
        st.wait_stream(torch.cuda.current_stream())
    outs = []
    for i, a in enumerate(mats):
        st = streams[i % 2]
        with torch.cuda.stream(st):
            outs.append(M.factor(a, "auto", seed=7, stream=st, sync=False))
    torch.cuda.synchronize()
    for (Q, R, info), (Qr, Rr, ir) in zip(outs, ref):
        assert torch.equal(Q, Qr) and torch.equal(R, Rr)
        assert M.read_infos(info)[0] == ir


def test_plan_execute_matches_factor(M):
    A = to_dev(W.test_matrix(10000, 40, 1e5, 909))
    Q1, R1, _ = M.factor(A, "fp32", seed=3)
    plan = M.Plan(10000, 40)
    Q2 = M.empty_colmajor(10000, 40)
    R2 = M.empty_colmajor(40, 40)
    plan.execute(A, Q2, R2, "fp32", seed=3)
    torch.cuda.synchronize()
    assert plan.last_info().status == 0
    assert torch.equal(Q1, Q2) and torch.equal(R1, R2)


def test_batched_matches_single(M):
    mats = [W.test_matrix(m, n, k, 1000 + i) for i, (m, n, k) in
            enumerate([(5000, 8, 1e2), (7000, 16, 1e6), (9000, 32, 1e10), (4096, 64, 1e3)])]
    As = [to_dev(a) for a in mats]
    Qs, Rs, infos = M.factor_batched(As, "auto", seeds=[1, 2, 3, 4])
    for a, A, Q, R, inf, sd in zip(mats, As, Qs, Rs, infos, [1, 2, 3, 4]):
        assert inf.status == 0
        Q1, R1, _ = M.factor(A, "auto", seed=sd)
        assert torch.equal(Q, Q1) and torch.equal(R, R1)
        assert MT.orthogonality(to_host(Q)) <= 1e-13


def test_bad_arguments_raise(M):
    A = to_dev(W.gaussian(100, 10, 1))
    with pytest.raises(M.MrcqrError) as e:
        M.factor(A, "fp16", s=5)  # s < n
    assert e.value.code == 1
    with pytest.raises(M.MrcqrError):
        M.factor(A, 9)
