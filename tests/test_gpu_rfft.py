"""The paper's own sketch operator (Algorithm 2, FFT and Select): real parts
of c DFT bins drawn from {0..m/2}, scaled by sqrt(c/m), c = 3n by default,
run on the same MFMA contraction as the DCT-II sketch. Whole factorizations
with it give the unique thin QR and follow the oracle's policy; a side by
side with the DCT-II at s = 2n and 3n reports orthogonality, kappa(Rc) and
time at m = 2^20."""
import numpy as np
import pytest

import workloads as W
from oracle import householder as HH, metrics as MT, mrcqr as OM, precision as P
from gpu_common import require_gpu, to_dev, to_host, progress, torch

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def M():
    return require_gpu()


def _run(M, plan, A, prec, seed, reps=0):
    m, n = A.shape
    Q, R = M.empty_colmajor(m, n), M.empty_colmajor(n, n)
    plan.execute(A, Q, R, prec, seed=seed)
    torch.cuda.synchronize()
    info = plan.last_info()
    ms = None
    if reps:
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        for i in range(reps):
            plan.execute(A, Q, R, prec, seed=seed + 1 + i)
        e1.record()
        torch.cuda.synchronize()
        ms = e0.elapsed_time(e1) / reps
        plan.execute(A, Q, R, prec, seed=seed)
        torch.cuda.synchronize()
    return Q, R, info, ms


@pytest.mark.parametrize("prec,kappa", [("fp16", 1e2), ("fp32", 1e6), ("fp64", 1e12), ("auto", 1e7), ("bf16", 1e2)])
def test_rfft_factor_gives_unique_qr_like_the_oracle(M, prec, kappa):
    m, n = 4096, 32
    progress(f"rfft factor {prec} kappa={kappa:g}")
    A = W.test_matrix(m, n, kappa, 41)
    plan = M.Plan(m, n, transform="rfft")  # c = 3n = 96
    Q, R, info, _ = _run(M, plan, to_dev(A), prec, 7)
    o = OM.factor(A, OM.AUTO if prec == "auto" else {"fp16": P.FP16, "fp32": P.FP32, "fp64": P.FP64,
                                                      "bf16": P.BF16}[prec], 7, transform=OM.RFFT)
    assert (info.status, info.precision_used, info.escalations) == (o.status, o.precision_used, o.escalations)
    assert info.status == 0, info
    Qh, Rh = to_host(Q), to_host(R)
    _, Ro = HH.householder_qr(A)
    assert MT.rel_diff(Rh, Ro) <= 50 * n * 2.0 ** -53 * kappa
    assert MT.orthogonality(Qh) <= 1e-13 and MT.residual(A, Qh, Rh, 1.0) <= 1e-13


@pytest.mark.parametrize("n", [64, 128])
def test_rfft_and_dct_side_by_side(M, n):
    m, kappa = 1 << 20, 1e4
    A_h = W.test_matrix(m, n, kappa, 11)
    A = to_dev(A_h)
    cases = [("dct", 2 * n), ("rfft", 2 * n)] + ([("dct", 3 * n), ("rfft", 3 * n)] if n <= 64 else [])
    for transform, s in cases:
        plan = M.Plan(m, n, s, transform=transform)
        for prec in ("fp16", "fp64"):
            Q, R, info, ms = _run(M, plan, A, prec, 3, reps=5)
            o = MT.orthogonality(to_host(Q))
            progress(f"side by side m=2^20 n={n} {transform} s={s} {prec}: {ms:.3f} ms/QR, orth {o:.2e}, "
                     f"kappa(Rc) {info.kappa_rc_est:.2f}, status {info.status}")
            assert info.status == 0 and o <= 1e-13, (transform, s, prec, info, o)
