"""Precision sweep at the full headline shape (m = 2^20, n = 128, s = 256):
kappa in {1e2, 1e4, 1e8, 1e12, 1e16} x sketch in {FP64, FP32, FP16, BF16}.
Checked against the regimes of Section "Adaptive Precision Selection" (FP16
below 1e4, FP32 below 1e8, FP64 for any kappa; BF16 below 1e2 by the same
u_p kappa < 1 rule): inside its regime a precision returns status 0 with
||I - Q^T Q||_2 <= 1e-13 and ||A - QR|| / ||A|| <= 1e-13; every result the
library accepts (status 0) meets the same bound; and once a precision fails
at some kappa it does not recover at a larger one. Each call is timed."""
import numpy as np
import pytest

import workloads as W
from oracle import metrics as MT
from gpu_common import require_gpu, to_host, progress, torch

pytestmark = pytest.mark.gpu

M_ROWS, N_COLS = 1 << 20, 128
KAPPAS = [1e2, 1e4, 1e8, 1e12, 1e16]
REGIME = {"fp64": 1e17, "fp32": 1e8, "fp16": 1e4, "bf16": 1e2}  # accurate for kappa <= bound


@pytest.fixture(scope="module")
def M():
    return require_gpu()


@pytest.mark.parametrize("prec", ["fp64", "fp32", "fp16", "bf16"])
def test_precision_sweep_full_size(M, prec):
    plan = M.Plan(M_ROWS, N_COLS)
    Q, R = M.empty_colmajor(M_ROWS, N_COLS), M.empty_colmajor(N_COLS, N_COLS)
    ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    failed_at = None
    rows = []
    for k in KAPPAS:
        A = W.device_test_matrix(M_ROWS, N_COLS, k, 600 + int(np.log10(k)))
        plan.execute(A, Q, R, prec, seed=9)  # warm-up of this input
        torch.cuda.synchronize()
        ev0.record()
        plan.execute(A, Q, R, prec, seed=9)
        ev1.record()
        torch.cuda.synchronize()
        ms = ev0.elapsed_time(ev1)
        info = plan.last_info()
        orth = res = float("nan")
        if info.status in (0, 7):
            Qh, Rh = to_host(Q), to_host(R)
            orth = MT.orthogonality(Qh)
            res = MT.residual(to_host(A), Qh, Rh, 1.0)
        rows.append((k, info.status, orth, res, ms))
        progress(f"sweep {prec} kappa={k:.0e}: status {info.status} orth {orth:.2e} res {res:.2e} "
                 f"kappa(Rc)~{info.kappa_rc_est:.3g} {ms:.3f} ms")
        assert info.status in (0, 3, 7), info
        if k <= REGIME[prec]:
            assert info.status == 0, (prec, k, info)
        if info.status == 0:
            assert orth <= 1e-13 and res <= 1e-13, (prec, k, orth, res)
            assert failed_at is None, (prec, k, "accepted after failing at", failed_at)
        elif failed_at is None:
            failed_at = k
        del A
