"""MRCQR (Algorithm 2) on the CPU, stage by stage, in the paper's order.

Stage 1 (precision p): draw D and S; at = fl_p(D A); Y = sketch; thin QR of
Y in p (single precision when p is half or bfloat16, as the paper does since
no half QR exists; see Section "Algorithm Description"); promote Rs to
float64 with diag(Rs) > 0.
Stage 2 (float64): A1 = A Rs^{-1}; [Q, R2] = CholQR(A1) (Algorithm 1).
Stage 3: R = R2 Rs.

Adaptive policy (a reading; the paper gives the regimes and the rerun rule
in Section "Adaptive Precision Selection" but no estimator): start at
`start` precision (half by default); after Stage 1 estimate kappa(Rs) by
ICE; if it reaches the regime bound of the current precision (1e4 for half,
1e8 for single) or Rs is not finite / has a zero pivot, redo Stage 1 one
level higher. After Stage 2 a posterior check on kappa(R2) = kappa(A1)
(Cholesky-QR loses orthogonality like kappa(A1)^2 u; the estimate is
condest.kappa_posterior, ICE combined with a few power steps on R2 and
R2^{-1}) triggers a rerun at the next level when it exceeds TAU_POSTERIOR
or the Cholesky breaks down, as many times as there is a next level: the
paper's self-correcting rerun.
"""
from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np

from . import rng, sketch as SK, householder as HH, cholqr as CQ, condest as CE
from . import precision as P

AUTO = 0
TAU = {P.FP16: 1e4, P.FP32: 1e8, P.FP64: float("inf")}
TAU_POSTERIOR = 20.0
LADDER = [P.FP16, P.FP32, P.FP64]

STATUS_OK = 0
STATUS_CHOL_BREAKDOWN = 3
STATUS_SKETCH_SINGULAR = 4
STATUS_POSTERIOR_WARN = 7


@dataclass
class Result:
    Q: np.ndarray | None
    R: np.ndarray | None
    status: int
    precision_used: int
    escalations: int
    kappa_rs: float
    kappa_rc: float
    chol_fail_index: int = -1
    intermediates: dict = field(default_factory=dict)


DCT, RFFT = "dct", "rfft"


def stage1(A: np.ndarray, prec: int, seed: int, s: int, transform: str = DCT):
    """Draw, sketch (DCT-II rows, or the paper's real DFT bins from
    {0..m/2}), QR of the sketch in the precision the paper fixes."""
    m, n = A.shape
    d = rng.signs(seed, m)
    if transform == RFFT:
        S = rng.sample_rows(seed, m // 2 + 1, s)
        Y = SK.sketch_rfft(A, S, d, prec)
    else:
        S = rng.sample_rows(seed, m, s)
        Y = SK.sketch(A, S, d, prec)
    qr_dtype = np.float64 if prec == P.FP64 else np.float32
    Rs = HH.householder_r(Y, dtype=qr_dtype).astype(np.float64)
    return S, d, Y, Rs


def stage2(A: np.ndarray, Rs: np.ndarray):
    B = CQ.trsm_right_upper(A, Rs)
    G = CQ.gram(B)
    Rc = CQ.cholesky_upper(G)
    Q = CQ.trsm_right_upper(B, Rc)
    return B, G, Rc, Q


def posterior_kappa(Rc: np.ndarray) -> float:
    """Estimate of kappa_2(Rc) for the posterior check (see condest)."""
    return CE.kappa_posterior(Rc, CQ.upper_inverse(Rc))


def _rs_ok(Rs: np.ndarray) -> bool:
    d = np.diag(Rs)
    return bool(np.all(np.isfinite(Rs)) and np.all(d > 0))


def factor(A: np.ndarray, precision: int, seed: int, s: int | None = None,
           start: int = P.FP16, keep: bool = False, transform: str = DCT) -> Result:
    A = np.asarray(A, dtype=np.float64)
    m, n = A.shape
    s = (3 * n if transform == RFFT else 2 * n) if s is None else s
    if precision != AUTO:
        S, d, Y, Rs = stage1(A, precision, seed, s, transform)
        krs = CE.kappa_est(Rs) if _rs_ok(Rs) else float("inf")
        inter = {"S": S, "d": d, "Y": Y, "Rs": Rs} if keep else {}
        if not _rs_ok(Rs):
            return Result(None, None, STATUS_SKETCH_SINGULAR, precision, 0, krs, float("nan"), -1, inter)
        try:
            B, G, Rc, Q = stage2(A, Rs)
        except CQ.CholeskyBreakdown as e:
            return Result(None, None, STATUS_CHOL_BREAKDOWN, precision, 0, krs, float("nan"), e.index, inter)
        krc = posterior_kappa(Rc)
        if keep:
            inter.update({"B": B, "G": G, "Rc": Rc})
        st = STATUS_OK if krc <= TAU_POSTERIOR else STATUS_POSTERIOR_WARN
        return Result(Q, CQ.trmm_upper(Rc, Rs), st, precision, 0, krs, krc, -1, inter)

    level = LADDER.index(start)
    escalations = 0
    while True:
        prec = LADDER[level]
        S, d, Y, Rs = stage1(A, prec, seed, s, transform)
        ok = _rs_ok(Rs)
        krs = CE.kappa_est(Rs) if ok else float("inf")
        if (not ok or krs >= TAU[prec]) and level + 1 < len(LADDER):
            level += 1
            escalations += 1
            continue
        if not ok:
            return Result(None, None, STATUS_SKETCH_SINGULAR, prec, escalations, krs, float("nan"))
        try:
            B, G, Rc, Q = stage2(A, Rs)
            krc = posterior_kappa(Rc)
            fail = -1
        except CQ.CholeskyBreakdown as e:
            krc, fail = float("inf"), e.index
        if krc > TAU_POSTERIOR and level + 1 < len(LADDER):
            level += 1
            escalations += 1
            continue
        if fail >= 0:
            return Result(None, None, STATUS_CHOL_BREAKDOWN, prec, escalations, krs, krc, fail)
        st = STATUS_OK if krc <= TAU_POSTERIOR else STATUS_POSTERIOR_WARN
        return Result(Q, CQ.trmm_upper(Rc, Rs), st, prec, escalations, krs, krc)


def reference_qr(A: np.ndarray):
    """The unique thin QR with diag(R) > 0, by float64 Householder."""
    return HH.householder_qr(A, dtype=np.float64, want_q=True)
