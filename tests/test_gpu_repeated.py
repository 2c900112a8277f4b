"""Repeated factorizations of similar matrices (Section "Adaptive Precision
Selection", repeated calls): the AUTO_CARRY policy starts each call from the
precision the previous call on the same workspace accepted. The precision
sequence, escalation counts and statuses must be those of the oracle's AUTO
started from the same precision; the record carries across graph replays
and is forgotten by mrcqr_regime_reset."""
import numpy as np
import pytest

import workloads as W
from oracle import metrics as MT, mrcqr as OM, precision as P
from gpu_common import require_gpu, to_dev, to_host, progress, torch

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def M():
    return require_gpu()


def _run(M, plan, A, precision, seed):
    Q, R = M.empty_colmajor(plan.m, plan.n), M.empty_colmajor(plan.n, plan.n)
    plan.execute(A, Q, R, precision, seed=seed)
    torch.cuda.synchronize()
    return Q, R, plan.last_info()


# n = 256 takes the column-panel path, which carries the record the same way
@pytest.mark.parametrize("m,n", [(1 << 15, 64), (4096, 256)])
def test_carry_sequence_matches_oracle(M, m, n):
    seed = 31
    # clear of the regime bounds: kappa 1e2 -> FP16, 1e6 -> FP32, 1e10 -> FP64
    kappas = [1e2, 1e6, 1e2, 1e10, 1e6, 1e2]
    plan = M.Plan(m, n)
    start = P.FP16
    seen = []
    for i, k in enumerate(kappas):
        progress(f"carry call {i} n={n} kappa={k:g}")
        A = W.test_matrix(m, n, k, 700 + i)
        Q, R, g = _run(M, plan, to_dev(A), "auto_carry", seed)
        o = OM.factor(A, OM.AUTO, seed=seed, start=start)
        assert (g.status, g.precision_used, g.escalations) == (o.status, o.precision_used, o.escalations), (i, g, o)
        assert g.status == 0
        assert MT.orthogonality(to_host(Q)) <= 1e-13
        assert MT.residual(A, to_host(Q), to_host(R), 1.0) <= 1e-13
        start = o.precision_used
        seen.append(g.precision)
    assert seen == ["fp16", "fp32", "fp32", "fp64", "fp64", "fp64"]

    plan.reset_regime()
    _, _, g = _run(M, plan, to_dev(W.test_matrix(m, n, 1e2, 799)), "auto_carry", seed)
    assert g.precision == "fp16" and g.escalations == 0
    # plain AUTO neither reads nor writes the record
    _, _, g = _run(M, plan, to_dev(W.test_matrix(m, n, 1e6, 798)), "auto", seed)
    assert g.precision == "fp32"
    _, _, g = _run(M, plan, to_dev(W.test_matrix(m, n, 1e2, 797)), "auto_carry", seed)
    assert g.precision == "fp16"


def test_carry_across_graph_replays(M):
    m, n, seed = 1 << 14, 48, 5
    kappas = [1e2, 1e6, 1e2, 1e10, 1e2]
    inputs = [to_dev(W.test_matrix(m, n, k, 720 + i)) for i, k in enumerate(kappas)]
    plan = M.Plan(m, n)
    A = M.empty_colmajor(m, n)
    Q, R = M.empty_colmajor(m, n), M.empty_colmajor(n, n)
    A.copy_(inputs[0])
    side = torch.cuda.Stream()
    side.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(side):
        plan.execute(A, Q, R, "auto_carry", seed=seed)  # warm-up outside the capture
    torch.cuda.current_stream().wait_stream(side)
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g):
        plan.execute(A, Q, R, "auto_carry", seed=seed)
    torch.cuda.synchronize()
    plan.reset_regime()
    torch.cuda.synchronize()

    fixed = M.Plan(m, n)
    seen = []
    for i, Ai in enumerate(inputs):
        progress(f"graph carry replay {i}")
        A.copy_(Ai)
        torch.cuda.synchronize()
        g.replay()
        torch.cuda.synchronize()
        info = plan.last_info()
        assert info.status == 0, info
        seen.append(info.precision)
        # the carried call computes what a call forced to its precision computes
        Qf, Rf, _ = _run(M, fixed, Ai, info.precision, seed)
        assert torch.equal(Q, Qf) and torch.equal(R, Rf), i
    assert seen == ["fp16", "fp32", "fp32", "fp64", "fp64"]


def test_power_loop_shape_captured(M):
    """64 graph-replayed calls at m = 2^21, n = 64 with kappa rising from 1e2
    to 1e14 (same U and V, sigma changing per call)."""
    m, n, calls, seed = 1 << 21, 64, 64, 3
    progress("power-loop shape: building U, V")
    U, _, V = W.test_matrix_factors(m, n, 1.0, 900)
    Ud = torch.from_numpy(np.ascontiguousarray(U.T)).cuda().t()
    VT = torch.from_numpy(np.ascontiguousarray(V.T)).cuda()  # V^T, row-major, contiguous
    kappas = W.rising_kappas(calls)
    plan = M.Plan(m, n)
    A = M.empty_colmajor(m, n)
    Q, R = M.empty_colmajor(m, n), M.empty_colmajor(n, n)

    def load(k):
        sig = torch.from_numpy(W.singular_values(n, float(kappas[k]))).cuda()
        A.copy_((Ud * sig[None, :]) @ VT)

    load(0)
    side = torch.cuda.Stream()
    side.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(side):
        plan.execute(A, Q, R, "auto_carry", seed=seed)
    torch.cuda.current_stream().wait_stream(side)
    torch.cuda.synchronize()
    graph = torch.cuda.CUDAGraph()
    with torch.cuda.graph(graph):
        plan.execute(A, Q, R, "auto_carry", seed=seed)
    # plain AUTO on the same sequence, for the per-call time it would take
    plan_auto = M.Plan(m, n)
    Q2, R2 = M.empty_colmajor(m, n), M.empty_colmajor(n, n)
    with torch.cuda.stream(side):
        plan_auto.execute(A, Q2, R2, "auto", seed=seed)
    torch.cuda.current_stream().wait_stream(side)
    torch.cuda.synchronize()
    graph_auto = torch.cuda.CUDAGraph()
    with torch.cuda.graph(graph_auto):
        plan_auto.execute(A, Q2, R2, "auto", seed=seed)
    torch.cuda.synchronize()
    plan.reset_regime()
    torch.cuda.synchronize()

    order = {"fp16": 0, "fp32": 1, "fp64": 2}
    precs, ms, ms_auto = [], [], []
    ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)

    def timed(gr):
        ev0.record()
        gr.replay()
        ev1.record()
        torch.cuda.synchronize()
        return ev0.elapsed_time(ev1)

    for k in range(calls):
        load(k)
        torch.cuda.synchronize()
        ms_auto.append(timed(graph_auto))
        ms.append(timed(graph))
        info = plan.last_info()
        ia = plan_auto.last_info()
        assert ia.status == 0 and order[ia.precision] <= order[info.precision], (k, ia, info)
        assert info.status == 0, (k, info)
        precs.append(info.precision)
        if k in (0, calls // 2, calls - 1):
            progress(f"power-loop call {k} kappa={kappas[k]:.2g} {info.precision}")
            Ah, Qh, Rh = to_host(A), to_host(Q), to_host(R)
            assert MT.orthogonality(Qh) <= 1e-13, k
            assert MT.residual(Ah, Qh, Rh, 1.0) <= 1e-13, k
    steps = [order[p] for p in precs]
    assert steps[0] == 0 and steps[-1] == 2
    assert all(a <= b for a, b in zip(steps, steps[1:])), precs
    for name, t in (("auto_carry", ms), ("auto", ms_auto)):
        progress(f"power-loop {name} per call: p50 {np.percentile(t, 50):.3f} ms, p99 {np.percentile(t, 99):.3f} ms, "
                 f"total {sum(t):.2f} ms")
    progress(f"power-loop precisions fp16/fp32/fp64 = {precs.count('fp16')}/{precs.count('fp32')}/{precs.count('fp64')}")
