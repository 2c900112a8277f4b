"""Repeated factorizations inside one captured HIP graph (the pattern of a
power or block-Krylov loop): the plan API enqueues a static launch sequence
that allocates nothing and decides the precision (AUTO escalation and the
posterior rerun) on the device, so a captured call replays for any input of
the plan's shape. Every replay is checked bitwise against the same call made
eagerly, with eager work (the input copy, a synchronization) between
replays."""
import numpy as np
import pytest

import workloads as W
from oracle import metrics as MT
from gpu_common import require_gpu, to_dev, to_host, progress, torch

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def M():
    return require_gpu()


# n = 256 takes the column-panel path (its launch sequence is as static)
@pytest.mark.parametrize("precision,n", [("auto", 64), ("fp16", 64), ("auto", 256), ("fp16", 256)])
def test_graph_replays_match_eager_calls(M, precision, n):
    m, seed = 1 << 14, 21
    progress(f"graph capture {precision} n={n}")
    plan = M.Plan(m, n)
    # kappa rising as in a repeated-call loop; AUTO goes fp16 -> fp32 -> fp64
    kappas = [1e2, 1e6, 1e10] if precision == "auto" else [1e2, 1e3]
    inputs = [to_dev(W.test_matrix(m, n, k, 100 + i)) for i, k in enumerate(kappas)]
    eager = []
    for Ai in inputs:
        Qe, Re = M.empty_colmajor(m, n), M.empty_colmajor(n, n)
        plan.execute(Ai, Qe, Re, precision, seed=seed)
        torch.cuda.synchronize()
        eager.append((Qe.clone(), Re.clone(), plan.last_info()))

    A = M.empty_colmajor(m, n)
    Q, R = M.empty_colmajor(m, n), M.empty_colmajor(n, n)
    A.copy_(inputs[0])
    side = torch.cuda.Stream()
    side.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(side):
        plan.execute(A, Q, R, precision, seed=seed)  # warm-up outside the capture
    torch.cuda.current_stream().wait_stream(side)
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g):
        plan.execute(A, Q, R, precision, seed=seed)
    torch.cuda.synchronize()

    order = [0, 1, 2, 1, 0] if len(inputs) == 3 else [0, 1, 0]
    for rep, i in enumerate(order):
        A.copy_(inputs[i])
        torch.cuda.synchronize()
        g.replay()
        torch.cuda.synchronize()
        Qe, Re, ie = eager[i]
        info = plan.last_info()
        assert torch.equal(Q, Qe) and torch.equal(R, Re), (rep, i)
        assert (info.status, info.precision_used, info.escalations) == (ie.status, ie.precision_used,
                                                                         ie.escalations), (rep, i, info, ie)
        assert info.status == 0, info
        assert MT.orthogonality(to_host(Q)) <= 1e-13
    if precision == "auto":
        assert [e[2].precision for e in eager] == ["fp16", "fp32", "fp64"]
