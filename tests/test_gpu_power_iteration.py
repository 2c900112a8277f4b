"""A randomized range finder with power steps built on the captured MRCQR
call with AUTO_CARRY (Section "Adaptive Precision Selection", repeated
calls): Y_q = (M M^T)^q M Omega for q = 0, 1, 2, ..., each factored in
turn. Without re-orthogonalization between the products the condition
number of Y_q grows like (sigma_1 / sigma_b)^(2q+1), so the carried
precision climbs FP16 -> FP32 -> FP64 over the calls and never falls back.
Every basis must be orthonormal to 1e-13 and reproduce Y_q to 1e-13, and
the tangent of the largest angle between span(Q_q) and the top-b left
singular subspace of M must contract by (sigma_{b+1} / sigma_b)^2 per
step, as subspace iteration guarantees. The products with M are plain
library GEMMs of the driver, outside the factorization."""
import numpy as np
import pytest

import workloads as W
from oracle import metrics as MT
from gpu_common import require_gpu, to_host, progress, torch

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def M():
    return require_gpu()


def test_range_finder_power_steps_carry_the_regime(M):
    m, N, b, iters, seed = 1 << 18, 256, 32, 4, 13
    progress("range finder: building M = U diag(0.9^i) V^T")
    U, _, V = W.test_matrix_factors(m, N, 1.0, 950)
    sig = 0.9 ** np.arange(N)
    Md = torch.from_numpy(np.asfortranarray((U * sig[None, :]) @ V.T).T.copy()).cuda().t()  # column-major m x N
    MdT = Md.t().contiguous()
    Ub = torch.from_numpy(np.ascontiguousarray(U[:, :b])).cuda()
    Om = torch.from_numpy(W.gaussian(N, b, 951, order="C")).cuda()

    plan = M.Plan(m, b)
    Y = M.empty_colmajor(m, b)
    Q, R = M.empty_colmajor(m, b), M.empty_colmajor(b, b)
    Z = Md @ Om  # the running product (M M^T)^q M Omega
    Y.copy_(Z)
    # warm-up outside the capture, then capture one call and reset the regime
    side = torch.cuda.Stream()
    side.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(side):
        plan.execute(Y, Q, R, "auto_carry", seed=seed)
    torch.cuda.current_stream().wait_stream(side)
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g):
        plan.execute(Y, Q, R, "auto_carry", seed=seed)
    torch.cuda.synchronize()
    plan.reset_regime()
    torch.cuda.synchronize()

    order = {"fp16": 0, "fp32": 1, "fp64": 2}
    precs, dists = [], []
    for k in range(iters + 1):
        if k > 0:
            Z = Md @ (MdT @ Z)
            Y.copy_(Z)
        torch.cuda.synchronize()
        g.replay()
        torch.cuda.synchronize()
        info = plan.last_info()
        assert info.status == 0, (k, info)
        Qh, Rh = to_host(Q), to_host(R)
        assert MT.orthogonality(Qh) <= 1e-13, k
        assert MT.residual(to_host(Y), Qh, Rh, 1.0) <= 1e-13, k
        # tangent of the largest principal angle between span(Q) and span(U_b):
        # cos from the smallest singular value of Q^T U_b, sin from the norm
        # of (I - Q Q^T) U_b (both b x b on the host)
        C = Q.t() @ Ub
        P = Ub - Q @ C
        cos_t = float(np.linalg.svd(C.cpu().numpy(), compute_uv=False).min())
        sin_t = float(np.sqrt(max(np.linalg.eigvalsh((P.t() @ P).cpu().numpy()).max(), 0.0)))
        dist = sin_t / cos_t
        precs.append(info.precision)
        dists.append(dist)
        progress(f"range finder q={k}: {info.precision} (escalations {info.escalations}), "
                 f"kappa(Rc)~{info.kappa_rc_est:.3g}, tan angle to top-{b} subspace {dist:.3e}")
    steps = [order[p] for p in precs]
    assert all(a <= b_ for a, b_ in zip(steps, steps[1:])), precs
    assert steps[0] == 0 and steps[-1] == 2, precs
    # subspace iteration on M M^T contracts the tangent at least by
    # (sigma_{b+1} / sigma_b)^2 = 0.81 per step in exact arithmetic; the
    # products in float64 perturb the weakest of the b directions of Y_q by
    # about u (sigma_1 / sigma_b)^(2q+1) < 1e-3 relative, hence the margin
    for a, c in zip(dists, dists[1:]):
        assert c <= 0.82 * a, dists
