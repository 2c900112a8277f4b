"""The repeated-QR drivers of the package (paper_2606_18411_amd.krylov):
block Krylov (block Arnoldi on M M^T with BCGS2, two factorizations per
block) and the
power-step range finder, both on one graph-captured MRCQR call with the
carried precision (Section "Adaptive Precision Selection", repeated calls).
The whole basis must be orthonormal to 1e-13, the carried precision must
never fall, and the basis must do its job: the Ritz values of M M^T on the
block Krylov basis converge to the known sigma_i^2, and the range finder's
subspace approaches the top singular subspace at the subspace-iteration
rate."""
import numpy as np
import pytest

import workloads as W
from gpu_common import require_gpu, to_host, progress, torch

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def M():
    return require_gpu()


@pytest.fixture(scope="module")
def op():
    m, N = 1 << 18, 256
    U, _, V = W.test_matrix_factors(m, N, 1.0, 960)
    sig = 0.9 ** np.arange(N)
    Md = torch.from_numpy(np.asfortranarray((U * sig[None, :]) @ V.T).T.copy()).cuda().t()
    Om = torch.from_numpy(W.gaussian(N, 32, 961, order="C")).cuda()
    return Md, U, sig, Om


def _monotone(precs):
    order = {"fp16": 0, "bf16": 0, "fp32": 1, "fp64": 2}
    s = [order[p] for p in precs]
    return all(a <= b for a, b in zip(s, s[1:]))


def test_block_krylov_basis(M, op):
    from paper_2606_18411_amd import krylov
    Md, U, sig, Om = op
    b, k = 32, 4
    progress("block Krylov: 5 blocks of 32")
    res = krylov.block_krylov(Md, b, k, seed=3, Omega=Om)
    progress(f"block Krylov: precisions {res.precisions}, basis orthogonality {res.orthogonality:.2e}")
    assert all(i.status == 0 for i in res.infos), res.infos
    assert _monotone(res.precisions)
    assert res.orthogonality <= 1e-13
    V = res.basis
    T = (V.t() @ Md) @ (Md.t() @ V)
    ritz = np.sort(np.linalg.eigvalsh(to_host(0.5 * (T + T.t()))))[::-1]
    lam = sig ** 2
    assert ritz[0] <= lam[0] * (1 + 1e-12)
    rel = np.abs(ritz[:8] - lam[:8]) / lam[:8]
    progress(f"block Krylov: top Ritz values relative error {rel.max():.2e}")
    assert rel.max() <= 1e-8


def test_power_range_driver(M, op):
    from paper_2606_18411_amd import krylov
    Md, U, sig, Om = op
    b, q = 32, 4
    Ub = torch.from_numpy(np.ascontiguousarray(U[:, :b])).cuda()
    tangents = []

    def on_step(j, Q, R, info):
        C = Q.t() @ Ub
        P = Ub - Q @ C
        cos_t = float(np.linalg.svd(to_host(C), compute_uv=False).min())
        sin_t = float(np.sqrt(max(np.linalg.eigvalsh(to_host(P.t() @ P)).max(), 0.0)))
        tangents.append(sin_t / cos_t)

    res = krylov.power_range(Md, b, q, seed=13, Omega=Om, on_step=on_step)
    progress(f"power range: precisions {res.precisions}, tangents {['%.3g' % t for t in tangents]}")
    assert all(i.status == 0 for i in res.infos)
    assert _monotone(res.precisions) and res.precisions[0] == "fp16" and res.precisions[-1] == "fp64"
    assert res.orthogonality <= 1e-13
    for a, c in zip(tangents, tangents[1:]):
        assert c <= 0.82 * a
