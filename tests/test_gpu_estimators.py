"""The two other condition estimators of Section "Adaptive Precision
Selection" on the GPU: the block 1-norm estimator (on a triangular factor,
and the paper's Gram bound from the Cholesky factor of A^T A) and the CholQR
probe, against the oracle, then side by side with the policy's ICE estimate
over a kappa sweep (misclassification of the precision regime and time)."""
import numpy as np
import pytest

import workloads as W
from oracle import cholqr as CQ, condest as CE, mrcqr as OM, precision as P, rng
from gpu_common import require_gpu, to_dev, to_host, progress, torch

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def M():
    return require_gpu()


@pytest.mark.parametrize("n,kappa", [(8, 10.0), (50, 1e6), (128, 1e3), (128, 1e12), (2, 5.0), (1, 1.0), (77, 1e9)])
def test_onenorm_estimate_matches_oracle(M, n, kappa):
    R = W.upper_triangular(n, kappa, 500 + n)
    k = float(to_host(M.condest_1norm(to_dev(R), seed=9))[0])
    ko = CE.kappa_1norm_tri(R, seed=9)
    assert abs(k - ko) <= 1e-8 * ko, (k, ko)


@pytest.mark.parametrize("n,kappa", [(16, 1e2), (64, 1e5), (128, 1e3)])
def test_gram_bound_matches_oracle(M, n, kappa):
    A = W.test_matrix(8192, n, kappa, 600 + n)
    G = to_dev(A.T @ A)
    Rg, fail, _ = M.cholesky(G)
    torch.cuda.synchronize()
    assert int(to_host(fail)[0]) == -1
    k = float(to_host(M.condest_1norm(Rg, G, seed=4))[0])
    ko = CE.kappa_bound_gram(to_host(Rg), seed=4)
    assert abs(k - ko) <= 1e-8 * ko, (k, ko)
    assert k >= 0.5 * kappa


@pytest.mark.parametrize("kappa", [1e2, 1e4, 1e6, 1e12])
def test_cholqr_probe_tracks_the_oracle(M, kappa):
    """q = ||I - Q^T Q|| is rounding noise of one CholQR pass, so GPU and
    oracle agree in magnitude, not digits; both are lower bounds on kappa
    and both report the breakdown past 1e8."""
    A = W.test_matrix(1 << 15, 32, kappa, 700)
    k = float(to_host(M.cholqr_probe(to_dev(A)))[0])
    ko = CE.probe_kappa(A, exact=False)
    if not np.isfinite(ko):
        assert not np.isfinite(k)
        return
    assert ko / 5 <= k <= ko * 5, (k, ko)
    assert k <= 2 * kappa


def _regime(k):
    return 0 if k < 1e4 else (1 if k < 1e8 else 2)


def test_estimators_side_by_side_over_kappa(M):
    """Regime misclassification (half < 1e4 <= single < 1e8 <= double) and time
    of each estimator at the paper's sweep shape, m = 2^17, n = 50, kappa =
    10^2 .. 10^12 in half decades: ICE and the block 1-norm estimate on the
    FP64 sketch factor Rs (one sketch, s = 2n), the Gram bound (needs A^T A and
    its Cholesky: one more pass over A), the CholQR probe (one CholQR pass).
    A result in a lower regime than kappa's own would be caught by the
    posterior check; a higher one only costs time."""
    m, n, s = 1 << 17, 50, 100
    ev = lambda: torch.cuda.Event(enable_timing=True)
    counts = {k: [0, 0, 0] for k in ("ice", "1norm", "gram", "probe")}  # low, right, high
    times = {k: 0.0 for k in counts}
    exps = np.arange(2.0, 12.01, 0.5)
    # warm-up of every kernel involved (first launches load code objects)
    A0 = to_dev(W.paper_sweep_matrix(m, n, 1e3, 799))
    S0 = M.draw(5, m, s)
    R0, _ = M.sketch_qr(M.sketch(A0, S0, 5, "fp64"), "fp64")
    M.condest_1norm(R0)
    G0 = M.gram(A0)
    M.condest_1norm(M.cholesky(G0)[0], G0)
    M.cholqr_probe(A0)
    torch.cuda.synchronize()
    for e in exps:
        kappa = 10.0 ** e
        A = to_dev(W.paper_sweep_matrix(m, n, kappa, 800 + int(2 * e)))
        t = {}
        e0, e1 = ev(), ev()
        e0.record()
        S = M.draw(5, m, s)
        Rs, kap_ice = M.sketch_qr(M.sketch(A, S, 5, "fp64"), "fp64")
        e1.record()
        torch.cuda.synchronize()
        t["ice"] = e0.elapsed_time(e1)
        e0.record()
        k1 = M.condest_1norm(Rs, seed=5)
        e1.record()
        torch.cuda.synchronize()
        t["1norm"] = t["ice"] + e0.elapsed_time(e1)
        e0.record()
        G = M.gram(A)
        Rg, fail, _ = M.cholesky(G)
        kg = M.condest_1norm(Rg, G, seed=5)
        e1.record()
        torch.cuda.synchronize()
        t["gram"] = e0.elapsed_time(e1)
        kg = float("inf") if int(to_host(fail)[0]) >= 0 else float(to_host(kg)[0])
        e0.record()
        kp = M.cholqr_probe(A)
        e1.record()
        torch.cuda.synchronize()
        t["probe"] = e0.elapsed_time(e1)
        est = {"ice": float(to_host(kap_ice)[0]), "1norm": float(to_host(k1)[0]), "gram": kg,
               "probe": float(to_host(kp)[0])}
        for k, v in est.items():
            d = _regime(v) - _regime(kappa)
            counts[k][0 if d < 0 else (1 if d == 0 else 2)] += 1
            times[k] += t[k]
        progress(f"estimators kappa=1e{e:.1f}: " + ", ".join(f"{k} {v:.2e}" for k, v in est.items()))
    for k in counts:
        lo, ok, hi = counts[k]
        progress(f"estimator {k}: regime below kappa's {lo}, right {ok}, above {hi} of {len(exps)}; "
                 f"mean {times[k] / len(exps):.3f} ms per estimate (step entry points, incl. their allocations)")
    # ICE and the probe are lower bounds: they never land above kappa's regime
    # except at a boundary by rounding; the 1-norm based ones never below it
    assert counts["1norm"][0] == 0 and counts["gram"][0] == 0
    assert counts["probe"][2] == 0
