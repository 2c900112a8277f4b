"""Repeated-QR drivers on the captured MRCQR call: the workloads the paper
names for sequences of similar factorizations (Section "Introduction" and
Section "Adaptive Precision Selection", repeated calls: block Arnoldi and
randomized SVD via power iteration), where one regime classification is
reused by the calls that follow.

Each driver factors its blocks with one MRCQR call of fixed shape captured
in a HIP graph and replayed per block, with the AUTO_CARRY policy by
default: a call starts from the precision the previous call accepted and
escalates on the device, so the precision follows the slowly worsening
conditioning of the sequence without a host round trip. The products with
the operator are plain float64 library GEMMs (torch.mm) of the driver, not
part of the factorization.
"""
from __future__ import annotations

from dataclasses import dataclass, field

import torch

from . import Plan, empty_colmajor


class CapturedQR:
    """One MRCQR call for (m, b) matrices captured in a HIP graph.

    call(W) copies W into the captured input, replays the graph and returns
    (Q, R, info); Q and R are the captured output buffers (overwritten by
    the next call: copy them to keep them)."""

    def __init__(self, m: int, b: int, precision: str = "auto_carry", seed: int = 0, transform: str = "dct",
                 device="cuda"):
        self.plan = Plan(m, b, device=device, transform=transform)
        self.A = empty_colmajor(m, b, device)
        self.Q = empty_colmajor(m, b, device)
        self.R = empty_colmajor(b, b, device)
        self.A.zero_()
        self.A.diagonal().fill_(1.0)  # any full-rank input for the warm-up call
        side = torch.cuda.Stream()
        side.wait_stream(torch.cuda.current_stream())
        with torch.cuda.stream(side):
            self.plan.execute(self.A, self.Q, self.R, precision, seed=seed)
        torch.cuda.current_stream().wait_stream(side)
        torch.cuda.synchronize()
        self.graph = torch.cuda.CUDAGraph()
        with torch.cuda.graph(self.graph):
            self.plan.execute(self.A, self.Q, self.R, precision, seed=seed)
        torch.cuda.synchronize()
        self.plan.reset_regime()
        torch.cuda.synchronize()

    def __call__(self, W: torch.Tensor):
        self.A.copy_(W)
        self.graph.replay()
        torch.cuda.synchronize()
        return self.Q, self.R, self.plan.last_info()

    def reset_regime(self) -> None:
        self.plan.reset_regime()
        torch.cuda.synchronize()


def basis_orthogonality(V: torch.Tensor, chunk: int = 1 << 15) -> float:
    """||I - V^T V||_2 with the Gram matrix summed over row chunks in float64."""
    G = None
    for i in range(0, V.shape[0], chunk):
        part = V[i:i + chunk].t() @ V[i:i + chunk]
        G = part if G is None else G + part
    E = torch.eye(V.shape[1], dtype=V.dtype, device=V.device) - G
    return float(torch.linalg.eigvalsh(0.5 * (E + E.t())).abs().max())


@dataclass
class RepeatedQRResult:
    """The output of a driver: the basis (m x columns), per call the info of
    the factorization, and the orthogonality of the whole basis."""
    basis: torch.Tensor
    infos: list = field(default_factory=list)
    orthogonality: float = float("nan")

    @property
    def precisions(self):
        return [i.precision for i in self.infos]


def power_range(M: torch.Tensor, b: int, q: int, seed: int = 0, precision: str = "auto_carry",
                Omega: torch.Tensor | None = None, on_step=None) -> RepeatedQRResult:
    """Randomized range finder with power steps, Y_j = (M M^T)^j M Omega for
    j = 0 .. q, each factored in turn by the captured call (no
    orthonormalization between the products, so kappa(Y_j) grows like
    (sigma_1 / sigma_b)^(2j+1) and the carried precision climbs). Returns the
    last basis; on_step(j, Q, R, info) is called after every factorization."""
    m, N = M.shape
    if Omega is None:
        gen = torch.Generator(device=M.device)
        gen.manual_seed(int(seed))
        Omega = torch.randn(N, b, dtype=M.dtype, device=M.device, generator=gen)
    qr = CapturedQR(m, b, precision, seed, device=M.device)
    Mt = M.t().contiguous()
    Z = M @ Omega
    res = RepeatedQRResult(basis=None)
    for j in range(q + 1):
        if j > 0:
            Z = M @ (Mt @ Z)
        Q, R, info = qr(Z)
        res.infos.append(info)
        if on_step is not None:
            on_step(j, Q, R, info)
    res.basis = Q.clone()
    res.orthogonality = basis_orthogonality(res.basis)
    return res


def block_krylov(M: torch.Tensor, b: int, k: int, seed: int = 0, precision: str = "auto_carry",
                 Omega: torch.Tensor | None = None) -> RepeatedQRResult:
    """Block Krylov basis of M M^T started from M Omega (block Arnoldi on the
    symmetric operator): V_0 = qr(M Omega), and for j = 1 .. k the block
    W = M M^T V_{j-1} is orthogonalized against V = [V_0 .. V_{j-1}] by block
    classical Gram-Schmidt with reorthogonalization (Barlow and
    Smoktunowicz's BCGS2): Q1 = qr(W - V V^T W), V_j = qr(Q1 - V V^T Q1),
    both factorizations by the captured call. Without the second pass the
    coupling V^T W left by the first projection is amplified by R^{-1} when
    W lies close to span(V), as it does once the Krylov space has converged.
    The basis [V_0 .. V_k] (m x (k+1) b) and its orthogonality are
    returned; infos holds both calls per block."""
    m, N = M.shape
    if Omega is None:
        gen = torch.Generator(device=M.device)
        gen.manual_seed(int(seed))
        Omega = torch.randn(N, b, dtype=M.dtype, device=M.device, generator=gen)
    qr = CapturedQR(m, b, precision, seed, device=M.device)
    Mt = M.t().contiguous()
    basis = torch.empty((k + 1) * b, m, dtype=M.dtype, device=M.device).t()  # column-major
    res = RepeatedQRResult(basis=basis)
    Q, _, info = qr(M @ Omega)
    res.infos.append(info)
    basis[:, :b].copy_(Q)
    for j in range(1, k + 1):
        W = M @ (Mt @ basis[:, (j - 1) * b:j * b])
        V = basis[:, :j * b]
        for _ in range(2):
            Q, _, info = qr(W - V @ (V.t() @ W))
            res.infos.append(info)
            W = Q.clone()
        basis[:, j * b:(j + 1) * b].copy_(W)
    res.orthogonality = basis_orthogonality(basis)
    return res
