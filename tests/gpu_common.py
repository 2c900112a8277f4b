"""Helpers shared by the GPU tests (host-side conversions only)."""
import numpy as np
import pytest

torch = pytest.importorskip("torch")


def require_gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2606_18411_amd as M
    M.lib()  # raises if the HIP library is missing: no silent fallback
    return M


def to_dev(x: np.ndarray):
    """float64 numpy (any order) -> column-major float64 CUDA tensor."""
    x = np.asarray(x, dtype=np.float64)
    t = torch.from_numpy(np.ascontiguousarray(x.T)).cuda()
    return t.t()


def to_host(t) -> np.ndarray:
    return t.detach().cpu().numpy()


def progress(msg: str):
    print(f"[case] {msg}", flush=True)


def _chunked_gram_dev(X, chunk: int = 8192) -> np.ndarray:
    """X^T X of a device matrix: float64 products of row chunks on the GPU,
    the chunk results summed pairwise in float64 on the host (the evaluation
    error stays far below 1e-13; a single product over all rows would not
    guarantee that)."""
    parts = [to_host(X[i:i + chunk].t() @ X[i:i + chunk]) for i in range(0, X.shape[0], chunk)]
    while len(parts) > 1:
        parts = [parts[i] + parts[i + 1] if i + 1 < len(parts) else parts[i] for i in range(0, len(parts), 2)]
    return parts[0]


def dev_orthogonality(Q) -> float:
    """||I - Q^T Q||_2 of a device Q."""
    E = np.eye(Q.shape[1]) - _chunked_gram_dev(Q)
    return float(np.max(np.abs(np.linalg.eigvalsh(0.5 * (E + E.T)))))


def dev_residual(A, Q, R) -> float:
    """||A - Q R||_2 / ||A||_2 of device matrices (2-norms from n x n Grams)."""
    E = A - Q @ R
    G = _chunked_gram_dev(E)
    GA = _chunked_gram_dev(A)
    en = np.sqrt(max(np.max(np.linalg.eigvalsh(0.5 * (G + G.T))), 0.0))
    return float(en / np.sqrt(np.max(np.linalg.eigvalsh(0.5 * (GA + GA.T)))))
