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
