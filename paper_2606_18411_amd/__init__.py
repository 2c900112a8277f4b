"""MRCQR on MI355X: mixed-precision randomized Cholesky-QR (arXiv 2606.18411).

A thin Python binding over the C ABI of libmrcqr.so (include/mrcqr.h). It
only marshals arguments: every step of the factorization runs in the HIP
kernels of the library. PyTorch supplies device memory and the stream.

Matrices are float64 CUDA tensors in column-major layout: shape (m, n) with
stride (1, ld), ld >= m (e.g. ``torch.empty(n, m).t()``); ``colmajor()``
converts.

If the library is not built, or is built but cannot be loaded, every call
raises RuntimeError; there is no fallback.
"""
from __future__ import annotations

import ctypes
import os
import struct
from dataclasses import dataclass

import torch

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libmrcqr.so")

PREC = {"auto": 0, "fp64": 1, "fp32": 2, "fp16": 3, "bf16": 4, "auto_carry": 5}
PREC_NAME = {v: k for k, v in PREC.items()}
STATUS = {
    0: "ok", 1: "invalid argument", 2: "non-finite sketch", 3: "cholesky breakdown",
    4: "sketch singular", 5: "workspace", 6: "device error", 7: "posterior warning", 8: "unsupported",
}
TRANSFORM = {"dct": 0, "rfft": 1}  # sketch transform: DCT-II rows, or the paper's real DFT bins
OK, ERR_ARG, ERR_NONFINITE, ERR_CHOL, ERR_SINGULAR, ERR_WORKSPACE, ERR_DEVICE, WARN_POSTERIOR, ERR_UNSUPPORTED = range(9)

_lib = None


class MrcqrError(RuntimeError):
    def __init__(self, code: int, where: str):
        super().__init__(f"{where}: {STATUS.get(code, code)} (code {code})")
        self.code = code


def lib() -> ctypes.CDLL:
    """Load libmrcqr.so (once); raise if it is missing."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is not built; run python -m paper_2606_18411_amd.build")
        L = ctypes.CDLL(LIB_PATH)
        i64, u64, i32, vp, sz = ctypes.c_int64, ctypes.c_uint64, ctypes.c_int, ctypes.c_void_p, ctypes.c_size_t
        sig = {
            "mrcqr_factor": (i32, [vp, i64, i64, i64, i32, u64, i64, vp, i64, vp, i64, vp, vp]),
            "mrcqr_plan_create": (i32, [i64, i64, i64, ctypes.POINTER(vp)]),
            "mrcqr_plan_create_ex": (i32, [i64, i64, i64, i32, ctypes.POINTER(vp)]),
            "mrcqr_sketch_ex": (i32, [vp, i64, i64, i64, vp, i64, u64, i32, i32, vp, i64, vp, sz, vp]),
            "mrcqr_plan_workspace_bytes": (sz, [vp]),
            "mrcqr_execute": (i32, [vp, vp, sz, vp, i64, i32, u64, vp, i64, vp, i64, vp, vp]),
            "mrcqr_plan_destroy": (i32, [vp]),
            "mrcqr_factor_batched": (i32, [ctypes.c_int32, vp, vp, vp, vp, vp, vp, vp, vp, vp, vp, vp, vp]),
            "mrcqr_draw": (i32, [u64, i64, i64, vp, vp, vp]),
            "mrcqr_sketch_workspace_bytes": (sz, [i64, i64, i64, i32]),
            "mrcqr_sketch": (i32, [vp, i64, i64, i64, vp, i64, u64, i32, vp, i64, vp, sz, vp]),
            "mrcqr_sketch_qr": (i32, [vp, i64, i64, i64, i32, vp, i64, vp, vp]),
            "mrcqr_trsm_workspace_bytes": (sz, [i64]),
            "mrcqr_trsm": (i32, [vp, i64, i64, i64, vp, i64, vp, i64, vp, sz, vp]),
            "mrcqr_cholqr2_workspace_bytes": (sz, [i64, i64]),
            "mrcqr_cholqr2": (i32, [vp, i64, i64, i64, vp, i64, vp, i64, vp, sz, vp, vp]),
            "mrcqr_gram_workspace_bytes": (sz, [i64, i64]),
            "mrcqr_gram": (i32, [vp, i64, i64, i64, vp, i64, vp, sz, vp]),
            "mrcqr_cholesky": (i32, [vp, i64, i64, vp, i64, vp, vp, vp]),
            "mrcqr_trmm": (i32, [vp, i64, vp, i64, i64, vp, i64, vp]),
            "mrcqr_tri_inverse": (i32, [vp, i64, i64, vp, i64, vp]),
            "mrcqr_form_q": (i32, [vp, i64, i64, i64, vp, i64, vp, i64, vp]),
            "mrcqr_condest": (i32, [vp, i64, i64, vp, vp]),
            "mrcqr_posterior_kappa": (i32, [vp, vp, i64, i64, vp, vp, vp]),
            "mrcqr_posterior_workspace_bytes": (sz, [i64]),
            "mrcqr_release_cache": (i32, []),
            "mrcqr_condest_1norm": (i32, [vp, vp, i64, i64, u64, vp, vp]),
            "mrcqr_cholqr_probe_workspace_bytes": (sz, [i64, i64]),
            "mrcqr_cholqr_probe": (i32, [vp, i64, i64, i64, vp, sz, vp, vp]),
            "mrcqr_regime_reset": (i32, [vp, vp, sz, vp]),
            "mrcqr_batch_plan_create": (i32, [i32, vp, vp, ctypes.POINTER(vp)]),
            "mrcqr_batch_plan_workspace_bytes": (sz, [vp]),
            "mrcqr_batch_plan_destroy": (i32, [vp]),
            "mrcqr_batch_execute": (i32, [vp, vp, sz, vp, vp, vp, vp, vp, vp, vp, vp, vp, vp]),
            "mrcqr_status_string": (ctypes.c_char_p, [i32]),
            "mrcqr_version": (i32, []),
        }
        for name, (res, args) in sig.items():
            f = getattr(L, name)
            f.restype = res
            f.argtypes = args
        _lib = L
    return _lib


def _check(code: int, where: str) -> None:
    if code != OK:
        raise MrcqrError(code, where)


def _stream(stream) -> int:
    if stream is None:
        return torch.cuda.current_stream().cuda_stream
    return stream.cuda_stream if hasattr(stream, "cuda_stream") else int(stream)


def _prec(p) -> int:
    return PREC[p] if isinstance(p, str) else int(p)


def colmajor(x: torch.Tensor) -> torch.Tensor:
    """Column-major copy (stride (1, m)) of a 2-D tensor unless it already is one."""
    if x.dim() != 2:
        raise ValueError("expected a 2-D tensor")
    if x.stride(0) == 1 and x.stride(1) >= max(1, x.shape[0]):
        return x
    return x.t().contiguous().t()


def empty_colmajor(m: int, n: int, device="cuda", dtype=torch.float64) -> torch.Tensor:
    return torch.empty((n, m), device=device, dtype=dtype).t()


def _ld(x: torch.Tensor) -> int:
    if x.dim() != 2 or (x.shape[0] > 1 and x.stride(0) != 1):
        raise ValueError("matrices must be column-major (stride(0) == 1)")
    return max(x.stride(1), x.shape[0], 1)


def _mat(x, rows: int, cols: int, name: str) -> None:
    """Check before any launch that x is a column-major float64 matrix of
    shape (rows, cols): the library can only check leading dimensions, so a
    wrong shape or dtype would turn into out-of-bounds device accesses."""
    if not isinstance(x, torch.Tensor) or x.dim() != 2:
        raise ValueError(f"{name} must be a 2-D tensor")
    if tuple(x.shape) != (rows, cols):
        raise ValueError(f"{name} has shape {tuple(x.shape)}, expected ({rows}, {cols})")
    if x.dtype != torch.float64:
        raise TypeError(f"{name} must be float64, got {x.dtype}")
    # a single row or column has no layout to check in that dimension
    if (rows > 1 and x.stride(0) != 1) or (cols > 1 and x.stride(1) < rows):
        raise ValueError(f"{name} must be column-major (stride (1, ld), ld >= {rows})")


def _same_cuda_device(named, device=None) -> None:
    """Every tensor of `named` ((name, tensor) pairs) is a CUDA tensor on one
    device (`device` when given). Checked after the shapes, last before the
    library is called."""
    for name, x in named:
        if not x.is_cuda:
            raise TypeError(f"{name} must be a CUDA tensor")
        if device is None:
            device = x.device
        elif x.device != torch.device(device):
            raise ValueError(f"{name} is on {x.device}, expected {device}")


@dataclass
class Info:
    status: int
    precision_used: int
    chol_fail_index: int
    escalations: int
    kappa_rs_est: float
    kappa_rc_est: float

    @property
    def precision(self) -> str:
        return PREC_NAME.get(self.precision_used, str(self.precision_used))

    @property
    def ok(self) -> bool:
        return self.status == OK

    @staticmethod
    def from_bytes(b: bytes) -> "Info":
        return Info(*struct.unpack("<iiiidd", b))


INFO_BYTES = 32


def read_infos(buf: torch.Tensor, count: int = 1):
    host = buf.cpu().numpy().tobytes()
    return [Info.from_bytes(host[i * INFO_BYTES:(i + 1) * INFO_BYTES]) for i in range(count)]


def factor(A: torch.Tensor, precision="fp16", seed: int = 0, s: int | None = None,
           Q: torch.Tensor | None = None, R: torch.Tensor | None = None, stream=None,
           sync: bool = True):
    """Thin QR A = Q R by MRCQR. Returns (Q, R, Info) (Info None if sync=False)."""
    if not isinstance(A, torch.Tensor) or A.dim() != 2:
        raise ValueError("A must be a 2-D tensor")
    m, n = A.shape
    _mat(A, m, n, "A")
    if Q is not None:
        _mat(Q, m, n, "Q")
    if R is not None:
        _mat(R, n, n, "R")
    _same_cuda_device([("A", A)] + ([("Q", Q)] if Q is not None else []) + ([("R", R)] if R is not None else []))
    if Q is None:
        Q = empty_colmajor(m, n, A.device)
    if R is None:
        R = empty_colmajor(n, n, A.device)
    info = torch.empty(INFO_BYTES, dtype=torch.uint8, device=A.device)
    code = lib().mrcqr_factor(A.data_ptr(), m, n, _ld(A), _prec(precision), seed & (2 ** 64 - 1), s or 0,
                              Q.data_ptr(), _ld(Q), R.data_ptr(), _ld(R), _stream(stream), info.data_ptr())
    _check(code, "mrcqr_factor")
    if not sync:
        return Q, R, info
    torch.cuda.synchronize(A.device)
    return Q, R, read_infos(info)[0]


def cholqr2(A: torch.Tensor, stream=None, sync: bool = True):
    """CholQR2 (Algorithm 1 twice), the paper's stability baseline.
    Returns (Q, R, Info)."""
    if not isinstance(A, torch.Tensor) or A.dim() != 2:
        raise ValueError("A must be a 2-D tensor")
    m, n = A.shape
    _mat(A, m, n, "A")
    _same_cuda_device([("A", A)])
    Q, R = empty_colmajor(m, n, A.device), empty_colmajor(n, n, A.device)
    wsb = int(lib().mrcqr_cholqr2_workspace_bytes(m, n))
    ws = torch.empty(max(wsb, 1), dtype=torch.uint8, device=A.device)
    info = torch.empty(INFO_BYTES, dtype=torch.uint8, device=A.device)
    _check(lib().mrcqr_cholqr2(A.data_ptr(), m, n, _ld(A), Q.data_ptr(), _ld(Q), R.data_ptr(), _ld(R),
                               ws.data_ptr(), wsb, _stream(stream), info.data_ptr()), "mrcqr_cholqr2")
    if not sync:
        return Q, R, info
    torch.cuda.synchronize(A.device)
    return Q, R, read_infos(info)[0]


class Plan:
    """A plan for fixed (m, n, s) with its own workspace; execute() allocates nothing.
    transform: "dct" (DCT-II rows, default s = 2n) or "rfft" (the paper's real
    DFT bins, default s = 3n)."""

    def __init__(self, m: int, n: int, s: int | None = None, device="cuda", transform: str = "dct"):
        p = ctypes.c_void_p()
        _check(lib().mrcqr_plan_create_ex(m, n, s or 0, TRANSFORM[transform], ctypes.byref(p)),
               "mrcqr_plan_create_ex")
        self.transform = transform
        self._p = p
        self.m, self.n = m, n
        self.workspace_bytes = int(lib().mrcqr_plan_workspace_bytes(p))
        # zero bytes: no AUTO_CARRY record, so the first carrying call starts from FP16
        self.workspace = torch.zeros(self.workspace_bytes, dtype=torch.uint8, device=device)
        self.info = torch.empty(INFO_BYTES, dtype=torch.uint8, device=device)

    def execute(self, A, Q, R, precision="fp16", seed: int = 0, stream=None):
        _mat(A, self.m, self.n, "A")
        _mat(Q, self.m, self.n, "Q")
        _mat(R, self.n, self.n, "R")
        _same_cuda_device([("A", A), ("Q", Q), ("R", R)], self.workspace.device)
        _check(lib().mrcqr_execute(self._p, self.workspace.data_ptr(), self.workspace_bytes, A.data_ptr(), _ld(A),
                                   _prec(precision), seed & (2 ** 64 - 1), Q.data_ptr(), _ld(Q), R.data_ptr(),
                                   _ld(R), _stream(stream), self.info.data_ptr()), "mrcqr_execute")

    def reset_regime(self, stream=None):
        """Forget the precision carried by 'auto_carry' calls on this plan."""
        _check(lib().mrcqr_regime_reset(self._p, self.workspace.data_ptr(), self.workspace_bytes,
                                        _stream(stream)), "mrcqr_regime_reset")

    def last_info(self) -> Info:
        return read_infos(self.info)[0]

    def __del__(self):
        try:
            if getattr(self, "_p", None) is not None and _lib is not None:
                _lib.mrcqr_plan_destroy(self._p)
        except Exception:
            pass


def _as_int64(u: int) -> int:
    return u - 2 ** 64 if u >= 2 ** 63 else u


class BatchPlan:
    """A batch of independent factorizations of shapes [(m, n), ...] (s = 2n),
    run as grouped launches; execute() allocates nothing once the per-member
    argument arrays (device tensors) are set with bind()."""

    def __init__(self, shapes, device="cuda"):
        k = len(shapes)
        ms = (ctypes.c_int64 * k)(*[int(m) for m, _ in shapes])
        ns = (ctypes.c_int64 * k)(*[int(n) for _, n in shapes])
        p = ctypes.c_void_p()
        _check(lib().mrcqr_batch_plan_create(k, ms, ns, ctypes.byref(p)), "mrcqr_batch_plan_create")
        self._p = p
        self.shapes = [(int(m), int(n)) for m, n in shapes]
        self.device = device
        self.workspace_bytes = int(lib().mrcqr_batch_plan_workspace_bytes(p))
        # zero bytes: no AUTO_CARRY records
        self.workspace = torch.zeros(self.workspace_bytes, dtype=torch.uint8, device=device)
        self.infos = torch.empty(INFO_BYTES * k, dtype=torch.uint8, device=device)
        self._args = None

    def bind(self, As, Qs, Rs, precisions, seeds):
        """Per-member arguments as device arrays (kept alive by the plan)."""
        dev = self.device
        k = len(self.shapes)
        if not (len(As) == len(Qs) == len(Rs) == k) or len(list(seeds)) != k:
            raise ValueError(f"expected {k} members in As, Qs, Rs and seeds")
        named = []
        for i, ((m, n), a, q, r) in enumerate(zip(self.shapes, As, Qs, Rs)):
            _mat(a, m, n, f"As[{i}]")
            _mat(q, m, n, f"Qs[{i}]")
            _mat(r, n, n, f"Rs[{i}]")
            named += [(f"As[{i}]", a), (f"Qs[{i}]", q), (f"Rs[{i}]", r)]
        _same_cuda_device(named, self.workspace.device)
        i64 = lambda vals: torch.tensor(vals, dtype=torch.int64, device=dev)
        precs = precisions if isinstance(precisions, (list, tuple)) else [precisions] * len(As)
        if len(precs) != k:
            raise ValueError(f"expected {k} precisions")
        self._args = (
            i64([a.data_ptr() for a in As]), i64([_ld(a) for a in As]),
            torch.tensor([_prec(q) for q in precs], dtype=torch.int32, device=dev),
            i64([_as_int64(int(x) & (2 ** 64 - 1)) for x in seeds]),  # uint64 bits in an int64 tensor
            i64([q.data_ptr() for q in Qs]), i64([_ld(q) for q in Qs]),
            i64([r.data_ptr() for r in Rs]), i64([_ld(r) for r in Rs]),
            (As, Qs, Rs),
        )

    def execute(self, stream=None, infos=True):
        a = self._args
        if a is None:
            raise RuntimeError("BatchPlan.execute before bind()")
        _check(lib().mrcqr_batch_execute(self._p, self.workspace.data_ptr(), self.workspace_bytes, a[0].data_ptr(),
                                         a[1].data_ptr(), a[2].data_ptr(), a[3].data_ptr(), a[4].data_ptr(),
                                         a[5].data_ptr(), a[6].data_ptr(), a[7].data_ptr(), _stream(stream),
                                         self.infos.data_ptr() if infos else None), "mrcqr_batch_execute")

    def last_infos(self):
        return read_infos(self.infos, len(self.shapes))

    def __del__(self):
        try:
            if getattr(self, "_p", None) is not None and _lib is not None:
                _lib.mrcqr_batch_plan_destroy(self._p)
        except Exception:
            pass


def factor_batched(As, precision="auto", seeds=None, stream=None):
    """Factor a list of column-major float64 CUDA matrices; returns (Qs, Rs, infos)."""
    k = len(As)
    for i, a in enumerate(As):
        if not isinstance(a, torch.Tensor) or a.dim() != 2:
            raise ValueError(f"As[{i}] must be a 2-D tensor")
        _mat(a, a.shape[0], a.shape[1], f"As[{i}]")
    _same_cuda_device([(f"As[{i}]", a) for i, a in enumerate(As)])
    seeds = list(seeds) if seeds is not None else list(range(k))
    precs = [precision] * k if isinstance(precision, (str, int)) else list(precision)
    Qs = [empty_colmajor(a.shape[0], a.shape[1], a.device) for a in As]
    Rs = [empty_colmajor(a.shape[1], a.shape[1], a.device) for a in As]
    arr = lambda ctype, vals: (ctype * k)(*vals)
    infos = torch.empty(INFO_BYTES * k, dtype=torch.uint8, device=As[0].device if k else "cuda")
    code = lib().mrcqr_factor_batched(
        k, arr(ctypes.c_void_p, [a.data_ptr() for a in As]), arr(ctypes.c_int64, [a.shape[0] for a in As]),
        arr(ctypes.c_int64, [a.shape[1] for a in As]), arr(ctypes.c_int64, [_ld(a) for a in As]),
        arr(ctypes.c_int32, [_prec(p) for p in precs]), arr(ctypes.c_uint64, [s & (2 ** 64 - 1) for s in seeds]),
        arr(ctypes.c_void_p, [q.data_ptr() for q in Qs]), arr(ctypes.c_int64, [_ld(q) for q in Qs]),
        arr(ctypes.c_void_p, [r.data_ptr() for r in Rs]), arr(ctypes.c_int64, [_ld(r) for r in Rs]),
        _stream(stream), infos.data_ptr() if k else None)
    _check(code, "mrcqr_factor_batched")
    torch.cuda.synchronize()
    return Qs, Rs, read_infos(infos, k) if k else []


# ---- individual steps ----------------------------------------------------

def draw(seed: int, m: int, s: int, signs: bool = False, device="cuda", stream=None):
    S = torch.empty(s, dtype=torch.int32, device=device)
    D = torch.empty(m, dtype=torch.int8, device=device) if signs else None
    _check(lib().mrcqr_draw(seed & (2 ** 64 - 1), m, s, S.data_ptr(), D.data_ptr() if D is not None else None,
                            _stream(stream)), "mrcqr_draw")
    return (S, D) if signs else S


def sketch(A: torch.Tensor, S: torch.Tensor, seed: int, precision="fp16", stream=None,
           transform: str = "dct") -> torch.Tensor:
    m, n = A.shape
    _mat(A, m, n, "A")
    if not (isinstance(S, torch.Tensor) and S.dim() == 1 and S.dtype == torch.int32):
        raise TypeError("S must be a 1-D int32 tensor")
    s = S.shape[0]
    _same_cuda_device([("A", A), ("S", S)])
    kmax = m // 2 + 1 if transform == "rfft" else m
    if s < 1 or s > kmax or int(S.min()) < 0 or int(S.max()) >= kmax:
        raise ValueError(f"S must hold 1..{kmax} indices in [0, {kmax})")
    Y = empty_colmajor(s, n, A.device)
    p = _prec(precision)
    wsb = int(lib().mrcqr_sketch_workspace_bytes(m, n, s, p))
    ws = torch.empty(max(wsb, 1), dtype=torch.uint8, device=A.device)
    _check(lib().mrcqr_sketch_ex(A.data_ptr(), m, n, _ld(A), S.data_ptr(), s, seed & (2 ** 64 - 1), p,
                                 TRANSFORM[transform], Y.data_ptr(), _ld(Y), ws.data_ptr(), wsb, _stream(stream)),
           "mrcqr_sketch_ex")
    return Y


def sketch_qr(Y: torch.Tensor, precision="fp32", stream=None):
    s, n = Y.shape
    _mat(Y, s, n, "Y")
    _same_cuda_device([("Y", Y)])
    Rs = empty_colmajor(n, n, Y.device)
    kappa = torch.empty(1, dtype=torch.float64, device=Y.device)
    _check(lib().mrcqr_sketch_qr(Y.data_ptr(), s, n, _ld(Y), _prec(precision), Rs.data_ptr(), _ld(Rs),
                                 kappa.data_ptr(), _stream(stream)), "mrcqr_sketch_qr")
    return Rs, kappa


def trsm(A: torch.Tensor, R: torch.Tensor, X: torch.Tensor | None = None, stream=None,
         workspace: torch.Tensor | None = None) -> torch.Tensor:
    m, n = A.shape
    _mat(A, m, n, "A")
    _mat(R, n, n, "R")
    if X is not None:
        _mat(X, m, n, "X")
    _same_cuda_device([("A", A), ("R", R)] + ([("X", X)] if X is not None else []))
    if X is None:
        X = empty_colmajor(m, n, A.device)
    wsb = int(lib().mrcqr_trsm_workspace_bytes(n))
    if workspace is None or workspace.numel() < wsb:
        workspace = torch.empty(max(wsb, 1), dtype=torch.uint8, device=A.device)
    _check(lib().mrcqr_trsm(A.data_ptr(), m, n, _ld(A), R.data_ptr(), _ld(R), X.data_ptr(), _ld(X),
                            workspace.data_ptr(), wsb, _stream(stream)), "mrcqr_trsm")
    return X


def gram(B: torch.Tensor, stream=None) -> torch.Tensor:
    m, n = B.shape
    _mat(B, m, n, "B")
    _same_cuda_device([("B", B)])
    G = empty_colmajor(n, n, B.device)
    wsb = int(lib().mrcqr_gram_workspace_bytes(m, n))
    ws = torch.empty(max(wsb, 1), dtype=torch.uint8, device=B.device)
    _check(lib().mrcqr_gram(B.data_ptr(), m, n, _ld(B), G.data_ptr(), _ld(G), ws.data_ptr(), wsb,
                            _stream(stream)), "mrcqr_gram")
    return G


def cholesky(G: torch.Tensor, stream=None):
    n = G.shape[0]
    _mat(G, n, n, "G")
    _same_cuda_device([("G", G)])
    Rc = empty_colmajor(n, n, G.device)
    fail = torch.empty(1, dtype=torch.int32, device=G.device)
    kappa = torch.empty(1, dtype=torch.float64, device=G.device)
    _check(lib().mrcqr_cholesky(G.data_ptr(), n, _ld(G), Rc.data_ptr(), _ld(Rc), fail.data_ptr(),
                                kappa.data_ptr(), _stream(stream)), "mrcqr_cholesky")
    return Rc, fail, kappa


def trmm(R2: torch.Tensor, R1: torch.Tensor, stream=None) -> torch.Tensor:
    n = R2.shape[0]
    _mat(R2, n, n, "R2")
    _mat(R1, n, n, "R1")
    _same_cuda_device([("R2", R2), ("R1", R1)])
    R = empty_colmajor(n, n, R2.device)
    _check(lib().mrcqr_trmm(R2.data_ptr(), _ld(R2), R1.data_ptr(), _ld(R1), n, R.data_ptr(), _ld(R),
                            _stream(stream)), "mrcqr_trmm")
    return R


def tri_inverse(R: torch.Tensor, stream=None) -> torch.Tensor:
    n = R.shape[0]
    _mat(R, n, n, "R")
    _same_cuda_device([("R", R)])
    X = empty_colmajor(n, n, R.device)
    _check(lib().mrcqr_tri_inverse(R.data_ptr(), n, _ld(R), X.data_ptr(), _ld(X), _stream(stream)),
           "mrcqr_tri_inverse")
    return X


def form_q(B: torch.Tensor, X: torch.Tensor, Q: torch.Tensor | None = None, stream=None) -> torch.Tensor:
    m, n = B.shape
    _mat(B, m, n, "B")
    _mat(X, n, n, "X")
    if Q is not None:
        _mat(Q, m, n, "Q")
    _same_cuda_device([("B", B), ("X", X)] + ([("Q", Q)] if Q is not None else []))
    if Q is None:
        Q = empty_colmajor(m, n, B.device)
    _check(lib().mrcqr_form_q(B.data_ptr(), m, n, _ld(B), X.data_ptr(), _ld(X), Q.data_ptr(), _ld(Q),
                              _stream(stream)), "mrcqr_form_q")
    return Q


def condest(R: torch.Tensor, stream=None) -> torch.Tensor:
    n = R.shape[0]
    _mat(R, n, n, "R")
    _same_cuda_device([("R", R)])
    kappa = torch.empty(1, dtype=torch.float64, device=R.device)
    _check(lib().mrcqr_condest(R.data_ptr(), n, _ld(R), kappa.data_ptr(), _stream(stream)), "mrcqr_condest")
    return kappa


def posterior_kappa(R: torch.Tensor, X: torch.Tensor, stream=None) -> torch.Tensor:
    """Power-step estimate sigma_max(R) sigma_max(X) (X = R^{-1}) used by the
    posterior check; R and X must share one leading dimension."""
    n = R.shape[0]
    _mat(R, n, n, "R")
    _mat(X, n, n, "X")
    _same_cuda_device([("R", R), ("X", X)])
    if _ld(R) != _ld(X):
        raise ValueError("R and X must have the same leading dimension")
    kappa = torch.empty(1, dtype=torch.float64, device=R.device)
    wsb = int(lib().mrcqr_posterior_workspace_bytes(n))
    ws = torch.empty(wsb, dtype=torch.uint8, device=R.device) if wsb else None
    _check(lib().mrcqr_posterior_kappa(R.data_ptr(), X.data_ptr(), n, _ld(R), kappa.data_ptr(),
                                       ws.data_ptr() if ws is not None else None, _stream(stream)),
           "mrcqr_posterior_kappa")
    return kappa


def condest_1norm(R: torch.Tensor, G: torch.Tensor | None = None, seed: int = 0, stream=None) -> torch.Tensor:
    """Block 1-norm estimate: kappa_1(R), or (with G = R^T R) the paper's bound
    sqrt(n ||G||_1 ||G^{-1}||_1)."""
    n = R.shape[0]
    _mat(R, n, n, "R")
    if G is not None:
        _mat(G, n, n, "G")
        if _ld(G) != _ld(R):
            raise ValueError("R and G must have the same leading dimension")
    _same_cuda_device([("R", R)] + ([("G", G)] if G is not None else []))
    kappa = torch.empty(1, dtype=torch.float64, device=R.device)
    _check(lib().mrcqr_condest_1norm(R.data_ptr(), G.data_ptr() if G is not None else None, n, _ld(R),
                                     seed & (2 ** 64 - 1), kappa.data_ptr(), _stream(stream)), "mrcqr_condest_1norm")
    return kappa


def cholqr_probe(A: torch.Tensor, stream=None) -> torch.Tensor:
    """The CholQR probe's lower bound on kappa_2(A) (+inf on breakdown)."""
    m, n = A.shape
    _mat(A, m, n, "A")
    _same_cuda_device([("A", A)])
    wsb = int(lib().mrcqr_cholqr_probe_workspace_bytes(m, n))
    ws = torch.empty(max(wsb, 1), dtype=torch.uint8, device=A.device)
    kappa = torch.empty(1, dtype=torch.float64, device=A.device)
    _check(lib().mrcqr_cholqr_probe(A.data_ptr(), m, n, _ld(A), ws.data_ptr(), wsb, kappa.data_ptr(),
                                    _stream(stream)), "mrcqr_cholqr_probe")
    return kappa


def release_cache() -> None:
    """Wait for and free the workspaces cached by factor() and factor_batched()."""
    _check(lib().mrcqr_release_cache(), "mrcqr_release_cache")


def version() -> int:
    return int(lib().mrcqr_version())
