"""mrcqr_factor_noalloc (the entry point for callers that cannot allocate)
against mrcqr_factor through the C ABI: bitwise-equal Q, R and info on two
calls in a row, the second with a smaller input, and a synchronous
MRCQR_ERR_WORKSPACE for a shape beyond its fixed workspace."""
import ctypes

import numpy as np
import pytest

import workloads as W
from oracle import metrics as MT
from gpu_common import require_gpu, to_dev, to_host, progress, torch

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def M():
    M = require_gpu()
    L = M.lib()
    i64, u64, i32, vp = ctypes.c_int64, ctypes.c_uint64, ctypes.c_int, ctypes.c_void_p
    L.mrcqr_factor_noalloc.argtypes = [vp, i64, i64, i64, i32, u64, i64, vp, i64, vp, i64, vp, vp]
    L.mrcqr_factor_noalloc.restype = i32
    L.mrcqr_factor_noalloc_max_workspace_bytes.restype = ctypes.c_size_t
    return M


def _noalloc(M, A, prec, seed):
    m, n = A.shape
    Q, R = M.empty_colmajor(m, n), M.empty_colmajor(n, n)
    info = torch.empty(M.INFO_BYTES, dtype=torch.uint8, device=A.device)
    code = M.lib().mrcqr_factor_noalloc(A.data_ptr(), m, n, A.stride(1), M.PREC[prec], seed, 0, Q.data_ptr(),
                                        Q.stride(1), R.data_ptr(), R.stride(1),
                                        torch.cuda.current_stream().cuda_stream, info.data_ptr())
    assert code == M.OK, code
    torch.cuda.synchronize()
    return Q, R, M.read_infos(info)[0]


def test_noalloc_matches_factor_twice_with_smaller_second_call(M):
    assert M.lib().mrcqr_factor_noalloc_max_workspace_bytes() == 64 << 20
    for (m, n, kappa, prec, seed) in [(40000, 64, 1e6, "auto", 3), (3000, 20, 1e3, "fp16", 4)]:
        progress(f"noalloc m={m} n={n} {prec}")
        A = to_dev(W.test_matrix(m, n, kappa, 77 + n))
        Q, R, info = _noalloc(M, A, prec, seed)
        Qr, Rr, ir = M.factor(A, prec, seed=seed)
        same = lambda x, y: (np.isnan(x) and np.isnan(y)) or x == y
        assert (info.status, info.precision_used, info.chol_fail_index, info.escalations) == \
            (ir.status, ir.precision_used, ir.chol_fail_index, ir.escalations), (info, ir)
        assert same(info.kappa_rs_est, ir.kappa_rs_est) and same(info.kappa_rc_est, ir.kappa_rc_est)
        assert info.status == 0, info
        assert torch.equal(Q, Qr) and torch.equal(R, Rr)
        assert MT.orthogonality(to_host(Q)) <= 1e-13


def test_noalloc_rejects_a_workspace_beyond_its_size(M):
    m, n = 1 << 16, 128  # about 161 MiB of workspace
    fake = ctypes.c_void_p(0x1000)
    code = M.lib().mrcqr_factor_noalloc(fake, m, n, m, 3, 1, 0, ctypes.c_void_p(0x2000), m,
                                        ctypes.c_void_p(0x3000), n, None, None)
    assert code == M.ERR_WORKSPACE
