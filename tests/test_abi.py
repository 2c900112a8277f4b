"""The C ABI library loads and exports every symbol include/mrcqr.h declares;
argument checks return synchronously without touching a GPU."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "mrcqr.h")
LIB = os.path.join(ROOT, "paper_2606_18411_amd", "libmrcqr.so")


def declared():
    txt = open(HEADER).read()
    txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
    return sorted(set(re.findall(r"\b(mrcqr_[a-z_0-9]+)\s*\(", txt)))


@pytest.fixture(scope="module")
def lib():
    if not os.path.exists(LIB):
        pytest.fail("libmrcqr.so is not built (python -m paper_2606_18411_amd.build)")
    return ctypes.CDLL(LIB)


def test_header_declares_the_path():
    names = declared()
    for must in ["mrcqr_factor", "mrcqr_factor_batched", "mrcqr_plan_create", "mrcqr_execute",
                 "mrcqr_draw", "mrcqr_sketch", "mrcqr_sketch_qr", "mrcqr_trsm", "mrcqr_gram",
                 "mrcqr_cholesky", "mrcqr_trmm", "mrcqr_condest", "mrcqr_status_string"]:
        assert must in names


def test_every_declared_symbol_is_exported(lib):
    for name in declared():
        assert hasattr(lib, name), name


def test_argument_errors_are_synchronous(lib):
    f = lib.mrcqr_factor
    i64, vp = ctypes.c_int64, ctypes.c_void_p
    f.argtypes = [vp, i64, i64, i64, ctypes.c_int, ctypes.c_uint64, i64, vp, i64, vp, i64, vp, vp]
    f.restype = ctypes.c_int
    fake = ctypes.c_void_p(0x1000)
    fake2 = ctypes.c_void_p(0x2000)
    # (m, n, lda, prec, s, ldq, ldr) -> expected code
    cases = [((100, 10, 100, 3, 0, 100, 10), 0 if False else None),
             ((100, 10, 99, 3, 0, 100, 10), 1),     # lda < m
             ((5, 10, 5, 3, 0, 5, 10), 1),          # m < n
             ((100, 10, 100, 3, 5, 100, 10), 1),    # s < n
             ((100, 10, 100, 3, 200, 100, 10), 1),  # s > m
             ((100, 10, 100, 7, 0, 100, 10), 1),    # bad precision
             ((100, 0, 100, 3, 0, 100, 1), 1),      # n = 0
             ((100, 10, 100, 3, 0, 100, 9), 1),     # ldr < n
             ((2000, 600, 2000, 3, 0, 2000, 600), 8)]  # n above this library's limit (512)
    for (m, n, lda, prec, s, ldq, ldr), want in cases:
        if want is None:
            continue
        assert f(fake, m, n, lda, prec, 0, s, fake2, ldq, fake2, ldr, None, None) == want
    assert f(None, 100, 10, 100, 3, 0, 0, fake2, 100, fake2, 10, None, None) == 1
    assert f(fake, 100, 10, 100, 3, 0, 0, fake, 100, fake2, 10, None, None) == 1  # Q aliases A
    # AUTO_CARRY needs a caller-owned workspace (plan API)
    assert f(fake, 100, 10, 100, 5, 0, 0, fake2, 100, fake2, 10, None, None) == 1


def test_step_entry_points_reject_shapes_synchronously(lib):
    vp, i64 = ctypes.c_void_p, ctypes.c_int64
    fake = ctypes.c_void_p(0x1000)
    lib.mrcqr_trmm.argtypes = [vp, i64, vp, i64, i64, vp, i64, vp]
    assert lib.mrcqr_trmm(fake, 600, fake, 600, 600, fake, 600, None) == 8
    assert lib.mrcqr_trmm(fake, 10, fake, 10, 11, fake, 11, None) == 1
    lib.mrcqr_posterior_kappa.argtypes = [vp, vp, i64, i64, vp, vp, vp]
    assert lib.mrcqr_posterior_kappa(fake, fake, 600, 600, fake, None, None) == 8
    assert lib.mrcqr_posterior_kappa(fake, None, 20, 20, fake, None, None) == 1
    assert lib.mrcqr_posterior_kappa(fake, fake, 20, 19, fake, None, None) == 1
    # n > 128 keeps its power vectors in a caller-owned workspace
    lib.mrcqr_posterior_workspace_bytes.restype = ctypes.c_size_t
    lib.mrcqr_posterior_workspace_bytes.argtypes = [i64]
    assert lib.mrcqr_posterior_workspace_bytes(128) == 0
    assert lib.mrcqr_posterior_workspace_bytes(300) >= 4 * 512 * 8
    assert lib.mrcqr_posterior_kappa(fake, fake, 300, 300, fake, None, None) == 5
    # nothing cached in this process: releasing touches no device
    assert lib.mrcqr_release_cache() == 0


def test_status_strings(lib):
    lib.mrcqr_status_string.restype = ctypes.c_char_p
    lib.mrcqr_status_string.argtypes = [ctypes.c_int]
    assert lib.mrcqr_status_string(0) == b"ok"
    assert b"Cholesky" in lib.mrcqr_status_string(3)
    assert lib.mrcqr_version() >= 100


def test_plan_workspace_layout_is_sane(lib):
    p = ctypes.c_void_p()
    lib.mrcqr_plan_create.argtypes = [ctypes.c_int64, ctypes.c_int64, ctypes.c_int64, ctypes.POINTER(ctypes.c_void_p)]
    lib.mrcqr_plan_workspace_bytes.restype = ctypes.c_size_t
    lib.mrcqr_plan_workspace_bytes.argtypes = [ctypes.c_void_p]
    lib.mrcqr_plan_destroy.argtypes = [ctypes.c_void_p]
    assert lib.mrcqr_plan_create(1 << 20, 128, 0, ctypes.byref(p)) == 0
    b = lib.mrcqr_plan_workspace_bytes(p)
    assert (1 << 20) * 128 * 8 < b < (1 << 20) * 128 * 8 * 1.5  # B dominates the workspace
    lib.mrcqr_plan_destroy(p)
    assert lib.mrcqr_plan_create(10, 20, 0, ctypes.byref(p)) == 1


def test_column_panel_shapes_and_workspaces(lib):
    """128 < n <= 512: accepted with s <= 1024 (the blocked sketch QR), with
    workspaces that hold B plus the n x n objects, the pair-Gram partials and
    the row-major copies for the condition estimates."""
    i64, vp, sz = ctypes.c_int64, ctypes.c_void_p, ctypes.c_size_t
    p = ctypes.c_void_p()
    lib.mrcqr_plan_create.argtypes = [i64, i64, i64, ctypes.POINTER(vp)]
    lib.mrcqr_plan_workspace_bytes.restype = sz
    lib.mrcqr_plan_workspace_bytes.argtypes = [vp]
    lib.mrcqr_plan_destroy.argtypes = [vp]
    m = 1 << 20
    for n in (129, 256, 300, 512):
        assert lib.mrcqr_plan_create(m, n, 0, ctypes.byref(p)) == 0, n
        b = lib.mrcqr_plan_workspace_bytes(p)
        assert m * n * 8 + 4 * n * n * 8 < b < m * n * 8 * 1.5, (n, b)
        lib.mrcqr_plan_destroy(p)
    assert lib.mrcqr_plan_create(m, 300, 1024, ctypes.byref(p)) == 0
    lib.mrcqr_plan_destroy(p)
    assert lib.mrcqr_plan_create(m, 300, 1025, ctypes.byref(p)) == 8  # sketch beyond the blocked QR
    assert lib.mrcqr_plan_create(m, 513, 0, ctypes.byref(p)) == 8
    assert lib.mrcqr_plan_create(400, 300, 0, ctypes.byref(p)) == 1  # s = 2n > m
    for name, args in (("mrcqr_trsm_workspace_bytes", (512,)), ("mrcqr_gram_workspace_bytes", (m, 512))):
        f = getattr(lib, name)
        f.restype = sz
        f.argtypes = [i64] * len(args)
        assert f(*args) > 0, name
    lib.mrcqr_gram_workspace_bytes.restype = sz
    assert lib.mrcqr_gram_workspace_bytes(m, 513) == 0
    lib.mrcqr_posterior_workspace_bytes.restype = sz
    lib.mrcqr_posterior_workspace_bytes.argtypes = [i64]
    assert lib.mrcqr_posterior_workspace_bytes(600) == 0  # nothing beyond n = 512


def test_noalloc_entry_rejects_shapes_beyond_its_array_synchronously(lib):
    """The no-allocation entry point answers MRCQR_ERR_WORKSPACE, before any
    device call, for shapes whose plan outgrows its fixed device array (every
    column-panel shape at m = 2^20), and MRCQR_ERR_ARG for bad arguments."""
    i64, vp = ctypes.c_int64, ctypes.c_void_p
    f = lib.mrcqr_factor_noalloc
    f.argtypes = [vp, i64, i64, i64, ctypes.c_int, ctypes.c_uint64, i64, vp, i64, vp, i64, vp, vp]
    lib.mrcqr_factor_noalloc_max_workspace_bytes.restype = ctypes.c_size_t
    cap = lib.mrcqr_factor_noalloc_max_workspace_bytes()
    assert cap >= 1 << 20
    a, q, r = vp(0x1000), vp(0x2000), vp(0x3000)
    m = 1 << 20
    for n in (128, 256, 512):
        assert m * n * 8 > cap
        assert f(a, m, n, m, 3, 0, 0, q, m, r, n, None, None) == 5, n
    assert f(a, m, 600, m, 3, 0, 0, q, m, r, 600, None, None) == 8
    assert f(None, m, 256, m, 3, 0, 0, q, m, r, 256, None, None) == 1


def test_batch_and_regime_argument_errors(lib):
    """The batch plan rejects bad member shapes, and the batch and regime
    entry points reject missing arguments, before any device call."""
    i64p = ctypes.POINTER(ctypes.c_int64)
    vp = ctypes.c_void_p
    lib.mrcqr_batch_plan_create.argtypes = [ctypes.c_int32, i64p, i64p, ctypes.POINTER(vp)]
    lib.mrcqr_batch_plan_create.restype = ctypes.c_int
    arr = lambda vals: (ctypes.c_int64 * len(vals))(*vals)
    p = vp()
    cases = [((), (), 1),                         # empty batch
             ((100, 64), (10, 40), 1),            # member 1: s = 2n > m
             ((1000, 1000), (10, 200), 8),        # member 1: n above this library's limit
             ((1000,), (0,), 1),                  # n = 0
             ((1 << 28,), (4,), 8)]               # m beyond the exact-phase row limit
    for ms, ns, want in cases:
        k = len(ms)
        got = lib.mrcqr_batch_plan_create(k, arr(ms) if k else None, arr(ns) if k else None, ctypes.byref(p))
        assert got == want, (ms, ns, got)
    assert lib.mrcqr_batch_plan_create(1, arr([100]), arr([10]), None) == 1  # no output pointer
    lib.mrcqr_batch_plan_workspace_bytes.restype = ctypes.c_size_t
    lib.mrcqr_batch_plan_workspace_bytes.argtypes = [vp]
    assert lib.mrcqr_batch_plan_workspace_bytes(None) == 0
    lib.mrcqr_batch_execute.argtypes = [vp] * 2 + [ctypes.c_size_t] + [vp] * 10
    lib.mrcqr_batch_execute.restype = ctypes.c_int
    assert lib.mrcqr_batch_execute(None, None, 0, *([None] * 10)) == 1
    lib.mrcqr_regime_reset.argtypes = [vp, vp, ctypes.c_size_t, vp]
    lib.mrcqr_regime_reset.restype = ctypes.c_int
    assert lib.mrcqr_regime_reset(None, None, 0, None) == 1
    # a plan without a workspace: MRCQR_ERR_WORKSPACE
    q = vp()
    lib.mrcqr_plan_create.argtypes = [ctypes.c_int64, ctypes.c_int64, ctypes.c_int64, ctypes.POINTER(vp)]
    assert lib.mrcqr_plan_create(4096, 32, 0, ctypes.byref(q)) == 0
    assert lib.mrcqr_regime_reset(q, None, 0, None) == 5
    lib.mrcqr_plan_destroy.argtypes = [vp]
    lib.mrcqr_plan_destroy(q)
