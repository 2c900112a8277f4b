"""The Python binding checks every tensor argument (shape, dtype, layout,
device) before the library is called, so a mismatched tensor raises instead
of becoming an out-of-bounds device access. Runs on the CPU: tensors that
pass every other check still fail on the device check."""
import pytest

torch = pytest.importorskip("torch")
import paper_2606_18411_amd as M  # noqa: E402


def cm(m, n, dtype=torch.float64):
    return torch.zeros((n, m), dtype=dtype).t()


def test_factor_checks_outputs_before_the_device():
    A = cm(64, 8)
    with pytest.raises(ValueError, match="Q has shape"):
        M.factor(A, Q=cm(64, 7))
    with pytest.raises(ValueError, match="R has shape"):
        M.factor(A, R=cm(8, 9))
    with pytest.raises(TypeError, match="R must be float64"):
        M.factor(A, R=cm(8, 8, torch.float32))
    with pytest.raises(ValueError, match="column-major"):
        M.factor(A, Q=torch.zeros(64, 8, dtype=torch.float64))
    with pytest.raises(TypeError, match="CUDA"):
        M.factor(A)


def test_step_functions_check_shapes():
    A, R = cm(64, 8), cm(8, 8)
    with pytest.raises(ValueError, match="R has shape"):
        M.trsm(A, cm(8, 9))
    with pytest.raises(ValueError, match="X has shape"):
        M.trsm(A, R, X=cm(63, 8))
    with pytest.raises(ValueError, match="X has shape"):
        M.form_q(A, cm(7, 7))
    with pytest.raises(ValueError, match="Q has shape"):
        M.form_q(A, R, Q=cm(64, 9))
    with pytest.raises(ValueError, match="R1 has shape"):
        M.trmm(R, cm(9, 9))
    with pytest.raises(ValueError, match="X has shape"):
        M.posterior_kappa(R, cm(8, 7))
    with pytest.raises(TypeError, match="int32"):
        M.sketch(A, torch.zeros(16, dtype=torch.int64), seed=1)
    with pytest.raises(TypeError, match="CUDA"):
        M.trsm(A, R)


def test_batched_entry_checks_members():
    with pytest.raises(ValueError, match="As\\[1\\] must be a 2-D"):
        M.factor_batched([cm(64, 8), torch.zeros(5, dtype=torch.float64)])
    with pytest.raises(TypeError, match="As\\[0\\] must be float64"):
        M.factor_batched([cm(64, 8, torch.float32)])


def test_single_column_and_single_row_need_no_layout():
    # a (m, 1) or (1, n) tensor may carry any stride in its size-1 dimension
    M._mat(torch.zeros(1000, 1, dtype=torch.float64).as_strided((1000, 1), (1, 1)), 1000, 1, "A")
    M._mat(torch.zeros(1, 1, dtype=torch.float64), 1, 1, "R")
    with pytest.raises(ValueError, match="column-major"):
        M._mat(torch.zeros(1000, 2, dtype=torch.float64), 1000, 2, "A")
