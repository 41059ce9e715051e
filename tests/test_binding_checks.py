"""CPU checks of the binding's argument validation: a vector of the wrong
dtype or length, or a multi-vector block of the wrong shape, is refused before
any launch (the kernels trust these shapes and would write out of bounds).

The containers are built from CPU tensors, so a call that passed validation
would stop at the device check; every mismatch must be reported first."""
import numpy as np
import pytest
import torch

from paper_0910_4836_amd import spmv as S

N_ROWS, N_COLS = 6, 9


def csr():
    rp = torch.tensor([0, 1, 2, 2, 3, 4, 5], dtype=torch.int32)
    col = torch.tensor([0, 3, 8, 1, 2], dtype=torch.int32)
    val = torch.ones(5, dtype=torch.float64)
    A = S.CSR(N_ROWS, N_COLS, rp, col, val)
    A.plan = torch.tensor([0, N_ROWS], dtype=torch.int32)      # skip planning (a library call)
    A.n_blocks = 1
    return A


def jds():
    return S.JDS(N_ROWS, N_COLS, torch.arange(N_ROWS, dtype=torch.int32), torch.arange(N_ROWS, dtype=torch.int32),
                 torch.zeros(2, dtype=torch.int32), np.zeros(2, np.int32), torch.zeros(1, dtype=torch.int32),
                 torch.zeros(1, dtype=torch.float64))


def dia():
    return S.DIA(N_ROWS, N_COLS, np.zeros(1, np.int32), torch.zeros(N_ROWS, dtype=torch.float64), csr())


def blocked():
    return S.Blocked(N_ROWS, N_COLS, 64, torch.arange(N_ROWS, dtype=torch.int32), torch.zeros(2, dtype=torch.int64),
                     torch.zeros(1, dtype=torch.int32), np.zeros(1, np.int32), torch.zeros(1, dtype=torch.int32),
                     torch.zeros(1, dtype=torch.float64), 0)


def single_vector_calls():
    A, J, D = csr(), jds(), dia()
    return {
        "spmv_crs": lambda x, y: S.spmv_crs(A, x, y),
        "spmv_jds": lambda x, y: S.spmv_jds(J, x, y),
        "spmv_dia": lambda x, y: S.spmv_dia(D, x, y),
    }


def test_one_triangle_checks_before_launch():
    """The one-triangle product takes FP64 vectors only and square storage."""
    U = S.SymCSR(S.CSR(N_ROWS, N_ROWS, torch.zeros(N_ROWS + 1, dtype=torch.int32), torch.zeros(0, dtype=torch.int32),
                       torch.zeros(0, dtype=torch.float64)))
    with pytest.raises(TypeError, match="float64"):
        S.spmv_crs_sym(U, torch.zeros(N_ROWS, dtype=torch.float32))
    with pytest.raises(ValueError, match="y has 5 elements"):
        S.spmv_crs_sym(U, torch.zeros(N_ROWS, dtype=torch.float64), torch.zeros(N_ROWS - 1, dtype=torch.float64))
    with pytest.raises(ValueError, match="must live on the GPU"):
        S.spmv_crs_sym(U, torch.zeros(N_ROWS, dtype=torch.float64))
    with pytest.raises(ValueError, match="square"):
        S.csr_upper_from_csr(csr())


@pytest.mark.parametrize("name", ["spmv_crs", "spmv_jds", "spmv_dia"])
def test_vector_mismatches_raise_before_launch(name):
    fn = single_vector_calls()[name]
    x = torch.zeros(N_COLS, dtype=torch.float64)
    with pytest.raises(ValueError, match="y is torch.float32 but x is torch.float64"):
        fn(x, torch.zeros(N_ROWS, dtype=torch.float32))
    with pytest.raises(ValueError, match="y has 5 elements"):
        fn(x, torch.zeros(N_ROWS - 1, dtype=torch.float64))
    with pytest.raises(ValueError, match="x has 8 elements"):
        fn(torch.zeros(N_COLS - 1, dtype=torch.float64), torch.zeros(N_ROWS, dtype=torch.float64))
    with pytest.raises(TypeError, match="x must be float64 or float32"):
        fn(torch.zeros(N_COLS, dtype=torch.bfloat16), None)
    with pytest.raises(TypeError, match="x must be float64 or float32"):
        fn(torch.zeros(N_COLS, dtype=torch.int32), None)
    # shapes right: the next check is the device one
    with pytest.raises(ValueError, match="must live on the GPU"):
        fn(x, torch.zeros(N_ROWS, dtype=torch.float64))


@pytest.mark.parametrize("name", ["spmm_crs", "spmm_jds", "spmm_jds_blocked"])
def test_block_mismatches_raise_before_launch(name):
    A, J, B = csr(), jds(), blocked()
    fn = {"spmm_crs": lambda X, Y: S.spmm_crs(A, X, Y), "spmm_jds": lambda X, Y: S.spmm_jds(J, X, Y),
          "spmm_jds_blocked": lambda X, Y: S.spmm_jds_blocked(B, X, Y)}[name]
    k = 3
    X = torch.zeros(k, N_COLS, dtype=torch.float64).t()           # column-major (n_cols, k)
    with pytest.raises(ValueError, match="Y is torch.float32 but X is torch.float64"):
        fn(X, torch.zeros(k, N_ROWS, dtype=torch.float32).t())
    with pytest.raises(ValueError, match=r"Y must be \(6, 3\)"):
        fn(X, torch.zeros(k + 1, N_ROWS, dtype=torch.float64).t())
    with pytest.raises(ValueError, match=r"Y must be \(6, 3\)"):
        fn(X, torch.zeros(k, N_ROWS - 1, dtype=torch.float64).t())
    with pytest.raises(ValueError, match=r"X must be \(9, k\)"):
        fn(torch.zeros(k, N_COLS - 1, dtype=torch.float64).t(), None)
    with pytest.raises(TypeError, match="X must be float64 or float32"):
        fn(torch.zeros(k, N_COLS, dtype=torch.bfloat16).t(), None)
    with pytest.raises(ValueError, match="column-major"):
        fn(torch.zeros(N_COLS, k, dtype=torch.float64), None)  # row-major
    with pytest.raises(ValueError, match="must live on the GPU"):
        fn(X, torch.zeros(k, N_ROWS, dtype=torch.float64).t())


def test_int32_is_a_payload_dtype_only():
    """int32 maps to the payload code the value-moving calls accept."""
    assert S.dtype_code(torch.int32) == 3
    with pytest.raises(TypeError):
        S.dtype_code(torch.int64)


def test_blocked_multi_vector_refuses_symmetric_permutation():
    B = blocked()
    B.symperm = True
    with pytest.raises(ValueError, match="symmetric-permutation"):
        S.spmm_jds_blocked(B, torch.zeros(3, N_COLS, dtype=torch.float64).t())


def test_coo_indices_must_be_int32():
    """int64 indices would be read as pairs of int32 halves: refused."""
    r = torch.zeros(3, dtype=torch.int64)
    c = torch.zeros(3, dtype=torch.int32)
    v = torch.ones(3, dtype=torch.float64)
    with pytest.raises(TypeError, match="int32"):
        S.csr_from_coo(4, 4, r, c, v)
    with pytest.raises(ValueError, match="one length"):
        S.csr_from_coo(4, 4, c, c, torch.ones(2, dtype=torch.float64))
