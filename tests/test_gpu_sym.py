"""One-triangle CRS of a symmetric matrix against the FP64 oracle.

Storage: the GPU upper triangle is bit-exact against oracle.csr_upper (entries
with col >= row, CRS order), for every payload dtype.
Products: y = alpha*(U + U^T - diag U) x + beta*y, each y_i a sum of its
row's terms in FP64 in an order the atomics leave open; every order meets
the FP64 bound, so the check is |y - y_ref| <= 1e-12 * sum_j |a_ij||x_j|
against both the triangle oracle and the full CRS oracle.  Integer inputs
have exact partial sums in any order: bit-exact.  FP32 / BF16 values are
exact in FP64, so their products are checked against the oracle on the
rounded values at the FP64 bound.
"""
import numpy as np
import pytest
import torch

import oracle
import synth
from gpu_common import FP64_TOL, gpu_csr, max_err, to_dev, to_np

pytestmark = pytest.mark.gpu
sp = pytest.importorskip("paper_0910_4836_amd")


def sym_case(name):
    rng = np.random.default_rng({"random": 1, "long": 2, "diagonals": 3, "arrow": 4, "tridiag": 5}[name])
    if name == "random":
        r, c, v, n, _ = synth.random_symmetric(3000, 0.004, rng, empty_rows=0.1)
    elif name == "long":
        # rows longer than a plan block (single-row blocks) and empty rows
        r, c, v, n, _ = synth.random_symmetric(9000, 0.0008, rng, empty_rows=0.2, long_rows=3, long_len=6000)
    elif name == "diagonals":
        r, c, v, n, _ = synth.sym_diagonals(n=30000, ndiag=12)
    elif name == "arrow":
        # a full last row and column: every block adds into y[n-1]
        n = 20000
        i = np.arange(n - 1)
        up_r = np.concatenate([np.arange(n), i])
        up_c = np.concatenate([np.arange(n), np.full(n - 1, n - 1)])
        up_v = rng.standard_normal(len(up_r))
        off = up_c > up_r
        r = np.concatenate([up_r, up_c[off]]).astype(np.int32)
        c = np.concatenate([up_c, up_r[off]]).astype(np.int32)
        v = np.concatenate([up_v, up_v[off]])
    else:
        # more than 256 short rows per plan block
        n = 50000
        i = np.arange(n)
        r = np.concatenate([i, i[:-1], i[1:]]).astype(np.int32)
        c = np.concatenate([i, i[1:], i[:-1]]).astype(np.int32)
        v0 = rng.standard_normal(n - 1)
        v = np.concatenate([rng.standard_normal(n), v0, v0])
    return r, c, v, n, rng


CASES = ["random", "long", "diagonals", "arrow", "tridiag"]


@pytest.mark.parametrize("dt", [torch.float64, torch.float32, torch.bfloat16, torch.int32])
@pytest.mark.parametrize("case", ["random", "long", "diagonals"])
def test_csr_upper_bit_exact(case, dt):
    r, c, v, n, _ = sym_case(case)
    R = oracle.csr_from_coo(n, n, r, c, v)
    Uo = oracle.csr_upper(R)
    A = gpu_csr(sp, r, c, v, n, n)
    if dt == torch.int32:
        pos = torch.arange(A.nnz, dtype=torch.int32, device=A.device)
        S = sp.csr_upper_from_csr(A.with_values(pos))
        # the payload carried through is the position of each kept entry
        keep = np.flatnonzero(R.col >= R.row_index())
        assert np.array_equal(to_np(S.upper.val), keep.astype(np.int32))
    else:
        S = sp.csr_upper_from_csr(A.with_values(sp.spmv_convert_values(A.val, dt)) if dt != torch.float64 else A)
        if dt == torch.float64:
            assert np.array_equal(to_np(S.upper.val).view(np.uint64), Uo.val.view(np.uint64))
    assert S.nnz == Uo.nnz
    assert np.array_equal(to_np(S.upper.row_ptr), Uo.row_ptr)
    assert np.array_equal(to_np(S.upper.col_idx), Uo.col)


@pytest.mark.parametrize("staged", [False, True])
@pytest.mark.parametrize("block_nnz", [256, 1024, 4096])
@pytest.mark.parametrize("case", CASES)
def test_crs_sym_fp64_parity(case, block_nnz, staged):
    r, c, v, n, rng = sym_case(case)
    R = oracle.csr_from_coo(n, n, r, c, v)
    Uo = oracle.csr_upper(R)
    A = gpu_csr(sp, r, c, v, n, n)
    S = sp.csr_upper_from_csr(A)
    sp.spmv_crs_plan(S.upper, block_nnz)
    S.upper.staged = staged                 # spmv_crs_sym_staged: entries walked in row order
    x = rng.uniform(-1, 1, n)
    y0 = rng.uniform(-1, 1, n)
    D = oracle.row_absdot(R, x) + np.abs(y0)
    xd = to_dev(x)
    for alpha, beta in ((1.0, 0.0), (-0.5, 2.0), (0.0, 1.0)):
        got = sp.spmv_crs_sym(S, xd, to_dev(y0), alpha, beta)
        for want in (oracle.spmv_crs_sym(Uo, x, y0, alpha, beta), oracle.spmv_crs(R, x, y0, alpha, beta)):
            e = max_err(got, want, D * max(abs(alpha), 1.0))
            assert e <= FP64_TOL, (case, alpha, beta, e)
    # beta == 0 ignores NaN in y
    got = sp.spmv_crs_sym(S, xd, torch.full((n,), float("nan"), dtype=torch.float64, device=A.device), 1.0, 0.0)
    assert torch.isfinite(got).all()


@pytest.mark.parametrize("staged", [False, True])
@pytest.mark.parametrize("case", ["random", "arrow", "tridiag"])
def test_crs_sym_integer_exact(case, staged):
    r, c, v, n, rng = sym_case(case)
    vi = np.where(v > 0, np.ceil(v * 4), np.floor(v * 4))              # integers, symmetric like v
    vi[vi == 0] = 1.0
    R = oracle.csr_from_coo(n, n, r, c, vi)
    A = gpu_csr(sp, r, c, vi, n, n)
    S = sp.csr_upper_from_csr(A)
    S.upper.staged = staged
    x = synth.integer_vector(n, rng)
    want = oracle.spmv_crs(R, x)
    for _ in range(2):
        assert np.array_equal(to_np(sp.spmv_crs_sym(S, to_dev(x))), want)


@pytest.mark.parametrize("staged", [False, True])
@pytest.mark.parametrize("vdt", [torch.float32, torch.bfloat16])
def test_crs_sym_reduced_values(vdt, staged):
    r, c, v, n, rng = sym_case("diagonals")
    if vdt == torch.float32:
        vq = oracle.round_f32(v).astype(np.float64)
    else:
        vq = oracle.bf16_bits_to_f64(oracle.round_bf16_bits(v))
    R = oracle.csr_from_coo(n, n, r, c, vq)
    A = gpu_csr(sp, r, c, v, n, n)
    S = sp.csr_upper_from_csr(A)
    Sq = S.with_values(sp.spmv_convert_values(S.upper.val, vdt))
    Sq.upper.staged = staged
    x = rng.uniform(-1, 1, n)
    got = sp.spmv_crs_sym(Sq, to_dev(x))
    assert max_err(got, oracle.spmv_crs(R, x), oracle.row_absdot(R, x)) <= FP64_TOL


def test_crs_sym_empty_and_errors():
    dev = "cuda"
    n = 7
    A = sp.CSR(n, n, torch.zeros(n + 1, dtype=torch.int32, device=dev), torch.zeros(0, dtype=torch.int32, device=dev),
               torch.zeros(0, dtype=torch.float64, device=dev))
    S = sp.csr_upper_from_csr(A)
    assert S.nnz == 0
    for staged in (False, True):
        S.upper.staged = staged
        y = torch.full((n,), 3.0, dtype=torch.float64, device=dev)
        out = sp.spmv_crs_sym(S, torch.ones(n, dtype=torch.float64, device=dev), y, 1.0, 0.5)
        assert torch.equal(out, torch.full((n,), 1.5, dtype=torch.float64, device=dev))
    r, c, v, n, rng = sym_case("random")
    S = sp.csr_upper_from_csr(gpu_csr(sp, r, c, v, n, n))
    with pytest.raises(TypeError):
        sp.spmv_crs_sym(S, torch.ones(n, dtype=torch.float32, device=dev))
    with pytest.raises(ValueError):
        sp.csr_upper_from_csr(gpu_csr(sp, r, c, v, n, n + 1))
