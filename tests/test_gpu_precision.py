"""Mixed-precision value storage (FP32 / BF16 values, FP32 accumulation, FP64 for
rows longer than 4096 entries) against the FP64 oracle run on the quantised values.

Per row, with L_i stored entries, D_i = sum_j |a_q,ij| |x_j| and u32 = 2^-24,
u64 = 2^-53, gamma_k(u) = k u / (1 - k u):
  rows with L_i <= 4096: x is rounded to FP32 (u32), each product once (u32)
      and L_i - 1 sums (u32)  ->  |y_i - (A_q x)_i| <= gamma_{L_i+1}(u32) D_i
  rows with L_i > 4096: exact FP64 products, FP64 sums
      ->  |y_i - (A_q x)_i| <= gamma_{L_i+1}(u64) D_i
  FP32 output vectors add one final rounding: + u32 D_i.
The quantisation itself (FP64 -> FP32 / BF16, one round-to-nearest-even step)
is checked bit for bit against the oracle's rounding.
"""
import numpy as np
import pytest
import torch

import oracle
import synth
from gpu_common import rand_coo, to_dev, to_np

pytestmark = pytest.mark.gpu
sp = pytest.importorskip("paper_0910_4836_amd")

U32, U64 = 2.0 ** -24, 2.0 ** -53


def gamma(k, u):
    return k * u / (1 - k * u)


def bound(L, D, vec_f32):
    b = np.where(L > 4096, gamma(L + 1, U64), gamma(L + 1, U32)) * D
    if vec_f32:
        b = b + U32 * D
    return b


def quantised(R, dt):
    if dt == torch.float32:
        return oracle.round_f32(R.val).astype(np.float64)
    return oracle.bf16_bits_to_f64(oracle.round_bf16_bits(R.val))


def kernels(A, vt):
    J = sp.jds_from_csr(A)
    B = sp.jds_blocked_from_jds(J, 64)
    S = sp.Split(A)
    RS = sp.RowSplit(A)
    As = A.with_values(A.val)
    if As.plan is None:
        sp.spmv_crs_plan(As)
    As.staged = True
    return {
        "crs_staged": lambda x: sp.spmv_crs(As, x),
        "jds_row_split": lambda x: sp.spmv_jds_row_split(RS, x),
        "blocked_row_split": lambda x: sp.spmv_jds_blocked_row_split(RS, x, rows_per_wave=16),
        "crs_split": lambda x: sp.spmv_crs_split(S, x),
        "jds_split": lambda x: sp.spmv_jds_split(S, x),
        "blocked_split": lambda x: sp.spmv_jds_blocked_split(S, x),
        "crs": lambda x: sp.spmv_crs(A, x),
        "crs_wave": lambda x: sp.spmv_crs(A, x, use_plan=False),
        "jds": lambda x: sp.spmv_jds(J, x),
        "jds_mi4": lambda x: sp.spmv_jds(J, x, max_iters=4),
        "jds_tiled": lambda x: sp.spmv_jds_tiled(J, x),
        "blocked_tiled": lambda x: sp.spmv_jds_blocked_tiled(B, x),
        "blocked": lambda x: sp.spmv_jds_blocked(B, x),
        "blocked_r16": lambda x: sp.spmv_jds_blocked(B, x, rows_per_wave=16),
    }


@pytest.mark.parametrize("vdt", [torch.float32, torch.bfloat16])
@pytest.mark.parametrize("xdt", [torch.float64, torch.float32])
def test_mixed_precision_bounds(vdt, xdt):
    # symmetric diagonals (the Hamiltonian-like shape) plus a few rows > 4096 entries
    n = 30000
    r, c, v, n, _ = synth.sym_diagonals(n=n, ndiag=12)
    rng = np.random.default_rng(5)
    long_rows = rng.choice(n, 3, replace=False)
    extra_r = np.repeat(long_rows, 5000).astype(np.int32)
    extra_c = np.concatenate([rng.choice(n, 5000, replace=False) for _ in long_rows]).astype(np.int32)
    r2 = np.concatenate([r, extra_r])
    c2 = np.concatenate([c, extra_c])
    v2 = np.concatenate([v, rng.standard_normal(len(extra_r))])
    R = oracle.csr_from_coo(n, n, r2, c2, v2)            # duplicates summed
    x = synth.uniform_vector(n, rng).astype(np.float32 if xdt == torch.float32 else np.float64)
    # GPU: FP64 CRS built on the device, values rounded on the device
    A64 = sp.csr_from_coo(n, n, to_dev(r2), to_dev(c2), to_dev(v2))
    assert np.array_equal(to_np(A64.val), R.val)
    Aq = A64.with_values(sp.spmv_convert_values(A64.val, vdt))
    Aq.plan = None
    vq = quantised(R, vdt)
    assert np.array_equal(to_np(Aq.val.to(torch.float64)), vq)
    Rq = oracle.CSR(n, n, R.row_ptr, R.col, vq)
    xx = x.astype(np.float64)
    want = oracle.spmv_crs(Rq, xx)
    D = oracle.row_absdot(Rq, xx)
    L = R.row_lengths()
    assert (L > 4096).sum() == 3
    lim = bound(L, D, xdt == torch.float32)
    for name, fn in kernels(Aq, xdt).items():
        got = to_np(fn(to_dev(x))).astype(np.float64)
        err = np.abs(got - want)
        assert np.all(err <= lim), f"{name}: worst ratio {np.max(err / np.maximum(lim, 1e-300)):.3f}"
        # the long rows really are accumulated in FP64
        assert np.all(err[L > 4096] <= gamma(5020, U64) * D[L > 4096] + (U32 * D[L > 4096] if xdt == torch.float32 else 0))
    # report (not pinned): total error against the unquantised FP64 product
    total = np.abs(to_np(kernels(Aq, xdt)["crs"](to_dev(x))) - oracle.spmv_crs(R, xx)) / np.maximum(D, 1e-300)
    print(f"\n{vdt} values, {xdt} vectors: max total rel error vs FP64 = {total.max():.3e}")


def test_fp64_values_fp32_vectors():
    r, c, v, nr, nc, rng = rand_coo(3, 5000, 5000, 0.003, long_rows=4, long_len=4500)
    R = oracle.csr_from_coo(nr, nc, r, c, v)
    x = rng.uniform(-1, 1, nc).astype(np.float32)
    A = sp.csr_from_coo(nr, nc, to_dev(r), to_dev(c), to_dev(v))
    want = oracle.spmv_crs(R, x.astype(np.float64))
    D = oracle.row_absdot(R, x.astype(np.float64))
    for name, fn in kernels(A, torch.float32).items():
        got = to_np(fn(to_dev(x))).astype(np.float64)
        assert np.all(np.abs(got - want) <= (U32 + gamma(R.row_lengths() + 1, U64)) * D), name


def test_integer_values_exact_in_every_precision():
    r, c, v, nr, nc, rng = rand_coo(9, 3000, 3000, 0.004, integer=True, long_rows=3, long_len=2900)
    x = synth.integer_vector(nc, rng)
    R = oracle.csr_from_coo(nr, nc, r, c, v)
    want = oracle.spmv_crs(R, x)
    for vdt in (torch.float32, torch.bfloat16):
        for xdt in (torch.float64, torch.float32):
            A = sp.csr_from_coo(nr, nc, to_dev(r), to_dev(c), to_dev(v))
            Aq = A.with_values(sp.spmv_convert_values(A.val, vdt))
            Aq.plan = None
            for name, fn in kernels(Aq, xdt).items():
                got = to_np(fn(to_dev(x).to(xdt))).astype(np.float64)
                assert np.array_equal(got, want), (vdt, xdt, name)
