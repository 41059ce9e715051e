"""Differentiable SpMV and the 20-step Chebyshev recurrence on the GPU (FP32)
against the FP64 oracle gradient (itself pinned by central differences and the
closed form on Laplacian sine modes in the CPU tests).

Tolerance (FP32 values and vectors): every step adds at most about
(L+1) u32 |A||y_k| per row (L = 20 entries, u32 = 2^-24) and a recurrence of
20 steps carries each such error forward at most ~20 times (the homogeneous
error recurrence e_{k+1} = 2 A e_k - e_{k-1} grows like the second-kind
Chebyshev polynomials, at most linearly for a spectrum inside [-1, 1]).  A
first-order worst case is 20 * 20 * 21 u32 ~ 5e-4 of the largest state; the
tests use 2e-3 norm-wise for states, loss and gradients (rounding errors of
random data stay far below the worst case).  FP64 runs use 1e-10.
"""
import numpy as np
import pytest
import torch

import oracle
import synth
from gpu_common import to_dev, to_np

pytestmark = pytest.mark.gpu
sp = pytest.importorskip("paper_0910_4836_amd")
from paper_0910_4836_amd import autograd as AG  # noqa: E402


def c5_like(n, band, dtype):
    r, c, v, n, _ = synth.banded_uniform(n=n, band=band, dtype=np.float64)
    vq = v.astype(dtype).astype(np.float64)
    R = oracle.csr_from_coo(n, n, r, c, vq)
    A = sp.csr_from_coo(n, n, to_dev(r), to_dev(c), to_dev(vq).to(torch.float32 if dtype == np.float32 else torch.float64))
    return R, A


def rel_inf(a, b):
    return np.abs(a - b).max() / np.abs(b).max()


@pytest.mark.parametrize("dtype,tol", [(np.float64, 1e-10), (np.float32, 2e-3)])
@pytest.mark.parametrize("transpose", ["crs", "jds"])
def test_chebyshev_loss_and_gradient(dtype, tol, transpose):
    n = 20000
    R, A = c5_like(n, 500, dtype)
    x = synth.uniform_vector(n, synth.rng_for(5, 3)).astype(dtype)
    loss_ref, dx_ref, dval_ref, ys = oracle.cheb_loss_grad(R, x.astype(np.float64), 20)
    tdt = torch.float32 if dtype == np.float32 else torch.float64
    op = AG.SpMVOperator(A, transpose=transpose)
    vals = op.J.jd_val.clone().requires_grad_(True)
    xt = to_dev(x).to(tdt).requires_grad_(True)
    loss = AG.chebyshev_loss(op, vals, xt, steps=20, checkpoint=5)
    loss.backward()
    assert abs(loss.item() - loss_ref) <= tol * abs(loss_ref)
    assert rel_inf(to_np(xt.grad).astype(np.float64), dx_ref) <= tol
    order = to_np(op.jds_src).astype(np.int64)
    assert rel_inf(to_np(vals.grad).astype(np.float64), dval_ref[order]) <= tol
    # forward states
    y20 = AG.cheb_states(op, vals.detach(), xt.detach(), 20)[20]
    assert rel_inf(to_np(y20).astype(np.float64), ys[20]) <= tol


def test_checkpointed_equals_stored_bit_for_bit():
    n = 8000
    R, A = c5_like(n, 300, np.float32)
    x = to_dev(synth.uniform_vector(n, synth.rng_for(5, 4)).astype(np.float32))
    op = AG.SpMVOperator(A)
    grads = []
    for ck in (1, 5, 7, 20):
        vals = op.J.jd_val.clone().requires_grad_(True)
        xt = x.clone().requires_grad_(True)
        AG.chebyshev_loss(op, vals, xt, 20, ck).backward()
        grads.append((to_np(vals.grad), to_np(xt.grad)))
    for gv, gx in grads[1:]:
        assert np.array_equal(gv, grads[0][0]) and np.array_equal(gx, grads[0][1])


def test_spmv_function_gradcheck_fp64():
    r, c, v, n, _, = synth.random_pattern(60, 60, 0.1, np.random.default_rng(2))[:5]
    A = sp.csr_from_coo(n, n, to_dev(r), to_dev(c), to_dev(v))
    op = AG.SpMVOperator(A)
    vals = op.J.jd_val.clone().requires_grad_(True)
    x = torch.randn(n, dtype=torch.float64, device="cuda", requires_grad=True)
    assert torch.autograd.gradcheck(lambda a, b: AG.spmv(op, a, b), (vals, x), eps=1e-6, atol=1e-9)
    # adjoint identity <g, A x> = <A^T g, x> and Euler identity sum(vals * dvals) = <g, A x>
    g = torch.randn(n, dtype=torch.float64, device="cuda")
    y = AG.spmv(op, vals, x)
    y.backward(g)
    gAx = float(torch.dot(g, y))
    assert abs(float(torch.dot(x.grad, x)) - gAx) <= 1e-12 * n
    assert abs(float(torch.dot(vals.grad, vals)) - gAx) <= 1e-12 * n


@pytest.mark.parametrize("transpose", ["crs", "jds"])
def test_transposed_values_follow_a_new_vals_tensor(transpose):
    """A^T's values are cached per vals tensor.  A new tensor of the same size
    (freed and reallocated in between, so the allocator may well hand out
    the old address, version 0 again) must not reuse the old transpose:
    dx = A^T g is checked against the oracle for both."""
    r, c, v, n, _ = synth.random_pattern(3000, 3000, 0.004, np.random.default_rng(11))[:5]
    A = sp.csr_from_coo(n, n, to_dev(r), to_dev(c), to_dev(v))
    op = AG.SpMVOperator(A, transpose=transpose)
    g = synth.uniform_vector(n, np.random.default_rng(12))
    order = to_np(op.jds_src).astype(np.int64)          # JDS slot -> CRS position
    R = oracle.csr_from_coo(n, n, r, c, v)
    assert R.nnz == A.nnz
    for seed in (1, 2, 3):
        crs_vals = np.random.default_rng(seed).standard_normal(R.nnz)
        Rv = oracle.CSR(n, n, R.row_ptr, R.col, crs_vals)
        vals = op.vals_from_crs(to_dev(crs_vals))
        assert np.array_equal(to_np(vals), crs_vals[order])
        dx = to_np(op.rmatvec(vals, to_dev(g)))
        want = oracle.spmv_crs_transposed(Rv, g)
        D = oracle.spmv_crs_transposed(oracle.CSR(n, n, R.row_ptr, R.col, np.abs(crs_vals)), np.abs(g))
        assert oracle.rel_err(dx, want, D).max() <= 1e-12, seed
        # an in-place change of the same tensor is seen too
        vals.mul_(2.0)
        dx2 = to_np(op.rmatvec(vals, to_dev(g)))
        assert oracle.rel_err(dx2, 2.0 * want, 2.0 * D).max() <= 1e-12, seed
        del vals
        torch.cuda.synchronize()


def test_int32_payload_through_the_conversions():
    """int32 values ride through CRS -> JDS -> blocked JDS, the permutation
    and the gather bit for bit (the position maps of the operator above)."""
    r, c, v, n, _ = synth.random_pattern(500, 400, 0.02, np.random.default_rng(13))[:5]
    R = oracle.csr_from_coo(n, 400, r, c, v)
    A = sp.csr_from_coo(n, 400, to_dev(r), to_dev(c), to_dev(v))
    pos = torch.arange(A.nnz, dtype=torch.int32, device="cuda")
    pos[::7] = -pos[::7] - 1                         # negative payloads too
    Jp = sp.jds_from_csr(A.with_values(pos))
    Jo = oracle.jds_from_csr(R)
    want = np.arange(R.nnz, dtype=np.int64)
    want[::7] = -want[::7] - 1
    # the JDS scatter is a permutation of entries: compare against the oracle's
    # JDS of the same positions
    Jw = oracle.jds_from_csr(oracle.CSR(n, 400, R.row_ptr, R.col, want.astype(np.float64)))
    assert Jp.jd_val.dtype == torch.int32
    assert np.array_equal(to_np(Jp.jd_val).astype(np.int64), Jw.jd_val.astype(np.int64))
    assert np.array_equal(to_np(Jp.perm), Jo.perm)
    B = sp.jds_blocked_from_jds(Jp, 64)
    Bw = oracle.blocked_from_jds(Jw, 64)
    assert np.array_equal(to_np(B.bl_val).astype(np.int64), Bw.bl_val.astype(np.int64))
    back = sp.jds_to_csr(Jp)
    assert np.array_equal(to_np(back.val).astype(np.int64), want)
    g = sp.spmv_gather_values(torch.tensor([2, 0, 1], dtype=torch.int32, device="cuda"), pos[:3])
    assert to_np(g).tolist() == [int(want[2]), int(want[0]), int(want[1])]
    p = sp.spmv_permute_vec(Jp.perm, pos[:n].clone())
    assert np.array_equal(to_np(p).astype(np.int64), want[:n][Jo.perm])
