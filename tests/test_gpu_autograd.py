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
