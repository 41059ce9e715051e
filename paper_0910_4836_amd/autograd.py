"""Differentiable SpMV and the checkpointed Chebyshev recurrence on the GPU.

``SpMVOperator`` holds a square sparse pattern in JDS storage (values in JDS
order are the differentiable parameter) together with a prebuilt storage of
its transpose and the map that fills A^T's values from A's.  Backward of
y = A x:
    dx    = A^T g       (a product with the prebuilt transpose: a gather per
                          entry, no atomics; CRS storage by default, which
                          keeps neighbouring rows' x windows together, or
                          JDS with transpose="jds")
    dval  = g[row] * x[col]   (spmv_grad_vals_jds, in JDS order)
All arithmetic runs in the library's kernels; this module only sequences calls.

``chebyshev_loss(op, vals, x, steps=20, checkpoint=5)`` returns
loss = ||y_steps||^2 for y_0 = x, y_1 = A y_0, y_{k+1} = 2 A y_k - y_{k-1}.
Its backward is the hand-written reverse sweep of the recurrence; only every
`checkpoint`-th pair of states is kept from the forward pass and each segment
is recomputed before it is swept (activation checkpointing).
"""
from __future__ import annotations

import weakref

import numpy as np
import torch

from . import spmv as S


class SpMVOperator:
    def __init__(self, A: S.CSR, unroll: int = 0, max_iters: int = 0, transpose: str = "crs", wg_waves: int = 0):
        if A.n_rows != A.n_cols:
            raise ValueError("the operator must be square")
        if transpose not in ("crs", "jds"):
            raise ValueError("transpose must be 'crs' or 'jds'")
        dev = A.device
        self.n = A.n_rows
        self.nnz = A.nnz
        self.unroll, self.max_iters, self.wg_waves = unroll, max_iters, wg_waves
        self.transpose = transpose
        # JDS of A, and of A with the CRS position of every entry as an int32
        # payload (the conversion moves values bit for bit)
        self.J = S.jds_from_csr(A)
        pos = torch.arange(self.nnz, dtype=torch.int32, device=dev)
        Jpos = S.jds_from_csr(A.with_values(pos))
        self.jds_src = Jpos.jd_val                                              # JDS slot -> CRS position
        jds_of_crs = S.spmv_permute_vec(self.jds_src, pos, inverse=True)      # CRS position -> JDS slot
        # A^T in CRS (pattern + map into A's CRS values)
        rowT, colT, tmap = S.spmv_transpose_csr(A)
        if transpose == "crs":
            # A^T CRS slot -> A CRS position -> A JDS slot
            self.tmapT = S.spmv_gather_values(tmap, jds_of_crs)
            self.AT = S.spmv_crs_plan(S.CSR(A.n_cols, A.n_rows, rowT, colT, None))
            self.JT = None
        else:
            AT = S.CSR(A.n_cols, A.n_rows, rowT, colT, tmap)
            JT = S.jds_from_csr(AT)
            # A^T JDS slot -> A CRS position -> A JDS slot
            self.tmapT = S.spmv_gather_values(JT.jd_val, jds_of_crs)
            self.JT = JT.with_values(None)
            self.AT = None
        self._valsT = None
        self._valsT_of = None        # weak reference to the vals tensor _valsT was built from
        self._valsT_key = None

    def vals_from_crs(self, crs_val: torch.Tensor) -> torch.Tensor:
        """A's values given in CRS order, rearranged into the operator's JDS order."""
        return S.spmv_gather_values(self.jds_src, crs_val)

    def transposed_values(self, vals: torch.Tensor) -> torch.Tensor:
        """A^T's values (one gather), reused while `vals` is the same tensor
        object with the same version counter, storage and dtype.  A new
        tensor is never taken for the old one, even when the allocator puts
        it at the address of a freed one."""
        key = (vals._version, vals.data_ptr(), vals.dtype)
        same = self._valsT_of is not None and self._valsT_of() is vals and self._valsT_key == key
        if self._valsT is None or not same:
            self._valsT = S.spmv_gather_values(self.tmapT, vals)
            self._valsT_of = weakref.ref(vals)
            self._valsT_key = key
        return self._valsT

    # y = alpha*A x + beta*y
    def matvec(self, vals, x, y=None, alpha=1.0, beta=0.0):
        return S.spmv_jds(self.J.with_values(vals), x, y, alpha, beta, self.unroll, self.max_iters, self.wg_waves)

    def rmatvec(self, vals, g, y=None, alpha=1.0, beta=0.0):
        vT = self.transposed_values(vals)
        if self.AT is not None:
            return S.spmv_crs(self.AT.with_values(vT), g, y, alpha, beta)
        return S.spmv_jds(self.JT.with_values(vT), g, y, alpha, beta, self.unroll, self.max_iters, self.wg_waves)

    def grad_vals(self, g, x, out=None, alpha=1.0, beta=0.0):
        return S.spmv_grad_vals_jds(self.J, g, x, out, alpha, beta)


class SpMVFunction(torch.autograd.Function):
    """y = A(vals) x with the hand-written backward."""

    @staticmethod
    def forward(ctx, vals, x, op: SpMVOperator):
        ctx.op = op
        ctx.save_for_backward(vals, x)
        return op.matvec(vals, x)

    @staticmethod
    def backward(ctx, g):
        vals, x = ctx.saved_tensors
        op = ctx.op
        g = g.contiguous()
        dvals = op.grad_vals(g, x) if ctx.needs_input_grad[0] else None
        dx = op.rmatvec(vals, g) if ctx.needs_input_grad[1] else None
        return dvals, dx, None


def spmv(op: SpMVOperator, vals, x):
    return SpMVFunction.apply(vals, x, op)


def _copy(v):
    out = torch.empty_like(v)
    return S.spmv_axpby(1.0, v, 0.0, out)


def _step(op, vals, y_k, y_km1):
    """y_{k+1} = 2 A y_k - y_{k-1} (one fused kernel call)."""
    out = _copy(y_km1)
    return op.matvec(vals, y_k, out, alpha=2.0, beta=-1.0)


def cheb_states(op, vals, x, steps):
    ys = [x, op.matvec(vals, x)]
    for _ in range(1, steps):
        ys.append(_step(op, vals, ys[-1], ys[-2]))
    return ys


class ChebyshevLoss(torch.autograd.Function):
    @staticmethod
    def forward(ctx, vals, x, op: SpMVOperator, steps: int, checkpoint: int):
        if steps < 1:
            raise ValueError("steps >= 1")
        ckpt = max(1, int(checkpoint))
        saved = {0: (x,)}
        y_prev, y = x, op.matvec(vals, x)
        for k in range(1, steps):
            if k % ckpt == 0:
                saved[k] = (_copy(y_prev), _copy(y))       # (y_{k-1}, y_k)
            y_prev, y = y, _step(op, vals, y, y_prev)
        loss = S.spmv_dot(y, y)[0]                       # FP64
        ctx.op, ctx.steps, ctx.ckpt, ctx.saved = op, steps, ckpt, saved
        ctx.save_for_backward(vals, x, y)
        return loss

    @staticmethod
    def backward(ctx, gl):
        vals, x, y_last = ctx.saved_tensors
        op, K, ckpt, saved = ctx.op, ctx.steps, ctx.ckpt, ctx.saved
        scale = float(gl.item()) if gl.numel() == 1 else 1.0
        n = x.numel()
        # adjoint states bar[k]; only three are live at a time
        bar = {K: S.spmv_axpby(2.0 * scale, y_last, 0.0, torch.empty_like(y_last))}
        dvals = torch.empty(op.nnz, dtype=vals.dtype, device=vals.device)
        first_dval = True

        def get_bar(k):
            if k not in bar:
                bar[k] = S.spmv_axpby(0.0, x, 0.0, torch.empty_like(x))   # alpha = beta = 0 writes zeros
            return bar[k]

        # segments [s, e): recompute y_{s-1}..y_e from the checkpoint at s
        starts = sorted(set([0] + [k for k in saved if k > 0]))
        for si in range(len(starts) - 1, -1, -1):
            s = starts[si]
            e = starts[si + 1] if si + 1 < len(starts) else K
            # forward states y_k for k in [s-1, e] (k <= K-1 needed)
            if s == 0:
                ys = {0: x, 1: op.matvec(vals, x)}
                lo = 1
            else:
                ys = {s - 1: saved[s][0], s: saved[s][1]}
                lo = s
            for k in range(lo, e - 1):
                ys[k + 1] = _step(op, vals, ys[k], ys[k - 1])
            # reverse sweep over steps k = e-1 .. max(s, 1) (step k makes y_{k+1})
            for k in range(min(e, K) - 1, max(s, 1) - 1, -1):
                bk1 = bar.pop(k + 1)
                op.rmatvec(vals, bk1, get_bar(k), alpha=2.0, beta=1.0)
                S.spmv_axpby(-1.0, bk1, 1.0, get_bar(k - 1))
                op.grad_vals(bk1, ys[k], dvals, alpha=2.0, beta=0.0 if first_dval else 1.0)
                first_dval = False
            if s == 0:
                b1 = bar.pop(1)
                op.rmatvec(vals, b1, get_bar(0), alpha=1.0, beta=1.0)
                op.grad_vals(b1, x, dvals, alpha=1.0, beta=0.0 if first_dval else 1.0)
                first_dval = False
        dx = bar.pop(0)
        return dvals, dx, None, None, None


def chebyshev_loss(op: SpMVOperator, vals, x, steps: int = 20, checkpoint: int = 5):
    return ChebyshevLoss.apply(vals, x, op, steps, checkpoint)
