"""Shared helpers for the GPU parity tests (inputs from synth, references from the oracle)."""
import numpy as np
import torch

import oracle
import synth

DEV = "cuda"
FP64_TOL = 1e-12      # max |y - y_ref| / sum_j |a_ij||x_j|, FP64 kernels


def to_dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).to(DEV)


def to_np(t):
    return t.detach().cpu().numpy()


def rand_coo(seed, n_rows, n_cols, density, **kw):
    rng = np.random.default_rng(seed)
    r, c, v, nr, nc = synth.random_pattern(n_rows, n_cols, density, rng, **kw)
    return r, c, v, nr, nc, rng


def gpu_csr(sp, r, c, v, n_rows, n_cols, dtype=torch.float64):
    return sp.csr_from_coo(n_rows, n_cols, to_dev(r), to_dev(c), to_dev(v).to(dtype))


def max_err(y_gpu, y_ref, D):
    return float(oracle.rel_err(to_np(y_gpu).astype(np.float64), y_ref, D).max(initial=0.0))
