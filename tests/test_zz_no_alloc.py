"""The allocation-free dot product (spmv_dot_noalloc, for callers that cannot
allocate) called through the C ABI against the workspace form spmv_dot: the
same kernels and summation tree, so the results must be bit-identical, on two
calls in a row (the second smaller, so partials left by the first are in the
scratch array and must not be read) and on an empty input; inputs beyond the
scratch array's capacity are refused before any device work."""
import ctypes

import numpy as np
import pytest
import torch

pytestmark = pytest.mark.gpu
sp = pytest.importorskip("paper_0910_4836_amd")
from paper_0910_4836_amd import _lib  # noqa: E402


def _ptr(t):
    return ctypes.c_void_p(t.data_ptr())


def _stream():
    return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)


def _dot_ws(lib, x, y, code):
    out = torch.full((1,), np.nan, dtype=torch.float64, device="cuda")
    ws = torch.empty(max(lib.spmv_dot_workspace_size(x.numel()), 1), dtype=torch.uint8, device="cuda")
    assert lib.spmv_dot(x.numel(), _ptr(x), _ptr(y), code, _ptr(out), _ptr(ws), ws.numel(), _stream()) == 0
    return out


def _dot_noalloc(lib, x, y, code):
    out = torch.full((1,), np.nan, dtype=torch.float64, device="cuda")
    st = lib.spmv_dot_noalloc(x.numel(), _ptr(x), _ptr(y), code, _ptr(out), _stream())
    assert st == 0, lib.spmv_last_error()
    return out


def test_noalloc_dot_matches_workspace_dot_twice():
    lib = _lib.load()
    g = torch.Generator(device="cuda")
    g.manual_seed(20091026)
    cases = [(3_000_001, torch.float64, _lib.F64), (10_007, torch.float32, _lib.F32)]
    for n, dt, code in cases:
        print(f"[noalloc] n={n} dtype={dt}", flush=True)
        x = (torch.rand(n, generator=g, device="cuda", dtype=torch.float64) * 2 - 1).to(dt)
        y = (torch.rand(n, generator=g, device="cuda", dtype=torch.float64) * 2 - 1).to(dt)
        got = _dot_noalloc(lib, x, y, code)
        want = _dot_ws(lib, x, y, code)
        torch.cuda.synchronize()
        assert got.item() == want.item(), (n, got.item(), want.item())
        # and the value itself: a sum of n FP64 products within n*2^-53*sum|x y|
        xs, ys = x.double().cpu().numpy(), y.double().cpu().numpy()
        assert abs(got.item() - float(np.dot(xs, ys))) <= n * 2.0 ** -53 * float(np.abs(xs * ys).sum())
    # empty input: exactly zero
    e = torch.empty(0, dtype=torch.float64, device="cuda")
    out = torch.full((1,), np.nan, dtype=torch.float64, device="cuda")
    assert lib.spmv_dot_noalloc(0, None, None, _lib.F64, _ptr(out), _stream()) == 0
    torch.cuda.synchronize()
    assert out.item() == 0.0
    del e
    # the binding
    x = torch.linspace(-1, 1, 5000, dtype=torch.float64, device="cuda")
    o = torch.empty(1, dtype=torch.float64, device="cuda")
    assert sp.spmv_dot_noalloc(x, x, o).item() == sp.spmv_dot(x, x).item()


def test_noalloc_dot_rejects_inputs_beyond_the_scratch():
    lib = _lib.load()
    x = torch.zeros(4, dtype=torch.float64, device="cuda")
    out = torch.zeros(1, dtype=torch.float64, device="cuda")
    # the size check comes first: nothing is read or launched
    st = lib.spmv_dot_noalloc(134_217_728 + 1, _ptr(x), _ptr(x), _lib.F64, _ptr(out), _stream())
    assert st == 3 and b"SPMV_DOT_NOALLOC_MAX_N" in lib.spmv_last_error()
    st = lib.spmv_dot_noalloc(4, _ptr(x), _ptr(x), _lib.BF16, _ptr(out), _stream())
    assert st == 1
