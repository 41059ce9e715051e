"""CPU oracle for the CRS / JDS SpMV library (plain serial FP64 C, via ctypes).

TEST INFRASTRUCTURE.  Only the test-suite, the package smoke check and the
benchmark's CPU-baseline leg may import this module.  The product path (the
HIP library and its Python binding) never does, and shares no code with it.

The arithmetic lives in ``oracle.c``; this wrapper only marshals numpy arrays.
Every routine there cites the part of the paper (Schubert, Hager, Fehske,
Section 2: storage schemes and the CRS / JDS kernels) that it writes out.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "oracle.c")
_LIB = os.path.join(_HERE, "liborc.so")

CFLAGS = ["-O2", "-ffp-contract=off", "-fno-fast-math", "-fPIC", "-shared", "-Wall"]


def build(force: bool = False) -> str:
    """Compile oracle.c with gcc (no FMA contraction)."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp"
        subprocess.check_call(["gcc", *CFLAGS, "-o", tmp, _SRC, "-lm"])
        os.replace(tmp, _LIB)
    return _LIB


_lib = None

_i32p = np.ctypeslib.ndpointer(np.int32, flags="C_CONTIGUOUS")
_i64p = np.ctypeslib.ndpointer(np.int64, flags="C_CONTIGUOUS")
_f64p = np.ctypeslib.ndpointer(np.float64, flags="C_CONTIGUOUS")
_u16p = np.ctypeslib.ndpointer(np.uint16, flags="C_CONTIGUOUS")
_i32, _i64, _f64, _int = C.c_int32, C.c_int64, C.c_double, C.c_int

_SIGS = {
    "orc_spmv_crs": (None, [_i32, _i32p, _i32p, _f64p, _f64p, _f64p, _f64, _f64]),
    "orc_row_absdot": (None, [_i32, _i32p, _i32p, _f64p, _f64p, _f64p]),
    "orc_spmm_crs": (None, [_i32, _i32p, _i32p, _f64p, _i32, _f64p, _i64, _f64p, _i64, _f64, _f64]),
    "orc_csr_from_coo": (_i64, [_i32, _i32, _i64, _i32p, _i32p, _f64p, _i32p, _i32p, _f64p]),
    "orc_jds_from_csr": (_i32, [_i32, _i32p, _i32p, _f64p, _int, _i32p, _i32p, _i32p, _i32, _i32p, _f64p]),
    "orc_jds_to_csr": (None, [_i32, _i32p, _i32p, _i32, _i32p, _f64p, _i32p, _i32p, _f64p]),
    "orc_spmv_jds": (None, [_i32, _i32p, _i32p, _i32, _i32p, _f64p, _f64p, _f64p, _f64, _f64, _int]),
    "orc_spmv_nujds": (None, [_i32, _i32p, _i32p, _i32, _i32p, _f64p, _f64p, _f64p, _f64, _f64, _int, _i32]),
    "orc_spmv_nbjds": (None, [_i32, _i32p, _i32p, _i32, _i32p, _f64p, _f64p, _f64p, _f64, _f64, _int, _i32]),
    "orc_jds_blocked_from_jds": (_i64, [_i32, _i32p, _i32, _i32p, _f64p, _i32, _int, _i64p, _i32p, _i32p, _f64p]),
    "orc_jds_blocked_windowed": (_i64, [_i32, _i32p, _i32p, _f64p, _i32, _i32, _i32p, _i64p, _i32p, C.c_void_p,
                                        C.c_void_p]),
    "orc_spmv_jds_blocked": (None, [_i32, _i32p, _i32, _i32, _i64p, _i32p, _i32p, _f64p, _f64p, _f64p, _f64, _f64, _int]),
    "orc_round_bf16": (None, [_f64p, _u16p, _i64]),
    "orc_csr_transpose": (None, [_i32, _i32, _i32p, _i32p, _i32p, _i32p, _i64p]),
    "orc_csr_upper": (_i64, [_i32, _i32p, _i32p, _f64p, C.c_void_p, C.c_void_p, C.c_void_p]),
    "orc_spmv_crs_sym": (None, [_i32, _i32p, _i32p, _f64p, _f64p, _f64p, _f64, _f64]),
    "orc_grad_vals_csr": (None, [_i32, _i32p, _i32p, _f64p, _f64p, _f64p, _f64, _f64]),
    "orc_spmv_crs_transposed": (None, [_i32, _i32, _i32p, _i32p, _f64p, _f64p, _f64p]),
    "orc_cheb_forward": (None, [_i32, _i32p, _i32p, _f64p, _f64p, _i32, _f64p]),
    "orc_cheb_adjoint": (_f64, [_i32, _i32p, _i32p, _f64p, _f64p, _i32, _f64p, _f64p]),
}


def lib():
    global _lib
    if _lib is None:
        path = _LIB if os.path.exists(_LIB) else build()
        if os.path.getmtime(path) < os.path.getmtime(_SRC):
            path = build()
        _lib = C.CDLL(path)
        for name, (res, args) in _SIGS.items():
            fn = getattr(_lib, name)
            fn.restype = res
            fn.argtypes = args
    return _lib


def _c(a, dt):
    return np.ascontiguousarray(a, dtype=dt)


# ---------------------------------------------------------------------------
# CRS


class CSR:
    """Host CRS matrix (row_ptr int32, col int32, val float64)."""

    def __init__(self, n_rows, n_cols, row_ptr, col, val):
        self.n_rows, self.n_cols = int(n_rows), int(n_cols)
        self.row_ptr = _c(row_ptr, np.int32)
        self.col = _c(col, np.int32)
        self.val = _c(val, np.float64)

    @property
    def nnz(self):
        return int(self.row_ptr[-1])

    def row_lengths(self):
        return np.diff(self.row_ptr.astype(np.int64))

    def row_index(self):
        return np.repeat(np.arange(self.n_rows, dtype=np.int64), self.row_lengths())


def csr_from_coo(n_rows, n_cols, row, col, val) -> CSR:
    row, col, val = _c(row, np.int32), _c(col, np.int32), _c(val, np.float64)
    nnz = len(row)
    row_ptr = np.zeros(n_rows + 1, np.int32)
    col_out = np.zeros(max(nnz, 1), np.int32)
    val_out = np.zeros(max(nnz, 1), np.float64)
    got = lib().orc_csr_from_coo(n_rows, n_cols, nnz, row, col, val, row_ptr, col_out, val_out)
    if got < 0:
        raise ValueError("COO index out of range")
    return CSR(n_rows, n_cols, row_ptr, col_out[:got], val_out[:got])


def spmv_crs(A: CSR, x, y=None, alpha=1.0, beta=0.0):
    x = _c(x, np.float64)
    out = np.zeros(A.n_rows, np.float64) if y is None else _c(y, np.float64).copy()
    lib().orc_spmv_crs(A.n_rows, A.row_ptr, A.col, A.val, x, out, alpha, beta)
    return out


def row_absdot(A: CSR, x):
    D = np.zeros(A.n_rows, np.float64)
    lib().orc_row_absdot(A.n_rows, A.row_ptr, A.col, A.val, _c(x, np.float64), D)
    return D


def spmm_crs(A: CSR, X, alpha=1.0, beta=0.0, Y=None):
    """X is (n_cols, k) in Fortran (column-major) order."""
    X = np.asfortranarray(X, dtype=np.float64)
    k = X.shape[1]
    Yo = np.zeros((A.n_rows, k), np.float64, order="F") if Y is None else np.asfortranarray(Y, dtype=np.float64).copy(order="F")
    xf = X.ravel(order="F")
    yf = Yo.ravel(order="F")
    lib().orc_spmm_crs(A.n_rows, A.row_ptr, A.col, A.val, k, xf, X.shape[0], yf, A.n_rows, alpha, beta)
    return yf.reshape((A.n_rows, k), order="F")


def spmv_crs_transposed(A: CSR, g):
    y = np.zeros(A.n_cols, np.float64)
    lib().orc_spmv_crs_transposed(A.n_rows, A.n_cols, A.row_ptr, A.col, A.val, _c(g, np.float64), y)
    return y


def transpose(A: CSR):
    """Returns (rowT_ptr, colT, tmap): A^T's pattern and A^T.val = A.val[tmap]."""
    rowT = np.zeros(A.n_cols + 1, np.int32)
    colT = np.zeros(max(A.nnz, 1), np.int32)
    tmap = np.zeros(max(A.nnz, 1), np.int64)
    lib().orc_csr_transpose(A.n_rows, A.n_cols, A.row_ptr, A.col, rowT, colT, tmap)
    return rowT, colT[:A.nnz], tmap[:A.nnz]


def csr_upper(A: CSR) -> CSR:
    """Upper triangle (col >= row) of a square matrix, each row in CRS order."""
    assert A.n_rows == A.n_cols
    n = A.n_rows
    m = int(lib().orc_csr_upper(n, A.row_ptr, A.col, A.val, None, None, None))
    rp = np.zeros(n + 1, np.int32)
    col = np.zeros(max(m, 1), np.int32)
    val = np.zeros(max(m, 1), np.float64)
    lib().orc_csr_upper(n, A.row_ptr, A.col, A.val, rp.ctypes.data_as(C.c_void_p), col.ctypes.data_as(C.c_void_p),
                        val.ctypes.data_as(C.c_void_p))
    return CSR(n, n, rp, col[:m], val[:m])


def spmv_crs_sym(U: CSR, x, y=None, alpha=1.0, beta=0.0):
    """y = alpha * (U + U^T - diag(U)) x + beta * y from the upper triangle U."""
    out = np.zeros(U.n_rows, np.float64) if y is None else _c(y, np.float64).copy()
    lib().orc_spmv_crs_sym(U.n_rows, U.row_ptr, U.col, U.val, _c(x, np.float64), out, alpha, beta)
    return out


def grad_vals(A: CSR, g, x, alpha=1.0, beta=0.0, out=None):
    o = np.zeros(max(A.nnz, 1), np.float64) if out is None else _c(out, np.float64).copy()
    lib().orc_grad_vals_csr(A.n_rows, A.row_ptr, A.col, _c(g, np.float64), _c(x, np.float64), o, alpha, beta)
    return o[:A.nnz]


# ---------------------------------------------------------------------------
# JDS family


class JDS:
    def __init__(self, n, perm, iperm, jd_ptr, jd_col, jd_val, symperm):
        self.n = n
        self.perm, self.iperm, self.jd_ptr = perm, iperm, jd_ptr
        self.jd_col, self.jd_val = jd_col, jd_val
        self.ndiag = len(jd_ptr) - 1
        self.symperm = bool(symperm)


def jds_from_csr(A: CSR, symperm=False) -> JDS:
    n = A.n_rows
    if symperm and A.n_rows != A.n_cols:
        raise ValueError("symmetric permutation needs a square matrix")
    perm = np.zeros(max(n, 1), np.int32)
    iperm = np.zeros(max(n, 1), np.int32)
    nnz = A.nnz
    jd_col = np.zeros(max(nnz, 1), np.int32)
    jd_val = np.zeros(max(nnz, 1), np.float64)
    cap = int(A.row_lengths().max()) + 1 if n else 1
    jd_ptr = np.zeros(cap, np.int32)
    nd = lib().orc_jds_from_csr(n, A.row_ptr, A.col, A.val, int(symperm), perm, iperm, jd_ptr, cap,
                                jd_col, jd_val)
    assert nd >= 0
    return JDS(n, perm[:n], iperm[:n], jd_ptr[:nd + 1], jd_col[:nnz], jd_val[:nnz], symperm)


def jds_to_csr(J: JDS, n_cols) -> CSR:
    n = J.n
    nnz = int(J.jd_ptr[-1])
    row_ptr = np.zeros(n + 1, np.int32)
    col = np.zeros(max(nnz, 1), np.int32)
    val = np.zeros(max(nnz, 1), np.float64)
    lib().orc_jds_to_csr(n, _c(J.perm, np.int32), _c(J.jd_ptr, np.int32), J.ndiag, _c(J.jd_col, np.int32),
                         _c(J.jd_val, np.float64), row_ptr, col, val)
    return CSR(n, n_cols, row_ptr, col[:nnz], val[:nnz])


def _jds_args(J):
    return (J.n, _c(J.perm, np.int32), _c(J.jd_ptr, np.int32), J.ndiag, _c(J.jd_col, np.int32),
            _c(J.jd_val, np.float64))


def spmv_jds(J: JDS, x, y=None, alpha=1.0, beta=0.0):
    out = np.zeros(J.n, np.float64) if y is None else _c(y, np.float64).copy()
    lib().orc_spmv_jds(*_jds_args(J), _c(x, np.float64), out, alpha, beta, int(J.symperm))
    return out


def spmv_nujds(J: JDS, x, unroll, y=None, alpha=1.0, beta=0.0):
    out = np.zeros(J.n, np.float64) if y is None else _c(y, np.float64).copy()
    lib().orc_spmv_nujds(*_jds_args(J), _c(x, np.float64), out, alpha, beta, int(J.symperm), unroll)
    return out


def spmv_nbjds(J: JDS, x, block, y=None, alpha=1.0, beta=0.0):
    out = np.zeros(J.n, np.float64) if y is None else _c(y, np.float64).copy()
    lib().orc_spmv_nbjds(*_jds_args(J), _c(x, np.float64), out, alpha, beta, int(J.symperm), block)
    return out


class Blocked:
    def __init__(self, n, perm, C, slice_ptr, slice_nd, bl_col, bl_val, symperm):
        self.n, self.perm, self.C = n, perm, C
        self.slice_ptr, self.slice_nd = slice_ptr, slice_nd
        self.bl_col, self.bl_val = bl_col, bl_val
        self.n_slices = len(slice_nd)
        self.symperm = symperm


def blocked_from_jds(J: JDS, C: int, sojds=False) -> Blocked:
    n = J.n
    ns = (n + C - 1) // C
    slice_ptr = np.zeros(ns + 1, np.int64)
    slice_nd = np.zeros(max(ns, 1), np.int32)
    # size: every block padded to its first row
    lens0 = np.diff(J.jd_ptr.astype(np.int64))
    first = np.arange(ns, dtype=np.int64) * C
    nd = np.array([(lens0 > f).sum() for f in first], dtype=np.int64) if ns else np.zeros(0, np.int64)
    total = int((nd * C).sum())
    bl_col = np.zeros(max(total, 1), np.int32)
    bl_val = np.zeros(max(total, 1), np.float64)
    got = lib().orc_jds_blocked_from_jds(n, _c(J.jd_ptr, np.int32), J.ndiag, _c(J.jd_col, np.int32),
                                         _c(J.jd_val, np.float64), C, int(sojds), slice_ptr, slice_nd,
                                         bl_col, bl_val)
    assert got == total
    return Blocked(n, J.perm, C, slice_ptr, slice_nd[:ns], bl_col[:total], bl_val[:total], J.symperm)


def blocked_windowed(A: CSR, C_: int, sigma: int) -> Blocked:
    """RBJDS storage over rows sorted by decreasing length inside windows of
    sigma consecutive rows (sigma a multiple of C_)."""
    n = A.n_rows
    ns = (n + C_ - 1) // C_
    perm = np.zeros(max(n, 1), np.int32)
    slice_ptr = np.zeros(ns + 1, np.int64)
    slice_nd = np.zeros(max(ns, 1), np.int32)
    total = lib().orc_jds_blocked_windowed(n, A.row_ptr, A.col, A.val, C_, sigma, perm, slice_ptr, slice_nd,
                                           None, None)          # sizes only
    if total < 0:
        raise ValueError("sigma must be a positive multiple of C")
    bl_col = np.zeros(max(total, 1), np.int32)
    bl_val = np.zeros(max(total, 1), np.float64)
    got = lib().orc_jds_blocked_windowed(n, A.row_ptr, A.col, A.val, C_, sigma, perm, slice_ptr, slice_nd,
                                         bl_col.ctypes.data, bl_val.ctypes.data)
    assert got == total
    return Blocked(n, perm[:n], C_, slice_ptr, slice_nd[:ns], bl_col[:total], bl_val[:total], False)


def spmv_blocked(B: Blocked, x, y=None, alpha=1.0, beta=0.0):
    out = np.zeros(B.n, np.float64) if y is None else _c(y, np.float64).copy()
    lib().orc_spmv_jds_blocked(B.n, _c(B.perm, np.int32), B.C, B.n_slices, _c(B.slice_ptr, np.int64),
                               _c(B.slice_nd, np.int32), _c(B.bl_col, np.int32), _c(B.bl_val, np.float64),
                               _c(x, np.float64), out, alpha, beta, int(B.symperm))
    return out


# ---------------------------------------------------------------------------
# reduced precision


def round_bf16_bits(v) -> np.ndarray:
    """bf16 bit patterns of ``v``: one round-to-nearest-even step from FP64."""
    v = _c(v, np.float64)
    out = np.zeros(max(len(v), 1), np.uint16)
    lib().orc_round_bf16(v, out, len(v))
    return out[:len(v)]


def bf16_bits_to_f64(bits) -> np.ndarray:
    b = np.asarray(bits, dtype=np.uint16).astype(np.uint32) << 16
    return b.view(np.float32).astype(np.float64)


def round_f32(v) -> np.ndarray:
    """float32 round-to-nearest-even of FP64 values (numpy's cast)."""
    return np.asarray(v, dtype=np.float64).astype(np.float32)


# ---------------------------------------------------------------------------
# error metric


def rel_err(y, y_ref, D) -> np.ndarray:
    """err_i = |y_i - y_ref_i| / D_i; a row with D_i = 0 must be exactly 0."""
    y = np.asarray(y, dtype=np.float64)
    y_ref = np.asarray(y_ref, dtype=np.float64)
    diff = np.abs(y - y_ref)
    out = np.zeros_like(diff)
    nz = D > 0
    out[nz] = diff[nz] / D[nz]
    out[~nz] = np.where(diff[~nz] == 0, 0.0, np.inf)
    return out


# ---------------------------------------------------------------------------
# Chebyshev recurrence


def cheb_forward(A: CSR, x, steps=20):
    n = A.n_rows
    ys = np.zeros((steps + 1) * n, np.float64)
    lib().orc_cheb_forward(n, A.row_ptr, A.col, A.val, _c(x, np.float64), steps, ys)
    return ys.reshape(steps + 1, n)


def cheb_loss_grad(A: CSR, x, steps=20):
    """Returns (loss, dx, dval, ys) for loss = ||y_steps||^2."""
    ys = cheb_forward(A, x, steps)
    n = A.n_rows
    dx = np.zeros(n, np.float64)
    dval = np.zeros(max(A.nnz, 1), np.float64)
    loss = lib().orc_cheb_adjoint(n, A.row_ptr, A.col, A.val, ys.ravel(), steps, dx, dval)
    return loss, dx, dval[:A.nnz], ys
