"""Python binding of libspmv.so: torch tensors in, C ABI calls out.

Each function has the name of the C entry point it wraps and only marshals
arguments: device pointers of torch tensors, sizes, dtype codes and the
current HIP stream.  Every computation runs in the library's HIP kernels.
Workspace and output buffers are allocated here as torch tensors (the library
itself never allocates).

Matrix containers:
  CSR      n_rows, n_cols, row_ptr, col_idx, val     (paper Section 2, CRS)
  JDS      perm, iperm, jd_ptr (+ host copy), jd_col, jd_val   (Section 2, JDS)
  Blocked  slice_ptr, slice_nd (+ host copy), bl_col, bl_val   (RBJDS / SOJDS)
"""
from __future__ import annotations

import ctypes as C
from dataclasses import dataclass, field
from typing import Optional, Tuple

import numpy as np
import torch

from . import _lib
from ._lib import BF16, F32, F64, I32, SOJDS, SYMPERM, SpmvError, call

# int32 is a payload type: the value-moving calls (conversions, permute,
# gather) copy it bit for bit; the arithmetic calls reject it.
_DTYPE_CODE = {torch.float64: F64, torch.float32: F32, torch.bfloat16: BF16, torch.int32: I32}
_VEC_DTYPES = (torch.float64, torch.float32)
_I32 = torch.int32


def dtype_code(t: torch.dtype) -> int:
    try:
        return _DTYPE_CODE[t]
    except KeyError:
        raise TypeError(f"unsupported dtype {t}") from None


def _p(t: Optional[torch.Tensor]):
    if t is None or t.data_ptr() == 0:
        return None
    return C.c_void_p(t.data_ptr())


def _stream():
    return C.c_void_p(torch.cuda.current_stream().cuda_stream)


def _dev(device=None):
    return torch.device(device) if device is not None else torch.device("cuda", torch.cuda.current_device())


def _ws(nbytes: int, device):
    return torch.empty(max(int(nbytes), 1), dtype=torch.uint8, device=device)


def _h_i32(a: np.ndarray):
    return a.ctypes.data_as(C.POINTER(C.c_int32))


def _h_i64(a: np.ndarray):
    return a.ctypes.data_as(C.POINTER(C.c_int64))


def _check_dev(*ts):
    for t in ts:
        if t is not None and not t.is_cuda:
            raise ValueError("tensors must live on the GPU")
        if t is not None and not t.is_contiguous():
            raise ValueError("tensors must be contiguous")


def version() -> str:
    return _lib.load().spmv_version().decode()


# --------------------------------------------------------------------------- containers


@dataclass
class CSR:
    n_rows: int
    n_cols: int
    row_ptr: torch.Tensor
    col_idx: torch.Tensor
    val: torch.Tensor
    plan: Optional[torch.Tensor] = None
    n_blocks: int = 0
    block_nnz: int = 0
    staged: bool = False        # spmv_crs runs the staged kernel (spmv_crs_staged) over the plan

    @property
    def nnz(self) -> int:
        return int(self.col_idx.numel())

    @property
    def device(self):
        return self.row_ptr.device

    def with_values(self, val: torch.Tensor) -> "CSR":
        return CSR(self.n_rows, self.n_cols, self.row_ptr, self.col_idx, val, self.plan, self.n_blocks,
                   self.block_nnz, self.staged)


@dataclass
class JDS:
    n: int
    n_cols: int
    perm: torch.Tensor
    iperm: torch.Tensor
    jd_ptr: torch.Tensor
    h_jd_ptr: np.ndarray
    jd_col: torch.Tensor
    jd_val: torch.Tensor
    symperm: bool = False
    tile_plans: dict = field(default_factory=dict, repr=False)   # (max_iters, rows_per_wave, wg_waves) -> plan

    @property
    def ndiag(self) -> int:
        return len(self.h_jd_ptr) - 1

    @property
    def nnz(self) -> int:
        return int(self.h_jd_ptr[-1])

    @property
    def flags(self) -> int:
        return SYMPERM if self.symperm else 0

    def with_values(self, val: torch.Tensor) -> "JDS":
        return JDS(self.n, self.n_cols, self.perm, self.iperm, self.jd_ptr, self.h_jd_ptr, self.jd_col, val,
                   self.symperm, self.tile_plans)


@dataclass
class Blocked:
    n: int
    n_cols: int
    C: int
    perm: torch.Tensor
    slice_ptr: torch.Tensor
    slice_nd: torch.Tensor
    h_slice_nd: np.ndarray
    bl_col: torch.Tensor
    bl_val: torch.Tensor
    padded: int
    symperm: bool = False
    sojds: bool = False
    sigma: int = 0                   # > 0: rows sorted by length inside windows of sigma rows
    tile_plans: dict = field(default_factory=dict, repr=False)   # (max_iters, rows_per_wave, wg_waves) -> plan

    @property
    def n_slices(self) -> int:
        return len(self.h_slice_nd)

    def with_values(self, val: torch.Tensor) -> "Blocked":
        return Blocked(self.n, self.n_cols, self.C, self.perm, self.slice_ptr, self.slice_nd, self.h_slice_nd,
                       self.bl_col, val, self.padded, self.symperm, self.sojds, self.sigma, self.tile_plans)


# --------------------------------------------------------------------------- setup


def csr_from_coo(n_rows: int, n_cols: int, row: torch.Tensor, col: torch.Tensor, val: torch.Tensor) -> CSR:
    """COO -> CRS on the GPU (spmv_csr_from_coo): sorted, duplicates summed in input order."""
    if row.dtype != _I32 or col.dtype != _I32:
        # the library reads 4-byte indices: an int64 tensor would be read as
        # pairs of int32 halves, a different matrix without an error
        raise TypeError(f"row and col must be int32, got {row.dtype} and {col.dtype}")
    if row.numel() != col.numel() or row.numel() != val.numel():
        raise ValueError(f"row, col and val must have one length, got {row.numel()}, {col.numel()}, {val.numel()}")
    _check_dev(row, col, val)
    dev = row.device
    nnz = int(row.numel())
    ws = _ws(_lib.load().spmv_csr_from_coo_workspace_size(n_rows, n_cols, nnz), dev)
    row_ptr = torch.empty(n_rows + 1, dtype=_I32, device=dev)
    col_out = torch.empty(max(nnz, 1), dtype=_I32, device=dev)
    val_out = torch.empty(max(nnz, 1), dtype=val.dtype, device=dev)
    h_nnz = C.c_int64(0)
    call("spmv_csr_from_coo", n_rows, n_cols, nnz, _p(row), _p(col), _p(val), dtype_code(val.dtype), _p(row_ptr),
         _p(col_out), _p(val_out), C.byref(h_nnz), _p(ws), ws.numel(), _stream())
    k = h_nnz.value
    return CSR(n_rows, n_cols, row_ptr, col_out[:k], val_out[:k])


def spmv_csr_validate(A: CSR) -> bool:
    ws = _ws(_lib.load().spmv_csr_validate_workspace_size(), A.device)
    ok = C.c_int32(0)
    call("spmv_csr_validate", A.n_rows, A.n_cols, A.nnz, _p(A.row_ptr), _p(A.col_idx), C.byref(ok), _p(ws),
         ws.numel(), _stream())
    return bool(ok.value)


def spmv_crs_plan(A: CSR, block_nnz: int = 0) -> CSR:
    """Builds (and stores on A) the row-block plan used by spmv_crs / spmm_crs."""
    nb = C.c_int32(0)
    st = _lib.load().spmv_crs_plan(A.n_rows, _p(A.row_ptr), block_nnz, None, 0, C.byref(nb), _stream())
    if st not in (0, 3):
        call("spmv_crs_plan", A.n_rows, _p(A.row_ptr), block_nnz, None, 0, C.byref(nb), _stream())
    plan = torch.empty(nb.value + 1, dtype=_I32, device=A.device)
    call("spmv_crs_plan", A.n_rows, _p(A.row_ptr), block_nnz, _p(plan), plan.numel(), C.byref(nb), _stream())
    A.plan, A.n_blocks, A.block_nnz = plan, nb.value, block_nnz
    return A


def jds_from_csr(A: CSR, symperm: bool = False) -> JDS:
    """CRS -> JDS on the GPU (spmv_jds_from_csr)."""
    lib = _lib.load()
    dev = A.device
    n, nnz = A.n_rows, A.nnz
    flags = SYMPERM if symperm else 0
    ws = _ws(lib.spmv_jds_from_csr_workspace_size(n, nnz), dev)
    perm = torch.empty(max(n, 1), dtype=_I32, device=dev)
    iperm = torch.empty(max(n, 1), dtype=_I32, device=dev)
    jd_col = torch.empty(max(nnz, 1), dtype=_I32, device=dev)
    jd_val = torch.empty(max(nnz, 1), dtype=A.val.dtype, device=dev)
    nd = C.c_int32(0)
    args = lambda cap, jp, hjp: (n, nnz, _p(A.row_ptr), _p(A.col_idx), _p(A.val), dtype_code(A.val.dtype), flags,
                                 _p(perm), _p(iperm), jp, cap, _p(jd_col), _p(jd_val), C.byref(nd), hjp, _p(ws),
                                 ws.numel(), _stream())
    st = lib.spmv_jds_from_csr(*args(0, None, None))
    if st not in (0, 3):
        call("spmv_jds_from_csr", *args(0, None, None))
    jd_ptr = torch.empty(nd.value + 1, dtype=_I32, device=dev)
    h_jd_ptr = np.zeros(nd.value + 1, dtype=np.int32)
    call("spmv_jds_from_csr", *args(nd.value + 1, _p(jd_ptr), _h_i32(h_jd_ptr)))
    return JDS(n, A.n_cols, perm[:n], iperm[:n], jd_ptr, h_jd_ptr, jd_col[:nnz], jd_val[:nnz], symperm)


def jds_to_csr(J: JDS) -> CSR:
    lib = _lib.load()
    dev = J.jd_ptr.device
    ws = _ws(lib.spmv_jds_to_csr_workspace_size(J.n), dev)
    row_ptr = torch.empty(J.n + 1, dtype=_I32, device=dev)
    col = torch.empty(max(J.nnz, 1), dtype=_I32, device=dev)
    val = torch.empty(max(J.nnz, 1), dtype=J.jd_val.dtype, device=dev)
    call("spmv_jds_to_csr", J.n, _p(J.perm), _p(J.jd_ptr), J.ndiag, _p(J.jd_col), _p(J.jd_val),
         dtype_code(J.jd_val.dtype), J.flags, _p(row_ptr), _p(col), _p(val), _p(ws), ws.numel(), _stream())
    return CSR(J.n, J.n_cols, row_ptr, col[:J.nnz], val[:J.nnz])


def jds_blocked_from_jds(J: JDS, C_: int = 64, sojds: bool = False) -> Blocked:
    """JDS -> blocked JDS with slices of C_ rows (spmv_jds_blocked_from_jds)."""
    lib = _lib.load()
    dev = J.jd_ptr.device
    flags = SOJDS if sojds else 0
    ns = -(-J.n // C_)
    ws = _ws(lib.spmv_jds_blocked_workspace_size(J.n, J.ndiag, C_, flags), dev)
    slice_ptr = torch.empty(ns + 1, dtype=torch.int64, device=dev)
    slice_nd = torch.empty(max(ns, 1), dtype=_I32, device=dev)
    h_slice_nd = np.zeros(max(ns, 1), dtype=np.int32)
    padded = C.c_int64(0)
    args = lambda cap, bc, bv: (J.n, _p(J.jd_ptr), J.ndiag, _p(J.jd_col), _p(J.jd_val), dtype_code(J.jd_val.dtype),
                                C_, flags, _p(slice_ptr), _p(slice_nd), bc, bv, cap, C.byref(padded),
                                _h_i32(h_slice_nd), _p(ws), ws.numel(), _stream())
    st = lib.spmv_jds_blocked_from_jds(*args(0, None, None))
    if st not in (0, 3):
        call("spmv_jds_blocked_from_jds", *args(0, None, None))
    tot = padded.value
    bl_col = torch.empty(max(tot, 1), dtype=_I32, device=dev)
    bl_val = torch.empty(max(tot, 1), dtype=J.jd_val.dtype, device=dev)
    if tot > 0:
        call("spmv_jds_blocked_from_jds", *args(tot, _p(bl_col), _p(bl_val)))
    return Blocked(J.n, J.n_cols, C_, J.perm, slice_ptr, slice_nd[:ns], h_slice_nd[:ns].copy(), bl_col[:tot],
                   bl_val[:tot], tot, J.symperm, sojds)


def jds_blocked_windowed_from_csr(A: CSR, C_: int = 64, sigma: int = 65536) -> Blocked:
    """CRS -> blocked JDS with rows sorted by length inside windows of sigma
    rows (spmv_jds_blocked_windowed_from_csr); sigma is rounded up to a
    multiple of C_."""
    lib = _lib.load()
    dev = A.device
    sigma = -(-int(sigma) // C_) * C_
    n = A.n_rows
    ns = -(-n // C_)
    ws = _ws(lib.spmv_jds_blocked_windowed_workspace_size(n), dev)
    perm = torch.empty(max(n, 1), dtype=_I32, device=dev)
    slice_ptr = torch.empty(ns + 1, dtype=torch.int64, device=dev)
    slice_nd = torch.empty(max(ns, 1), dtype=_I32, device=dev)
    h_slice_nd = np.zeros(max(ns, 1), dtype=np.int32)
    padded = C.c_int64(0)
    args = lambda cap, bc, bv: (n, A.nnz, _p(A.row_ptr), _p(A.col_idx), _p(A.val), dtype_code(A.val.dtype), C_,
                                sigma, _p(perm), _p(slice_ptr), _p(slice_nd), bc, bv, cap, C.byref(padded),
                                _h_i32(h_slice_nd), _p(ws), ws.numel(), _stream())
    st = lib.spmv_jds_blocked_windowed_from_csr(*args(0, None, None))
    if st not in (0, 3):
        call("spmv_jds_blocked_windowed_from_csr", *args(0, None, None))
    tot = padded.value
    bl_col = torch.empty(max(tot, 1), dtype=_I32, device=dev)
    bl_val = torch.empty(max(tot, 1), dtype=A.val.dtype, device=dev)
    if tot > 0:
        call("spmv_jds_blocked_windowed_from_csr", *args(tot, _p(bl_col), _p(bl_val)))
    return Blocked(n, A.n_cols, C_, perm[:n], slice_ptr, slice_nd[:ns], h_slice_nd[:ns].copy(), bl_col[:tot],
                   bl_val[:tot], tot, False, False, sigma)


def spmv_jds_blocked_tiles(B: Blocked, max_iters: int = 0, rows_per_wave: int = 0, wg_waves: int = 0):
    """The tile plan of B for spmv_jds_blocked_tiled (spmv_jds_blocked_tiles),
    built once per launch shape and kept on B: (tiles, n_tiles, h_plan)."""
    key = (max_iters, rows_per_wave, wg_waves)
    if key not in B.tile_plans:
        lib = _lib.load()
        nt = C.c_int64(0)
        h_plan = np.zeros(10, dtype=np.int64)
        args = lambda t, cap: (B.n, B.C, B.n_slices, _h_i32(B.h_slice_nd), max_iters, rows_per_wave, wg_waves, t,
                               cap, C.byref(nt), _h_i64(h_plan), _stream())
        st = lib.spmv_jds_blocked_tiles(*args(None, 0))
        if st not in (0, 3):
            call("spmv_jds_blocked_tiles", *args(None, 0))
        tiles = torch.empty(max(2 * nt.value, 1), dtype=_I32, device=B.bl_col.device)
        call("spmv_jds_blocked_tiles", *args(_p(tiles), tiles.numel()))
        B.tile_plans[key] = (tiles, nt.value, h_plan)
    return B.tile_plans[key]


def spmv_jds_blocked_tiled(B: Blocked, x: torch.Tensor, y: Optional[torch.Tensor] = None, alpha: float = 1.0,
                           beta: float = 0.0, unroll: int = 0, max_iters: int = 0, rows_per_wave: int = 0,
                           wg_waves: int = 0) -> torch.Tensor:
    """y = alpha*A x + beta*y with the blocked-JDS kernel launched from B's
    tile plan (spmv_jds_blocked_tiled): each XCD walks its eighth of the
    slices in order."""
    y = _out_vec(y, B.n, x, beta, B.n_cols)
    tiles, nt, h_plan = spmv_jds_blocked_tiles(B, max_iters, rows_per_wave, wg_waves)
    flags = (SYMPERM if B.symperm else 0) | (SOJDS if B.sojds else 0)
    call("spmv_jds_blocked_tiled", B.n, _p(B.perm), B.C, B.n_slices, _p(B.slice_ptr), _p(B.slice_nd), _p(B.bl_col),
         _p(B.bl_val), dtype_code(B.bl_val.dtype), _p(x), _p(y), dtype_code(x.dtype), float(alpha), float(beta),
         _p(tiles), nt, _h_i64(h_plan), unroll, flags, _stream())
    return y


def spmv_convert_values(t: torch.Tensor, dtype: torch.dtype) -> torch.Tensor:
    """Rounds (round-to-nearest-even, one step) or widens values to ``dtype``."""
    _check_dev(t)
    out = torch.empty(t.shape, dtype=dtype, device=t.device)
    call("spmv_convert_values", t.numel(), _p(t), dtype_code(t.dtype), _p(out), dtype_code(dtype), _stream())
    return out


def spmv_transpose_csr(A: CSR):
    """Returns (rowT_ptr, colT, tmap): A^T's pattern, its values being A.val[tmap]."""
    lib = _lib.load()
    dev = A.device
    ws = _ws(lib.spmv_transpose_workspace_size(A.n_rows, A.n_cols, A.nnz), dev)
    rowT = torch.empty(A.n_cols + 1, dtype=_I32, device=dev)
    colT = torch.empty(max(A.nnz, 1), dtype=_I32, device=dev)
    tmap = torch.empty(max(A.nnz, 1), dtype=_I32, device=dev)
    call("spmv_transpose_csr", A.n_rows, A.n_cols, A.nnz, _p(A.row_ptr), _p(A.col_idx), _p(rowT), _p(colT),
         _p(tmap), _p(ws), ws.numel(), _stream())
    return rowT, colT[:A.nnz], tmap[:A.nnz]


# --------------------------------------------------------------------------- compute


def _out_vec(y, n, x, beta, n_cols):
    """Checks x and y against the product's shape and returns y (a new vector
    if None).  The kernels read n_cols elements of x and write n elements of
    y in x's dtype with no device-side bounds checks, so a short or mistyped
    vector is refused here, before any launch."""
    if x.dtype not in _VEC_DTYPES:
        raise TypeError(f"x must be float64 or float32, got {x.dtype}")
    if x.numel() < n_cols:
        raise ValueError(f"x has {x.numel()} elements, the matrix has {n_cols} columns")
    if y is not None:
        if y.dtype != x.dtype:
            raise ValueError(f"y is {y.dtype} but x is {x.dtype}; both vectors take one dtype")
        if y.numel() < n:
            raise ValueError(f"y has {y.numel()} elements, the matrix has {n} rows")
    _check_dev(x)
    if y is None:
        if beta != 0.0:
            raise ValueError("beta != 0 needs y")
        return torch.empty(n, dtype=x.dtype, device=x.device)
    _check_dev(y)
    return y


def spmv_crs(A: CSR, x: torch.Tensor, y: Optional[torch.Tensor] = None, alpha: float = 1.0, beta: float = 0.0,
             use_plan: bool = True) -> torch.Tensor:
    """y = alpha*A x + beta*y with the CRS kernels (spmv_crs; spmv_crs_staged
    when A.staged is set and the plan is used)."""
    y = _out_vec(y, A.n_rows, x, beta, A.n_cols)
    if use_plan and A.plan is None:
        spmv_crs_plan(A)
    plan = A.plan if use_plan else None
    call("spmv_crs_staged" if (use_plan and A.staged) else "spmv_crs", A.n_rows, A.n_cols, _p(A.row_ptr), _p(A.col_idx), _p(A.val), dtype_code(A.val.dtype), _p(x),
         _p(y), dtype_code(x.dtype), float(alpha), float(beta), _p(plan), A.n_blocks if use_plan else 0,
         A.block_nnz if use_plan else 0, _stream())
    return y


def spmv_jds(J: JDS, x: torch.Tensor, y: Optional[torch.Tensor] = None, alpha: float = 1.0, beta: float = 0.0,
             unroll: int = 0, max_iters: int = 0, wg_waves: int = 0) -> torch.Tensor:
    """y = alpha*A x + beta*y with the JDS kernel (spmv_jds)."""
    y = _out_vec(y, J.n, x, beta, J.n_cols)
    call("spmv_jds", J.n, _p(J.perm), _p(J.jd_ptr), _h_i32(J.h_jd_ptr), J.ndiag, _p(J.jd_col), _p(J.jd_val),
         dtype_code(J.jd_val.dtype), _p(x), _p(y), dtype_code(x.dtype), float(alpha), float(beta), unroll, max_iters,
         wg_waves, J.flags, _stream())
    return y


def spmv_jds_tiles(J: JDS, max_iters: int = 0, rows_per_wave: int = 0, wg_waves: int = 0):
    """The XCD-local tile plan of J for spmv_jds_tiled (spmv_jds_tiles), built
    once per launch shape and kept on J: (tiles, n_tiles, h_plan)."""
    key = (max_iters, rows_per_wave, wg_waves)
    if key not in J.tile_plans:
        lib = _lib.load()
        nt = C.c_int64(0)
        h_plan = np.zeros(10, dtype=np.int64)
        args = lambda t, cap: (J.n, _h_i32(J.h_jd_ptr), J.ndiag, max_iters, rows_per_wave, wg_waves, t, cap,
                               C.byref(nt), _h_i64(h_plan), _stream())
        st = lib.spmv_jds_tiles(*args(None, 0))
        if st not in (0, 3):
            call("spmv_jds_tiles", *args(None, 0))
        tiles = torch.empty(max(2 * nt.value, 1), dtype=_I32, device=J.jd_ptr.device)
        call("spmv_jds_tiles", *args(_p(tiles), tiles.numel()))
        J.tile_plans[key] = (tiles, nt.value, h_plan)
    return J.tile_plans[key]


def spmv_jds_tiled(J: JDS, x: torch.Tensor, y: Optional[torch.Tensor] = None, alpha: float = 1.0, beta: float = 0.0,
                   unroll: int = 0, max_iters: int = 0, rows_per_wave: int = 0, wg_waves: int = 0) -> torch.Tensor:
    """y = alpha*A x + beta*y with the JDS kernel launched from J's XCD-local
    tile plan (spmv_jds_tiled)."""
    y = _out_vec(y, J.n, x, beta, J.n_cols)
    tiles, nt, h_plan = spmv_jds_tiles(J, max_iters, rows_per_wave, wg_waves)
    call("spmv_jds_tiled", J.n, _p(J.perm), _p(J.jd_ptr), J.ndiag, _p(J.jd_col), _p(J.jd_val),
         dtype_code(J.jd_val.dtype), _p(x), _p(y), dtype_code(x.dtype), float(alpha), float(beta), _p(tiles), nt,
         _h_i64(h_plan), unroll, J.flags, _stream())
    return y


def spmv_jds_blocked(B: Blocked, x: torch.Tensor, y: Optional[torch.Tensor] = None, alpha: float = 1.0,
                     beta: float = 0.0, rows_per_wave: int = 0, unroll: int = 0, max_iters: int = 0,
                     wg_waves: int = 0) -> torch.Tensor:
    """y = alpha*A x + beta*y with the blocked-JDS kernel (spmv_jds_blocked)."""
    y = _out_vec(y, B.n, x, beta, B.n_cols)
    flags = (SYMPERM if B.symperm else 0) | (SOJDS if B.sojds else 0)
    call("spmv_jds_blocked", B.n, _p(B.perm), B.C, B.n_slices, _p(B.slice_ptr), _p(B.slice_nd),
         _h_i32(B.h_slice_nd), _p(B.bl_col), _p(B.bl_val), dtype_code(B.bl_val.dtype), _p(x), _p(y),
         dtype_code(x.dtype), float(alpha), float(beta), rows_per_wave, unroll, max_iters, wg_waves, flags, _stream())
    return y


def colmajor(n: int, k: int, dtype, device) -> torch.Tensor:
    """An n x k column-major block (a transposed view of a (k, n) tensor)."""
    return torch.empty(k, n, dtype=dtype, device=device).t()


def _ld(X: torch.Tensor, n: int) -> int:
    if X.dim() != 2 or X.stride(0) != 1 or X.shape[0] != n:
        raise ValueError("multi-vector blocks must be column-major (n, k) with unit row stride")
    return X.stride(1) if X.shape[1] > 1 else n


def _check_blocks(X: torch.Tensor, Y: Optional[torch.Tensor], n_rows: int, n_cols: int) -> None:
    """X must be (n_cols, k) and Y (n_rows, k), column-major, one vector dtype:
    the kernels trust these shapes, so a mismatch is refused before launch."""
    if X.dtype not in _VEC_DTYPES:
        raise TypeError(f"X must be float64 or float32, got {X.dtype}")
    if X.dim() != 2 or X.shape[0] != n_cols:
        raise ValueError(f"X must be ({n_cols}, k), got {tuple(X.shape)}")
    if Y is not None:
        if Y.dtype != X.dtype:
            raise ValueError(f"Y is {Y.dtype} but X is {X.dtype}; both blocks take one dtype")
        if Y.dim() != 2 or tuple(Y.shape) != (n_rows, X.shape[1]):
            raise ValueError(f"Y must be ({n_rows}, {X.shape[1]}), got {tuple(Y.shape)}")
    _ld(X, n_cols)
    if Y is not None:
        _ld(Y, n_rows)
    for t in (X, Y):
        if t is not None and not t.is_cuda:
            raise ValueError("tensors must live on the GPU")


def spmm_workspace(n_cols: int, k: int, dtype, device) -> torch.Tensor:
    """Workspace for the interleaved multi-vector path (a row-major copy of X)."""
    return _ws(_lib.load().spmm_workspace_size(n_cols, k, dtype_code(dtype)), device)


def spmm_crs(A: CSR, X: torch.Tensor, Y: Optional[torch.Tensor] = None, alpha: float = 1.0, beta: float = 0.0,
             ws: Optional[torch.Tensor] = None, interleave: bool = True) -> torch.Tensor:
    """Y = alpha*A X + beta*Y for a column-major block X (spmm_crs)."""
    _check_blocks(X, Y, A.n_rows, A.n_cols)
    if A.plan is None:
        spmv_crs_plan(A)
    k = X.shape[1]
    if Y is None:
        Y = colmajor(A.n_rows, k, X.dtype, X.device)
    if interleave and ws is None:
        ws = spmm_workspace(A.n_cols, k, X.dtype, X.device)
    call("spmm_crs", A.n_rows, A.n_cols, _p(A.row_ptr), _p(A.col_idx), _p(A.val), dtype_code(A.val.dtype), k, _p(X),
         _ld(X, A.n_cols), _p(Y), _ld(Y, A.n_rows), dtype_code(X.dtype), float(alpha), float(beta), _p(A.plan),
         A.n_blocks, A.block_nnz, _p(ws) if interleave else None, ws.numel() if (interleave and ws is not None) else 0,
         _stream())
    return Y


def spmm_jds(J: JDS, X: torch.Tensor, Y: Optional[torch.Tensor] = None, alpha: float = 1.0, beta: float = 0.0,
             ws: Optional[torch.Tensor] = None, interleave: bool = True) -> torch.Tensor:
    """Y = alpha*A X + beta*Y for a column-major block X (spmm_jds)."""
    _check_blocks(X, Y, J.n, J.n_cols)
    k = X.shape[1]
    if Y is None:
        Y = colmajor(J.n, k, X.dtype, X.device)
    if interleave and ws is None:
        ws = spmm_workspace(J.n_cols, k, X.dtype, X.device)
    call("spmm_jds", J.n, J.n_cols, _p(J.perm), _p(J.jd_ptr), _h_i32(J.h_jd_ptr), J.ndiag, _p(J.jd_col),
         _p(J.jd_val), dtype_code(J.jd_val.dtype), k, _p(X), _ld(X, J.n_cols), _p(Y), _ld(Y, J.n), dtype_code(X.dtype),
         float(alpha), float(beta), J.flags, _p(ws) if interleave else None,
         ws.numel() if (interleave and ws is not None) else 0, _stream())
    return Y


def spmm_jds_blocked_plan(B: Blocked, k: int, max_groups: int = 0,
                          xcd_ranges: Optional[bool] = None) -> Tuple[torch.Tensor, int]:
    """Plan of spmm_jds_blocked for k vectors and its grid size (cached on B
    per k rounded up to a power of two and the two launch choices).
    Defaults, measured on the power-law matrix at k = 8 and 32: the windowed
    order takes up to 4 lane groups per row and XCD ranges of equal work
    (its rows stay together); the global order one group per row, records
    dealt to the XCDs in turn (its deep slices spread over all of them)."""
    K2 = 1
    while K2 < k and K2 < 64:
        K2 *= 2
    if xcd_ranges is None:
        xcd_ranges = B.sigma > 0
    if max_groups == 0:
        max_groups = 4 if B.sigma > 0 else 1
    key = ("spmm", K2, max_groups, bool(xcd_ranges))
    if key not in B.tile_plans:
        words, grid = C.c_int32(0), C.c_int32(0)
        args = lambda pl, cap: (B.n, B.C, B.n_slices, _h_i32(B.h_slice_nd), K2, max_groups, int(bool(xcd_ranges)),
                                pl, cap, C.byref(words), C.byref(grid), _stream())
        st = _lib.load().spmm_jds_blocked_plan(*args(None, 0))
        if st not in (0, 3):
            call("spmm_jds_blocked_plan", *args(None, 0))
        plan = torch.empty(max(words.value, 1), dtype=_I32, device=B.perm.device)
        call("spmm_jds_blocked_plan", *args(_p(plan), plan.numel()))
        B.tile_plans[key] = (plan, grid.value)
    return B.tile_plans[key]


def spmm_jds_blocked(B: Blocked, X: torch.Tensor, Y: Optional[torch.Tensor] = None, alpha: float = 1.0,
                     beta: float = 0.0, ws: Optional[torch.Tensor] = None, max_groups: int = 0,
                     xcd_ranges: Optional[bool] = None) -> torch.Tensor:
    """Y = alpha*A X + beta*Y over blocked-JDS storage, global or windowed
    order (spmm_jds_blocked; X staged row-major in ws, 1 <= k <= 64)."""
    if B.symperm:
        raise ValueError("spmm_jds_blocked: symmetric-permutation storage is not supported")
    _check_blocks(X, Y, B.n, B.n_cols)
    k = X.shape[1]
    if not 1 <= k <= 64:
        raise ValueError("spmm_jds_blocked: k must be in [1, 64]")
    if Y is None:
        Y = colmajor(B.n, k, X.dtype, X.device)
    if ws is None:
        ws = spmm_workspace(B.n_cols, k, X.dtype, X.device)
    plan, grid = spmm_jds_blocked_plan(B, k, max_groups, xcd_ranges)
    call("spmm_jds_blocked", B.n, B.n_cols, _p(B.perm), B.C, B.n_slices, _p(B.slice_ptr), _p(B.slice_nd),
         _p(B.bl_col), _p(B.bl_val), dtype_code(B.bl_val.dtype), k, _p(X), _ld(X, B.n_cols), _p(Y), _ld(Y, B.n),
         dtype_code(X.dtype), float(alpha), float(beta), _p(plan), grid, _p(ws), ws.numel(), _stream())
    return Y


def spmv_permute_vec(perm: torch.Tensor, v: torch.Tensor, inverse: bool = False) -> torch.Tensor:
    out = torch.empty_like(v)
    call("spmv_permute_vec", v.numel(), _p(perm), _p(v), _p(out), dtype_code(v.dtype), int(inverse), _stream())
    return out


def spmv_gather_values(map_: torch.Tensor, v: torch.Tensor) -> torch.Tensor:
    """out[i] = v[map_[i]]; every element moves bit for bit (int32 included)."""
    out = torch.empty(map_.numel(), dtype=v.dtype, device=v.device)
    call("spmv_gather_values", map_.numel(), _p(map_), _p(v), _p(out), dtype_code(v.dtype), _stream())
    return out


def spmv_axpby(alpha: float, x: torch.Tensor, beta: float, y: torch.Tensor) -> torch.Tensor:
    """y = alpha*x + beta*y in place (beta == 0 never reads y)."""
    call("spmv_axpby", x.numel(), float(alpha), _p(x), float(beta), _p(y), dtype_code(x.dtype), _stream())
    return y


def spmv_dot(x: torch.Tensor, y: torch.Tensor, out: Optional[torch.Tensor] = None) -> torch.Tensor:
    """sum_i x_i y_i in FP64 with a fixed summation tree; a 1-element device tensor."""
    if out is None:
        out = torch.empty(1, dtype=torch.float64, device=x.device)
    ws = _ws(_lib.load().spmv_dot_workspace_size(x.numel()), x.device)
    call("spmv_dot", x.numel(), _p(x), _p(y), dtype_code(x.dtype), _p(out), _p(ws), ws.numel(), _stream())
    return out


def spmv_dot_noalloc(x: torch.Tensor, y: torch.Tensor, out: torch.Tensor) -> torch.Tensor:
    """sum_i x_i y_i into the 1-element FP64 device tensor `out`, with the
    library's own scratch array instead of a workspace (no allocation here or
    in the library; bit-identical to spmv_dot)."""
    _check_dev(x, y, out)
    if x.dtype not in _VEC_DTYPES or y.dtype != x.dtype or y.numel() != x.numel():
        raise ValueError("x and y must be float64 or float32 vectors of one dtype and length")
    if out.dtype != torch.float64 or out.numel() < 1:
        raise ValueError("out must be a float64 device tensor")
    call("spmv_dot_noalloc", x.numel(), _p(x), _p(y), dtype_code(x.dtype), _p(out), _stream())
    return out


def spmv_grad_vals_jds(J: JDS, g: torch.Tensor, x: torch.Tensor, out: Optional[torch.Tensor] = None,
                       alpha: float = 1.0, beta: float = 0.0) -> torch.Tensor:
    """dval[e] = alpha*g[row_e]*x[col_e] + beta*dval[e] over the JDS entries."""
    if out is None:
        if beta != 0.0:
            raise ValueError("beta != 0 needs out")
        out = torch.empty(J.nnz, dtype=g.dtype, device=g.device)
    call("spmv_grad_vals_jds", J.n, _p(J.perm), _p(J.jd_ptr), _h_i32(J.h_jd_ptr), J.ndiag, J.nnz, _p(J.jd_col),
         _p(g), _p(x), _p(out), dtype_code(g.dtype), float(alpha), float(beta), J.flags, _stream())
    return out


def spmv_stream_triad(a, b, c, s: float):
    call("spmv_stream_triad", a.numel(), _p(b), _p(c), _p(a), float(s), _stream())


def spmv_stream_copy(a, b):
    call("spmv_stream_copy", a.numel(), _p(b), _p(a), _stream())


def spmv_stream_read(b, part):
    call("spmv_stream_read", b.numel(), _p(b), _p(part), part.numel(), _stream())


def spmv_stride_probe(n, b, part, a=None, ind=None, k=1, ind_max=None):
    """s += b[j(i)] or s += a[i]*b[j(i)] for i < n, j(i) = k*i or ind[i]
    (spmv_stride_probe); with `ind`, `ind_max` is its largest entry (known to
    the caller that built it)."""
    if ind is not None and ind_max is None:
        raise ValueError("ind needs ind_max")
    need = ind_max + 1 if ind is not None else k * (n - 1) + 1
    if n > 0 and b.numel() < need:
        raise ValueError("b is too short for the index stream")
    if a is not None and a.numel() < n:
        raise ValueError("a is shorter than n")
    call("spmv_stride_probe", n, 1 if a is not None else 0, _p(a), _p(b), _p(ind), k, _p(part), part.numel(),
         _stream())


def spmv_gather_probe(idx, x, part):
    call("spmv_gather_probe", idx.numel(), _p(idx), _p(x), _p(part), part.numel(), _stream())


# --------------------------------------------------------------------------- column-split forms


def _ptr_array(ts):
    return (C.c_void_p * len(ts))(*[t.data_ptr() if t is not None and t.data_ptr() else None for t in ts])


class Split:
    """A matrix cut into SPLIT_PARTS column blocks (spmv_split_columns); part k
    is an ordinary CRS matrix over the rows that hold one of its entries, and
    gets JDS / blocked-JDS forms on demand."""

    def __init__(self, A: CSR, width: int = 0, block_nnz: int = 0):
        lib = _lib.load()
        P = _lib.SPLIT_PARTS
        dev = A.device
        self.n, self.n_cols = A.n_rows, A.n_cols
        nnz = A.nnz
        cap = min(nnz, P * A.n_rows)
        ws = _ws(lib.spmv_split_columns_workspace_size(A.n_rows, nnz), dev)
        self.row_ptr_all = torch.empty(cap + P, dtype=_I32, device=dev)
        self.dest_all = torch.empty(max(cap, 1), dtype=_I32, device=dev)
        self.slot_ptr = torch.empty(A.n_rows + 1, dtype=_I32, device=dev)
        self.col = torch.empty(max(nnz, 1), dtype=_I32, device=dev)
        self.val = torch.empty(max(nnz, 1), dtype=A.val.dtype, device=dev)
        self.bounds = np.zeros(P + 1, dtype=np.int64)
        self.row_off = np.zeros(P + 1, dtype=np.int64)
        call("spmv_split_columns", A.n_rows, A.n_cols, nnz, _p(A.row_ptr), _p(A.col_idx), _p(A.val),
             dtype_code(A.val.dtype), width, _p(self.row_ptr_all), _p(self.dest_all), _p(self.slot_ptr), _p(self.col),
             _p(self.val), _h_i64(self.bounds), _h_i64(self.row_off), _p(ws), ws.numel(), _stream())
        self.n_slots = int(self.row_off[P])
        self.ws = _ws(lib.spmv_split_workspace_size(self.n_slots), dev)
        self.parts = [self.part_csr(k) for k in range(P)]
        # CRS plans of the parts, one after the other
        plans, self.plan_off, self.n_blocks = [], np.zeros(P, np.int32), np.zeros(P, np.int32)
        off = 0
        for k, Ak in enumerate(self.parts):
            spmv_crs_plan(Ak, block_nnz)
            plans.append(Ak.plan[:Ak.n_blocks + 1])
            self.plan_off[k], self.n_blocks[k] = off, Ak.n_blocks
            off += Ak.n_blocks + 1
        self.plan_all = torch.cat(plans)
        self.block_nnz = block_nnz
        self.jds = None
        self.blocked = {}

    def part_rows(self, k: int) -> int:
        return int(self.row_off[k + 1] - self.row_off[k])

    def part_dest(self, k: int) -> torch.Tensor:
        """Slot of each compressed row of part k."""
        return self.dest_all[int(self.row_off[k]):int(self.row_off[k + 1])]

    def part_csr(self, k: int) -> CSR:
        nk, r0 = self.part_rows(k), int(self.row_off[k])
        a, b = int(self.bounds[k]), int(self.bounds[k + 1])
        return CSR(nk, self.n_cols, self.row_ptr_all[r0 + k:r0 + k + nk + 1], self.col[a:b], self.val[a:b])

    def with_values(self, val: torch.Tensor) -> "Split":
        """Same structure, values (part-major order) of another dtype."""
        S = Split.__new__(Split)
        S.__dict__.update(self.__dict__)
        S.val = val
        S.parts = [S.part_csr(k) for k in range(_lib.SPLIT_PARTS)]
        for Ak, A0 in zip(S.parts, self.parts):
            Ak.plan, Ak.n_blocks, Ak.block_nnz = A0.plan, A0.n_blocks, A0.block_nnz
        S.jds = None
        S.blocked = {}
        S._jds_args = None
        S._blocked_args = {}
        return S

    def jds_parts(self):
        """JDS of every part, its perm mapped to slots (rows of the part go
        straight to their slots)."""
        if self.jds is None:
            self.jds = []
            for k, Ak in enumerate(self.parts):
                J = jds_from_csr(Ak)
                if J.n > 0:
                    J.perm = spmv_gather_values(J.perm[:J.n], self.part_dest(k))
                self.jds.append(J)
        return self.jds

    def blocked_parts(self, C_: int = 64):
        if C_ not in self.blocked:
            self.blocked[C_] = [jds_blocked_from_jds(J, C_) for J in self.jds_parts()]
        return self.blocked[C_]


def spmv_crs_split(S: Split, x, y=None, alpha=1.0, beta=0.0):
    y = _out_vec(y, S.n, x, beta, S.n_cols)
    call("spmv_crs_split", S.n, S.n_cols, _p(S.row_ptr_all), _p(S.dest_all), _p(S.slot_ptr), _p(S.col), _p(S.val),
         _h_i64(S.bounds), _h_i64(S.row_off), dtype_code(S.val.dtype), _p(S.plan_all), _h_i32(S.plan_off),
         _h_i32(S.n_blocks), S.block_nnz, _p(x), _p(y), dtype_code(x.dtype), float(alpha), float(beta), _p(S.ws),
         S.ws.numel(), _stream())
    return y


def _jds_split_args(S: Split):
    """ctypes arrays describing the JDS parts, built once per Split."""
    if getattr(S, "_jds_args", None) is None:
        Js = S.jds_parts()
        hptr = (C.c_void_p * len(Js))(*[J.h_jd_ptr.ctypes.data for J in Js])
        ndiag = np.array([J.ndiag for J in Js], dtype=np.int32)
        S._jds_args = (Js, _ptr_array([J.perm for J in Js]), _ptr_array([J.jd_ptr for J in Js]), hptr, ndiag,
                       _ptr_array([J.jd_col for J in Js]), _ptr_array([J.jd_val for J in Js]))
    return S._jds_args


def spmv_jds_split(S: Split, x, y=None, alpha=1.0, beta=0.0, unroll=0, max_iters=0, wg_waves=0):
    y = _out_vec(y, S.n, x, beta, S.n_cols)
    Js, perm, jp, hptr, ndiag, col, val = _jds_split_args(S)
    call("spmv_jds_split", S.n, _p(S.slot_ptr), _h_i64(S.row_off), perm, jp, hptr, _h_i32(ndiag), col, val,
         dtype_code(Js[0].jd_val.dtype), _p(x), _p(y), dtype_code(x.dtype), float(alpha), float(beta), unroll,
         max_iters, wg_waves, _p(S.ws), S.ws.numel(), _stream())
    return y


def _blocked_split_args(S: Split, C_: int):
    cache = S.__dict__.setdefault("_blocked_args", {})
    if C_ not in cache:
        Bs = S.blocked_parts(C_)
        hnd = (C.c_void_p * len(Bs))(*[B.h_slice_nd.ctypes.data for B in Bs])
        cache[C_] = (Bs, _ptr_array([B.perm for B in Bs]), _ptr_array([B.slice_ptr for B in Bs]),
                     _ptr_array([B.slice_nd for B in Bs]), hnd, _ptr_array([B.bl_col for B in Bs]),
                     _ptr_array([B.bl_val for B in Bs]))
    return cache[C_]


def spmv_jds_blocked_split(S: Split, x, y=None, alpha=1.0, beta=0.0, C_=64, rows_per_wave=0, unroll=0,
                           max_iters=0, wg_waves=0):
    y = _out_vec(y, S.n, x, beta, S.n_cols)
    Bs, perm, sptr, snd, hnd, col, val = _blocked_split_args(S, C_)
    call("spmv_jds_blocked_split", S.n, C_, _p(S.slot_ptr), _h_i64(S.row_off), perm, sptr, snd, hnd, col, val,
         dtype_code(Bs[0].bl_val.dtype), _p(x), _p(y), dtype_code(x.dtype), float(alpha), float(beta), rows_per_wave,
         unroll, max_iters, wg_waves, _p(S.ws), S.ws.numel(), _stream())
    return y


# --------------------------------------------------------------------------- row-split forms


class RowSplit:
    """A matrix cut into SPLIT_PARTS contiguous row blocks of about nnz/8
    entries each (spmv_split_rows); part k is an ordinary CRS matrix (views of
    the original column and value arrays) and gets JDS / blocked-JDS forms on
    demand, with permutations local to the part."""

    def __init__(self, A: CSR):
        lib = _lib.load()
        P = _lib.SPLIT_PARTS
        dev = A.device
        self.n, self.n_cols = A.n_rows, A.n_cols
        ws = _ws(lib.spmv_split_rows_workspace_size(), dev)
        self.row_ptr_parts = torch.empty(A.n_rows + P, dtype=_I32, device=dev)
        self.bounds = np.zeros(P + 1, dtype=np.int64)
        self.entry_bounds = np.zeros(P + 1, dtype=np.int64)
        call("spmv_split_rows", A.n_rows, A.nnz, _p(A.row_ptr), _p(self.row_ptr_parts), _h_i64(self.bounds),
             _h_i64(self.entry_bounds), _p(ws), ws.numel(), _stream())
        self.A = A
        self.parts = [self.part_csr(k) for k in range(P)]
        self.jds = None
        self.blocked = {}

    def part_rows(self, k: int) -> int:
        return int(self.bounds[k + 1] - self.bounds[k])

    def part_csr(self, k: int) -> CSR:
        nk, r0 = self.part_rows(k), int(self.bounds[k])
        a, b = int(self.entry_bounds[k]), int(self.entry_bounds[k + 1])
        return CSR(nk, self.n_cols, self.row_ptr_parts[r0 + k:r0 + k + nk + 1], self.A.col_idx[a:b],
                   self.A.val[a:b])

    def jds_parts(self):
        if self.jds is None:
            self.jds = [jds_from_csr(Ak) for Ak in self.parts]
        return self.jds

    def blocked_parts(self, C_: int = 64):
        if C_ not in self.blocked:
            self.blocked[C_] = [jds_blocked_from_jds(J, C_) for J in self.jds_parts()]
        return self.blocked[C_]

    def with_values(self, dtype: torch.dtype) -> "RowSplit":
        """Same structure with the values rounded (or widened) to ``dtype``."""
        R = RowSplit.__new__(RowSplit)
        R.__dict__.update(self.__dict__)
        R.A = self.A.with_values(spmv_convert_values(self.A.val, dtype))
        R.parts = [R.part_csr(k) for k in range(_lib.SPLIT_PARTS)]
        R.jds = [J.with_values(spmv_convert_values(J.jd_val, dtype)) for J in self.jds_parts()]
        R.blocked = {C_: [B.with_values(spmv_convert_values(B.bl_val, dtype)) for B in Bs]
                     for C_, Bs in self.blocked.items()}
        R._jds_args = None
        R._blocked_args = {}
        return R


def _jds_row_split_args(R: RowSplit):
    if getattr(R, "_jds_args", None) is None:
        Js = R.jds_parts()
        hptr = (C.c_void_p * len(Js))(*[J.h_jd_ptr.ctypes.data for J in Js])
        ndiag = np.array([J.ndiag for J in Js], dtype=np.int32)
        R._jds_args = (Js, _ptr_array([J.perm for J in Js]), _ptr_array([J.jd_ptr for J in Js]), hptr, ndiag,
                       _ptr_array([J.jd_col for J in Js]), _ptr_array([J.jd_val for J in Js]))
    return R._jds_args


def spmv_jds_row_split(R: RowSplit, x, y=None, alpha=1.0, beta=0.0, unroll=0, max_iters=0, wg_waves=0):
    y = _out_vec(y, R.n, x, beta, R.n_cols)
    Js, perm, jp, hptr, ndiag, col, val = _jds_row_split_args(R)
    call("spmv_jds_row_split", R.n, _h_i64(R.bounds), perm, jp, hptr, _h_i32(ndiag), col, val,
         dtype_code(Js[0].jd_val.dtype), _p(x), _p(y), dtype_code(x.dtype), float(alpha), float(beta), unroll,
         max_iters, wg_waves, _stream())
    return y


def _blocked_row_split_args(R: RowSplit, C_: int):
    cache = R.__dict__.setdefault("_blocked_args", {})
    if C_ not in cache:
        Bs = R.blocked_parts(C_)
        hnd = (C.c_void_p * len(Bs))(*[B.h_slice_nd.ctypes.data for B in Bs])
        cache[C_] = (Bs, _ptr_array([B.perm for B in Bs]), _ptr_array([B.slice_ptr for B in Bs]),
                     _ptr_array([B.slice_nd for B in Bs]), hnd, _ptr_array([B.bl_col for B in Bs]),
                     _ptr_array([B.bl_val for B in Bs]))
    return cache[C_]


def spmv_jds_blocked_row_split(R: RowSplit, x, y=None, alpha=1.0, beta=0.0, C_=64, rows_per_wave=0, unroll=0,
                               max_iters=0, wg_waves=0):
    y = _out_vec(y, R.n, x, beta, R.n_cols)
    Bs, perm, sptr, snd, hnd, col, val = _blocked_row_split_args(R, C_)
    call("spmv_jds_blocked_row_split", R.n, C_, _h_i64(R.bounds), perm, sptr, snd, hnd, col, val,
         dtype_code(Bs[0].bl_val.dtype), _p(x), _p(y), dtype_code(x.dtype), float(alpha), float(beta), rows_per_wave,
         unroll, max_iters, wg_waves, _stream())
    return y


# --------------------------------------------------------------------------- DIA + CRS hybrid


@dataclass
class SymCSR:
    """A symmetric n x n matrix stored as its upper triangle U (entries with
    col >= row, CRS order): A = U + U^T - diag(U)."""
    upper: CSR

    @property
    def n(self) -> int:
        return self.upper.n_rows

    @property
    def nnz(self) -> int:
        """Stored entries (those of U)."""
        return self.upper.nnz

    @property
    def device(self):
        return self.upper.device

    def with_values(self, val: torch.Tensor) -> "SymCSR":
        return SymCSR(self.upper.with_values(val))


def csr_upper_from_csr(A: CSR) -> SymCSR:
    """Full CRS of a symmetric matrix -> its upper triangle on the GPU
    (spmv_csr_upper_from_csr; entries below the diagonal are not read)."""
    if A.n_rows != A.n_cols:
        raise ValueError("one-triangle storage needs a square matrix")
    lib = _lib.load()
    dev = A.device
    n = A.n_rows
    ws = _ws(lib.spmv_csr_upper_workspace_size(n), dev)
    m = C.c_int64(0)
    args = lambda rp, uc, uv: (n, A.nnz, _p(A.row_ptr), _p(A.col_idx), _p(A.val), dtype_code(A.val.dtype),
                               C.byref(m), rp, uc, uv, _p(ws), ws.numel(), _stream())
    call("spmv_csr_upper_from_csr", *args(None, None, None))
    k = m.value
    rp = torch.empty(n + 1, dtype=_I32, device=dev)
    col = torch.empty(max(k, 1), dtype=_I32, device=dev)
    val = torch.empty(max(k, 1), dtype=A.val.dtype, device=dev)
    call("spmv_csr_upper_from_csr", *args(_p(rp), _p(col), _p(val)))
    return SymCSR(CSR(n, n, rp, col[:k], val[:k]))


def spmv_crs_sym(S: SymCSR, x: torch.Tensor, y: Optional[torch.Tensor] = None, alpha: float = 1.0,
                 beta: float = 0.0) -> torch.Tensor:
    """y = alpha*A x + beta*y from the upper triangle (spmv_crs_sym, or
    spmv_crs_sym_staged when S.upper.staged is set; FP64 x and y; the
    mirrored terms are added with atomics, so y may differ in the last bits
    between runs)."""
    U = S.upper
    if x.dtype != torch.float64:
        raise TypeError("spmv_crs_sym: x must be float64")
    y = _out_vec(y, U.n_rows, x, beta, U.n_cols)
    if U.plan is None:
        spmv_crs_plan(U)
    call("spmv_crs_sym_staged" if U.staged else "spmv_crs_sym", U.n_rows, _p(U.row_ptr), _p(U.col_idx), _p(U.val),
         dtype_code(U.val.dtype), _p(x), _p(y), dtype_code(x.dtype), float(alpha), float(beta), _p(U.plan), U.n_blocks, U.block_nnz, _stream())
    return y


REM_WINDOW, REM_SLICE = 256, 16


@dataclass
class Slices:
    """A CRS matrix in window-sorted slices (spmv_csr_to_slices): rows sorted
    by decreasing length inside windows of 256, slices of 16 positions."""
    n_rows: int
    slice_ptr: torch.Tensor      # int64, n_slices + 1
    slice_nd: torch.Tensor       # int32, the slice's first (longest) row's length
    slot_row: torch.Tensor       # uint8, window-local row at each sorted position
    bl_col: torch.Tensor         # padded slots, col = -1 in padding
    bl_val: torch.Tensor

    def with_values(self, val: torch.Tensor) -> "Slices":
        return Slices(self.n_rows, self.slice_ptr, self.slice_nd, self.slot_row, self.bl_col, val)


def csr_to_slices(A: CSR) -> Slices:
    """CRS -> window-sorted slices on the GPU (spmv_csr_to_slices)."""
    lib = _lib.load()
    dev = A.device
    n = A.n_rows
    ns = (n + REM_SLICE - 1) // REM_SLICE
    ws = _ws(lib.spmv_csr_slices_workspace_size(n), dev)
    sp_ = torch.empty(ns + 1, dtype=torch.int64, device=dev)
    nd = torch.empty(max(ns, 1), dtype=_I32, device=dev)
    rows = torch.empty(max(n, 1), dtype=torch.uint8, device=dev)
    padded = C.c_int64(0)
    args = lambda col, val, cap: (n, _p(A.row_ptr), _p(A.col_idx), _p(A.val), dtype_code(A.val.dtype), _p(sp_),
                                  _p(nd), _p(rows), col, val, cap, C.byref(padded), _p(ws), ws.numel(), _stream())
    call("spmv_csr_to_slices", *args(None, None, 0))
    m = padded.value
    col = torch.empty(max(m, 1), dtype=_I32, device=dev)
    val = torch.empty(max(m, 1), dtype=A.val.dtype, device=dev)
    call("spmv_csr_to_slices", *args(_p(col), _p(val), max(m, 1)))
    return Slices(n, sp_, nd[:ns], rows[:n], col[:m], val[:m])


@dataclass
class DIA:
    """Densely stored diagonals (offset col - row) plus a remainder, in CRS or
    (rem_slices) in window-sorted slices."""
    n_rows: int
    n_cols: int
    offsets: np.ndarray          # int32, ascending, host
    dia_val: torch.Tensor        # ndia * n_rows values, diagonal after diagonal
    rem: CSR                     # the entries on no stored diagonal
    symmetric: bool = False      # offsets >= 0, each diagonal also serves its mirror
    rem_slices: Optional[Slices] = None

    @property
    def ndia(self) -> int:
        return len(self.offsets)

    def with_values(self, dia_val: torch.Tensor, rem_val: Optional[torch.Tensor] = None) -> "DIA":
        """Same structure, other values (rem_val: the remainder CRS's values;
        the sliced copy, if any, is rebuilt from them)."""
        rem = self.rem if rem_val is None else self.rem.with_values(rem_val)
        D = DIA(self.n_rows, self.n_cols, self.offsets, dia_val, rem, self.symmetric, self.rem_slices)
        if self.rem_slices is not None and rem_val is not None and rem.nnz:
            D.rem_slices = csr_to_slices(rem)
        return D


def dia_from_csr(A: CSR, max_diags: int = 0, symmetric: bool = False, sliced: bool = False) -> DIA:
    """CRS -> DIA + CRS hybrid on the GPU (spmv_dia_from_csr; with
    symmetric=True, spmv_dia_sym_from_csr: upper diagonals only, each also
    standing for its mirror, for a square matrix symmetric on them).  With
    sliced=True the remainder is also laid out in window-sorted slices
    (spmv_csr_to_slices) and spmv_dia uses them."""
    lib = _lib.load()
    dev = A.device
    if symmetric and A.n_rows != A.n_cols:
        raise ValueError("symmetric storage needs a square matrix")
    ws = _ws(lib.spmv_dia_workspace_size(A.n_rows, A.n_cols), dev)
    offs = np.zeros(_lib.DIA_MAX, dtype=np.int32)
    nd = C.c_int32(0)
    rem_nnz = C.c_int64(0)
    shape = (A.n_rows,) if symmetric else (A.n_rows, A.n_cols)
    fn = "spmv_dia_sym_from_csr" if symmetric else "spmv_dia_from_csr"
    args = lambda dv, rp, rc, rv: (*shape, A.nnz, _p(A.row_ptr), _p(A.col_idx), _p(A.val),
                                   dtype_code(A.val.dtype), max_diags, _h_i32(offs), C.byref(nd), C.byref(rem_nnz),
                                   dv, rp, rc, rv, _p(ws), ws.numel(), _stream())
    call(fn, *args(None, None, None, None))
    k, m = nd.value, rem_nnz.value
    dia_val = torch.empty(max(k * A.n_rows, 1), dtype=A.val.dtype, device=dev)
    rem_rp = torch.empty(A.n_rows + 1, dtype=_I32, device=dev)
    rem_col = torch.empty(max(m, 1), dtype=_I32, device=dev)
    rem_val = torch.empty(max(m, 1), dtype=A.val.dtype, device=dev)
    call(fn, *args(_p(dia_val), _p(rem_rp), _p(rem_col), _p(rem_val)))
    D = DIA(A.n_rows, A.n_cols, offs[:k].copy(), dia_val[:k * A.n_rows],
            CSR(A.n_rows, A.n_cols, rem_rp, rem_col[:m], rem_val[:m]), symmetric)
    if sliced:
        D.rem_slices = csr_to_slices(D.rem)
    return D


def spmv_dia(D: DIA, x: torch.Tensor, y: Optional[torch.Tensor] = None, alpha: float = 1.0,
             beta: float = 0.0) -> torch.Tensor:
    """y = alpha*A x + beta*y over the DIA + CRS hybrid (spmv_dia)."""
    y = _out_vec(y, D.n_rows, x, beta, D.n_cols)
    has_rem = D.rem.nnz > 0
    if D.rem_slices is not None:
        R = D.rem_slices
        call("spmv_dia_sliced", D.n_rows, D.n_cols, D.ndia, _h_i32(D.offsets), _p(D.dia_val),
             dtype_code(D.dia_val.dtype), *((_p(R.slice_ptr), _p(R.slice_nd), _p(R.slot_row), _p(R.bl_col),
                                             _p(R.bl_val)) if has_rem else (None,) * 5),
             _p(x), _p(y), dtype_code(x.dtype), float(alpha), float(beta), int(D.symmetric), _stream())
        return y
    shape = (D.n_rows,) if D.symmetric else (D.n_rows, D.n_cols)
    call("spmv_dia_sym" if D.symmetric else "spmv_dia", *shape, D.ndia, _h_i32(D.offsets), _p(D.dia_val),
         dtype_code(D.dia_val.dtype), _p(D.rem.row_ptr) if has_rem else None,
         _p(D.rem.col_idx) if has_rem else None, _p(D.rem.val) if has_rem else None, _p(x), _p(y),
         dtype_code(x.dtype), float(alpha), float(beta), _stream())
    return y


# --------------------------------------------------------------------------- many matrices


class Batched:
    """Many blocked-JDS matrices (float32) run by one persistent launch (spmv_batched).

    ``mats`` is a list of Blocked matrices (float32 values).  Their arrays are
    concatenated once; x and y of all matrices are concatenated in order.
    """

    def __init__(self, mats, rows_per_wave: int = 64, unroll: int = 0, n_workgroups: int = 0):
        if not mats:
            raise ValueError("no matrices")
        dev = mats[0].bl_val.device
        for B in mats:
            if B.bl_val.dtype != torch.float32:
                raise TypeError("batched form takes float32 values")
        self.n_mat = len(mats)
        self.n_rows = np.array([B.n for B in mats], dtype=np.int32)
        self.n_cols = np.array([B.n_cols for B in mats], dtype=np.int64)
        self.C = np.array([B.C for B in mats], dtype=np.int32)
        self.row_base = np.concatenate([[0], np.cumsum(self.n_rows.astype(np.int64))[:-1]]).astype(np.int64)
        self.col_base = np.concatenate([[0], np.cumsum(self.n_cols)[:-1]]).astype(np.int64)
        self.total_rows = int(self.n_rows.astype(np.int64).sum())
        self.total_cols = int(self.n_cols.sum())
        ns = np.array([B.n_slices for B in mats], dtype=np.int64)
        self.slice_base = np.concatenate([[0], np.cumsum(ns)[:-1]]).astype(np.int64)
        el_base = np.concatenate([[0], np.cumsum([B.padded for B in mats])[:-1]]).astype(np.int64)
        # absolute slice offsets on the host, from each matrix's device slice_ptr
        self.h_slice_ptr = np.concatenate(
            [B.slice_ptr[:-1].cpu().numpy() + el_base[m] for m, B in enumerate(mats)]).astype(np.int64)
        self.h_slice_nd = np.concatenate([B.h_slice_nd for B in mats]).astype(np.int32)
        self.bl_col = torch.cat([B.bl_col for B in mats])
        self.bl_val = torch.cat([B.bl_val for B in mats])
        self.perm = torch.cat([B.perm for B in mats])
        self.rows_per_wave, self.unroll, self.n_workgroups = rows_per_wave, unroll, n_workgroups
        self.mats_C = int(self.C[0]) if bool((self.C == self.C[0]).all()) else None
        self.nnz_padded = int(self.bl_val.numel())
        self._plan(dev)

    def _plan(self, dev):
        lib = _lib.load()
        nt = C.c_int64(0)
        args = lambda p, cap: (self.n_mat, _h_i32(self.n_rows), _h_i32(self.C), _h_i64(self.slice_base),
                               _h_i64(self.row_base), _h_i64(self.col_base), _h_i64(self.h_slice_ptr),
                               _h_i32(self.h_slice_nd), self.rows_per_wave, p, cap, C.byref(nt), _stream())
        st = lib.spmv_batched_plan(*args(None, 0))
        if st not in (0, 3):
            call("spmv_batched_plan", *args(None, 0))
        self.n_tiles = nt.value
        self.plan = torch.empty(max(self.n_tiles * _lib.BATCHED_PLAN_WORDS, 1), dtype=_I32, device=dev)
        call("spmv_batched_plan", *args(_p(self.plan), self.plan.numel()))

    def __call__(self, x: torch.Tensor, y: Optional[torch.Tensor] = None) -> torch.Tensor:
        if y is None:
            y = torch.empty(self.total_rows, dtype=torch.float32, device=x.device)
        call("spmv_batched", self.n_tiles, _p(self.plan), _p(self.perm), _p(self.bl_col), _p(self.bl_val), _p(x),
             _p(y), self.unroll, self.n_workgroups, _stream())
        return y


# --------------------------------------------------------------------------- HIP graphs


class Graph:
    """Captures the library calls made inside ``with g.capture():`` on a side stream."""

    def __init__(self):
        self.exec = None
        self.stream = torch.cuda.Stream()

    def capture(self):
        g = self

        class _Ctx:
            def __enter__(self_):
                g.stream.wait_stream(torch.cuda.current_stream())
                self_.ctx = torch.cuda.stream(g.stream)
                self_.ctx.__enter__()
                call("spmv_graph_begin", C.c_void_p(g.stream.cuda_stream))

            def __exit__(self_, et, ev, tb):
                h = C.c_void_p()
                try:
                    call("spmv_graph_end", C.c_void_p(g.stream.cuda_stream), C.byref(h))
                finally:
                    self_.ctx.__exit__(et, ev, tb)
                torch.cuda.current_stream().wait_stream(g.stream)
                g.exec = h
                return False

        return _Ctx()

    def replay(self):
        call("spmv_graph_launch", self.exec, _stream())

    def __del__(self):
        if getattr(self, "exec", None):
            try:
                _lib.load().spmv_graph_destroy(self.exec)
            except Exception:
                pass
