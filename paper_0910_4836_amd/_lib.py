"""ctypes loader for libspmv.so: argument types of every C entry point.

The library must be built (``python -m paper_0910_4836_amd.build`` or
``__graft_entry__.build()``); there is no fallback path.
"""
from __future__ import annotations

import ctypes as C
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libspmv.so")

F64, F32, BF16, I32 = 0, 1, 2, 3     # I32: payload of the value-moving calls only
SYMPERM, SOJDS = 1, 2
WIDE_ROW_NNZ = 4096
BATCHED_PLAN_WORDS = 12
SPLIT_PARTS = 8
DIA_MAX = 64           # SPMV_DIA_MAX

STATUS = {0: "ok", 1: "invalid argument", 2: "bad matrix format", 3: "output capacity too small",
          4: "unsupported", 5: "HIP runtime error"}


class SpmvError(RuntimeError):
    def __init__(self, status, func, msg):
        super().__init__(f"{func}: {STATUS.get(status, status)}: {msg}")
        self.status = status


_p = C.c_void_p
_i32, _i64, _u32, _f64, _sz, _int = C.c_int32, C.c_int64, C.c_uint32, C.c_double, C.c_size_t, C.c_int
_i32p = C.POINTER(C.c_int32)
_i64p = C.POINTER(C.c_int64)
_vpp = C.POINTER(C.c_void_p)

SIGNATURES = {
    "spmv_status_string": (C.c_char_p, [_int]),
    "spmv_last_error": (C.c_char_p, []),
    "spmv_version": (C.c_char_p, []),
    "spmv_csr_from_coo_workspace_size": (_sz, [_i32, _i32, _i64]),
    "spmv_csr_from_coo": (_int, [_i32, _i32, _i64, _p, _p, _p, _int, _p, _p, _p, _i64p, _p, _sz, _p]),
    "spmv_csr_validate_workspace_size": (_sz, []),
    "spmv_csr_validate": (_int, [_i32, _i32, _i64, _p, _p, _i32p, _p, _sz, _p]),
    "spmv_jds_from_csr_workspace_size": (_sz, [_i32, _i64]),
    "spmv_jds_from_csr": (_int, [_i32, _i64, _p, _p, _p, _int, _u32, _p, _p, _p, _i32, _p, _p, _i32p, _i32p,
                                 _p, _sz, _p]),
    "spmv_jds_to_csr_workspace_size": (_sz, [_i32]),
    "spmv_jds_to_csr": (_int, [_i32, _p, _p, _i32, _p, _p, _int, _u32, _p, _p, _p, _p, _sz, _p]),
    "spmv_jds_blocked_workspace_size": (_sz, [_i32, _i32, _i32, _u32]),
    "spmv_jds_blocked_from_jds": (_int, [_i32, _p, _i32, _p, _p, _int, _i32, _u32, _p, _p, _p, _p, _i64, _i64p,
                                         _i32p, _p, _sz, _p]),
    "spmv_crs_plan": (_int, [_i32, _p, _i32, _p, _i32, _i32p, _p]),
    "spmv_jds_blocked_windowed_workspace_size": (_sz, [_i32]),
    "spmv_jds_blocked_windowed_from_csr": (_int, [_i32, _i64, _p, _p, _p, _int, _i32, _i32, _p, _p, _p, _p, _p,
                                                  _i64, _i64p, _i32p, _p, _sz, _p]),
    "spmv_jds_blocked_tiles": (_int, [_i32, _i32, _i32, _i32p, _i32, _i32, _i32, _p, _i64, _i64p, _i64p, _p]),
    "spmv_jds_blocked_tiled": (_int, [_i32, _p, _i32, _i32, _p, _p, _p, _p, _int, _p, _p, _int, _f64, _f64, _p,
                                      _i64, _i64p, _i32, _u32, _p]),
    "spmv_jds_tiles": (_int, [_i32, _i32p, _i32, _i32, _i32, _i32, _p, _i64, _i64p, _i64p, _p]),
    "spmv_jds_tiled": (_int, [_i32, _p, _p, _i32, _p, _p, _int, _p, _p, _int, _f64, _f64, _p, _i64, _i64p, _i32,
                              _u32, _p]),
    "spmv_convert_values": (_int, [_i64, _p, _int, _p, _int, _p]),
    "spmv_transpose_workspace_size": (_sz, [_i32, _i32, _i64]),
    "spmv_transpose_csr": (_int, [_i32, _i32, _i64, _p, _p, _p, _p, _p, _p, _sz, _p]),
    "spmv_crs": (_int, [_i32, _i32, _p, _p, _p, _int, _p, _p, _int, _f64, _f64, _p, _i32, _i32, _p]),
    "spmv_crs_staged": (_int, [_i32, _i32, _p, _p, _p, _int, _p, _p, _int, _f64, _f64, _p, _i32, _i32, _p]),
    "spmv_jds": (_int, [_i32, _p, _p, _i32p, _i32, _p, _p, _int, _p, _p, _int, _f64, _f64, _i32, _i32, _i32, _u32,
                        _p]),
    "spmv_jds_blocked": (_int, [_i32, _p, _i32, _i32, _p, _p, _i32p, _p, _p, _int, _p, _p, _int, _f64, _f64, _i32,
                                _i32, _i32, _i32, _u32, _p]),
    "spmv_permute_vec": (_int, [_i32, _p, _p, _p, _int, _int, _p]),
    "spmv_gather_values": (_int, [_i64, _p, _p, _p, _int, _p]),
    "spmv_axpby": (_int, [_i64, _f64, _p, _f64, _p, _int, _p]),
    "spmv_dot_workspace_size": (_sz, [_i64]),
    "spmv_dot": (_int, [_i64, _p, _p, _int, _p, _p, _sz, _p]),
    "spmv_dot_noalloc": (_int, [_i64, _p, _p, _int, _p, _p]),
    "spmm_workspace_size": (_sz, [_i32, _i32, _int]),
    "spmm_crs": (_int, [_i32, _i32, _p, _p, _p, _int, _i32, _p, _i64, _p, _i64, _int, _f64, _f64, _p, _i32, _i32,
                        _p, _sz, _p]),
    "spmm_jds": (_int, [_i32, _i32, _p, _p, _i32p, _i32, _p, _p, _int, _i32, _p, _i64, _p, _i64, _int, _f64, _f64,
                        _u32, _p, _sz, _p]),
    "spmm_jds_blocked_plan": (_int, [_i32, _i32, _i32, _i32p, _i32, _i32, _i32, _p, _i32, _i32p, _i32p, _p]),
    "spmm_jds_blocked": (_int, [_i32, _i32, _p, _i32, _i32, _p, _p, _p, _p, _int, _i32, _p, _i64, _p, _i64, _int,
                                _f64, _f64, _p, _i32, _p, _sz, _p]),
    "spmv_grad_vals_jds": (_int, [_i32, _p, _p, _i32p, _i32, _i64, _p, _p, _p, _p, _int, _f64, _f64, _u32, _p]),
    "spmv_split_columns_workspace_size": (_sz, [_i32, _i64]),
    "spmv_split_columns": (_int, [_i32, _i32, _i64, _p, _p, _p, _int, _i32, _p, _p, _p, _p, _p, _i64p, _i64p, _p, _sz,
                                  _p]),
    "spmv_split_workspace_size": (_sz, [_i64]),
    "spmv_crs_split": (_int, [_i32, _i32, _p, _p, _p, _p, _p, _i64p, _i64p, _int, _p, _i32p, _i32p, _i32, _p, _p, _int,
                              _f64, _f64, _p, _sz, _p]),
    "spmv_jds_split": (_int, [_i32, _p, _i64p, _vpp, _vpp, _vpp, _i32p, _vpp, _vpp, _int, _p, _p, _int, _f64, _f64,
                              _i32, _i32, _i32, _p, _sz, _p]),
    "spmv_jds_blocked_split": (_int, [_i32, _i32, _p, _i64p, _vpp, _vpp, _vpp, _vpp, _vpp, _vpp, _int, _p, _p, _int,
                                      _f64, _f64, _i32, _i32, _i32, _i32, _p, _sz, _p]),
    "spmv_split_rows_workspace_size": (_sz, []),
    "spmv_split_rows": (_int, [_i32, _i64, _p, _p, _i64p, _i64p, _p, _sz, _p]),
    "spmv_jds_row_split": (_int, [_i32, _i64p, _vpp, _vpp, _vpp, _i32p, _vpp, _vpp, _int, _p, _p, _int, _f64, _f64,
                                  _i32, _i32, _i32, _p]),
    "spmv_jds_blocked_row_split": (_int, [_i32, _i32, _i64p, _vpp, _vpp, _vpp, _vpp, _vpp, _vpp, _int, _p, _p, _int,
                                          _f64, _f64, _i32, _i32, _i32, _i32, _p]),
    "spmv_stride_probe": (_int, [_i64, _i32, _p, _p, _p, _i64, _p, _i64, _p]),
    "spmv_dia_workspace_size": (_sz, [_i32, _i32]),
    "spmv_dia_from_csr": (_int, [_i32, _i32, _i64, _p, _p, _p, _int, _i32, _i32p, _i32p, _i64p, _p, _p, _p, _p, _p,
                                 _sz, _p]),
    "spmv_dia": (_int, [_i32, _i32, _i32, _i32p, _p, _int, _p, _p, _p, _p, _p, _int, _f64, _f64, _p]),
    "spmv_dia_sym_from_csr": (_int, [_i32, _i64, _p, _p, _p, _int, _i32, _i32p, _i32p, _i64p, _p, _p, _p, _p, _p,
                                     _sz, _p]),
    "spmv_dia_sym": (_int, [_i32, _i32, _i32p, _p, _int, _p, _p, _p, _p, _p, _int, _f64, _f64, _p]),
    "spmv_csr_slices_workspace_size": (_sz, [_i32]),
    "spmv_csr_to_slices": (_int, [_i32, _p, _p, _p, _int, _p, _p, _p, _p, _p, _i64, _i64p, _p, _sz, _p]),
    "spmv_dia_sliced": (_int, [_i32, _i32, _i32, _i32p, _p, _int, _p, _p, _p, _p, _p, _p, _p, _int, _f64, _f64,
                                  _int, _p]),
    "spmv_csr_upper_workspace_size": (_sz, [_i32]),
    "spmv_csr_upper_from_csr": (_int, [_i32, _i64, _p, _p, _p, _int, _i64p, _p, _p, _p, _p, _sz, _p]),
    "spmv_crs_sym": (_int, [_i32, _p, _p, _p, _int, _p, _p, _int, _f64, _f64, _p, _i32, _i32, _p]),
    "spmv_crs_sym_staged": (_int, [_i32, _p, _p, _p, _int, _p, _p, _int, _f64, _f64, _p, _i32, _i32, _p]),
    "spmv_batched_plan": (_int, [_i32, _i32p, _i32p, _i64p, _i64p, _i64p, _i64p, _i32p, _i32, _p, _i64, _i64p,
                                 _p]),
    "spmv_batched": (_int, [_i64, _p, _p, _p, _p, _p, _p, _i32, _i32, _p]),
    "spmv_graph_begin": (_int, [_p]),
    "spmv_graph_end": (_int, [_p, _vpp]),
    "spmv_graph_launch": (_int, [_p, _p]),
    "spmv_graph_destroy": (_int, [_p]),
    "spmv_stream_triad": (_int, [_i64, _p, _p, _p, _f64, _p]),
    "spmv_stream_copy": (_int, [_i64, _p, _p, _p]),
    "spmv_stream_read": (_int, [_i64, _p, _p, _i64, _p]),
    "spmv_gather_probe": (_int, [_i64, _p, _p, _p, _i64, _p]),
}

_lib = None


def load():
    """Loads libspmv.so and declares every entry point; raises if it is missing."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError(f"{LIB_PATH} is not built; run __graft_entry__.build() "
                              "(python -m paper_0910_4836_amd.build)")
        lib = C.CDLL(LIB_PATH)
        for name, (res, args) in SIGNATURES.items():
            fn = getattr(lib, name)
            fn.restype = res
            fn.argtypes = args
        _lib = lib
    return _lib


def call(name, *args):
    """Calls entry point ``name``; a non-zero status raises SpmvError."""
    lib = load()
    st = getattr(lib, name)(*args)
    if st != 0:
        msg = lib.spmv_last_error().decode()
        raise SpmvError(st, name, msg)
    return st
