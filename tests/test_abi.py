"""CPU checks of the C ABI: the library loads, exports every declared entry point,
the Python binding declares them all, and the product path never touches the oracle."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "spmv.h")
PKG = os.path.join(ROOT, "paper_0910_4836_amd")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    names = re.findall(r"\b((?:spmv|spmm)_[a-z0-9_]+)\s*\(", text)
    return sorted(set(names))


def test_header_declares_the_boundary():
    names = declared_functions()
    for must in ["spmv_csr_from_coo", "spmv_jds_from_csr", "spmv_crs", "spmv_jds", "spmv_jds_blocked",
                 "spmv_jds_blocked_from_jds", "spmm_crs", "spmm_jds", "spmv_batched", "spmv_batched_plan",
                 "spmv_transpose_csr", "spmv_grad_vals_jds", "spmv_convert_values"]:
        assert must in names


def test_library_exports_every_declared_symbol():
    from paper_0910_4836_amd import _lib
    lib = ctypes.CDLL(_lib.LIB_PATH)
    missing = [n for n in declared_functions() if not hasattr(lib, n)]
    assert not missing, missing


def test_binding_declares_every_symbol():
    from paper_0910_4836_amd import _lib
    assert sorted(_lib.SIGNATURES) == declared_functions()
    lib = _lib.load()
    assert lib.spmv_version().decode() == "1.0.0"
    assert lib.spmv_status_string(3).decode() == "output capacity too small"


def test_host_side_validation_without_gpu():
    """Argument checks run on the host before any device work."""
    from paper_0910_4836_amd import _lib
    lib = _lib.load()
    st = lib.spmv_crs(-1, 0, None, None, None, 0, None, None, 0, 1.0, 0.0, None, 0, 0, None)
    assert st == 1 and b"negative" in lib.spmv_last_error()
    st = lib.spmv_jds(10, None, None, None, 0, None, None, 0, None, None, 0, 1.0, 0.0, 3, 0, 0, 0, None)
    assert st == 1 and b"unroll" in lib.spmv_last_error()
    st = lib.spmv_jds_blocked(10, None, 96, 1, None, None, None, None, None, 0, None, None, 0, 1.0, 0.0, 0, 0, 0,
                              0, 0, None)
    assert st == 1 and b"multiple of 64" in lib.spmv_last_error()
    st = lib.spmv_crs(10, 10, None, None, None, 7, None, None, 0, 1.0, 0.0, None, 0, 0, None)
    assert st == 1 and b"dtype" in lib.spmv_last_error()
    # the staged CRS kernel needs a plan and a block size within [256, 4096]
    p = ctypes.c_void_p(16)           # a non-null stand-in, never dereferenced (the checks fail first)
    st = lib.spmv_crs_staged(10, 10, p, p, p, 0, p, p, 0, 1.0, 0.0, None, 1, 1024, None)
    assert st == 1 and b"plan" in lib.spmv_last_error()
    st = lib.spmv_crs_staged(10, 10, p, p, p, 0, p, p, 0, 1.0, 0.0, p, 1, 8192, None)
    assert st == 1 and b"block_nnz" in lib.spmv_last_error()
    st = lib.spmv_crs_staged(10, 10, p, p, p, 9, p, p, 0, 1.0, 0.0, p, 1, 1024, None)
    assert st == 1 and b"dtype" in lib.spmv_last_error()
    assert lib.spmv_crs_staged(0, 10, None, None, None, 0, None, None, 0, 1.0, 0.0, None, 0, 0, None) == 0
    # row-split bounds must run from 0 to n without decreasing
    import numpy as np
    from paper_0910_4836_amd import spmv as spmv_mod
    for bad in ([0, 2, 1, 3, 4, 5, 6, 7, 10], [0, 1, 2, 3, 4, 5, 6, 7, 9]):
        b = np.array(bad, dtype=np.int64)
        st = lib.spmv_jds_row_split(10, spmv_mod._h_i64(b), None, None, None, None, None, None, 0, None, None, 0, 1.0,
                                    0.0, 0, 0, 0, None)
        assert st == 1 and b"h_bounds" in lib.spmv_last_error()
        st = lib.spmv_jds_blocked_row_split(10, 64, spmv_mod._h_i64(b), None, None, None, None, None, None, 0, None, None,
                                            0, 1.0, 0.0, 0, 0, 0, 0, None)
        assert st == 1 and b"h_bounds" in lib.spmv_last_error()
    st = lib.spmv_jds_row_split(10, None, None, None, None, None, None, None, 0, None, None, 0, 1.0, 0.0, 0, 0, 0,
                                None)
    assert st == 1 and b"h_bounds" in lib.spmv_last_error()
    # DIA offsets: at most SPMV_DIA_MAX, increasing, inside the matrix
    offs = np.array([0, 5, 3], dtype=np.int32)
    st = lib.spmv_dia(10, 10, 3, spmv_mod._h_i32(offs), 1, 0, None, None, None, 1, 1, 0, 1.0, 0.0, None)
    assert st == 1 and b"increase" in lib.spmv_last_error()
    offs = np.array([-10], dtype=np.int32)
    st = lib.spmv_dia(10, 10, 1, spmv_mod._h_i32(offs), 1, 0, None, None, None, 1, 1, 0, 1.0, 0.0, None)
    assert st == 1 and b"outside" in lib.spmv_last_error()
    st = lib.spmv_dia(10, 10, 65, None, None, 0, None, None, None, None, None, 0, 1.0, 0.0, None)
    assert st == 1 and b"ndia" in lib.spmv_last_error()
    # launch shape: 4, 8 or 16 wavefronts per workgroup
    st = lib.spmv_jds(10, None, None, None, 0, None, None, 0, None, None, 0, 1.0, 0.0, 0, 0, 12, 0, None)
    assert st == 1 and b"wg_waves" in lib.spmv_last_error()
    # symmetric DIA: upper diagonals only
    offs = np.array([-3], dtype=np.int32)
    st = lib.spmv_dia_sym(10, 1, spmv_mod._h_i32(offs), 1, 0, None, None, None, 1, 1, 0, 1.0, 0.0, None)
    assert st == 1 and b">= 0" in lib.spmv_last_error()
    # DIA with the remainder in window-sorted slices: square for symmetric
    # storage; a remainder needs its slot rows
    st = lib.spmv_dia_sliced(10, 12, 0, None, None, 0, None, None, None, None, None, 1, 1, 0, 1.0, 0.0, 1, None)
    assert st == 1 and b"square" in lib.spmv_last_error()
    st = lib.spmv_dia_sliced(10, 10, 0, None, None, 0, 1, 1, None, 1, 1, 1, 1, 0, 1.0, 0.0, 0, None)
    assert st == 1 and b"null remainder slices" in lib.spmv_last_error()
    st = lib.spmv_csr_to_slices(10, 1, 1, 1, 0, 1, 1, 1, None, None, 0, spmv_mod.C.byref(spmv_mod.C.c_int64(0)), 1,
                                16, None)
    assert st == 1 and b"workspace" in lib.spmv_last_error()
    st = lib.spmv_csr_to_slices(-1, None, None, None, 0, None, None, None, None, None, 0, None, None, 0, None)
    assert st == 1 and b"n_rows < 0" in lib.spmv_last_error()
    # access-pattern probe: a stride of at least 1
    st = lib.spmv_stride_probe(100, 0, None, None, None, 0, None, 0, None)
    assert st == 1 and b"k < 1" in lib.spmv_last_error()


def test_product_path_does_not_use_the_oracle():
    for dirpath, _, files in os.walk(PKG):
        for f in files:
            if f.endswith((".py", ".hip", ".hpp", ".cpp", ".h")):
                text = open(os.path.join(dirpath, f)).read()
                assert not re.search(r"\boracle\b", text), f"{f} mentions the oracle"
                assert "synth" not in text, f"{f} imports the input generator"


def test_missing_library_fails_loudly(tmp_path, monkeypatch):
    from paper_0910_4836_amd import _lib
    monkeypatch.setattr(_lib, "_lib", None)
    monkeypatch.setattr(_lib, "LIB_PATH", str(tmp_path / "absent.so"))
    with pytest.raises(ImportError):
        _lib.load()
