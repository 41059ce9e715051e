"""MI355X (gfx950) CRS / JDS sparse matrix-vector library.

The kernels and the C ABI live in ``libspmv.so`` (sources in ``csrc/``, API in
``include/spmv.h``); this package is its Python binding.  The operations follow
Schubert, Hager and Fehske, "Performance limitations for sparse matrix-vector
multiplications on current multicore environments", Section 2.
"""
from ._lib import SpmvError, load as load_library  # noqa: F401
from .spmv import (  # noqa: F401
    CSR, DIA, JDS, SymCSR, Slices, Batched, csr_to_slices, Blocked, Graph, RowSplit, Split, colmajor, csr_from_coo, dia_from_csr, dtype_code,
    jds_blocked_from_jds, jds_from_csr, jds_to_csr, spmm_crs, spmm_jds, spmm_jds_blocked, spmm_workspace, spmv_axpby,
    spmv_convert_values, spmv_crs, spmv_crs_plan, spmv_crs_split, spmv_csr_validate, spmv_dia, spmv_dot,
    spmv_dot_noalloc, jds_blocked_windowed_from_csr, spmv_jds_blocked_tiles, spmv_jds_blocked_tiled,
    spmv_jds_tiles, spmv_jds_tiled,
    spmv_gather_probe, spmv_gather_values, spmv_grad_vals_jds, spmv_jds, spmv_jds_blocked,
    spmv_jds_blocked_row_split, spmv_jds_blocked_split, spmv_jds_row_split, spmv_jds_split, spmv_permute_vec,
    csr_upper_from_csr, spmv_crs_sym, spmv_stream_copy, spmv_stream_read, spmv_stream_triad, spmv_stride_probe, spmv_transpose_csr, version)
