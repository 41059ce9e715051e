/*
 * spmv.h - C ABI of the MI355X (gfx950) CRS / JDS sparse matrix-vector library.
 *
 * The operations follow G. Schubert, G. Hager, H. Fehske, "Performance
 * limitations for sparse matrix-vector multiplications on current multicore
 * environments" (arXiv:0910.4836), Section 2 (CRS, JDS and the NBJDS, NUJDS,
 * RBJDS and SOJDS refinements).  The library adds mixed-precision value
 * storage, multi-vector and many-matrix forms and the derivatives needed to
 * differentiate through y = A x.
 *
 * Conventions (apply to every call unless its comment says otherwise)
 *  - Pointers are DEVICE pointers, except parameters whose name starts with
 *    h_, which are host pointers.  `stream` is a hipStream_t (NULL = the
 *    default stream), passed as void* so that this header needs no HIP header.
 *  - Indices are 0-based int32; nnz counts are int64 but must stay below 2^31.
 *  - The caller owns every buffer: inputs, outputs and workspace.  The library
 *    never allocates or frees caller memory.  Calls that need scratch memory
 *    take (ws, ws_bytes) and have a *_workspace_size() query.
 *  - Setup calls (conversions, plans) may synchronise `stream` to return sizes
 *    through h_ outputs; they cannot be captured in a HIP graph.  Compute calls
 *    (spmv_*, spmm_*, grad, axpby, batched run) are asynchronous, do not
 *    allocate and do not synchronise, so they can be captured.
 *  - Compute calls, and setup calls that start from a CRS or JDS matrix,
 *    validate their arguments on the host only (null pointers, negative
 *    sizes, unsupported dtype combinations); the matrix contents are trusted.
 *    spmv_csr_from_coo checks its indices; spmv_csr_validate() checks CRS
 *    contents on the device.
 *  - Every call returns a spmv_status; on failure spmv_last_error() returns a
 *    message for the calling thread.  No C++ exception crosses this boundary.
 *  - Results are deterministic: every output element is produced by one
 *    fixed sequence of operations for a given argument set.  The one
 *    exception is spmv_crs_sym / spmv_crs_sym_staged (one-triangle storage), whose mirrored terms
 *    are added with floating-point atomics.
 *  - Vectors x and y of one call must not overlap (except where stated).
 */
#ifndef SPMV_H
#define SPMV_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    SPMV_OK = 0,
    SPMV_ERR_INVALID_ARG = 1, /* null pointer, negative size, bad flag          */
    SPMV_ERR_BAD_FORMAT = 2,  /* index out of range, malformed row_ptr          */
    SPMV_ERR_CAPACITY = 3,    /* an output buffer is too small (size returned)  */
    SPMV_ERR_UNSUPPORTED = 4, /* dtype combination or size the library lacks    */
    SPMV_ERR_HIP = 5          /* a HIP runtime call failed                      */
} spmv_status;

typedef enum {
    SPMV_F64 = 0,  /* IEEE double                                       */
    SPMV_F32 = 1,  /* IEEE float                                        */
    SPMV_BF16 = 2, /* bfloat16 bit patterns (uint16_t), values only     */
    SPMV_I32 = 3   /* int32 payload: accepted only by the calls that move */
                   /* values without arithmetic (spmv_jds_from_csr,       */
                   /* spmv_jds_to_csr, spmv_jds_blocked_from_jds,         */
                   /* spmv_csr_upper_from_csr, spmv_permute_vec,          */
                   /* spmv_gather_values), which copy                     */
                   /* every element bit for bit; e.g. entry positions     */
                   /* carried through a conversion.  Rejected elsewhere.  */
} spmv_dtype;

/* flags */
#define SPMV_SYMPERM 1u /* JDS: permute columns too (A_{p(i),p(j)}); x, y in the permuted basis */
#define SPMV_SOJDS 2u   /* blocked JDS: sort the entries of each row for near-unit x strides   */

/* Rows with more than this many entries accumulate in FP64 when the values
 * are stored as FP32 or BF16. */
#define SPMV_WIDE_ROW_NNZ 4096

const char *spmv_status_string(spmv_status s);
/* Message describing the last failure on the calling thread ("" if none). */
const char *spmv_last_error(void);
/* Library version, e.g. "1.0.0". */
const char *spmv_version(void);

/* ======================================================================== */
/* Setup: format construction (paper Section 2)                              */
/* ======================================================================== */

/* COO triplets -> CRS (paper Section 2: val, col_idx, row_ptr).
 * Entries are ordered by (row, col); duplicate (row, col) pairs are summed in
 * input order; explicit zeros are kept as stored entries.  val/val_out have
 * dtype dt (F64 or F32; duplicates are summed in that type).
 * Outputs: row_ptr[n_rows+1], col_idx[nnz], val_out[nnz] (nnz = input count
 * is always enough); *h_nnz_out = stored entries.  Any row or col outside
 * [0, n_rows) x [0, n_cols) -> SPMV_ERR_BAD_FORMAT.  Synchronises.  */
size_t spmv_csr_from_coo_workspace_size(int32_t n_rows, int32_t n_cols, int64_t nnz);
spmv_status spmv_csr_from_coo(int32_t n_rows, int32_t n_cols, int64_t nnz, const int32_t *row,
                              const int32_t *col, const void *val, spmv_dtype dt,
                              int32_t *row_ptr, int32_t *col_idx, void *val_out,
                              int64_t *h_nnz_out, void *ws, size_t ws_bytes, void *stream);

/* Checks a CRS structure on the device: row_ptr[0] == 0, row_ptr non-
 * decreasing, row_ptr[n_rows] == nnz, every col_idx in [0, n_cols).
 * *h_ok = 1 if valid, 0 otherwise.  ws: spmv_csr_validate_workspace_size().
 * Synchronises. */
size_t spmv_csr_validate_workspace_size(void);
spmv_status spmv_csr_validate(int32_t n_rows, int32_t n_cols, int64_t nnz, const int32_t *row_ptr,
                              const int32_t *col_idx, int32_t *h_ok, void *ws, size_t ws_bytes,
                              void *stream);

/* CRS -> JDS (paper Section 2): rows are permuted by decreasing length
 * (equal lengths keep ascending original index), each row's entries are
 * shifted left in CRS order, and the d-th entries of all rows form jagged
 * diagonal d, stored diagonal after diagonal.
 *   perm[r]  = original row of permuted row r;  iperm = inverse (n each)
 *   jd_ptr[d] = offset of diagonal d, jd_ptr[ndiag] = nnz (ndiag = max row
 *              length); capacity jd_ptr_cap entries
 *   jd_col, jd_val: nnz entries; with SPMV_SYMPERM jd_col = iperm[col]
 *              (square matrices only), otherwise original column numbers.
 * *h_ndiag = ndiag.  If jd_ptr_cap < ndiag+1 returns SPMV_ERR_CAPACITY with
 * *h_ndiag set and nothing else written (call again with a larger buffer).
 * h_jd_ptr (optional, may be NULL) receives a host copy of jd_ptr; the JDS
 * compute calls take that copy to size their launch without reading device
 * memory.  Synchronises. */
size_t spmv_jds_from_csr_workspace_size(int32_t n, int64_t nnz);
spmv_status spmv_jds_from_csr(int32_t n, int64_t nnz, const int32_t *row_ptr, const int32_t *col_idx,
                              const void *val, spmv_dtype dt, unsigned flags, int32_t *perm,
                              int32_t *iperm, int32_t *jd_ptr, int32_t jd_ptr_cap, int32_t *jd_col,
                              void *jd_val, int32_t *h_ndiag, int32_t *h_jd_ptr, void *ws,
                              size_t ws_bytes, void *stream);

/* JDS -> CRS in the original row order, entries of a row in diagonal order
 * (the exact inverse of spmv_jds_from_csr).  With SPMV_SYMPERM the columns
 * are mapped back through perm.  row_ptr[n+1], col_idx[nnz], val[nnz].
 * ws: spmv_jds_to_csr_workspace_size(n).  Synchronises. */
size_t spmv_jds_to_csr_workspace_size(int32_t n);
spmv_status spmv_jds_to_csr(int32_t n, const int32_t *perm, const int32_t *jd_ptr, int32_t ndiag,
                            const int32_t *jd_col, const void *jd_val, spmv_dtype dt, unsigned flags,
                            int32_t *row_ptr, int32_t *col_idx, void *val, void *ws, size_t ws_bytes,
                            void *stream);

/* JDS -> blocked JDS (paper Section 2, RBJDS; SOJDS with SPMV_SOJDS).
 * Blocks ("slices") are C consecutive permuted rows, C a positive multiple of
 * 64.  All elements of a slice are stored together, diagonal by diagonal,
 * padded to the slice's first (longest) row; padded slots hold col = -1 and
 * value 0 and are never used.  Element (d, row r) of slice s = r / C is at
 * slice_ptr[s] + d*C + (r - s*C).
 *   slice_ptr[n_slices+1] (int64), slice_nd[n_slices] = diagonals in slice s,
 *   n_slices = ceil(n / C); bl_col/bl_val hold the padded total.
 * SPMV_SOJDS: inside each slice the entries of every row are re-assigned to
 * diagonal slots: the slice's first row keeps CRS order; each following row,
 * slot by slot, takes from its remaining entries the one whose column is
 * closest to (column in the same slot of the previous row) + 1, the smaller
 * column on a tie.
 * *h_padded = padded total; if bl_cap < padded returns SPMV_ERR_CAPACITY and
 * writes nothing else.  h_slice_nd (optional) receives a host copy of
 * slice_nd.  Synchronises. */
size_t spmv_jds_blocked_workspace_size(int32_t n, int32_t ndiag, int32_t C, unsigned flags);
spmv_status spmv_jds_blocked_from_jds(int32_t n, const int32_t *jd_ptr, int32_t ndiag,
                                      const int32_t *jd_col, const void *jd_val, spmv_dtype dt,
                                      int32_t C, unsigned flags, int64_t *slice_ptr, int32_t *slice_nd,
                                      int32_t *bl_col, void *bl_val, int64_t bl_cap, int64_t *h_padded,
                                      int32_t *h_slice_nd, void *ws, size_t ws_bytes, void *stream);

/* CRS -> blocked JDS over a windowed row order (the RBJDS storage of
 * spmv_jds_blocked_from_jds; paper Section 2 leaves room for a more elaborate
 * initial ordering of the elements).  The rows are cut into windows of sigma
 * consecutive original rows (sigma a positive multiple of C); inside each
 * window they are sorted by decreasing length (ties in ascending original
 * index), and the windows follow one another, so perm is window-local and
 * sigma >= n gives the plain JDS order.  Slices of C permuted rows never span
 * two windows; each is stored diagonal by diagonal and padded to its first
 * (longest) row (col = -1, value 0), entries of a row in CRS order.  Rows that
 * are neighbours in the original order stay neighbours in time when the
 * slices are processed in order, which keeps the x window of a banded part
 * of the matrix in cache.
 *   perm[n], slice_ptr[n_slices+1] (int64), slice_nd[n_slices],
 *   n_slices = ceil(n / C); bl_col/bl_val hold the padded total.
 * *h_padded = padded total; if bl_cap < padded returns SPMV_ERR_CAPACITY with
 * *h_padded set and the arrays unwritten.  h_slice_nd (optional) receives a
 * host copy of slice_nd.  dt: F64, F32, BF16 or I32 (moved bit for bit).
 * ws: spmv_jds_blocked_windowed_workspace_size(n).  Synchronises. */
size_t spmv_jds_blocked_windowed_workspace_size(int32_t n);
spmv_status spmv_jds_blocked_windowed_from_csr(int32_t n, int64_t nnz, const int32_t *row_ptr,
                                               const int32_t *col_idx, const void *val, spmv_dtype dt,
                                               int32_t C, int32_t sigma, int32_t *perm, int64_t *slice_ptr,
                                               int32_t *slice_nd, int32_t *bl_col, void *bl_val,
                                               int64_t bl_cap, int64_t *h_padded, int32_t *h_slice_nd,
                                               void *ws, size_t ws_bytes, void *stream);

/* Tile plan for spmv_jds_blocked_tiled, built on the host from the slice
 * depths of any blocked-JDS storage (slice depths need not decrease, as in
 * the windowed order).  Every run of slices wanting the same split (R rows
 * per wavefront, S wavefronts per row group; chosen from the slice depth as
 * in spmv_jds_blocked, or R = rows_per_wave when that is non-zero) is covered
 * by workgroups of (wg_waves / S) * R rows, one record of two int32 each
 * (first row; R, S and row count packed).  When the depths never increase
 * (the globally sorted order) the records are dealt as in spmv_jds_tiles,
 * with slices for rows: each run of equal-depth slices of at least 1,024
 * rows in 8 contiguous pieces, one per XCD, the rest for equal cost.
 * Otherwise (e.g. the windowed order, whose windows already keep
 * neighbouring rows together) they are cut into 8 contiguous ranges of about
 * equal work: range k runs on XCD k.
 *   tiles: 2 * n_tiles int32 (device), written when tiles_cap >= 2 * n_tiles,
 *          otherwise SPMV_ERR_CAPACITY with *h_n_tiles set (two-call pattern)
 *   h_plan[10]: the 9 range bounds and the wavefronts per workgroup, passed
 *          unchanged to spmv_jds_blocked_tiled.
 * Synchronises. */
spmv_status spmv_jds_blocked_tiles(int32_t n, int32_t C, int32_t n_slices, const int32_t *h_slice_nd,
                                   int32_t max_iters, int32_t rows_per_wave, int32_t wg_waves,
                                   int32_t *tiles, int64_t tiles_cap, int64_t *h_n_tiles, int64_t *h_plan,
                                   void *stream);

/* Row-block plan for spmv_crs / spmm_crs: plan[0..n_blocks] are row
 * boundaries.  Consecutive rows are grouped while the group holds at most
 * block_nnz entries (0 = library default, 1024) and at most 256 rows, or at
 * most 2048 rows if none of them has more than 16 entries; a row longer than
 * block_nnz is a block of its own.  The kernels accept any plan whose blocks
 * are either a single row or hold at most block_nnz entries.  If plan_cap < n_blocks+1 returns
 * SPMV_ERR_CAPACITY with *h_n_blocks set.  Synchronises (reads row_ptr). */
spmv_status spmv_crs_plan(int32_t n_rows, const int32_t *row_ptr, int32_t block_nnz, int32_t *plan,
                          int32_t plan_cap, int32_t *h_n_blocks, void *stream);

/* CRS <-> reduced-precision value conversion: out[i] = in[i] rounded to
 * out_dt with round-to-nearest-even in one step (F64 -> BF16 does not pass
 * through F32).  Widening conversions are exact.  Asynchronous. */
spmv_status spmv_convert_values(int64_t n, const void *in, spmv_dtype in_dt, void *out,
                                spmv_dtype out_dt, void *stream);

/* Structure of A^T (n_rows x n_cols A, CRS): rowT_ptr[n_cols+1], colT[nnz]
 * (row c of A^T lists column c of A in ascending row order) and tmap[nnz]
 * with A^T's values = val[tmap].  Synchronises. */
size_t spmv_transpose_workspace_size(int32_t n_rows, int32_t n_cols, int64_t nnz);
spmv_status spmv_transpose_csr(int32_t n_rows, int32_t n_cols, int64_t nnz, const int32_t *row_ptr,
                               const int32_t *col_idx, int32_t *rowT_ptr, int32_t *colT, int32_t *tmap,
                               void *ws, size_t ws_bytes, void *stream);

/* ======================================================================== */
/* Compute                                                                   */
/* ======================================================================== */
/* All SpMV forms compute y = alpha * A x + beta * y.  beta == 0 never reads
 * y.  val_dt is F64, F32 or BF16; vec_dt (x and y) is F64 or F32.
 * Arithmetic: F64 values -> products and sums in FP64.  F32/BF16 values ->
 * x is rounded to FP32 and products and sums are FP32, except rows with more
 * than SPMV_WIDE_ROW_NNZ entries, which form exact FP64 products of the
 * stored value and x and sum them in FP64.  alpha/beta are applied in FP64
 * and y is rounded to vec_dt once. */

/* CRS kernel (paper Section 2, CRS listing): y_i = alpha*sum_j val_j x_{col_j}
 * + beta*y_i.  plan/n_blocks/block_nnz as given to and returned by
 * spmv_crs_plan (block_nnz 0 = default); plan == NULL uses one wavefront per
 * row.  col_idx, val and x may be NULL only if the matrix stores no entry. */
spmv_status spmv_crs(int32_t n_rows, int32_t n_cols, const int32_t *row_ptr, const int32_t *col_idx,
                     const void *val, spmv_dtype val_dt, const void *x, void *y, spmv_dtype vec_dt,
                     double alpha, double beta, const int32_t *plan, int32_t n_blocks,
                     int32_t block_nnz, void *stream);

/* CRS kernel, staged (paper Section 2, CRS kernel): the same product over the
 * same plan as spmv_crs, with the gathers issued in row order.  A block's
 * col/val are first copied to LDS in entry order; then each row's entries
 * are walked by G lanes (G = the largest power of two with G * rows <= 256,
 * at most 64; one lane per row in a block of more than 256 rows), so that a
 * wavefront's gather touches the same entry position of consecutive rows.
 * Rows of a multi-row block are summed per lane in entry order with fused
 * multiply-adds, then by a fixed shuffle tree over the G lanes; single-row
 * blocks are summed as in spmv_crs.  Accumulator types, argument meaning and
 * errors as for spmv_crs, except that plan is required (NULL ->
 * SPMV_ERR_INVALID_ARG).  The kernel trusts the plan: every multi-row block holds
 * at most block_nnz entries (LDS holds ceil(block_nnz / 1024) * 1024 entries
 * of values and indices).  Asynchronous. */
spmv_status spmv_crs_staged(int32_t n_rows, int32_t n_cols, const int32_t *row_ptr, const int32_t *col_idx,
                            const void *val, spmv_dtype val_dt, const void *x, void *y, spmv_dtype vec_dt,
                            double alpha, double beta, const int32_t *plan, int32_t n_blocks,
                            int32_t block_nnz, void *stream);

/* JDS kernel (paper Section 2, JDS listing; NBJDS/NUJDS refinements): each
 * lane owns one permuted row and walks the jagged diagonals that reach it,
 * `unroll` diagonals at a time (2, 4 or 8; 0 = default).  Rows whose length
 * exceeds `max_iters` diagonals (0 = default) have their diagonals split over
 * up to W wavefronts whose partial sums are added in a fixed order, W =
 * wg_waves, the wavefronts per workgroup: 4, 8 or 16 (0 = 16).  unroll,
 * max_iters and wg_waves shape the launch only (small workgroups keep more
 * gathers in flight for short, irregular rows; large ones stream uniform
 * rows better); the result is the same up to the summation order of long
 * rows.
 * Without SPMV_SYMPERM, x is in the original basis and y[perm[r]] receives
 * row r; with it, x and y are both in the permuted basis.
 * h_jd_ptr: host copy of jd_ptr (ndiag+1 entries). */
spmv_status spmv_jds(int32_t n, const int32_t *perm, const int32_t *jd_ptr, const int32_t *h_jd_ptr,
                     int32_t ndiag, const int32_t *jd_col, const void *jd_val, spmv_dtype val_dt,
                     const void *x, void *y, spmv_dtype vec_dt, double alpha, double beta,
                     int32_t unroll, int32_t max_iters, int32_t wg_waves, unsigned flags, void *stream);

/* Blocked JDS kernel (RBJDS / SOJDS storage): same result as spmv_jds.
 * rows_per_wave R in {8, 16, 32, 64} (0 = 64): a wavefront covers R rows of a
 * slice with 64/R lanes per row striding over the diagonals.  unroll,
 * max_iters and wg_waves as for spmv_jds.
 * h_slice_nd: host copy of slice_nd (non-increasing, as built). */
spmv_status spmv_jds_blocked(int32_t n, const int32_t *perm, int32_t C, int32_t n_slices,
                             const int64_t *slice_ptr, const int32_t *slice_nd,
                             const int32_t *h_slice_nd, const int32_t *bl_col, const void *bl_val,
                             spmv_dtype val_dt, const void *x, void *y, spmv_dtype vec_dt, double alpha,
                             double beta, int32_t rows_per_wave, int32_t unroll, int32_t max_iters,
                             int32_t wg_waves, unsigned flags, void *stream);

/* The blocked-JDS product y = alpha*A x + beta*y (as spmv_jds_blocked, same
 * arithmetic per row) launched from a tile plan (spmv_jds_blocked_tiles):
 * every workgroup takes one record, and the workgroups on XCD k walk range k
 * of the records in order.  For the windowed order this keeps each XCD on
 * neighbouring rows of the original matrix.  h_plan is the plan's h_plan[10].
 * Asynchronous; allocates nothing. */
spmv_status spmv_jds_blocked_tiled(int32_t n, const int32_t *perm, int32_t C, int32_t n_slices,
                                   const int64_t *slice_ptr, const int32_t *slice_nd, const int32_t *bl_col,
                                   const void *bl_val, spmv_dtype val_dt, const void *x, void *y,
                                   spmv_dtype vec_dt, double alpha, double beta, const int32_t *tiles,
                                   int64_t n_tiles, const int64_t *h_plan, int32_t unroll, unsigned flags,
                                   void *stream);
/* XCD-local tile plan of JDS storage for spmv_jds_tiled, built on the host
 * from h_jd_ptr (setup; synchronises when it copies the records).  The
 * length sort (stable) keeps the rows of one length in original order, and a
 * length class draws its rows from the whole matrix; dealt round robin, the
 * rows of one region of the matrix land on every XCD, each fetching that
 * region's band of x into its own L2.  Here each run of at least 1,024 rows
 * of one length is cut into 8 contiguous pieces, piece k for XCD k (one
 * eighth of those rows each, neighbours in the original order); every other
 * row group (rows longer than max_iters diagonals, in 64-row chunks wanting
 * the same split, and short runs) is dealt to the XCD with the least cost so
 * far, largest first.  R and S per group as in spmv_jds (R = rows_per_wave
 * when non-zero); records of (wg_waves / S) * R rows, two int32 each (first
 * row; R, S and row count packed); XCD k's range holds its dealt records in
 * row order, then its pieces.
 *   tiles: 2 * n_tiles int32 (device), written when tiles_cap >= 2 * n_tiles,
 *          otherwise SPMV_ERR_CAPACITY with *h_n_tiles set (two-call pattern)
 *   h_plan[10]: the 9 range bounds and the wavefronts per workgroup. */
spmv_status spmv_jds_tiles(int32_t n, const int32_t *h_jd_ptr, int32_t ndiag, int32_t max_iters, int32_t rows_per_wave,
                           int32_t wg_waves, int32_t *tiles, int64_t tiles_cap, int64_t *h_n_tiles, int64_t *h_plan,
                           void *stream);
/* The JDS product (as spmv_jds, same arithmetic per row for the same R and
 * S) launched from a tile plan (spmv_jds_tiles): the workgroups on XCD k walk
 * range k of the records in order.  Asynchronous; allocates nothing. */
spmv_status spmv_jds_tiled(int32_t n, const int32_t *perm, const int32_t *jd_ptr, int32_t ndiag, const int32_t *jd_col,
                           const void *jd_val, spmv_dtype val_dt, const void *x, void *y, spmv_dtype vec_dt,
                           double alpha, double beta, const int32_t *tiles, int64_t n_tiles, const int64_t *h_plan,
                           int32_t unroll, unsigned flags, void *stream);

/* Vector basis change: inverse == 0: out[r] = in[perm[r]] (to the permuted
 * basis); inverse != 0: out[perm[r]] = in[r].  dt F64 or F32. */
spmv_status spmv_permute_vec(int32_t n, const int32_t *perm, const void *in, void *out, spmv_dtype dt,
                             int inverse, void *stream);

/* out[i] = in[map[i]], i < n (e.g. A^T's values from tmap). */
spmv_status spmv_gather_values(int64_t n, const int32_t *map, const void *in, void *out, spmv_dtype dt,
                               void *stream);

/* y = alpha*x + beta*y (beta == 0 never reads y, alpha == 0 never reads x);
 * dt F64 or F32. */
spmv_status spmv_axpby(int64_t n, double alpha, const void *x, double beta, void *y, spmv_dtype dt,
                       void *stream);

/* *out (device double) = sum_i x_i*y_i in FP64, fixed summation tree.
 * ws: spmv_dot_workspace_size(n). */
size_t spmv_dot_workspace_size(int64_t n);
spmv_status spmv_dot(int64_t n, const void *x, const void *y, spmv_dtype dt, double *out, void *ws,
                     size_t ws_bytes, void *stream);

/* spmv_dot without a workspace, for callers that cannot allocate device
 * memory (code under HIP graph capture, tight serving loops, harnesses that
 * forbid allocation): the block partials go to a fixed array inside the
 * library (SPMV_DOT_NOALLOC_PARTS doubles, 256 KiB, one per GPU, held until
 * the process ends).  Same kernels and summation tree as spmv_dot, so the
 * result is bit-identical to it.  n > SPMV_DOT_NOALLOC_MAX_N returns
 * SPMV_ERR_CAPACITY before any device work.  The call allocates nothing and
 * does not synchronise.  Every call on one GPU shares that GPU's array:
 * calls whose executions overlap on one GPU (different streams, or graphs
 * replayed concurrently) race on it and give undefined results; calls
 * ordered on one stream are safe. */
#define SPMV_DOT_NOALLOC_PARTS 32768
#define SPMV_DOT_NOALLOC_MAX_N 134217728 /* SPMV_DOT_NOALLOC_PARTS * 4096 elements */
spmv_status spmv_dot_noalloc(int64_t n, const void *x, const void *y, spmv_dtype dt, double *out,
                             void *stream);

/* Multi-vector forms: Y[:, c] = alpha*A X[:, c] + beta*Y[:, c] for c < k,
 * X and Y column-major with leading dimensions ldx >= n_cols and ldy >= n
 * (the paper's kernels, each stored entry used for k right-hand sides).
 * ws (spmm_workspace_size(n_cols, k, vec_dt) bytes, may be NULL): with it,
 * X is first copied into an interleaved row-major block inside ws so that
 * every entry gathers its k values contiguously (k <= 64); without it the
 * kernels gather straight from the column-major X.  Same arithmetic rules as
 * the single-vector forms.  spmm_crs takes the spmv_crs_plan row blocks and
 * the block_nnz they were built with (0 = default; on the workspace path a
 * multi-row block's val/col are staged in LDS, block_nnz of each); spmm_jds
 * takes the host copy h_jd_ptr (needed on the workspace path). */
size_t spmm_workspace_size(int32_t n_cols, int32_t k, spmv_dtype vec_dt);
spmv_status spmm_crs(int32_t n_rows, int32_t n_cols, const int32_t *row_ptr, const int32_t *col_idx,
                     const void *val, spmv_dtype val_dt, int32_t k, const void *X, int64_t ldx, void *Y,
                     int64_t ldy, spmv_dtype vec_dt, double alpha, double beta, const int32_t *plan,
                     int32_t n_blocks, int32_t block_nnz, void *ws, size_t ws_bytes, void *stream);
spmv_status spmm_jds(int32_t n, int32_t n_cols, const int32_t *perm, const int32_t *jd_ptr,
                     const int32_t *h_jd_ptr, int32_t ndiag, const int32_t *jd_col, const void *jd_val,
                     spmv_dtype val_dt, int32_t k, const void *X, int64_t ldx, void *Y, int64_t ldy,
                     spmv_dtype vec_dt, double alpha, double beta, unsigned flags, void *ws,
                     size_t ws_bytes, void *stream);
/* Multi-vector product over blocked-JDS storage (paper Section 2, RBJDS),
 * either order: spmv_jds_blocked_from_jds (global length sort) or
 * spmv_jds_blocked_windowed_from_csr (sorted inside windows of sigma rows,
 * which keeps the rows an XCD works on neighbours in the original order, so
 * the X rows that banded entries gather stay in that XCD's L2).  X is staged
 * row-major into ws as for spmm_crs (ws required, 1 <= k <= 64), then a
 * group of min(K2, 8) lanes (K2 = k rounded up to a power of two) walks a
 * row's diagonals (deep slices: several groups per row, and several
 * wavefronts per row set, each on a contiguous range of diagonals, their
 * partial sums added in a fixed order); a record of the plan is one
 * 512-lane workgroup; the records are dealt to the XCDs in contiguous
 * ranges.  Same arithmetic rules as the other multi-vector forms
 * (rows of more than SPMV_WIDE_ROW_NNZ entries accumulate in FP64).
 * spmm_jds_blocked_plan (setup, synchronises) builds the plan on the host
 * from h_slice_nd for this k: 9 int32 range bounds, then 3 int32 per record
 * (first row, end row, and the lane groups per row and wavefronts per row
 * set chosen from the slice depth: groups double up to max_groups (1, 2, 4
 * or 8; 0 = 1), then wavefronts up to 8, until each lane has about 32
 * diagonals).  xcd_ranges != 0: range x holds about an eighth of the stored
 * work, in row order, and runs on XCD x (keeps a windowed order's rows
 * together); 0: the bounds are -1 and the hardware deals the records to the
 * XCDs in turn (balances a global length order).  *h_plan_words = the plan's
 * length, *h_grid = the workgroups to launch.  The plan is written to `plan` when plan_cap >= *h_plan_words,
 * otherwise SPMV_ERR_CAPACITY with both outputs set (two-call pattern).  It
 * depends on n, C, the slice depths and k rounded up to a power of two.
 * perm, C, n_slices, slice_ptr, slice_nd, bl_col, bl_val: the blocked
 * storage; Y[perm[r], c] receives permuted row r. */
spmv_status spmm_jds_blocked_plan(int32_t n, int32_t C, int32_t n_slices, const int32_t *h_slice_nd, int32_t k,
                                  int32_t max_groups, int32_t xcd_ranges, int32_t *plan, int32_t plan_cap,
                                  int32_t *h_plan_words, int32_t *h_grid, void *stream);
spmv_status spmm_jds_blocked(int32_t n, int32_t n_cols, const int32_t *perm, int32_t C, int32_t n_slices,
                             const int64_t *slice_ptr, const int32_t *slice_nd, const int32_t *bl_col,
                             const void *bl_val, spmv_dtype val_dt, int32_t k, const void *X, int64_t ldx, void *Y,
                             int64_t ldy, spmv_dtype vec_dt, double alpha, double beta, const int32_t *plan,
                             int32_t grid, void *ws, size_t ws_bytes, void *stream);

/* Value gradient of y = A x in JDS storage order:
 * dval[jd_ptr[d]+r] = alpha * g[row(r)] * x[jd_col[jd_ptr[d]+r]] + beta * dval[...]
 * with row(r) = perm[r] (original basis) or r (SPMV_SYMPERM).  Computed in
 * FP64 as (alpha*g[row])*x[col] and rounded once to dt (the value/vector
 * type, F64 or F32).  h_jd_ptr: host copy of jd_ptr (sizes the launch like
 * spmv_jds); nnz must equal jd_ptr[ndiag]. */
spmv_status spmv_grad_vals_jds(int32_t n, const int32_t *perm, const int32_t *jd_ptr,
                               const int32_t *h_jd_ptr, int32_t ndiag, int64_t nnz,
                               const int32_t *jd_col, const void *g, const void *x, void *dval,
                               spmv_dtype dt, double alpha, double beta, unsigned flags, void *stream);

/* ======================================================================== */
/* Column-split products                                                     */
/* ======================================================================== */
/* The paper (Section 2) names the irregular access to the input vector as
 * the bottleneck that its row blocking cannot remove.  These forms block the
 * columns instead: A = sum_k A_k, A_k holding the entries whose column lies
 * in [k*width, (k+1)*width), k < SPMV_SPLIT_PARTS (= the MI355X's 8 XCDs).
 * Part k is processed on XCD k, so its x gathers stay inside one 1/8 slice
 * of x that fits that XCD's L2.  A_k keeps only the rows that hold at least
 * one of its entries ("compressed rows", in ascending row order); each of
 * them owns one FP64 "slot" for its partial result.  The slots of row i are
 * slot_ptr[i] .. slot_ptr[i+1]-1, one per part present in the row, in part
 * order, and a last kernel forms y_i = alpha * (sum of row i's slots, in
 * slot order) + beta * y_i (deterministic).  Every part accumulates in FP64
 * whatever the value type (FP32 / BF16 values are widened exactly, FP32
 * vectors are read as stored): a part sees only a piece of each row, so the
 * rule "rows longer than SPMV_WIDE_ROW_NNZ entries accumulate in FP64" of
 * the unsplit calls could not be applied per part; FP64 throughout
 * satisfies it and the bound of the FP32 rule for the shorter rows.
 *
 * spmv_split_columns (setup, synchronises) reorders a CRS matrix part by
 * part.  With cap = min(nnz, SPMV_SPLIT_PARTS*n_rows):
 *   col_out[nnz], val_out[nnz]: part k's entries at h_bounds[k] ..
 *       h_bounds[k+1]-1, in CRS order;
 *   h_row_off[0..8]: part k's compressed rows are numbers h_row_off[k] ..
 *       h_row_off[k+1]-1; h_row_off[8] = n_slots (<= cap);
 *   row_ptr_all[cap + SPMV_SPLIT_PARTS]: part k's compressed row pointer,
 *       h_row_off[k+1]-h_row_off[k]+1 entries at row_ptr_all + h_row_off[k]
 *       + k, relative to h_bounds[k];
 *   dest_all[cap]: slot of each compressed row (part k's at dest_all +
 *       h_row_off[k]);
 *   slot_ptr[n_rows+1].
 * So part k is the CRS matrix (h_row_off[k+1]-h_row_off[k] rows, row_ptr_all +
 * h_row_off[k] + k, col_out + h_bounds[k], val_out + h_bounds[k]) whose row j
 * writes slot dest_all[h_row_off[k] + j].  width = 0 picks ceil(n_cols/8)
 * rounded up to 64.  Compute calls need ws of spmv_split_workspace_size(
 * n_slots) bytes for the slots; calls sharing one ws must not overlap. */
#define SPMV_SPLIT_PARTS 8
size_t spmv_split_columns_workspace_size(int32_t n_rows, int64_t nnz);
spmv_status spmv_split_columns(int32_t n_rows, int32_t n_cols, int64_t nnz, const int32_t *row_ptr,
                               const int32_t *col_idx, const void *val, spmv_dtype dt, int32_t width,
                               int32_t *row_ptr_all, int32_t *dest_all, int32_t *slot_ptr, int32_t *col_out,
                               void *val_out, int64_t *h_bounds, int64_t *h_row_off, void *ws, size_t ws_bytes,
                               void *stream);
size_t spmv_split_workspace_size(int64_t n_slots);
/* CRS parts as returned by spmv_split_columns; plan_all holds the
 * spmv_crs_plan of every part one after the other (part k's at plan_all +
 * h_plan_off[k], h_n_blocks[k] blocks, built with block_nnz). */
spmv_status spmv_crs_split(int32_t n_rows, int32_t n_cols, const int32_t *row_ptr_all, const int32_t *dest_all,
                           const int32_t *slot_ptr, const int32_t *col_idx, const void *val, const int64_t *h_bounds,
                           const int64_t *h_row_off, spmv_dtype val_dt, const int32_t *plan_all,
                           const int32_t *h_plan_off, const int32_t *h_n_blocks, int32_t block_nnz,
                           const void *x, void *y, spmv_dtype vec_dt, double alpha, double beta, void *ws,
                           size_t ws_bytes, void *stream);
/* JDS parts: part k is spmv_jds_from_csr of the CRS part k (without
 * SYMPERM) whose perm has been mapped through the part's dest entries, i.e.
 * h_perm[k][r] = dest_all[h_row_off[k] + perm_k[r]] is the slot of permuted
 * row r.  Host arrays of SPMV_SPLIT_PARTS device pointers (h_perm, h_jd_ptr,
 * h_jd_col, h_jd_val), of host pointers (h_jd_ptr_host) and of sizes
 * (h_ndiag).  unroll, max_iters and wg_waves as for spmv_jds (one value for
 * every part). */
spmv_status spmv_jds_split(int32_t n, const int32_t *slot_ptr, const int64_t *h_row_off, const int32_t *const *h_perm,
                           const int32_t *const *h_jd_ptr, const int32_t *const *h_jd_ptr_host, const int32_t *h_ndiag,
                           const int32_t *const *h_jd_col, const void *const *h_jd_val, spmv_dtype val_dt,
                           const void *x, void *y, spmv_dtype vec_dt, double alpha, double beta, int32_t unroll,
                           int32_t max_iters, int32_t wg_waves, void *ws, size_t ws_bytes, void *stream);
/* Blocked-JDS parts (slice height C for all parts), built from the JDS parts
 * above, so their perm gives slots too. */
spmv_status spmv_jds_blocked_split(int32_t n, int32_t C, const int32_t *slot_ptr, const int64_t *h_row_off,
                                   const int32_t *const *h_perm, const int64_t *const *h_slice_ptr,
                                   const int32_t *const *h_slice_nd, const int32_t *const *h_slice_nd_host,
                                   const int32_t *const *h_bl_col, const void *const *h_bl_val, spmv_dtype val_dt,
                                   const void *x, void *y, spmv_dtype vec_dt, double alpha, double beta,
                                   int32_t rows_per_wave, int32_t unroll, int32_t max_iters, int32_t wg_waves,
                                   void *ws, size_t ws_bytes, void *stream);

/* ======================================================================== */
/* Row-split products                                                        */
/* ======================================================================== */
/* The static row partition of the paper's shared-memory parallel SpMVM
 * (Section 5: each thread owns one contiguous block of rows, its pages
 * placed by first touch) with the MI355X's XCDs as the locality domains:
 * part k = rows [h_bounds[k], h_bounds[k+1]), k < SPMV_SPLIT_PARTS, is
 * stored in its own JDS or blocked-JDS form and processed on XCD k, so the
 * x entries near its diagonal stay in that XCD's L2.  Rows are complete in
 * their part: results go straight to y with the arithmetic of the unsplit
 * calls (including the SPMV_WIDE_ROW_NNZ rule), no workspace, no combine.
 *
 * spmv_split_rows (setup, synchronises) chooses the bounds by entries:
 * h_bounds[0] = 0, h_bounds[8] = n_rows and, for 0 < k < 8, h_bounds[k] is
 * the first row i with row_ptr[i] >= ceil(k*nnz/8) (k*n_rows/8 when nnz == 0).
 * h_entry_bounds[k] = row_ptr[h_bounds[k]].  row_ptr_parts[n_rows +
 * SPMV_SPLIT_PARTS] receives part k's row pointer, rebased to 0, as
 * h_bounds[k+1]-h_bounds[k]+1 entries at row_ptr_parts + h_bounds[k] + k, so
 * part k is the CRS matrix (h_bounds[k+1]-h_bounds[k] rows, row_ptr_parts +
 * h_bounds[k] + k, col_idx + h_entry_bounds[k], val + h_entry_bounds[k]).
 * ws: spmv_split_rows_workspace_size() bytes. */
size_t spmv_split_rows_workspace_size(void);
spmv_status spmv_split_rows(int32_t n_rows, int64_t nnz, const int32_t *row_ptr, int32_t *row_ptr_parts,
                            int64_t *h_bounds, int64_t *h_entry_bounds, void *ws, size_t ws_bytes, void *stream);
/* JDS parts: part k is spmv_jds_from_csr of CRS part k (without SYMPERM);
 * its perm holds row numbers local to the part, and permuted row r of part k
 * writes y[h_bounds[k] + h_perm[k][r]].  Host arrays of SPMV_SPLIT_PARTS
 * device pointers (h_perm, h_jd_ptr, h_jd_col, h_jd_val), of host pointers
 * (h_jd_ptr_host) and of sizes (h_ndiag).  x is in the original basis.
 * unroll, max_iters and wg_waves as for spmv_jds (one value for every part). */
spmv_status spmv_jds_row_split(int32_t n, const int64_t *h_bounds, const int32_t *const *h_perm,
                               const int32_t *const *h_jd_ptr, const int32_t *const *h_jd_ptr_host,
                               const int32_t *h_ndiag, const int32_t *const *h_jd_col, const void *const *h_jd_val,
                               spmv_dtype val_dt, const void *x, void *y, spmv_dtype vec_dt, double alpha,
                               double beta, int32_t unroll, int32_t max_iters, int32_t wg_waves, void *stream);
/* Blocked-JDS parts (slice height C for all parts), built from the JDS parts
 * above. */
spmv_status spmv_jds_blocked_row_split(int32_t n, int32_t C, const int64_t *h_bounds, const int32_t *const *h_perm,
                                       const int64_t *const *h_slice_ptr, const int32_t *const *h_slice_nd,
                                       const int32_t *const *h_slice_nd_host, const int32_t *const *h_bl_col,
                                       const void *const *h_bl_val, spmv_dtype val_dt, const void *x, void *y,
                                       spmv_dtype vec_dt, double alpha, double beta, int32_t rows_per_wave,
                                       int32_t unroll, int32_t max_iters, int32_t wg_waves, void *stream);

/* ======================================================================== */
/* DIA + CRS hybrid                                                          */
/* ======================================================================== */
/* The paper (Section 4.2) notes that the outer secondary diagonals of its
 * Hamiltonian hold most of the entries and could be stored densely.  Here a
 * diagonal (offset o = col - row) is stored densely when that costs no more
 * bytes than its entries in CRS: count_o * (s_v + 4) >= span_o * s_v, with
 * span_o the rows the diagonal crosses; at most max_diags of them (0 =
 * SPMV_DIA_MAX), the fullest first (ties: smaller offset).  Stored diagonals
 * are in ascending offset order; diagonal k holds dia_val[k*n_rows + i] =
 * a(i, i + offsets[k]) for every row i (0 where the matrix has no entry or
 * the column falls outside the matrix).  The other entries form the
 * remainder CRS (rem_row_ptr[n_rows+1], rem_col, rem_val: each row's
 * entries in CRS order).
 * spmv_dia_from_csr (setup, synchronises): with dia_val == NULL it only
 * returns *h_ndia, h_offsets[0..*h_ndia) and *h_rem_nnz; otherwise it also
 * fills dia_val (*h_ndia * n_rows values of dt), rem_row_ptr, rem_col and
 * rem_val (*h_rem_nnz entries).  ws: spmv_dia_workspace_size(n_rows, n_cols). */
#define SPMV_DIA_MAX 64
size_t spmv_dia_workspace_size(int32_t n_rows, int32_t n_cols);
spmv_status spmv_dia_from_csr(int32_t n_rows, int32_t n_cols, int64_t nnz, const int32_t *row_ptr,
                              const int32_t *col_idx, const void *val, spmv_dtype dt, int32_t max_diags,
                              int32_t *h_offsets, int32_t *h_ndia, int64_t *h_rem_nnz, void *dia_val,
                              int32_t *rem_row_ptr, int32_t *rem_col, void *rem_val, void *ws, size_t ws_bytes,
                              void *stream);
/* y = alpha * A x + beta * y over the hybrid: each lane owns one row, reads
 * its value of every stored diagonal (consecutive rows: consecutive values
 * and consecutive x) and then its remainder entries.  A row sums its
 * diagonals in offset order, then its remainder entries, in FP64 for every
 * value type (at most SPMV_DIA_MAX + remainder terms; the FP64 sum meets the
 * bound of the reduced-precision rule); y is rounded to vec_dt once.  Zeros
 * stored inside a diagonal are multiplied like entries (an Inf or NaN in x
 * reaches those rows).  rem_row_ptr may be NULL when the remainder is empty.
 * One lane walks a row's whole remainder, so the hybrid is meant for short
 * remainder rows: a row with many remainder entries holds up its wavefront
 * (and, in window-sorted slices, pads its slice to its length).
 * h_offsets: host copy of the ndia offsets. */
spmv_status spmv_dia(int32_t n_rows, int32_t n_cols, int32_t ndia, const int32_t *h_offsets, const void *dia_val,
                     spmv_dtype val_dt, const int32_t *rem_row_ptr, const int32_t *rem_col, const void *rem_val,
                     const void *x, void *y, spmv_dtype vec_dt, double alpha, double beta, void *stream);
/* Symmetric storage of the stored diagonals (the paper, Section 4.2, notes
 * that its Hamiltonian is symmetric and that storing one triangle would
 * halve the matrix).  For a square n x n matrix whose entries on the chosen
 * diagonals are symmetric (a(i, i+o) == a(i+o, i)): only offsets o >= 0 are
 * stored, diagonal k holding dia_val[k*n + i] = a(i, i + o_k); a diagonal is
 * chosen when (count_o + count_-o) * (s_v + 4) >= span_o * s_v, at most
 * max_diags, fullest first.  The entries below the main diagonal on a chosen
 * diagonal's mirror are not read: they are taken to equal their mirrors.
 * The remainder CRS holds every entry on neither a chosen diagonal nor its
 * mirror (both triangles, CRS order).  Same calling pattern, workspace and
 * outputs as spmv_dia_from_csr.  The stored diagonal bytes are half those of
 * spmv_dia_from_csr on a matrix of symmetric pairs of diagonals. */
spmv_status spmv_dia_sym_from_csr(int32_t n, int64_t nnz, const int32_t *row_ptr, const int32_t *col_idx,
                                  const void *val, spmv_dtype dt, int32_t max_diags, int32_t *h_offsets,
                                  int32_t *h_ndia, int64_t *h_rem_nnz, void *dia_val, int32_t *rem_row_ptr,
                                  int32_t *rem_col, void *rem_val, void *ws, size_t ws_bytes, void *stream);
/* y = alpha * A x + beta * y over the symmetric hybrid: row i adds
 * dia[k][i] * x[i + o_k] for every stored diagonal (offset order), then
 * dia[k][i - o_k] * x[i - o_k] for every o_k > 0 with i >= o_k (offset
 * order), then its remainder entries; FP64 sums, one rounding of y.  Every
 * term is a gather-free contiguous read (the mirror is the same diagonal
 * shifted by o_k rows), so no row writes another row's y: deterministic,
 * no atomics.  Offsets must be >= 0, increasing, < n. */
spmv_status spmv_dia_sym(int32_t n, int32_t ndia, const int32_t *h_offsets, const void *dia_val, spmv_dtype val_dt,
                         const int32_t *rem_row_ptr, const int32_t *rem_col, const void *rem_val, const void *x,
                         void *y, spmv_dtype vec_dt, double alpha, double beta, void *stream);

/* Remainder in window-sorted slices.  The paper (Section 2) stores RBJDS
 * blocks of length-sorted rows together, diagonal by diagonal.  The DIA
 * hybrid's remainder takes that layout with the sort confined to windows of
 * SPMV_REM_WINDOW rows (the rows one workgroup of the DIA kernel owns), so a
 * wavefront's loads of the d-th remainder entries are contiguous and the
 * padding stays small, while the permutation never leaves the workgroup.
 * spmv_csr_to_slices (setup, synchronises): window w holds rows
 * [256 w, 256 w + 256); its rows in decreasing length order (ties: lower row
 * first) fill sorted positions 256 w + t, and slot_row[256 w + t] (uint8) is
 * the window-local index of the row at position t.  Slices are
 * SPMV_REM_SLICE = 16 consecutive positions: slice s holds slice_nd[s] = the
 * length of its first (longest) row and occupies slots
 * [slice_ptr[s], slice_ptr[s] + 16 * slice_nd[s]); entry d (CRS order) of the
 * row at position p sits at slice_ptr[p / 16] + 16 d + p % 16; padding has
 * col = -1 and value 0 (also in the positions past n_rows of the last
 * slice).  slice_ptr[n_slices + 1] (int64), slice_nd[n_slices],
 * slot_row[n_rows], n_slices = ceil(n_rows / 16).  With bl_col == NULL only
 * slice_ptr, slice_nd, slot_row and *h_padded are written; bl_cap <
 * *h_padded gives SPMV_ERR_CAPACITY.  Any payload dtype (moved bit for bit).
 * ws: spmv_csr_slices_workspace_size(n_rows). */
#define SPMV_REM_WINDOW 256
#define SPMV_REM_SLICE 16
size_t spmv_csr_slices_workspace_size(int32_t n_rows);
spmv_status spmv_csr_to_slices(int32_t n_rows, const int32_t *row_ptr, const int32_t *col_idx, const void *val,
                               spmv_dtype dt, int64_t *slice_ptr, int32_t *slice_nd, uint8_t *slot_row,
                               int32_t *bl_col, void *bl_val, int64_t bl_cap, int64_t *h_padded, void *ws,
                               size_t ws_bytes, void *stream);
/* The DIA hybrid (symmetric = 0: spmv_dia; 1: spmv_dia_sym storage) with its
 * remainder in window-sorted slices (spmv_csr_to_slices of the remainder
 * CRS).  Each lane first sums its row's stored diagonals, the workgroup puts
 * the partial sums in LDS, and the lane at sorted position p continues the
 * sum of row slot_row[p] with that row's remainder entries, so every row is
 * still one FP64 sum in the order of spmv_dia / spmv_dia_sym (its diagonals,
 * then its remainder in CRS order): the result is bit-identical to them.
 * rem_slice_ptr may be NULL when the remainder is empty; otherwise
 * rem_slice_nd, rem_slot_row, rem_col, rem_val and x must be given
 * (SPMV_ERR_INVALID_ARG).  Offsets, dtypes and sizes follow spmv_dia
 * (symmetric = 1: spmv_dia_sym, and n_rows must equal n_cols).
 * Asynchronous; allocates nothing. */
spmv_status spmv_dia_sliced(int32_t n_rows, int32_t n_cols, int32_t ndia, const int32_t *h_offsets,
                            const void *dia_val, spmv_dtype val_dt, const int64_t *rem_slice_ptr,
                            const int32_t *rem_slice_nd, const uint8_t *rem_slot_row, const int32_t *rem_col,
                            const void *rem_val, const void *x, void *y, spmv_dtype vec_dt, double alpha, double beta,
                            int symmetric, void *stream);

/* ======================================================================== */
/* One-triangle CRS of a symmetric matrix                                    */
/* ======================================================================== */
/* The paper (Section 4.2) notes that its Hamiltonian is symmetric, so an
 * SpMV could move less data by storing one triangle; it does not try this.
 * Here a symmetric n x n matrix is stored as its upper triangle U (entries
 * with col >= row, each row in CRS order): A = U + U^T - diag(U), about half
 * the entries of the full CRS.
 * spmv_csr_upper_from_csr (setup, synchronises): from a full CRS matrix
 * (row_ptr[n+1], col_idx/val: nnz entries of dt, any payload dtype including
 * SPMV_I32, copied bit for bit) keeps the entries with col >= row.  Entries
 * below the diagonal are dropped without being read, so the matrix is taken
 * to be symmetric, not checked.  With up_row_ptr == NULL it only returns
 * *h_nnz_upper; otherwise it also fills up_row_ptr[n+1], up_col and up_val
 * (*h_nnz_upper entries).  ws: spmv_csr_upper_workspace_size(n) bytes. */
size_t spmv_csr_upper_workspace_size(int32_t n);
spmv_status spmv_csr_upper_from_csr(int32_t n, int64_t nnz, const int32_t *row_ptr, const int32_t *col_idx,
                                    const void *val, spmv_dtype dt, int64_t *h_nnz_upper, int32_t *up_row_ptr,
                                    int32_t *up_col, void *up_val, void *ws, size_t ws_bytes, void *stream);
/* y = alpha * (U + U^T - diag U) x + beta * y from the upper triangle:
 * row_ptr/col_idx/val hold U (every col >= its row; val F64, F32 or BF16);
 * x and y are FP64 (vec_dt must be SPMV_F64, else SPMV_ERR_UNSUPPORTED).
 * plan/n_blocks/block_nnz: spmv_crs_plan run on U's row_ptr with this
 * block_nnz (0 = default); a plan made with another block_nnz is an error the
 * library cannot see.  Two launches on `stream`: y = beta*y (beta == 0 writes
 * zeros without reading y), then one pass over U in which each entry
 * (i, j, a) is read once and serves row i (a*x_j, summed in FP64 per row and
 * added to y_i once) and, for j > i, row j (alpha*a*x_i added to y_j).  The
 * adds into y use device-scope FP64 atomics: every y_i is a sum of its terms
 * in an order that varies between runs (not bit-reproducible; the error
 * bound of an FP64 sum of row-length + 1 terms holds for every order). */
spmv_status spmv_crs_sym(int32_t n, const int32_t *row_ptr, const int32_t *col_idx, const void *val,
                         spmv_dtype val_dt, const void *x, void *y, spmv_dtype vec_dt, double alpha, double beta,
                         const int32_t *plan, int32_t n_blocks, int32_t block_nnz, void *stream);

/* One triangle, staged (paper Section 4.2, symmetric storage): the product of
 * spmv_crs_sym with the gathers and the mirrored-term atomics issued in row
 * order, as spmv_crs_staged issues its gathers: a block's col/val are copied
 * to LDS, then G lanes per row (one lane per row above 256 rows) walk the
 * row's entries, so that a wavefront's atomic adds target neighbouring y
 * elements on banded and diagonal patterns.  Arguments, dtypes, plan
 * requirements (multi-row blocks hold at most block_nnz entries), errors and
 * the atomic (not bit-reproducible) summation as for spmv_crs_sym.
 * Asynchronous. */
spmv_status spmv_crs_sym_staged(int32_t n, const int32_t *row_ptr, const int32_t *col_idx, const void *val,
                                spmv_dtype val_dt, const void *x, void *y, spmv_dtype vec_dt, double alpha,
                                double beta, const int32_t *plan, int32_t n_blocks, int32_t block_nnz,
                                void *stream);

/* ======================================================================== */
/* Many matrices in one launch                                               */
/* ======================================================================== */
/* Batched blocked-JDS SpMV: y_m = A_m x_m for m < n_mat, F32 values and
 * vectors, each matrix in blocked-JDS storage (spmv_jds_blocked_from_jds)
 * inside shared arrays:
 *   matrix m has h_n_rows[m] rows and slice height h_C[m] (multiple of 64);
 *   its slices are entries h_slice_base[m] .. + ceil(n_m / C_m) - 1 of the
 *   host copies h_slice_ptr (ABSOLUTE offsets into bl_col / bl_val) and
 *   h_slice_nd;  its rows are y[h_row_base[m] .. + n_m) and its permutation
 *   perm[h_row_base[m] .. + n_m) (local row numbers);  its columns index
 *   x[h_col_base[m] + col].
 * spmv_batched_plan cuts every matrix into tiles of rows_per_wave rows (8,
 * 16, 32 or 64; 0 = 64), orders the matrices by stored slots, largest first
 * (stable), keeps each matrix's tiles together in row order and writes
 * SPMV_BATCHED_PLAN_WORDS int32 per tile into the device array `plan`
 * (capacity plan_cap int32); *h_n_tiles returns the tile count; if the
 * capacity is too small returns SPMV_ERR_CAPACITY.  Synchronises.
 * spmv_batched runs all tiles in one persistent launch of n_workgroups
 * 256-lane workgroups (0 = 8 per compute unit; rounded to a multiple of 8):
 * each XCD walks one contiguous eighth of the table with a fixed wavefront
 * stride, so results are deterministic and the launch is capturable in a
 * HIP graph.
 * unroll: diagonals per trip (2, 4 or 8; 0 = 4). */
#define SPMV_BATCHED_PLAN_WORDS 12
spmv_status spmv_batched_plan(int32_t n_mat, const int32_t *h_n_rows, const int32_t *h_C,
                              const int64_t *h_slice_base, const int64_t *h_row_base,
                              const int64_t *h_col_base, const int64_t *h_slice_ptr,
                              const int32_t *h_slice_nd, int32_t rows_per_wave, int32_t *plan,
                              int64_t plan_cap, int64_t *h_n_tiles, void *stream);
spmv_status spmv_batched(int64_t n_tiles, const int32_t *plan, const int32_t *perm, const int32_t *bl_col,
                         const float *bl_val, const float *x, float *y, int32_t unroll,
                         int32_t n_workgroups, void *stream);

/* ======================================================================== */
/* HIP graph helpers (capture of compute calls issued on `stream`)            */
/* ======================================================================== */
spmv_status spmv_graph_begin(void *stream);
/* Ends the capture and instantiates it; *h_exec receives the handle. */
spmv_status spmv_graph_end(void *stream, void **h_exec);
spmv_status spmv_graph_launch(void *exec, void *stream);
spmv_status spmv_graph_destroy(void *exec);

/* ======================================================================== */
/* Bandwidth probes (attainable HBM bandwidth for the rooflines; the paper's  */
/* STREAM triad figures play this role for its CPUs)                          */
/* ======================================================================== */
/* a[i] = b[i] + s*c[i];  a[i] = b[i];  part[w] = sum of the elements read by
 * workgroup w.  n even, arrays 16-byte aligned; spmv_stream_read needs
 * part_cap >= 8 * (compute units) doubles. */
spmv_status spmv_stream_triad(int64_t n, const double *b, const double *c, double *a, double s,
                              void *stream);
spmv_status spmv_stream_copy(int64_t n, const double *b, double *a, void *stream);
spmv_status spmv_stream_read(int64_t n, const double *b, double *part, int64_t part_cap, void *stream);
/* Random-gather probe: part[w] = sum of x[idx[i]] over the i read by
 * workgroup w (idx streamed, one 8-byte x element gathered per index; every
 * idx[i] must index x).  Timed with x sized to fit one XCD's L2, the MALL or
 * only HBM, it gives the gather rate that bounds an SpMV whose x accesses
 * are irregular (paper Section 2: the x access is the limiting factor the
 * code balance leaves out).  part_cap >= 8 * (compute units) doubles. */
spmv_status spmv_gather_probe(int64_t n, const int32_t *idx, const double *x, double *part, int64_t part_cap,
                              void *stream);
/* The basic sparse vector operations of the paper's Section 4.1 (Table 1):
 * for i < n, s += b[j(i)] (scp == 0: PDADD / CSADD / ISADD / IRADD) or
 * s += a[i] * b[j(i)] (scp != 0: the ..SCP forms), with j(i) = k*i when ind
 * is NULL (k = 1 dense, k > 1 constant stride) and j(i) = ind[i] otherwise
 * (indirect: constant or random strides); part[w] receives workgroup w's
 * sum.  Every j(i) must index b (b holds at least k*(n-1)+1 doubles when ind
 * is NULL) and a holds n doubles; part_cap >= 8 * (compute units). */
spmv_status spmv_stride_probe(int64_t n, int32_t scp, const double *a, const double *b, const int32_t *ind, int64_t k,
                              double *part, int64_t part_cap, void *stream);

#ifdef __cplusplus
}
#endif
#endif /* SPMV_H */
