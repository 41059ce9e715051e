/*
 * Plain serial FP64 oracle for the CRS / JDS sparse matrix-vector library.
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product path may call this code:
 * only the tests, the smoke check and the benchmark's CPU-baseline leg load it.
 * It shares no source, header or table with the HIP library; the two meet only
 * through the seeded inputs of the synthetic-matrix module.
 *
 * Every routine is the plain definition of what it computes, in the order the
 * paper states it (Schubert, Hager, Fehske, "Performance limitations for sparse
 * matrix-vector multiplications on current multicore environments").  Built
 * with -O2 -ffp-contract=off so that a*b+c is a rounded product followed by a
 * rounded sum, never a fused multiply-add.
 *
 * Indices are 0-based (the paper's listings are 1-based Fortran).
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

typedef int32_t i32;
typedef int64_t i64;

/* ------------------------------------------------------------------------ */
/* CRS: paper Section 2, the CRS kernel listing.                              */

/* y[i] = alpha * sum_{j in row i} val[j]*x[col[j]] + beta * y[i].
 * The row sum runs left to right over the stored entries, starting at 0.
 * beta == 0 never reads y (so NaN garbage in y is ignored). */
void orc_spmv_crs(i32 n_rows, const i32 *row_ptr, const i32 *col, const double *val,
                  const double *x, double *y, double alpha, double beta)
{
    for (i32 i = 0; i < n_rows; ++i) {
        double s = 0.0;
        for (i32 j = row_ptr[i]; j < row_ptr[i + 1]; ++j)
            s = s + val[j] * x[col[j]];
        if (beta == 0.0)
            y[i] = alpha * s;
        else
            y[i] = alpha * s + beta * y[i];
    }
}

/* Row scale for the error metric: D[i] = sum_j |val[j]| * |x[col[j]]|. */
void orc_row_absdot(i32 n_rows, const i32 *row_ptr, const i32 *col, const double *val,
                    const double *x, double *D)
{
    for (i32 i = 0; i < n_rows; ++i) {
        double s = 0.0;
        for (i32 j = row_ptr[i]; j < row_ptr[i + 1]; ++j)
            s = s + fabs(val[j]) * fabs(x[col[j]]);
        D[i] = s;
    }
}

/* Multi-RHS: Y[:, c] = alpha*A*X[:, c] + beta*Y[:, c], column-major blocks. */
void orc_spmm_crs(i32 n_rows, const i32 *row_ptr, const i32 *col, const double *val,
                  i32 k, const double *X, i64 ldx, double *Y, i64 ldy, double alpha, double beta)
{
    for (i32 c = 0; c < k; ++c)
        orc_spmv_crs(n_rows, row_ptr, col, val, X + (i64)c * ldx, Y + (i64)c * ldy, alpha, beta);
}

/* ------------------------------------------------------------------------ */
/* COO -> CRS.  The paper's CRS definition (Section 2): per row, the values and
 * column indices of its entries, and row_ptr giving where each row starts.
 * Reading for unspecified points: entries sorted by (row, col); duplicate
 * (row, col) pairs are summed in input order; explicit zeros are kept. */

typedef struct { i32 r, c; i64 k; } coo_key;

static int coo_cmp(const void *pa, const void *pb)
{
    const coo_key *a = (const coo_key *)pa, *b = (const coo_key *)pb;
    if (a->r != b->r) return a->r < b->r ? -1 : 1;
    if (a->c != b->c) return a->c < b->c ? -1 : 1;
    if (a->k != b->k) return a->k < b->k ? -1 : 1;
    return 0;
}

/* Returns the number of stored entries, or -1 if an index is out of range. */
i64 orc_csr_from_coo(i32 n_rows, i32 n_cols, i64 nnz, const i32 *row, const i32 *col,
                     const double *val, i32 *row_ptr, i32 *col_out, double *val_out)
{
    for (i64 k = 0; k < nnz; ++k)
        if (row[k] < 0 || row[k] >= n_rows || col[k] < 0 || col[k] >= n_cols)
            return -1;
    coo_key *keys = (coo_key *)malloc(sizeof(coo_key) * (size_t)(nnz > 0 ? nnz : 1));
    for (i64 k = 0; k < nnz; ++k) {
        keys[k].r = row[k];
        keys[k].c = col[k];
        keys[k].k = k;
    }
    qsort(keys, (size_t)nnz, sizeof(coo_key), coo_cmp);
    for (i32 i = 0; i <= n_rows; ++i) row_ptr[i] = 0;
    i64 out = 0;
    for (i64 k = 0; k < nnz; ++k) {
        if (out > 0 && keys[k].r == keys[k - 1].r && keys[k].c == keys[k - 1].c) {
            val_out[out - 1] = val_out[out - 1] + val[keys[k].k];
        } else {
            col_out[out] = keys[k].c;
            val_out[out] = val[keys[k].k];
            row_ptr[keys[k].r + 1] += 1;
            ++out;
        }
    }
    for (i32 i = 0; i < n_rows; ++i) row_ptr[i + 1] += row_ptr[i];
    free(keys);
    return out;
}

/* ------------------------------------------------------------------------ */
/* JDS: paper Section 2.  Rows are permuted so that row length decreases with
 * the new row index; every row's entries are shifted left (kept in their CRS
 * order); the d-th entries of all rows that have one form jagged diagonal d,
 * stored one after another; jd_ptr[d] is where diagonal d starts.
 *
 * perm[r] = original row of permuted row r; equal lengths keep ascending
 * original index (stable).  iperm is the inverse.  With symperm != 0 the
 * columns are renumbered too (jd_col = iperm[col]), the paper's A_{p(i),p(j)};
 * otherwise columns keep the original numbering.
 *
 * Returns ndiag = max row length, or -(ndiag+1)-1 if jd_ptr_cap < ndiag+1. */

typedef struct { i32 len, row; } len_key;

static int len_cmp(const void *pa, const void *pb)
{
    const len_key *a = (const len_key *)pa, *b = (const len_key *)pb;
    if (a->len != b->len) return a->len > b->len ? -1 : 1;   /* descending length */
    if (a->row != b->row) return a->row < b->row ? -1 : 1;   /* then ascending row */
    return 0;
}

i32 orc_jds_from_csr(i32 n, const i32 *row_ptr, const i32 *col, const double *val, int symperm,
                     i32 *perm, i32 *iperm, i32 *jd_ptr, i32 jd_ptr_cap, i32 *jd_col, double *jd_val)
{
    len_key *keys = (len_key *)malloc(sizeof(len_key) * (size_t)(n > 0 ? n : 1));
    i32 ndiag = 0;
    for (i32 i = 0; i < n; ++i) {
        keys[i].len = row_ptr[i + 1] - row_ptr[i];
        keys[i].row = i;
        if (keys[i].len > ndiag) ndiag = keys[i].len;
    }
    if (jd_ptr_cap < ndiag + 1) {
        free(keys);
        return -(ndiag + 1) - 1;
    }
    qsort(keys, (size_t)n, sizeof(len_key), len_cmp);
    for (i32 r = 0; r < n; ++r) {
        perm[r] = keys[r].row;
        iperm[keys[r].row] = r;
    }
    /* diagonal d holds one entry for every row longer than d; rows are sorted,
     * so those are the permuted rows 0 .. count-1 */
    jd_ptr[0] = 0;
    for (i32 d = 0; d < ndiag; ++d) {
        i32 count = 0;
        while (count < n && keys[count].len > d) count++;   /* lengths descend */
        jd_ptr[d + 1] = jd_ptr[d] + count;
    }
    for (i32 d = 0; d < ndiag; ++d) {
        i32 count = jd_ptr[d + 1] - jd_ptr[d];
        for (i32 r = 0; r < count; ++r) {
            i32 src = row_ptr[perm[r]] + d;
            jd_col[jd_ptr[d] + r] = symperm ? iperm[col[src]] : col[src];
            jd_val[jd_ptr[d] + r] = val[src];
        }
    }
    free(keys);
    return ndiag;
}

/* Inverse of the above (without symperm): back to CRS in the original row
 * order, in-row order = diagonal order. */
void orc_jds_to_csr(i32 n, const i32 *perm, const i32 *jd_ptr, i32 ndiag, const i32 *jd_col,
                    const double *jd_val, i32 *row_ptr, i32 *col, double *val)
{
    for (i32 i = 0; i <= n; ++i) row_ptr[i] = 0;
    for (i32 d = 0; d < ndiag; ++d)
        for (i32 r = 0; r < jd_ptr[d + 1] - jd_ptr[d]; ++r)
            row_ptr[perm[r] + 1] += 1;
    for (i32 i = 0; i < n; ++i) row_ptr[i + 1] += row_ptr[i];
    for (i32 d = 0; d < ndiag; ++d)
        for (i32 r = 0; r < jd_ptr[d + 1] - jd_ptr[d]; ++r) {
            i32 dst = row_ptr[perm[r]] + d;
            col[dst] = jd_col[jd_ptr[d] + r];
            val[dst] = jd_val[jd_ptr[d] + r];
        }
}

/* Store the permuted-basis result back: y[perm[r]] = alpha*res[r] + beta*y[perm[r]]
 * (original basis) or y[r] = ... (symperm: x and y are both in the permuted basis). */
static void jds_store(i32 n, const i32 *perm, int symperm, const double *res, double *y,
                      double alpha, double beta)
{
    for (i32 r = 0; r < n; ++r) {
        i32 t = symperm ? r : perm[r];
        if (beta == 0.0)
            y[t] = alpha * res[r];
        else
            y[t] = alpha * res[r] + beta * y[t];
    }
}

/* Plain JDS kernel (paper Section 2, the JDS listing): for each jagged diagonal,
 * for every row it reaches, resvec(row) += val * invec(col).  The result vector
 * starts at zero.  Row r then sums its entries in diagonal order, which is its
 * CRS order, so this equals orc_spmv_crs in the permuted basis bit for bit. */
void orc_spmv_jds(i32 n, const i32 *perm, const i32 *jd_ptr, i32 ndiag, const i32 *jd_col,
                  const double *jd_val, const double *x, double *y, double alpha, double beta,
                  int symperm)
{
    double *res = (double *)calloc((size_t)(n > 0 ? n : 1), sizeof(double));
    for (i32 d = 0; d < ndiag; ++d) {
        i32 len = jd_ptr[d + 1] - jd_ptr[d];
        i32 off = jd_ptr[d];
        for (i32 r = 0; r < len; ++r)
            res[r] = res[r] + jd_val[off + r] * x[jd_col[off + r]];
    }
    jds_store(n, perm, symperm, res, y, alpha, beta);
    free(res);
}

/* NUJDS (paper Section 2): outer-loop unrolling, each result element updated by
 * `unroll` consecutive jagged diagonals in one sweep.  Per row the additions
 * still happen in diagonal order. */
void orc_spmv_nujds(i32 n, const i32 *perm, const i32 *jd_ptr, i32 ndiag, const i32 *jd_col,
                    const double *jd_val, const double *x, double *y, double alpha, double beta,
                    int symperm, i32 unroll)
{
    double *res = (double *)calloc((size_t)(n > 0 ? n : 1), sizeof(double));
    for (i32 d0 = 0; d0 < ndiag; d0 += unroll) {
        i32 dend = d0 + unroll < ndiag ? d0 + unroll : ndiag;
        i32 len0 = jd_ptr[d0 + 1] - jd_ptr[d0];       /* the longest of the group */
        for (i32 r = 0; r < len0; ++r)
            for (i32 d = d0; d < dend; ++d)
                if (r < jd_ptr[d + 1] - jd_ptr[d])
                    res[r] = res[r] + jd_val[jd_ptr[d] + r] * x[jd_col[jd_ptr[d] + r]];
    }
    jds_store(n, perm, symperm, res, y, alpha, beta);
    free(res);
}

/* NBJDS (paper Section 2): the diagonals are cut into blocks of `block` rows;
 * each block is finished for all diagonals that reach it before the next
 * block starts, skipping through val/col_idx of the unchanged JDS storage. */
void orc_spmv_nbjds(i32 n, const i32 *perm, const i32 *jd_ptr, i32 ndiag, const i32 *jd_col,
                    const double *jd_val, const double *x, double *y, double alpha, double beta,
                    int symperm, i32 block)
{
    double *res = (double *)calloc((size_t)(n > 0 ? n : 1), sizeof(double));
    for (i32 b0 = 0; b0 < n; b0 += block) {
        i32 b1 = b0 + block < n ? b0 + block : n;
        for (i32 d = 0; d < ndiag; ++d) {
            i32 len = jd_ptr[d + 1] - jd_ptr[d];
            if (len <= b0) break;                    /* diagonals only get shorter */
            i32 end = len < b1 ? len : b1;
            for (i32 r = b0; r < end; ++r)
                res[r] = res[r] + jd_val[jd_ptr[d] + r] * x[jd_col[jd_ptr[d] + r]];
        }
    }
    jds_store(n, perm, symperm, res, y, alpha, beta);
    free(res);
}

/* ------------------------------------------------------------------------ */
/* RBJDS / SOJDS storage (paper Section 2): all elements of a block of C
 * consecutive permuted rows are stored together.  Reading: inside a block the
 * order is diagonal by diagonal (so block size 1 is row by row, and one block
 * of n rows is plain JDS); every block is padded to its first (longest) row,
 * padded slots hold col = -1 and val = 0 and are skipped.
 *   slice_ptr[s] = start of block s (slice_ptr[n_slices] = padded total)
 *   slice_nd[s]  = number of diagonals in block s
 *   element (d, row r of block s) lives at slice_ptr[s] + d*C + (r - s*C).
 * With sojds != 0 the entries inside each row are re-assigned to diagonal
 * slots: the first row of a block keeps its order; every following row, slot
 * by slot, takes from its not-yet-placed entries the one whose column is
 * closest to (previous row's column in that slot) + 1, the smaller column on a
 * tie.  Returns the padded total. */
i64 orc_jds_blocked_from_jds(i32 n, const i32 *jd_ptr, i32 ndiag, const i32 *jd_col,
                             const double *jd_val, i32 C, int sojds, i64 *slice_ptr,
                             i32 *slice_nd, i32 *bl_col, double *bl_val)
{
    i32 n_slices = (n + C - 1) / C;
    i64 total = 0;
    for (i32 s = 0; s < n_slices; ++s) {
        i32 first = s * C;
        i32 nd = 0;                       /* length of the block's first row */
        while (nd < ndiag && jd_ptr[nd + 1] - jd_ptr[nd] > first) nd++;
        slice_ptr[s] = total;
        slice_nd[s] = nd;
        total += (i64)nd * C;
    }
    slice_ptr[n_slices] = total;
    i32 *taken = NULL;
    if (sojds) taken = (i32 *)malloc(sizeof(i32) * (size_t)(ndiag > 0 ? ndiag : 1));
    for (i32 s = 0; s < n_slices; ++s) {
        for (i32 rl = 0; rl < C; ++rl) {
            i32 r = s * C + rl;
            i32 len = 0;                  /* diagonals that reach row r */
            if (r < n)
                while (len < ndiag && jd_ptr[len + 1] - jd_ptr[len] > r) len++;
            if (sojds && r < n) for (i32 d = 0; d < len; ++d) taken[d] = 0;
            for (i32 d = 0; d < slice_nd[s]; ++d) {
                i64 dst = slice_ptr[s] + (i64)d * C + rl;
                if (d >= len) {
                    bl_col[dst] = -1;
                    bl_val[dst] = 0.0;
                    continue;
                }
                i32 pick = d;                          /* CRS order by default */
                if (sojds && rl > 0) {
                    i64 prev = slice_ptr[s] + (i64)d * C + (rl - 1);
                    i64 want = (i64)bl_col[prev] + 1;
                    pick = -1;
                    i64 best = 0;
                    for (i32 e = 0; e < len; ++e) {
                        if (taken[e]) continue;
                        i64 c = jd_col[jd_ptr[e] + r];
                        i64 dist = c > want ? c - want : want - c;
                        if (pick < 0 || dist < best ||
                            (dist == best && c < jd_col[jd_ptr[pick] + r])) {
                            pick = e;
                            best = dist;
                        }
                    }
                }
                if (sojds) taken[pick] = 1;
                bl_col[dst] = jd_col[jd_ptr[pick] + r];
                bl_val[dst] = jd_val[jd_ptr[pick] + r];
            }
        }
    }
    free(taken);
    return total;
}

/* RBJDS storage over a windowed row order (paper Section 2 notes that a more
 * elaborate initial ordering of the elements can pay off).  Reading: the rows
 * are cut into windows of sigma consecutive original rows (sigma a multiple
 * of C; the last window may be shorter), each window is sorted by decreasing
 * row length with ties in ascending original index, and the windows follow
 * one another; sigma >= n is the plain JDS order.  Blocks of C consecutive
 * permuted rows then never span two windows, are stored diagonal by diagonal
 * and padded to their first (longest) row exactly as in the RBJDS builder
 * above (col = -1, value 0 in padded slots), entries of a row in CRS order.
 *   perm[r] = original row of permuted row r
 * slice_ptr / slice_nd / bl_col / bl_val as above.  Returns the padded total,
 * or -1 if sigma is not a positive multiple of C. */
i64 orc_jds_blocked_windowed(i32 n, const i32 *row_ptr, const i32 *col, const double *val, i32 C, i32 sigma,
                             i32 *perm, i64 *slice_ptr, i32 *slice_nd, i32 *bl_col, double *bl_val)
{
    if (C <= 0 || sigma <= 0 || sigma % C != 0) return -1;
    len_key *keys = (len_key *)malloc(sizeof(len_key) * (size_t)(n > 0 ? n : 1));
    for (i32 w0 = 0; w0 < n; w0 += sigma) {
        i32 w1 = w0 + sigma < n ? w0 + sigma : n;
        for (i32 i = w0; i < w1; ++i) {
            keys[i].len = row_ptr[i + 1] - row_ptr[i];
            keys[i].row = i;
        }
        qsort(keys + w0, (size_t)(w1 - w0), sizeof(len_key), len_cmp);
    }
    for (i32 r = 0; r < n; ++r) perm[r] = keys[r].row;
    i32 n_slices = (n + C - 1) / C;
    i64 total = 0;
    for (i32 s = 0; s < n_slices; ++s) {
        slice_ptr[s] = total;
        slice_nd[s] = keys[s * C].len;          /* the block's first row is its longest */
        total += (i64)slice_nd[s] * C;
    }
    slice_ptr[n_slices] = total;
    if (bl_col) {
        for (i32 s = 0; s < n_slices; ++s) {
            for (i32 rl = 0; rl < C; ++rl) {
                i32 r = s * C + rl;
                i32 len = r < n ? keys[r].len : 0;
                for (i32 d = 0; d < slice_nd[s]; ++d) {
                    i64 dst = slice_ptr[s] + (i64)d * C + rl;
                    if (d < len) {
                        i32 src = row_ptr[perm[r]] + d;
                        bl_col[dst] = col[src];
                        bl_val[dst] = val[src];
                    } else {
                        bl_col[dst] = -1;
                        bl_val[dst] = 0.0;
                    }
                }
            }
        }
    }
    free(keys);
    return total;
}

/* RBJDS kernel: block by block, diagonal by diagonal inside the block, so the
 * block's part of the result vector stays in cache (paper Section 2). */
void orc_spmv_jds_blocked(i32 n, const i32 *perm, i32 C, i32 n_slices, const i64 *slice_ptr,
                          const i32 *slice_nd, const i32 *bl_col, const double *bl_val,
                          const double *x, double *y, double alpha, double beta, int symperm)
{
    double *res = (double *)calloc((size_t)(n > 0 ? n : 1), sizeof(double));
    for (i32 s = 0; s < n_slices; ++s)
        for (i32 d = 0; d < slice_nd[s]; ++d)
            for (i32 rl = 0; rl < C; ++rl) {
                i32 r = s * C + rl;
                i64 k = slice_ptr[s] + (i64)d * C + rl;
                if (r >= n || bl_col[k] < 0) continue;
                res[r] = res[r] + bl_val[k] * x[bl_col[k]];
            }
    jds_store(n, perm, symperm, res, y, alpha, beta);
    free(res);
}

/* ------------------------------------------------------------------------ */
/* Reduced-precision value storage.  bf16 keeps 8 significant bits and float's
 * exponent range.  One round-to-nearest-even step straight from the double
 * (no intermediate float, which could round twice).  Output is the bf16 bit
 * pattern. */
void orc_round_bf16(const double *in, uint16_t *out, i64 n)
{
    for (i64 i = 0; i < n; ++i) {
        double v = in[i];
        double q;
        if (isnan(v)) {
            out[i] = 0x7fc0;
            continue;
        }
        double a = fabs(v);
        if (a < ldexp(1.0, -126)) {
            /* bf16 subnormal range: multiples of 2^-133 */
            q = nearbyint(ldexp(a, 133));
            q = ldexp(q, -133);
        } else if (isinf(a)) {
            q = a;
        } else {
            int e;
            double m = frexp(a, &e);                  /* a = m * 2^e, 0.5 <= m < 1 */
            double t = nearbyint(ldexp(m, 8));        /* 8 significant bits, ties to even */
            q = ldexp(t, e - 8);
            /* beyond the largest finite bf16 (0x7f7f) rounding goes to infinity */
            if (q > ldexp(255.0, 127 - 7)) q = INFINITY;
        }
        float f = (float)q;                           /* exact: q has <= 8 bits */
        uint32_t bits;
        memcpy(&bits, &f, 4);
        bits >>= 16;
        if (signbit(v)) bits |= 0x8000u;
        out[i] = (uint16_t)bits;
    }
}

/* ------------------------------------------------------------------------ */
/* One-triangle storage of a symmetric matrix.  Section 4.2 observes that the
 * Hamiltonian is symmetric (Hermitian), which would let an SpMV move less
 * data; the paper does not pursue it.  Reading: A is stored as its upper
 * triangle U (entries with col >= row, each row in CRS order) and
 * A = U + U^T - diag(U).  Entries below the diagonal are dropped unread.
 * Returns nnz(U); with out_row_ptr == NULL nothing is written. */
i64 orc_csr_upper(i32 n, const i32 *row_ptr, const i32 *col, const double *val,
                  i32 *out_row_ptr, i32 *out_col, double *out_val)
{
    i64 p = 0;
    if (out_row_ptr) out_row_ptr[0] = 0;
    for (i32 i = 0; i < n; ++i) {
        for (i32 j = row_ptr[i]; j < row_ptr[i + 1]; ++j) {
            if (col[j] < i) continue;
            if (out_row_ptr) {
                out_col[p] = col[j];
                out_val[p] = val[j];
            }
            ++p;
        }
        if (out_row_ptr) out_row_ptr[i + 1] = (i32)p;
    }
    return p;
}

/* y = alpha * (U + U^T - diag(U)) x + beta * y from the upper triangle U.
 * Row i's sum is taken in ascending column order, as orc_spmv_crs takes it
 * on the full matrix with sorted rows: first the mirrored entries a(k, i),
 * k < i, in ascending k, then row i of U left to right.  beta == 0 never
 * reads y. */
void orc_spmv_crs_sym(i32 n, const i32 *row_ptr, const i32 *col, const double *val,
                      const double *x, double *y, double alpha, double beta)
{
    double *lo = (double *)calloc((size_t)(n > 0 ? n : 1), sizeof(double));
    /* lo[j] = sum over k < j of a(k, j) * x[k]; rows k are visited in
     * ascending order, so each lo[j] adds its terms in ascending k */
    for (i32 k = 0; k < n; ++k)
        for (i32 e = row_ptr[k]; e < row_ptr[k + 1]; ++e)
            if (col[e] > k) lo[col[e]] = lo[col[e]] + val[e] * x[k];
    for (i32 i = 0; i < n; ++i) {
        double s = lo[i];
        for (i32 e = row_ptr[i]; e < row_ptr[i + 1]; ++e)
            s = s + val[e] * x[col[e]];
        if (beta == 0.0)
            y[i] = alpha * s;
        else
            y[i] = alpha * s + beta * y[i];
    }
    free(lo);
}

/* ------------------------------------------------------------------------ */
/* Transpose of a CRS pattern: row c of A^T lists the entries of column c of A
 * in ascending original row order; tmap[t] is the position in A of entry t of
 * A^T, so A^T's values are val[tmap]. */
void orc_csr_transpose(i32 n_rows, i32 n_cols, const i32 *row_ptr, const i32 *col,
                       i32 *rowT_ptr, i32 *colT, i64 *tmap)
{
    for (i32 c = 0; c <= n_cols; ++c) rowT_ptr[c] = 0;
    for (i32 i = 0; i < n_rows; ++i)
        for (i32 j = row_ptr[i]; j < row_ptr[i + 1]; ++j)
            rowT_ptr[col[j] + 1] += 1;
    for (i32 c = 0; c < n_cols; ++c) rowT_ptr[c + 1] += rowT_ptr[c];
    i32 *fill = (i32 *)calloc((size_t)(n_cols > 0 ? n_cols : 1), sizeof(i32));
    for (i32 i = 0; i < n_rows; ++i)
        for (i32 j = row_ptr[i]; j < row_ptr[i + 1]; ++j) {
            i32 c = col[j];
            i32 t = rowT_ptr[c] + fill[c]++;
            colT[t] = i;
            tmap[t] = j;
        }
    free(fill);
}

/* Derivative of y = A x with respect to the stored values: y_i depends on
 * val[j] (j in row i) through val[j]*x[col[j]], so dL/dval[j] = g[i]*x[col[j]]
 * with g = dL/dy.  out[j] = alpha*g[i]*x[col[j]] + beta*out[j]. */
void orc_grad_vals_csr(i32 n_rows, const i32 *row_ptr, const i32 *col, const double *g,
                       const double *x, double *out, double alpha, double beta)
{
    for (i32 i = 0; i < n_rows; ++i)
        for (i32 j = row_ptr[i]; j < row_ptr[i + 1]; ++j) {
            double p = g[i] * x[col[j]];
            out[j] = (beta == 0.0) ? alpha * p : alpha * p + beta * out[j];
        }
}

/* Transposed product y = A^T g straight from the CRS arrays (the definition). */
void orc_spmv_crs_transposed(i32 n_rows, i32 n_cols, const i32 *row_ptr, const i32 *col,
                             const double *val, const double *g, double *y)
{
    for (i32 c = 0; c < n_cols; ++c) y[c] = 0.0;
    for (i32 i = 0; i < n_rows; ++i)
        for (i32 j = row_ptr[i]; j < row_ptr[i + 1]; ++j)
            y[col[j]] = y[col[j]] + val[j] * g[i];
}

/* ------------------------------------------------------------------------ */
/* Chebyshev recurrence driven by the SpMV: y0 = x, y1 = A y0,
 * y_{k+1} = 2 A y_k - y_{k-1}; ys holds y0..y_steps (n each). */
void orc_cheb_forward(i32 n, const i32 *row_ptr, const i32 *col, const double *val,
                      const double *x, i32 steps, double *ys)
{
    memcpy(ys, x, sizeof(double) * (size_t)n);
    if (steps < 1) return;
    orc_spmv_crs(n, row_ptr, col, val, ys, ys + n, 1.0, 0.0);
    for (i32 k = 1; k < steps; ++k) {
        double *yn = ys + (i64)(k + 1) * n;
        orc_spmv_crs(n, row_ptr, col, val, ys + (i64)k * n, yn, 2.0, 0.0);
        for (i32 i = 0; i < n; ++i)
            yn[i] = yn[i] - ys[(i64)(k - 1) * n + i];
    }
}

/* Reverse sweep of the recurrence for loss = sum_i y_steps[i]^2, written from
 * the chain rule on each step:
 *   ybar_steps = 2 y_steps
 *   step k (y_{k+1} = 2 A y_k - y_{k-1}), k = steps-1 .. 1:
 *       ybar_k += 2 A^T ybar_{k+1};  ybar_{k-1} -= ybar_{k+1};
 *       dval += 2 ybar_{k+1}[row] * y_k[col]
 *   step 0 (y_1 = A y_0): ybar_0 += A^T ybar_1;  dval += ybar_1[row] * y_0[col]
 *   dx = ybar_0.
 * ys from orc_cheb_forward; dval has nnz entries. Returns the loss. */
double orc_cheb_adjoint(i32 n, const i32 *row_ptr, const i32 *col, const double *val,
                        const double *ys, i32 steps, double *dx, double *dval)
{
    i32 nnz = row_ptr[n];
    double *bar = (double *)calloc((size_t)(steps + 1) * (size_t)(n > 0 ? n : 1), sizeof(double));
    double *t = (double *)malloc(sizeof(double) * (size_t)(n > 0 ? n : 1));
    double loss = 0.0;
    const double *yK = ys + (i64)steps * n;
    for (i32 i = 0; i < n; ++i) {
        loss = loss + yK[i] * yK[i];
        bar[(i64)steps * n + i] = 2.0 * yK[i];
    }
    for (i32 j = 0; j < nnz; ++j) dval[j] = 0.0;
    for (i32 k = steps - 1; k >= 1; --k) {
        double *bk1 = bar + (i64)(k + 1) * n;
        orc_spmv_crs_transposed(n, n, row_ptr, col, val, bk1, t);
        for (i32 i = 0; i < n; ++i) {
            bar[(i64)k * n + i] = bar[(i64)k * n + i] + 2.0 * t[i];
            bar[(i64)(k - 1) * n + i] = bar[(i64)(k - 1) * n + i] - bk1[i];
        }
        orc_grad_vals_csr(n, row_ptr, col, bk1, ys + (i64)k * n, dval, 2.0, 1.0);
    }
    if (steps >= 1) {
        orc_spmv_crs_transposed(n, n, row_ptr, col, val, bar + n, t);
        for (i32 i = 0; i < n; ++i) bar[i] = bar[i] + t[i];
        orc_grad_vals_csr(n, row_ptr, col, bar + n, ys, dval, 1.0, 1.0);
    } else {
        /* loss = |x|^2 directly */
    }
    memcpy(dx, bar, sizeof(double) * (size_t)n);
    free(bar);
    free(t);
    return loss;
}
