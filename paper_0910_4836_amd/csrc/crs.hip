// CRS sparse matrix-vector product (paper Section 2, the CRS kernel: each row
// is a sparse scalar product of its stored values with the gathered x).
//
// gfx950 design: the rows are cut, once per matrix, into blocks of consecutive
// rows holding at most block_nnz entries and at most 256 rows (2048 rows when
// none of them has more than 16 entries); a row longer than block_nnz is a
// block of its own.  One 256-lane workgroup per block:
//   * multi-row block ("stream" mode): the lanes walk the block's entries in
//     order - fully coalesced val/col reads, independent x gathers, four in
//     flight per lane - and park the products in LDS; then G lanes per row
//     (G = 256/rows, a power of two up to 64) add their row's products and
//     combine with a fixed shuffle tree, or, in a block of more than 256 short
//     rows, one lane adds each row.  (Measured and dropped: eight loads in
//     flight, row offsets staged in LDS, lane groups sized per row - none
//     helps the gather-bound power-law rows, and they cost 3-25% on uniform
//     rows.)
//   * single-row block ("vector" mode): all 256 lanes stride over the row with
//     fused multiply-adds, then a fixed wave tree and an ordered sum over the
//     four waves.
//   * staged kernel (a separate entry point over the same plans): the block's
//     col/val are copied to LDS in entry order, then the lanes walk the rows
//     and gather in row order, so that a wavefront's gather holds the same
//     entry position of consecutive rows.  It pays on banded and diagonal
//     matrices (fewer x lines per gather instruction for the address units),
//     not on the power-law rows; the autotuner picks per matrix.
// Every y element is written once by one lane; no atomics; the summation order
// depends only on the plan, so results are reproducible.
// Blocks are remapped so that each XCD walks a contiguous range of rows: the
// band part of x stays in that XCD's L2.
#include <algorithm>
#include <vector>

#include "common.hpp"

namespace spmv {

constexpr int CRS_THREADS = 256;
constexpr int CRS_DEFAULT_BLOCK_NNZ = 1024;
constexpr int CRS_MAX_BLOCK_NNZ = 4096;
constexpr int CRS_MAX_BLOCK_ROWS = 256;          // rows of a block in general
constexpr int CRS_MAX_SHORT_BLOCK_ROWS = 2048;   // rows of a block of short rows only
constexpr int CRS_SHORT_ROW = 16;                // "short": at most this many entries
constexpr int CRS_STREAM_U = 4;                  // stream mode: entries per lane per trip
constexpr int CRS_LDS_ROUND = CRS_STREAM_U * CRS_THREADS;   // products per trip

// LDS bytes of a block kernel: block_nnz products rounded up to whole trips.
inline size_t crs_lds_bytes(int32_t block_nnz, size_t acc_bytes)
{
    return (size_t)ceil_div(block_nnz, CRS_LDS_ROUND) * CRS_LDS_ROUND * acc_bytes;
}

template <bool WIDE, typename VT, typename XT, typename OT>
__device__ __forceinline__ void crs_vector_row(const int32_t *__restrict__ col, const VT *__restrict__ val,
                                               const XT *__restrict__ x, OT *__restrict__ y, int32_t row,
                                               int32_t e0, int32_t e1, double alpha, double beta,
                                               double *red, const int32_t *__restrict__ out_idx)
{
    typedef typename Acc<WIDE>::T acc_t;
    acc_t s = 0;
    int32_t k = e0 + (int32_t)threadIdx.x;
    constexpr int U = 4;
    for (; k + (U - 1) * CRS_THREADS < e1; k += U * CRS_THREADS) {
        int32_t c[U];
        VT v[U];
#pragma unroll
        for (int u = 0; u < U; ++u) {
            c[u] = ld_stream(col + k + u * CRS_THREADS);
            v[u] = ld_stream(val + k + u * CRS_THREADS);
        }
        XT xv[U];
#pragma unroll
        for (int u = 0; u < U; ++u) xv[u] = x[c[u]];
#pragma unroll
        for (int u = 0; u < U; ++u) s = Acc<WIDE>::mac(s, v[u], xv[u]);
    }
    for (; k < e1; k += CRS_THREADS) s = Acc<WIDE>::mac(s, ld_stream(val + k), x[ld_stream(col + k)]);
    // partials are added in the accumulator type; LDS holds them as double (exact)
    acc_t t = group_sum(s, WAVE);
    if (lane_id() == 0) red[threadIdx.x / WAVE] = (double)t;
    __syncthreads();
    if (threadIdx.x == 0) {
        acc_t tot = (acc_t)red[0];
        for (int w = 1; w < CRS_THREADS / WAVE; ++w) tot += (acc_t)red[w];
        write_y(y, out_idx ? out_idx[row] : row, (double)tot, alpha, beta);
    }
}

// Row sums of a multi-row block whose products sit in LDS (prod[k] = product
// of entry e0 + k): G lanes per row (G = largest power of two <= 256/nr, at
// most 64) with a fixed shuffle tree, or, in a block of more than 256 short
// rows, one lane per row adding its products in order.
// rs, re: the bounds of row r0 + t / G (G as below), loaded by the caller
// (for blocks of at most 256 rows) before the products, off the critical path.
template <typename acc_t, typename OT>
__device__ __forceinline__ void crs_row_sums(const int32_t *__restrict__ row_ptr, const acc_t *prod, int32_t r0,
                                             int32_t nr, int32_t e0, OT *__restrict__ y, double alpha, double beta,
                                             const int32_t *__restrict__ out_idx, int32_t rs, int32_t re)
{
    const int t = (int)threadIdx.x;
    if (nr > CRS_THREADS) {
        // many short rows (the planner admits more than 256 rows only when
        // none has more than 16 entries): one lane per row, rows t, t+256, ...
        for (int32_t g = t; g < nr; g += CRS_THREADS) {
            const int32_t rs = row_ptr[r0 + g] - e0, re = row_ptr[r0 + g + 1] - e0;
            acc_t s = 0;
            for (int32_t k = rs; k < re; ++k) s += prod[k];
            const int32_t row = r0 + g;
            write_y(y, out_idx ? out_idx[row] : row, (double)s, alpha, beta);
        }
        return;
    }
    int G = 64;
    while (G > 1 && G * nr > CRS_THREADS) G >>= 1;
    const int g = t / G, l = t % G;
    acc_t s = 0;
    if (g < nr)
        for (int32_t k = rs - e0 + l; k < re - e0; k += G) s += prod[k];
    s = group_sum(s, G);
    if (g < nr && l == 0) {
        const int32_t row = r0 + g;
        write_y(y, out_idx ? out_idx[row] : row, (double)s, alpha, beta);
    }
}

// One plan block b (rows plan[b] .. plan[b+1]) of y = alpha*A x + beta*y;
// row r's result goes to y[out_idx[r]] if out_idx is given, else to y[r].
// WIDE_ALL: accumulate every row in FP64 (the column-split parts, whose rows
// are pieces of rows whose full length the block does not see).
template <typename VT, typename XT, typename OT, bool WIDE_ALL = false>
__device__ __forceinline__ void crs_block_body(const int32_t *__restrict__ row_ptr, const int32_t *__restrict__ col,
                                               const VT *__restrict__ val, const XT *__restrict__ x,
                                               OT *__restrict__ y, const int32_t *__restrict__ plan, int64_t b,
                                               double alpha, double beta, double *smem_d, double *red,
                                               const int32_t *__restrict__ out_idx = nullptr)
{
    constexpr bool F64 = IsF64<VT>::value || WIDE_ALL;
    typedef typename Acc<F64>::T acc_t;
    acc_t *prod = reinterpret_cast<acc_t *>(smem_d);
    const int32_t r0 = plan[b], r1 = plan[b + 1];
    const int32_t e0 = row_ptr[r0], e1 = row_ptr[r1];
    const int32_t nr = r1 - r0, ne = e1 - e0;
    const int t = (int)threadIdx.x;

    if (nr == 1) {
        if (!F64 && ne > SPMV_WIDE_ROW_NNZ)
            crs_vector_row<true, VT, XT, OT>(col, val, x, y, r0, e0, e1, alpha, beta, red, out_idx);
        else
            crs_vector_row<F64, VT, XT, OT>(col, val, x, y, r0, e0, e1, alpha, beta, red, out_idx);
        return;
    }

    // the row bounds the row sums need, loaded now so that their latency
    // overlaps that of the entries and gathers
    int32_t rs = 0, re = 0;
    if (nr <= CRS_THREADS) {
        int G = 64;
        while (G > 1 && G * nr > CRS_THREADS) G >>= 1;
        const int g = t / G;
        if (g < nr) {
            rs = row_ptr[r0 + g];
            re = row_ptr[r0 + g + 1];
        }
    }

    // stream mode: products of the whole block into LDS (ne <= block_nnz);
    // each lane issues its U loads of val/col, then its U gathers, all before
    // it waits on any of them.  Lanes past the block's end load its last
    // entry again and store into LDS slots past ne, which hold
    // CRS_LDS_ROUND-rounded room and are never read: no branch around a
    // load, so the compiler cannot sink a gather behind a wait for another.
    constexpr int U = CRS_STREAM_U;
    if (ne > 0) {
        for (int32_t k0 = 0; k0 < ne; k0 += U * CRS_THREADS) {
            int32_t c[U];
            VT v[U];
#pragma unroll
            for (int u = 0; u < U; ++u) {
                const int32_t k = min(k0 + u * CRS_THREADS + t, ne - 1);
                c[u] = ld_stream(col + e0 + k);
                v[u] = ld_stream(val + e0 + k);
            }
            XT xv[U];
#pragma unroll
            for (int u = 0; u < U; ++u) xv[u] = x[c[u]];
#pragma unroll
            for (int u = 0; u < U; ++u) prod[k0 + u * CRS_THREADS + t] = Acc<F64>::mac((acc_t)0, v[u], xv[u]);
        }
    }
    __syncthreads();
    crs_row_sums<acc_t>(row_ptr, prod, r0, nr, e0, y, alpha, beta, out_idx, rs, re);
}

template <typename VT, typename XT>
__global__ __launch_bounds__(CRS_THREADS) void crs_block_kernel(const int32_t *__restrict__ row_ptr,
                                                                const int32_t *__restrict__ col,
                                                                const VT *__restrict__ val,
                                                                const XT *__restrict__ x, XT *__restrict__ y,
                                                                const int32_t *__restrict__ plan,
                                                                double alpha, double beta)
{
    extern __shared__ double smem_d[];
    __shared__ double red[CRS_THREADS / WAVE];
    crs_block_body<VT, XT, XT>(row_ptr, col, val, x, y, plan, xcd_remap(blockIdx.x, gridDim.x), alpha, beta, smem_d,
                               red);
}

// Staged CRS: the same plan blocks, with the gathers issued in row order
// instead of entry order.  The block's col/val stream into LDS first
// (coalesced, as in stream mode); then G lanes per row (one lane per row in a
// block of more than 256 short rows) walk their row's staged entries, keep
// CRS_STAGE_U gathers in flight, and accumulate with fused multiply-adds.  A
// wavefront's gather instruction then holds the same entry position of
// consecutive rows: on banded and diagonal patterns those are neighbouring
// columns, a few x lines per instruction instead of one per diagonal the
// entry-order walk crosses, which is what the address units pay for.
constexpr int CRS_STAGE_U = 8;

// LDS of the staged kernel: values then column indices of block_nnz entries,
// each array rounded up to whole trips of the staging loop.
inline size_t crs_staged_lds_bytes(int32_t block_nnz, size_t val_bytes)
{
    return (size_t)ceil_div(block_nnz, CRS_LDS_ROUND) * CRS_LDS_ROUND * (val_bytes + sizeof(int32_t));
}

template <typename acc_t, bool F64, typename VT, typename XT>
__device__ __forceinline__ acc_t crs_staged_row(const VT *vs, const int32_t *cs, const XT *__restrict__ x,
                                                int32_t a, int32_t z, int l, int G)
{
    acc_t s = 0;
    for (int32_t k = a + l; k < z; k += CRS_STAGE_U * G) {
        int32_t c[CRS_STAGE_U];
        VT v[CRS_STAGE_U];
#pragma unroll
        for (int u = 0; u < CRS_STAGE_U; ++u) {
            const int32_t kk = min(k + u * G, z - 1);
            c[u] = cs[kk];
            v[u] = vs[kk];
        }
        XT xv[CRS_STAGE_U];
#pragma unroll
        for (int u = 0; u < CRS_STAGE_U; ++u) xv[u] = x[c[u]];
#pragma unroll
        for (int u = 0; u < CRS_STAGE_U; ++u)
            if (k + u * G < z) s = Acc<F64>::mac(s, v[u], xv[u]);
    }
    return s;
}

template <typename VT, typename XT>
__global__ __launch_bounds__(CRS_THREADS) void crs_staged_kernel(const int32_t *__restrict__ row_ptr,
                                                                 const int32_t *__restrict__ col,
                                                                 const VT *__restrict__ val,
                                                                 const XT *__restrict__ x, XT *__restrict__ y,
                                                                 const int32_t *__restrict__ plan, int32_t lds_cap,
                                                                 double alpha, double beta)
{
    extern __shared__ double smem_d[];
    __shared__ double red[CRS_THREADS / WAVE];
    constexpr bool F64 = IsF64<VT>::value;
    typedef typename Acc<F64>::T acc_t;
    const int64_t b = xcd_remap(blockIdx.x, gridDim.x);
    const int32_t r0 = plan[b], r1 = plan[b + 1];
    const int32_t e0 = row_ptr[r0], e1 = row_ptr[r1];
    const int32_t nr = r1 - r0, ne = e1 - e0;
    const int t = (int)threadIdx.x;

    if (nr == 1) {
        if (!F64 && ne > SPMV_WIDE_ROW_NNZ)
            crs_vector_row<true, VT, XT, XT>(col, val, x, y, r0, e0, e1, alpha, beta, red, nullptr);
        else
            crs_vector_row<F64, VT, XT, XT>(col, val, x, y, r0, e0, e1, alpha, beta, red, nullptr);
        return;
    }

    // row bounds, loaded before the staging so that their latency overlaps it:
    // for at most 256 rows, row g = t / G of the G-lane groups; for more (all
    // of at most 16 entries, at most 2048 rows), rows t + 256 j, j < 8
    constexpr int MAXJ = CRS_MAX_SHORT_BLOCK_ROWS / CRS_THREADS;
    int G = 64;
    while (G > 1 && G * nr > CRS_THREADS) G >>= 1;
    const int g = t / G, l = t % G;
    int32_t lo[MAXJ], hi[MAXJ];
    if (nr <= CRS_THREADS) {
        lo[0] = g < nr ? row_ptr[r0 + g] : 0;
        hi[0] = g < nr ? row_ptr[r0 + g + 1] : 0;
    } else {
#pragma unroll
        for (int j = 0; j < MAXJ; ++j) {
            const int32_t q = t + j * CRS_THREADS;
            lo[j] = q < nr ? row_ptr[r0 + q] : 0;
            hi[j] = q < nr ? row_ptr[r0 + q + 1] : 0;
        }
    }

    // stage the block's entries (ne <= lds_cap; lanes past the end reload
    // the last entry into slots past ne, which lds_cap covers)
    VT *vs = reinterpret_cast<VT *>(smem_d);
    int32_t *cs = reinterpret_cast<int32_t *>(vs + lds_cap);
    constexpr int U = CRS_STREAM_U;
    for (int32_t k0 = 0; k0 < ne; k0 += U * CRS_THREADS) {
        int32_t c[U];
        VT v[U];
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const int32_t k = min(k0 + u * CRS_THREADS + t, ne - 1);
            c[u] = ld_stream(col + e0 + k);
            v[u] = ld_stream(val + e0 + k);
        }
#pragma unroll
        for (int u = 0; u < U; ++u) {
            cs[k0 + u * CRS_THREADS + t] = c[u];
            vs[k0 + u * CRS_THREADS + t] = v[u];
        }
    }
    __syncthreads();

    if (nr <= CRS_THREADS) {
        acc_t s = 0;
        if (g < nr) s = crs_staged_row<acc_t, F64>(vs, cs, x, lo[0] - e0, hi[0] - e0, l, G);
        s = group_sum(s, G);
        if (g < nr && l == 0) write_y(y, (int64_t)r0 + g, (double)s, alpha, beta);
        return;
    }
#pragma unroll
    for (int j = 0; j < MAXJ; ++j) {
        const int32_t q = t + j * CRS_THREADS;
        if (q < nr) {
            const acc_t s = crs_staged_row<acc_t, F64>(vs, cs, x, lo[j] - e0, hi[j] - e0, 0, 1);
            write_y(y, (int64_t)r0 + q, (double)s, alpha, beta);
        }
    }
    // rows past 2048 (a caller's plan may hold more rows than the planner's)
    for (int32_t q = t + MAXJ * CRS_THREADS; q < nr; q += CRS_THREADS) {
        const acc_t s = crs_staged_row<acc_t, F64>(vs, cs, x, row_ptr[r0 + q] - e0, row_ptr[r0 + q + 1] - e0, 0, 1);
        write_y(y, (int64_t)r0 + q, (double)s, alpha, beta);
    }
}

// Column-split CRS: part k (columns of the k-th eighth, compressed to the rows
// that hold one of its entries) runs on XCD k (workgroup b -> part b % 8) and
// writes each row's partial result into its slot.
struct CrsSplitTab {
    int64_t base[SPLIT_PARTS];        // part k's first entry in col / val
    int32_t row_off[SPLIT_PARTS];     // part k's first compressed row
    int32_t plan_off[SPLIT_PARTS];
    int32_t n_blocks[SPLIT_PARTS];
};

template <typename VT, typename XT>
__global__ __launch_bounds__(CRS_THREADS) void crs_split_kernel(const int32_t *__restrict__ row_ptr_all,
                                                                const int32_t *__restrict__ dest_all,
                                                                const int32_t *__restrict__ col,
                                                                const VT *__restrict__ val,
                                                                const XT *__restrict__ x,
                                                                double *__restrict__ slots,
                                                                const int32_t *__restrict__ plan_all, CrsSplitTab T)
{
    extern __shared__ double smem_d[];
    __shared__ double red[CRS_THREADS / WAVE];
    const int k = (int)(blockIdx.x % SPLIT_PARTS);
    const int64_t b = blockIdx.x / SPLIT_PARTS;
    if (b >= T.n_blocks[k]) return;
    crs_block_body<VT, XT, double, true>(row_ptr_all + T.row_off[k] + k, col + T.base[k], val + T.base[k], x, slots,
                                         plan_all + T.plan_off[k], b, 1.0, 0.0, smem_d, red,
                                         dest_all + T.row_off[k]);
}

// One wavefront per row: the default when no plan is given.
template <typename VT, typename XT>
__global__ __launch_bounds__(CRS_THREADS) void crs_wave_kernel(int32_t n_rows, const int32_t *__restrict__ row_ptr,
                                                               const int32_t *__restrict__ col,
                                                               const VT *__restrict__ val,
                                                               const XT *__restrict__ x, XT *__restrict__ y,
                                                               double alpha, double beta)
{
    constexpr bool F64 = IsF64<VT>::value;
    const int64_t row = xcd_remap(blockIdx.x, gridDim.x) * (CRS_THREADS / WAVE) + threadIdx.x / WAVE;
    if (row >= n_rows) return;
    const int32_t e0 = row_ptr[row], e1 = row_ptr[row + 1];
    if (!F64 && e1 - e0 > SPMV_WIDE_ROW_NNZ) {
        double s = 0;
        for (int32_t k = e0 + lane_id(); k < e1; k += WAVE) s = Acc<true>::mac(s, val[k], x[col[k]]);
        s = group_sum(s, WAVE);
        if (lane_id() == 0) write_y(y, row, s, alpha, beta);
    } else {
        typename Acc<F64>::T s = 0;
        for (int32_t k = e0 + lane_id(); k < e1; k += WAVE) s = Acc<F64>::mac(s, val[k], x[col[k]]);
        s = group_sum(s, WAVE);
        if (lane_id() == 0) write_y(y, row, (double)s, alpha, beta);
    }
}

// Multi-vector CRS: the same row blocks; G lanes per row, each lane keeps KB
// column accumulators so a row's entries are read once per KB columns of X.
template <int KB, typename VT, typename XT>
__global__ __launch_bounds__(CRS_THREADS) void spmm_crs_kernel(const int32_t *__restrict__ row_ptr,
                                                               const int32_t *__restrict__ col,
                                                               const VT *__restrict__ val, const XT *__restrict__ X,
                                                               int64_t ldx, XT *__restrict__ Y, int64_t ldy, int32_t k,
                                                               const int32_t *__restrict__ plan, double alpha,
                                                               double beta)
{
    constexpr bool F64 = IsF64<VT>::value;
    __shared__ double red[CRS_THREADS / WAVE][KB];
    const int64_t b = xcd_remap(blockIdx.x, gridDim.x);
    const int c0 = blockIdx.y * KB;
    const int kb = k - c0 < KB ? k - c0 : KB;
    const int32_t r0 = plan[b], r1 = plan[b + 1];
    const int32_t nr = r1 - r0;
    const XT *__restrict__ Xc = X + (int64_t)c0 * ldx;
    XT *__restrict__ Yc = Y + (int64_t)c0 * ldy;
    if (nr == 1) {
        const int32_t e0 = row_ptr[r0], e1 = row_ptr[r1];
        const bool wide = !F64 && e1 - e0 > SPMV_WIDE_ROW_NNZ;
        double acc[KB];
#pragma unroll
        for (int j = 0; j < KB; ++j) acc[j] = 0.0;
        if (F64 || wide) {
            for (int32_t e = e0 + (int32_t)threadIdx.x; e < e1; e += CRS_THREADS) {
                const int32_t c = ld_stream(col + e);
                const VT v = ld_stream(val + e);
#pragma unroll
                for (int j = 0; j < KB; ++j)
                    if (j < kb) acc[j] = Acc<true>::mac(acc[j], v, Xc[c + (int64_t)j * ldx]);
            }
#pragma unroll
            for (int j = 0; j < KB; ++j) acc[j] = group_sum(acc[j], WAVE);
        } else {
            float accf[KB];
#pragma unroll
            for (int j = 0; j < KB; ++j) accf[j] = 0.0f;
            for (int32_t e = e0 + (int32_t)threadIdx.x; e < e1; e += CRS_THREADS) {
                const int32_t c = ld_stream(col + e);
                const VT v = ld_stream(val + e);
#pragma unroll
                for (int j = 0; j < KB; ++j)
                    if (j < kb) accf[j] = Acc<false>::mac(accf[j], v, Xc[c + (int64_t)j * ldx]);
            }
#pragma unroll
            for (int j = 0; j < KB; ++j) acc[j] = (double)group_sum(accf[j], WAVE);
        }
        if (lane_id() == 0) {
#pragma unroll
            for (int j = 0; j < KB; ++j) red[threadIdx.x / WAVE][j] = acc[j];
        }
        __syncthreads();
        if (threadIdx.x < (unsigned)kb) {
            const int j = (int)threadIdx.x;
            if (F64 || wide) {
                double t = red[0][j];
                for (int w = 1; w < CRS_THREADS / WAVE; ++w) t += red[w][j];
                write_y(Yc + (int64_t)j * ldy, r0, t, alpha, beta);
            } else {
                float t = (float)red[0][j];
                for (int w = 1; w < CRS_THREADS / WAVE; ++w) t += (float)red[w][j];
                write_y(Yc + (int64_t)j * ldy, r0, (double)t, alpha, beta);
            }
        }
        return;
    }
    typedef typename Acc<F64>::T acc_t;
    int G = 64;
    while (G > 1 && G * nr > CRS_THREADS) G >>= 1;
    const int l = (int)threadIdx.x % G;
    // blocks of more than 256 (short) rows take several rounds of 256 rows
    for (int32_t g = (int32_t)threadIdx.x / G; g - (int32_t)threadIdx.x / G < nr; g += CRS_THREADS / G) {
        acc_t acc[KB];
#pragma unroll
        for (int j = 0; j < KB; ++j) acc[j] = 0;
        if (g < nr) {
            const int32_t rs = row_ptr[r0 + g], re = row_ptr[r0 + g + 1];
            for (int32_t e = rs + l; e < re; e += G) {
                const int32_t c = ld_stream(col + e);
                const VT v = ld_stream(val + e);
#pragma unroll
                for (int j = 0; j < KB; ++j)
                    if (j < kb) acc[j] = Acc<F64>::mac(acc[j], v, Xc[c + (int64_t)j * ldx]);
            }
        }
#pragma unroll
        for (int j = 0; j < KB; ++j) acc[j] = group_sum(acc[j], G);
        if (g < nr && l == 0) {
#pragma unroll
            for (int j = 0; j < KB; ++j)
                if (j < kb) write_y(Yc + (int64_t)j * ldy, (int64_t)r0 + g, (double)acc[j], alpha, beta);
        }
    }
}

// ---------------------------------------------------------------- one triangle
// y = alpha * (U + U^T - diag U) x + beta * y from the upper triangle U of a
// symmetric matrix.  y is first scaled by beta (sym_scale_kernel); then every
// plan block of U streams its entries once: entry (i, j, a) gives the product
// a*x[j] for row i's own sum (LDS, as in the CRS block kernel) and, for j > i,
// adds alpha*a*x[i] to y[j] with a device-scope FP64 atomic add; each row's
// own sum goes to y[i] with one more atomic add.  The order of the adds into
// a y entry is not fixed, so y is not bit-reproducible from run to run.
__global__ __launch_bounds__(256) void sym_scale_kernel(double *__restrict__ y, int64_t n, double beta)
{
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        y[i] = beta == 0.0 ? 0.0 : beta * y[i];
}

// LDS of the triangle kernel: FP64 products rounded up to whole trips, then
// one int16 row number per entry.
inline size_t crs_sym_lds_bytes(int32_t block_nnz)
{
    return (size_t)ceil_div(block_nnz, CRS_LDS_ROUND) * CRS_LDS_ROUND * 8 + (size_t)block_nnz * 2;
}

template <typename VT>
__global__ __launch_bounds__(CRS_THREADS) void crs_sym_kernel(const int32_t *__restrict__ row_ptr,
                                                              const int32_t *__restrict__ col,
                                                              const VT *__restrict__ val,
                                                              const double *__restrict__ x, double *__restrict__ y,
                                                              const int32_t *__restrict__ plan, int32_t block_nnz,
                                                              double alpha)
{
    extern __shared__ double smem_d[];
    __shared__ double red[CRS_THREADS / WAVE];
    const int64_t b = xcd_remap(blockIdx.x, gridDim.x);
    const int32_t r0 = plan[b], r1 = plan[b + 1];
    const int32_t e0 = row_ptr[r0], e1 = row_ptr[r1];
    const int32_t nr = r1 - r0, ne = e1 - e0;
    const int t = (int)threadIdx.x;

    if (nr == 1) {
        // one (long) row: lanes stride over its entries
        const double xi = x[r0];
        double s = 0.0;
        for (int32_t e = e0 + t; e < e1; e += CRS_THREADS) {
            const int32_t c = ld_stream(col + e);
            const double a = to_f64(ld_stream(val + e));
            s = fma(a, x[c], s);
            if (c > r0) unsafeAtomicAdd(y + c, alpha * (a * xi));
        }
        s = group_sum(s, WAVE);
        if (lane_id() == 0) red[t / WAVE] = s;
        __syncthreads();
        if (t == 0) {
            double tot = red[0];
            for (int w = 1; w < CRS_THREADS / WAVE; ++w) tot += red[w];
            unsafeAtomicAdd(y + r0, alpha * tot);
        }
        return;
    }

    int G = 64;
    while (G > 1 && G * nr > CRS_THREADS) G >>= 1;
    const int g = t / G, l = t % G;
    int32_t rs = 0, re = 0;
    if (nr <= CRS_THREADS && g < nr) {
        rs = row_ptr[r0 + g];
        re = row_ptr[r0 + g + 1];
    }

    // the row of every entry of the block, into LDS
    const int32_t rounded = (block_nnz + CRS_LDS_ROUND - 1) / CRS_LDS_ROUND * CRS_LDS_ROUND;
    double *prod = smem_d;
    int16_t *rid = reinterpret_cast<int16_t *>(smem_d + rounded);
    if (nr <= CRS_THREADS) {
        if (g < nr)
            for (int32_t k = rs - e0 + l; k < re - e0; k += G) rid[k] = (int16_t)g;
    } else {
        for (int32_t q = t; q < nr; q += CRS_THREADS)
            for (int32_t k = row_ptr[r0 + q] - e0; k < row_ptr[r0 + q + 1] - e0; ++k) rid[k] = (int16_t)q;
    }
    __syncthreads();

    // stream the entries: own-row products into LDS, mirrored terms to y
    constexpr int U = CRS_STREAM_U;
    if (ne > 0) {
        for (int32_t k0 = 0; k0 < ne; k0 += U * CRS_THREADS) {
            int32_t c[U], i[U];
            VT v[U];
#pragma unroll
            for (int u = 0; u < U; ++u) {
                const int32_t k = min(k0 + u * CRS_THREADS + t, ne - 1);
                c[u] = ld_stream(col + e0 + k);
                v[u] = ld_stream(val + e0 + k);
                i[u] = r0 + rid[k];
            }
            double xj[U], xi[U];
#pragma unroll
            for (int u = 0; u < U; ++u) {
                xj[u] = x[c[u]];
                xi[u] = x[i[u]];
            }
#pragma unroll
            for (int u = 0; u < U; ++u) {
                const int32_t k = k0 + u * CRS_THREADS + t;
                const double a = to_f64(v[u]);
                prod[k] = a * xj[u];
                if (k < ne && c[u] > i[u]) unsafeAtomicAdd(y + c[u], alpha * (a * xi[u]));
            }
        }
    }
    __syncthreads();

    // each row's own sum, in entry order per lane, then a fixed shuffle tree
    if (nr > CRS_THREADS) {
        for (int32_t q = t; q < nr; q += CRS_THREADS) {
            double acc = 0.0;
            for (int32_t k = row_ptr[r0 + q] - e0; k < row_ptr[r0 + q + 1] - e0; ++k) acc += prod[k];
            unsafeAtomicAdd(y + r0 + q, alpha * acc);
        }
        return;
    }
    double acc = 0.0;
    if (g < nr)
        for (int32_t k = rs - e0 + l; k < re - e0; k += G) acc += prod[k];
    acc = group_sum(acc, G);
    if (g < nr && l == 0) unsafeAtomicAdd(y + r0 + g, alpha * acc);
}

// One triangle, staged: the block's col/val copied to LDS as in the staged
// CRS kernel, then G lanes per row (one lane per row above 256 rows) walk
// their row's entries in row order.  Each lane adds its products into its
// row's sum and sends the mirrored terms (col > row) to y with FP64 atomics;
// a wavefront's atomic instruction then targets the same entry position of
// consecutive rows, i.e. neighbouring y elements on banded and diagonal
// patterns, instead of one y window per diagonal the entry-order walk
// crosses.  Each row's own sum goes to y with one more atomic add.
template <typename VT>
__device__ __forceinline__ void crs_sym_staged_row(const VT *vs, const int32_t *cs, const double *__restrict__ x,
                                                   double *__restrict__ y, int32_t i, int32_t a, int32_t z,
                                                   int l, int G, double alpha, double &s)
{
    const double axi = alpha * x[i];
    for (int32_t k = a + l; k < z; k += CRS_STAGE_U * G) {
        int32_t c[CRS_STAGE_U];
        VT v[CRS_STAGE_U];
#pragma unroll
        for (int u = 0; u < CRS_STAGE_U; ++u) {
            const int32_t kk = min(k + u * G, z - 1);
            c[u] = cs[kk];
            v[u] = vs[kk];
        }
        double xj[CRS_STAGE_U];
#pragma unroll
        for (int u = 0; u < CRS_STAGE_U; ++u) xj[u] = x[c[u]];
#pragma unroll
        for (int u = 0; u < CRS_STAGE_U; ++u)
            if (k + u * G < z) {
                const double av = to_f64(v[u]);
                s = fma(av, xj[u], s);
                if (c[u] > i) unsafeAtomicAdd(y + c[u], av * axi);
            }
    }
}

template <typename VT>
__global__ __launch_bounds__(CRS_THREADS) void crs_sym_staged_kernel(const int32_t *__restrict__ row_ptr,
                                                                     const int32_t *__restrict__ col,
                                                                     const VT *__restrict__ val,
                                                                     const double *__restrict__ x,
                                                                     double *__restrict__ y,
                                                                     const int32_t *__restrict__ plan,
                                                                     int32_t lds_cap, double alpha)
{
    extern __shared__ double smem_d[];
    const int64_t b = xcd_remap(blockIdx.x, gridDim.x);
    const int32_t r0 = plan[b], r1 = plan[b + 1];
    const int32_t e0 = row_ptr[r0], e1 = row_ptr[r1];
    const int32_t nr = r1 - r0, ne = e1 - e0;
    const int t = (int)threadIdx.x;
    if (nr == 1) {
        // one (long) row: lanes stride over its entries, straight from memory
        __shared__ double red[CRS_THREADS / WAVE];
        const double xi = x[r0];
        double s = 0.0;
        for (int32_t e = e0 + t; e < e1; e += CRS_THREADS) {
            const int32_t c = ld_stream(col + e);
            const double a = to_f64(ld_stream(val + e));
            s = fma(a, x[c], s);
            if (c > r0) unsafeAtomicAdd(y + c, alpha * (a * xi));
        }
        s = group_sum(s, WAVE);
        if (lane_id() == 0) red[t / WAVE] = s;
        __syncthreads();
        if (t == 0) {
            double tot = red[0];
            for (int w = 1; w < CRS_THREADS / WAVE; ++w) tot += red[w];
            unsafeAtomicAdd(y + r0, alpha * tot);
        }
        return;
    }
    constexpr int MAXJ = CRS_MAX_SHORT_BLOCK_ROWS / CRS_THREADS;
    int G = 64;
    while (G > 1 && G * nr > CRS_THREADS) G >>= 1;
    const int g = t / G, l = t % G;
    int32_t lo[MAXJ], hi[MAXJ];
    if (nr <= CRS_THREADS) {
        lo[0] = g < nr ? row_ptr[r0 + g] : 0;
        hi[0] = g < nr ? row_ptr[r0 + g + 1] : 0;
    } else {
#pragma unroll
        for (int j = 0; j < MAXJ; ++j) {
            const int32_t q = t + j * CRS_THREADS;
            lo[j] = q < nr ? row_ptr[r0 + q] : 0;
            hi[j] = q < nr ? row_ptr[r0 + q + 1] : 0;
        }
    }
    VT *vs = reinterpret_cast<VT *>(smem_d);
    int32_t *cs = reinterpret_cast<int32_t *>(vs + lds_cap);
    constexpr int U = CRS_STREAM_U;
    for (int32_t k0 = 0; k0 < ne; k0 += U * CRS_THREADS) {
        int32_t c[U];
        VT v[U];
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const int32_t k = min(k0 + u * CRS_THREADS + t, ne - 1);
            c[u] = ld_stream(col + e0 + k);
            v[u] = ld_stream(val + e0 + k);
        }
#pragma unroll
        for (int u = 0; u < U; ++u) {
            cs[k0 + u * CRS_THREADS + t] = c[u];
            vs[k0 + u * CRS_THREADS + t] = v[u];
        }
    }
    __syncthreads();
    if (nr <= CRS_THREADS) {
        double s = 0.0;
        if (g < nr) crs_sym_staged_row(vs, cs, x, y, r0 + g, lo[0] - e0, hi[0] - e0, l, G, alpha, s);
        s = group_sum(s, G);
        if (g < nr && l == 0) unsafeAtomicAdd(y + r0 + g, alpha * s);
        return;
    }
#pragma unroll
    for (int j = 0; j < MAXJ; ++j) {
        const int32_t q = t + j * CRS_THREADS;
        if (q < nr) {
            double s = 0.0;
            crs_sym_staged_row(vs, cs, x, y, r0 + q, lo[j] - e0, hi[j] - e0, 0, 1, alpha, s);
            unsafeAtomicAdd(y + r0 + q, alpha * s);
        }
    }
    for (int32_t q = t + MAXJ * CRS_THREADS; q < nr; q += CRS_THREADS) {
        double s = 0.0;
        crs_sym_staged_row(vs, cs, x, y, r0 + q, row_ptr[r0 + q] - e0, row_ptr[r0 + q + 1] - e0, 0, 1, alpha, s);
        unsafeAtomicAdd(y + r0 + q, alpha * s);
    }
}

template <typename VT>
static spmv_status launch_crs_sym(int32_t n, const int32_t *row_ptr, const int32_t *col, const void *val,
                                  const double *x, double *y, double alpha, double beta, const int32_t *plan,
                                  int32_t n_blocks, int32_t block_nnz, bool staged, hipStream_t s)
{
    const int64_t sgrid = std::min<int64_t>(ceil_div(n, 256), 8192);
    sym_scale_kernel<<<(unsigned)sgrid, 256, 0, s>>>(y, n, beta);
    SPMV_CHECK_LAUNCH("spmv_crs_sym scale");
    if (n_blocks == 0) return SPMV_OK;
    if (staged) {
        const int32_t cap = (int32_t)(ceil_div(block_nnz, CRS_LDS_ROUND) * CRS_LDS_ROUND);
        crs_sym_staged_kernel<VT><<<n_blocks, CRS_THREADS, crs_staged_lds_bytes(block_nnz, sizeof(VT)), s>>>(
            row_ptr, col, (const VT *)val, x, y, plan, cap, alpha);
    } else {
        crs_sym_kernel<VT><<<n_blocks, CRS_THREADS, crs_sym_lds_bytes(block_nnz), s>>>(
            row_ptr, col, (const VT *)val, x, y, plan, block_nnz, alpha);
    }
    SPMV_CHECK_LAUNCH("spmv_crs_sym");
    return SPMV_OK;
}

template <typename VT, typename XT>
static spmv_status launch_spmm_crs(const int32_t *row_ptr, const int32_t *col, const void *val, int32_t k,
                                   const void *X, int64_t ldx, void *Y, int64_t ldy, double alpha, double beta,
                                   const int32_t *plan, int32_t n_blocks, hipStream_t s)
{
    constexpr int KB = 8;
    dim3 grid((unsigned)n_blocks, (unsigned)ceil_div(k, KB));
    spmm_crs_kernel<KB, VT, XT><<<grid, CRS_THREADS, 0, s>>>(row_ptr, col, (const VT *)val, (const XT *)X, ldx,
                                                            (XT *)Y, ldy, k, plan, alpha, beta);
    SPMV_CHECK_LAUNCH("spmm_crs");
    return SPMV_OK;
}

template <typename VT, typename XT>
static spmv_status launch_crs(int32_t n_rows, const int32_t *row_ptr, const int32_t *col, const void *val,
                              const void *x, void *y, double alpha, double beta, const int32_t *plan,
                              int32_t n_blocks, int32_t block_nnz, hipStream_t s)
{
    if (plan) {
        if (n_blocks == 0) return SPMV_OK;
        const size_t lds = crs_lds_bytes(block_nnz, IsF64<VT>::value ? 8 : 4);
        crs_block_kernel<VT, XT><<<n_blocks, CRS_THREADS, lds, s>>>(row_ptr, col, (const VT *)val, (const XT *)x,
                                                                   (XT *)y, plan, alpha, beta);
    } else {
        int64_t grid = ceil_div(n_rows, CRS_THREADS / WAVE);
        crs_wave_kernel<VT, XT><<<(unsigned)grid, CRS_THREADS, 0, s>>>(n_rows, row_ptr, col, (const VT *)val,
                                                                       (const XT *)x, (XT *)y, alpha, beta);
    }
    SPMV_CHECK_LAUNCH("spmv_crs");
    return SPMV_OK;
}

template <typename VT, typename XT>
static spmv_status launch_crs_staged(const int32_t *row_ptr, const int32_t *col, const void *val, const void *x,
                                     void *y, double alpha, double beta, const int32_t *plan, int32_t n_blocks,
                                     int32_t block_nnz, hipStream_t s)
{
    if (n_blocks == 0) return SPMV_OK;
    const int32_t cap = (int32_t)(ceil_div(block_nnz, CRS_LDS_ROUND) * CRS_LDS_ROUND);
    crs_staged_kernel<VT, XT><<<n_blocks, CRS_THREADS, crs_staged_lds_bytes(block_nnz, sizeof(VT)), s>>>(
        row_ptr, col, (const VT *)val, (const XT *)x, (XT *)y, plan, cap, alpha, beta);
    SPMV_CHECK_LAUNCH("spmv_crs_staged");
    return SPMV_OK;
}

int32_t crs_default_block_nnz() { return CRS_DEFAULT_BLOCK_NNZ; }

// Greedy host planner shared by spmv_crs_plan and the multi-vector planner.
void crs_plan_rows(int32_t n_rows, const int32_t *rp, int32_t T, std::vector<int32_t> &out)
{
    out.clear();
    out.push_back(0);
    int32_t start = 0;
    int64_t cur = 0, longest = 0;
    for (int32_t r = 0; r < n_rows; ++r) {
        const int64_t len = (int64_t)rp[r + 1] - rp[r];
        const int32_t nr = r - start;
        const int64_t lg = std::max(longest, len);
        const int32_t row_cap = lg <= CRS_SHORT_ROW ? CRS_MAX_SHORT_BLOCK_ROWS : CRS_MAX_BLOCK_ROWS;
        if (nr > 0 && (cur + len > T || nr >= row_cap)) {
            out.push_back(r);
            start = r;
            cur = 0;
            longest = 0;
        }
        if (len > T) {                 // a long row is a block of its own
            out.push_back(r + 1);
            start = r + 1;
            cur = 0;
            longest = 0;
            continue;
        }
        cur += len;
        longest = std::max(longest, len);
    }
    if (start < n_rows) out.push_back(n_rows);
}

}  // namespace spmv

using namespace spmv;

extern "C" {

spmv_status spmv_crs_plan(int32_t n_rows, const int32_t *row_ptr, int32_t block_nnz, int32_t *plan,
                          int32_t plan_cap, int32_t *h_n_blocks, void *stream)
{
    SPMV_REQUIRE(n_rows >= 0, "spmv_crs_plan: n_rows < 0");
    SPMV_REQUIRE(h_n_blocks, "spmv_crs_plan: null h_n_blocks");
    SPMV_REQUIRE(row_ptr, "spmv_crs_plan: null row_ptr");
    if (block_nnz == 0) block_nnz = CRS_DEFAULT_BLOCK_NNZ;
    SPMV_REQUIRE(block_nnz >= CRS_THREADS && block_nnz <= CRS_MAX_BLOCK_NNZ,
                 "spmv_crs_plan: block_nnz must be in [256, 4096]");
    hipStream_t s = as_stream(stream);
    std::vector<int32_t> rp((size_t)n_rows + 1);
    SPMV_HIP(hipMemcpyAsync(rp.data(), row_ptr, sizeof(int32_t) * rp.size(), hipMemcpyDeviceToHost, s));
    SPMV_HIP(hipStreamSynchronize(s));
    for (int32_t r = 0; r < n_rows; ++r)
        if (rp[r + 1] < rp[r]) return fail(SPMV_ERR_BAD_FORMAT, "spmv_crs_plan: row_ptr decreases");
    std::vector<int32_t> blocks;
    crs_plan_rows(n_rows, rp.data(), block_nnz, blocks);
    int32_t nb = (int32_t)blocks.size() - 1;
    *h_n_blocks = nb;
    if (!plan || plan_cap < nb + 1) return fail(SPMV_ERR_CAPACITY, "spmv_crs_plan: plan capacity < n_blocks+1");
    SPMV_HIP(hipMemcpyAsync(plan, blocks.data(), sizeof(int32_t) * blocks.size(), hipMemcpyHostToDevice, s));
    SPMV_HIP(hipStreamSynchronize(s));
    return SPMV_OK;
}

spmv_status spmv_crs(int32_t n_rows, int32_t n_cols, const int32_t *row_ptr, const int32_t *col_idx,
                     const void *val, spmv_dtype val_dt, const void *x, void *y, spmv_dtype vec_dt, double alpha,
                     double beta, const int32_t *plan, int32_t n_blocks, int32_t block_nnz, void *stream)
{
    SPMV_REQUIRE(n_rows >= 0 && n_cols >= 0, "spmv_crs: negative size");
    SPMV_REQUIRE(valid_dtype(val_dt) && valid_vec_dtype(vec_dt), "spmv_crs: bad dtype");
    if (n_rows == 0) return SPMV_OK;
    SPMV_REQUIRE(row_ptr && y, "spmv_crs: null row_ptr or y");
    if (plan) {
        SPMV_REQUIRE(n_blocks >= 0, "spmv_crs: n_blocks < 0");
        if (block_nnz == 0) block_nnz = CRS_DEFAULT_BLOCK_NNZ;
        SPMV_REQUIRE(block_nnz >= CRS_THREADS && block_nnz <= CRS_MAX_BLOCK_NNZ,
                     "spmv_crs: block_nnz must be in [256, 4096]");
    }
    hipStream_t s = as_stream(stream);
#define CRS_CASE(VDT, VT, XDT, XT)                                                                          \
    if (val_dt == VDT && vec_dt == XDT)                                                                     \
        return launch_crs<VT, XT>(n_rows, row_ptr, col_idx, val, x, y, alpha, beta, plan, n_blocks, block_nnz, s);
    CRS_CASE(SPMV_F64, double, SPMV_F64, double)
    CRS_CASE(SPMV_F32, float, SPMV_F64, double)
    CRS_CASE(SPMV_BF16, bf16, SPMV_F64, double)
    CRS_CASE(SPMV_F32, float, SPMV_F32, float)
    CRS_CASE(SPMV_BF16, bf16, SPMV_F32, float)
    CRS_CASE(SPMV_F64, double, SPMV_F32, float)
#undef CRS_CASE
    return fail(SPMV_ERR_UNSUPPORTED, "spmv_crs: dtype combination");
}

spmv_status spmv_crs_staged(int32_t n_rows, int32_t n_cols, const int32_t *row_ptr, const int32_t *col_idx,
                            const void *val, spmv_dtype val_dt, const void *x, void *y, spmv_dtype vec_dt,
                            double alpha, double beta, const int32_t *plan, int32_t n_blocks, int32_t block_nnz,
                            void *stream)
{
    SPMV_REQUIRE(n_rows >= 0 && n_cols >= 0, "spmv_crs_staged: negative size");
    SPMV_REQUIRE(valid_dtype(val_dt) && valid_vec_dtype(vec_dt), "spmv_crs_staged: bad dtype");
    if (n_rows == 0) return SPMV_OK;
    SPMV_REQUIRE(row_ptr && y && plan, "spmv_crs_staged: null row_ptr, y or plan");
    SPMV_REQUIRE(n_blocks >= 0, "spmv_crs_staged: n_blocks < 0");
    if (block_nnz == 0) block_nnz = CRS_DEFAULT_BLOCK_NNZ;
    SPMV_REQUIRE(block_nnz >= CRS_THREADS && block_nnz <= CRS_MAX_BLOCK_NNZ,
                 "spmv_crs_staged: block_nnz must be in [256, 4096]");
    hipStream_t s = as_stream(stream);
#define CRSS_CASE(VDT, VT, XDT, XT)                                                                          \
    if (val_dt == VDT && vec_dt == XDT)                                                                      \
        return launch_crs_staged<VT, XT>(row_ptr, col_idx, val, x, y, alpha, beta, plan, n_blocks, block_nnz, s);
    CRSS_CASE(SPMV_F64, double, SPMV_F64, double)
    CRSS_CASE(SPMV_F32, float, SPMV_F64, double)
    CRSS_CASE(SPMV_BF16, bf16, SPMV_F64, double)
    CRSS_CASE(SPMV_F32, float, SPMV_F32, float)
    CRSS_CASE(SPMV_BF16, bf16, SPMV_F32, float)
    CRSS_CASE(SPMV_F64, double, SPMV_F32, float)
#undef CRSS_CASE
    return fail(SPMV_ERR_UNSUPPORTED, "spmv_crs_staged: dtype combination");
}

static spmv_status crs_sym_entry(int32_t n, const int32_t *row_ptr, const int32_t *col_idx, const void *val,
                                 spmv_dtype val_dt, const void *x, void *y, spmv_dtype vec_dt, double alpha,
                                 double beta, const int32_t *plan, int32_t n_blocks, int32_t block_nnz, bool staged,
                                 void *stream)
{
    SPMV_REQUIRE(n >= 0, "spmv_crs_sym: negative size");
    SPMV_REQUIRE(valid_dtype(val_dt), "spmv_crs_sym: bad value dtype");
    if (vec_dt != SPMV_F64) return fail(SPMV_ERR_UNSUPPORTED, "spmv_crs_sym: x and y must be FP64");
    if (n == 0) return SPMV_OK;
    SPMV_REQUIRE(row_ptr && x && y && plan, "spmv_crs_sym: null pointer");
    SPMV_REQUIRE(n_blocks >= 0, "spmv_crs_sym: n_blocks < 0");
    if (block_nnz == 0) block_nnz = CRS_DEFAULT_BLOCK_NNZ;
    SPMV_REQUIRE(block_nnz >= CRS_THREADS && block_nnz <= CRS_MAX_BLOCK_NNZ,
                 "spmv_crs_sym: block_nnz must be in [256, 4096]");
    hipStream_t s = as_stream(stream);
    const double *xd = (const double *)x;
    double *yd = (double *)y;
    switch (val_dt) {
    case SPMV_F64: return launch_crs_sym<double>(n, row_ptr, col_idx, val, xd, yd, alpha, beta, plan, n_blocks,
                                                 block_nnz, staged, s);
    case SPMV_F32: return launch_crs_sym<float>(n, row_ptr, col_idx, val, xd, yd, alpha, beta, plan, n_blocks,
                                                block_nnz, staged, s);
    case SPMV_BF16: return launch_crs_sym<bf16>(n, row_ptr, col_idx, val, xd, yd, alpha, beta, plan, n_blocks,
                                                block_nnz, staged, s);
    default: return fail(SPMV_ERR_UNSUPPORTED, "spmv_crs_sym: value dtype");
    }
}

spmv_status spmv_crs_sym(int32_t n, const int32_t *row_ptr, const int32_t *col_idx, const void *val,
                         spmv_dtype val_dt, const void *x, void *y, spmv_dtype vec_dt, double alpha, double beta,
                         const int32_t *plan, int32_t n_blocks, int32_t block_nnz, void *stream)
{
    return crs_sym_entry(n, row_ptr, col_idx, val, val_dt, x, y, vec_dt, alpha, beta, plan, n_blocks, block_nnz,
                         false, stream);
}

spmv_status spmv_crs_sym_staged(int32_t n, const int32_t *row_ptr, const int32_t *col_idx, const void *val,
                                spmv_dtype val_dt, const void *x, void *y, spmv_dtype vec_dt, double alpha,
                                double beta, const int32_t *plan, int32_t n_blocks, int32_t block_nnz, void *stream)
{
    return crs_sym_entry(n, row_ptr, col_idx, val, val_dt, x, y, vec_dt, alpha, beta, plan, n_blocks, block_nnz,
                         true, stream);
}

spmv_status spmv_crs_split(int32_t n_rows, int32_t n_cols, const int32_t *row_ptr_all, const int32_t *dest_all,
                           const int32_t *slot_ptr, const int32_t *col_idx, const void *val, const int64_t *h_bounds,
                           const int64_t *h_row_off, spmv_dtype val_dt, const int32_t *plan_all,
                           const int32_t *h_plan_off, const int32_t *h_n_blocks, int32_t block_nnz, const void *x,
                           void *y, spmv_dtype vec_dt, double alpha, double beta, void *ws, size_t ws_bytes,
                           void *stream)
{
    SPMV_REQUIRE(n_rows >= 0 && n_cols >= 0, "spmv_crs_split: negative size");
    SPMV_REQUIRE(valid_dtype(val_dt) && valid_vec_dtype(vec_dt), "spmv_crs_split: bad dtype");
    if (n_rows == 0) return SPMV_OK;
    SPMV_REQUIRE(row_ptr_all && slot_ptr && plan_all && h_plan_off && h_n_blocks && h_bounds && h_row_off && y,
                 "spmv_crs_split: null pointer");
    const int64_t n_slots = h_row_off[SPLIT_PARTS];
    SPMV_REQUIRE(n_slots >= 0 && n_slots <= (int64_t)SPLIT_PARTS * n_rows, "spmv_crs_split: bad h_row_off");
    SPMV_REQUIRE(n_slots == 0 || dest_all, "spmv_crs_split: null dest_all");
    SPMV_REQUIRE(ws && ws_bytes >= spmv_split_workspace_size(n_slots), "spmv_crs_split: workspace too small");
    if (block_nnz == 0) block_nnz = CRS_DEFAULT_BLOCK_NNZ;
    SPMV_REQUIRE(block_nnz >= CRS_THREADS && block_nnz <= CRS_MAX_BLOCK_NNZ,
                 "spmv_crs_split: block_nnz must be in [256, 4096]");
    CrsSplitTab T{};
    int64_t max_nb = 0;
    for (int k = 0; k < SPLIT_PARTS; ++k) {
        SPMV_REQUIRE(h_n_blocks[k] >= 0 && h_plan_off[k] >= 0, "spmv_crs_split: bad part plan");
        SPMV_REQUIRE(h_row_off[k] >= 0 && h_row_off[k] <= h_row_off[k + 1], "spmv_crs_split: bad h_row_off");
        SPMV_REQUIRE(h_n_blocks[k] == 0 || h_row_off[k + 1] > h_row_off[k], "spmv_crs_split: plan of an empty part");
        T.base[k] = h_bounds[k];
        T.row_off[k] = (int32_t)h_row_off[k];
        T.plan_off[k] = h_plan_off[k];
        T.n_blocks[k] = h_n_blocks[k];
        max_nb = std::max<int64_t>(max_nb, h_n_blocks[k]);
    }
    hipStream_t s = as_stream(stream);
    double *slots = (double *)ws;
    const unsigned grid = (unsigned)(max_nb * SPLIT_PARTS);
    if (grid) {
#define CSPLIT_CASE(VDT, VT, XDT, XT)                                                                          \
    if (val_dt == VDT && vec_dt == XDT) {                                                                      \
        const size_t lds = crs_lds_bytes(block_nnz, 8);                                                        \
        crs_split_kernel<VT, XT><<<grid, CRS_THREADS, lds, s>>>(row_ptr_all, dest_all, col_idx, (const VT *)val, \
                                                               (const XT *)x, slots, plan_all, T);             \
    } else
        CSPLIT_CASE(SPMV_F64, double, SPMV_F64, double)
        CSPLIT_CASE(SPMV_F32, float, SPMV_F64, double)
        CSPLIT_CASE(SPMV_BF16, bf16, SPMV_F64, double)
        CSPLIT_CASE(SPMV_F32, float, SPMV_F32, float)
        CSPLIT_CASE(SPMV_BF16, bf16, SPMV_F32, float)
        CSPLIT_CASE(SPMV_F64, double, SPMV_F32, float)
        return fail(SPMV_ERR_UNSUPPORTED, "spmv_crs_split: dtype combination");
#undef CSPLIT_CASE
        SPMV_CHECK_LAUNCH("spmv_crs_split");
    }
    return launch_combine(n_rows, slot_ptr, slots, y, vec_dt, alpha, beta, s);
}

}  // extern "C"

// Multi-vector CRS straight from the column-major X (no workspace); called by
// spmm_crs, which validated the arguments.
spmv_status spmv::spmm_crs_colmajor(int32_t n_rows, int32_t n_cols, const int32_t *row_ptr, const int32_t *col_idx,
                                    const void *val, spmv_dtype val_dt, int32_t k, const void *X, int64_t ldx,
                                    void *Y, int64_t ldy, spmv_dtype vec_dt, double alpha, double beta,
                                    const int32_t *plan, int32_t n_blocks, hipStream_t s)
{
    (void)n_rows;
    (void)n_cols;
    if (n_blocks == 0) return SPMV_OK;
#define SPMM_CASE(VDT, VT, XDT, XT)           \
    if (val_dt == VDT && vec_dt == XDT)       \
        return launch_spmm_crs<VT, XT>(row_ptr, col_idx, val, k, X, ldx, Y, ldy, alpha, beta, plan, n_blocks, s);
    SPMM_CASE(SPMV_F64, double, SPMV_F64, double)
    SPMM_CASE(SPMV_F32, float, SPMV_F32, float)
    SPMM_CASE(SPMV_F32, float, SPMV_F64, double)
    SPMM_CASE(SPMV_BF16, bf16, SPMV_F32, float)
    SPMM_CASE(SPMV_BF16, bf16, SPMV_F64, double)
    SPMM_CASE(SPMV_F64, double, SPMV_F32, float)
#undef SPMM_CASE
    return fail(SPMV_ERR_UNSUPPORTED, "spmm_crs: dtype combination");
}
