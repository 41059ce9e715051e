// Multi-vector products Y = alpha*A X + beta*Y, X and Y column-major (k columns).
//
// A column-major X makes every stored entry gather k separate 8-byte values
// from k far-apart columns: k L2 lines per entry.  With a workspace the
// library first copies X into an interleaved (row-major) block Xr, one
// transposing pass at streaming speed, and then every entry gathers its k
// values as one contiguous run of k*8 bytes.  Each row is handled by a group
// of LPR lanes (K2 = k rounded up to a power of two, at most 64; LPR = K2 up
// to 8, then 8 or 16), lane j owning columns j, j + LPR, ...: val/col are read
// once per entry for all k columns and each gather load of a group is
// contiguous.  Long rows get several groups whose partial sums meet in LDS and
// are added in a fixed order.  Y is written column-major directly.
//
// Without a workspace the column-major kernels of crs.hip / jds.hip run.
#include <algorithm>
#include <vector>

#include "common.hpp"

namespace spmv {

// Workgroup sizes, measured on the power-law matrix: the CRS kernel's rows
// are handled in rounds that each wait on their gathers, and 128-lane groups
// for k <= 8 keep more rounds in flight (10-14% faster than 256); the JDS
// kernel's classes favour larger groups (512: 3-5% faster than 256).
// CRS workgroup size: one wavefront for FP32 vectors (against 128 lanes:
// 1.14x faster at k = 8, 1.01x at k = 32; 256 lanes at k = 32: 1.13x slower),
// 128 lanes for FP64 up to k = 8 (64: 4% slower), 256 above (128: 5% slower).
template <int K2, typename XT>
constexpr int mm_crs_threads() { return sizeof(XT) == 4 ? 64 : (K2 <= 8 ? 128 : 256); }
// Lanes per row group (LPR) for k > 8: each lane owns k / LPR columns, so a
// wavefront keeps 64 / LPR rows' gathers in flight.  Measured on the
// power-law matrix at k = 32: CRS is fastest with 16 lanes for FP64 vectors
// (8 lanes: 11% slower, 32: 1% slower) and 8 for FP32 (1.30x faster than
// 32); JDS with 8 for both.
template <int K2, typename XT>
constexpr int mm_crs_lpr() { return K2 <= 8 ? K2 : (sizeof(XT) == 8 ? 16 : 8); }
template <int K2, typename XT>
constexpr int mm_jds_lpr() { return K2 <= 8 ? K2 : 8; }
constexpr int MM_JDS_THREADS = 512;
constexpr int MM_MAX_K2 = 64;
constexpr int MM_JP_LDS = 4097;            // jd_ptr entries staged in LDS (ndiag <= 4096)
// Rows of a multi-row CRS block whose offsets can be staged in LDS: twice
// the block's entries (a block of non-empty rows has at most block_nnz), at
// most 2048 (the planner's largest block of short rows).
__host__ __device__ constexpr int32_t mm_rp_lds(int32_t block_nnz)
{
    return 2 * block_nnz < 2048 ? 2 * block_nnz : 2048;
}
// Y tile of a multi-row CRS block with FP64 vectors and K2 >= 16: rows x K2
// doubles when they fit in this many (8 KB).  Measured on the power-law
// matrix: k = 32 1.07x faster (Y written 0.84 instead of 1.0 GB); at k = 8
// the tile halves the Y writes but its LDS costs a third of the occupancy of
// the 128-lane workgroups, 1.14x slower, so small k writes directly.
constexpr int MM_YTILE_ELEMS = 1024;
template <int K2>
constexpr size_t mm_ytile_bytes() { return K2 >= 16 ? sizeof(double) * MM_YTILE_ELEMS + 16 : 0; }

// Xr[c*k + j] = X[c + j*ldx] (2 <= k <= 64): a block of STAGE_ELEMS / k rows
// through LDS.  Reads walk each column's run of rows (coalesced), writes walk
// the block's contiguous stretch of Xr (coalesced).  Each lane issues all
// of its STAGE_PER_LANE reads before its LDS stores, and all of its LDS reads
// before its global stores, so a lane keeps 8 loads in flight.  (k = 1
// needs no staging: X itself is the row-major block.)
constexpr int STAGE_ELEMS = 2048;
constexpr int STAGE_THREADS = 256;
constexpr int STAGE_PER_LANE = STAGE_ELEMS / STAGE_THREADS;

template <typename T>
__global__ __launch_bounds__(STAGE_THREADS) void stage_rowmajor_kernel(int64_t n, int32_t k, const T *__restrict__ X,
                                                                       int64_t ldx, T *__restrict__ Xr)
{
    __shared__ T tile[STAGE_ELEMS + STAGE_ELEMS / 2];   // rows * (k + 1) for k >= 2
    const int rows = STAGE_ELEMS / k;                   // rows of this block
    const int64_t c0 = (int64_t)blockIdx.x * rows;
    const int nr = n - c0 < rows ? (int)(n - c0) : rows;
    const int tot = nr * k;
    const int stride = k + 1;                           // padded LDS rows
    const int t = (int)threadIdx.x;
    T v[STAGE_PER_LANE];
#pragma unroll
    for (int e = 0; e < STAGE_PER_LANE; ++e) {
        const int f = t + e * STAGE_THREADS;            // f < rows * k <= STAGE_ELEMS
        const int r = min(f % rows, nr - 1), j = min(f / rows, k - 1);
        v[e] = X[c0 + r + (int64_t)j * ldx];
    }
#pragma unroll
    for (int e = 0; e < STAGE_PER_LANE; ++e) {
        const int f = t + e * STAGE_THREADS;
        const int r = f % rows, j = f / rows;
        if (r < nr && j < k) tile[r * stride + j] = v[e];
    }
    __syncthreads();
#pragma unroll
    for (int e = 0; e < STAGE_PER_LANE; ++e) {
        const int f = min(t + e * STAGE_THREADS, tot - 1);
        v[e] = tile[(f / k) * stride + f % k];
    }
#pragma unroll
    for (int e = 0; e < STAGE_PER_LANE; ++e) {
        const int f = t + e * STAGE_THREADS;
        if (f < tot) Xr[c0 * k + f] = v[e];
    }
}

// One group of LPR lanes per (row, part): lane j accumulates columns j,
// j + LPR, ..., j + (CPL-1)*LPR over entries e_begin, e_begin + e_step, ...
template <int LPR, int CPL, bool WIDE, typename VT, typename XT>
__device__ __forceinline__ void mm_group_sum(const int32_t *__restrict__ col, const VT *__restrict__ val,
                                             const XT *__restrict__ Xr, int32_t k, int j, int64_t e_begin,
                                             int64_t e_end, int64_t e_step, double (&out)[CPL])
{
    typedef typename Acc<WIDE>::T acc_t;
    acc_t s[CPL];
#pragma unroll
    for (int t = 0; t < CPL; ++t) s[t] = 0;
    // entries per trip: eight gathers in flight per lane (U * CPL = 8);
    // measured at k = 8 (U = 8: 4-11% faster than 4) and k = 32 FP32 (U = 2)
    constexpr int U = CPL >= 8 ? 1 : 8 / CPL;
    int64_t e = e_begin;
    for (; e + (U - 1) * e_step < e_end; e += U * e_step) {
        int32_t c[U];
        VT v[U];
#pragma unroll
        for (int u = 0; u < U; ++u) {
            c[u] = col[e + u * e_step];
            v[u] = val[e + u * e_step];
        }
        XT xv[U][CPL];
#pragma unroll
        for (int u = 0; u < U; ++u)
#pragma unroll
            for (int t = 0; t < CPL; ++t)
                xv[u][t] = t * LPR + j < k ? Xr[(int64_t)c[u] * k + t * LPR + j] : XT(0);
#pragma unroll
        for (int u = 0; u < U; ++u)
#pragma unroll
            for (int t = 0; t < CPL; ++t) s[t] = Acc<WIDE>::mac(s[t], v[u], xv[u][t]);
    }
    for (; e < e_end; e += e_step) {
        const int32_t c = col[e];
        const VT v = val[e];
#pragma unroll
        for (int t = 0; t < CPL; ++t) {
            const XT xv = t * LPR + j < k ? Xr[(int64_t)c * k + t * LPR + j] : XT(0);
            s[t] = Acc<WIDE>::mac(s[t], v, xv);
        }
    }
#pragma unroll
    for (int t = 0; t < CPL; ++t) out[t] = (double)s[t];
}

// Entry-balanced multi-row block (staged in LDS): group g takes the g-th of
// NG equal shares [cs, ce) of the block's entries, walks them in order and
// sums row by row, so no group waits on a longer row than its neighbours.
// A row that starts and ends inside the share is written directly; a row
// crossing a share boundary leaves its pieces in LDS (tail: the piece in the
// share where it starts; lead: its pieces in later shares) and the group
// where it starts adds them in share order.  Empty rows (beta*y) are written
// by the group whose share holds their position; those after the last entry
// by the last group.
template <int LPR, int CPL, int NG, int K2, bool WIDE, typename VT, typename XT>
__device__ __forceinline__ void mm_crs_balanced(const int32_t *rp, int32_t r0, int32_t r1,
                                                const int32_t *col_s, const VT *val_s,
                                                const XT *__restrict__ Xr, int32_t k, XT *__restrict__ Y,
                                                int64_t ldy, double alpha, double beta, int g, int j,
                                                double (*lead)[K2], double (*tail)[K2], int32_t *lead_row,
                                                int32_t *tail_row, double *ytile)
{
    typedef typename Acc<WIDE>::T acc_t;
    constexpr int U = CPL >= 8 ? 1 : 8 / CPL;
    const int32_t E = rp[r1 - r0];
    const int32_t cs = (int32_t)((int64_t)g * E / NG), ce = (int32_t)((int64_t)(g + 1) * E / NG);
    // with a tile (blocks of few rows), finished rows wait in LDS and the
    // block writes them at the end, column by column, in runs of consecutive
    // rows: whole lines of a column leave together instead of 8-byte pieces
    auto put = [&](int32_t row, const acc_t *v) {
#pragma unroll
        for (int t = 0; t < CPL; ++t)
            if (t * LPR + j < k) {
                if (ytile) ytile[(int64_t)(t * LPR + j) * (r1 - r0) + (row - r0)] = (double)v[t];
                else write_y(Y + (int64_t)(t * LPR + j) * ldy, row, (double)v[t], alpha, beta);
            }
    };
    acc_t zero[CPL];
#pragma unroll
    for (int t = 0; t < CPL; ++t) zero[t] = 0;
    if (j == 0) lead_row[g] = tail_row[g] = -1;
    __syncthreads();
    // first row starting at or after entry cs
    int32_t lo = r0, hi = r1 + 1;
    while (lo < hi) {
        const int32_t mid = (lo + hi) >> 1;
        if (rp[mid - r0] < cs) lo = mid + 1;
        else hi = mid;
    }
    if (cs == ce) {
        if (g == NG - 1)
            for (int32_t r = lo; r < r1; ++r) put(r, zero);
    } else {
        int32_t cr;
        bool here;
        if (lo > r1 || rp[lo - r0] > cs) {
            cr = lo - 1;                                   // the row holding entry cs started before it
            here = false;
        } else {
            cr = lo;
            here = true;
            while (cr < r1 && rp[cr + 1 - r0] == cs) put(cr++, zero);    // empty rows at cs
        }
        int32_t bnd = rp[cr + 1 - r0];
        acc_t s[CPL];
#pragma unroll
        for (int t = 0; t < CPL; ++t) s[t] = 0;
        for (int32_t e = cs; e < ce; e += U) {
            int32_t c[U];
            VT v[U];
#pragma unroll
            for (int u = 0; u < U; ++u) {
                const int32_t q = e + u < ce ? e + u : ce - 1;
                c[u] = col_s[q];
                v[u] = val_s[q];
            }
            XT xv[U][CPL];
#pragma unroll
            for (int u = 0; u < U; ++u)
#pragma unroll
                for (int t = 0; t < CPL; ++t)
                    xv[u][t] = t * LPR + j < k ? Xr[(int64_t)c[u] * k + t * LPR + j] : XT(0);
#pragma unroll
            for (int u = 0; u < U; ++u) {
                if (e + u >= ce) break;
                while (e + u == bnd) {                      // row cr ended before this entry
                    if (here) {
                        put(cr, s);
                    } else {
#pragma unroll
                        for (int t = 0; t < CPL; ++t) lead[g][t * LPR + j] = (double)s[t];
                        if (j == 0) lead_row[g] = cr;
                    }
#pragma unroll
                    for (int t = 0; t < CPL; ++t) s[t] = 0;
                    ++cr;
                    here = true;
                    while (cr < r1 && rp[cr + 1 - r0] == e + u) put(cr++, zero);   // empty rows
                    bnd = rp[cr + 1 - r0];
                }
#pragma unroll
                for (int t = 0; t < CPL; ++t) s[t] = Acc<WIDE>::mac(s[t], v[u], xv[u][t]);
            }
        }
        if (bnd == ce) {                                    // row cr ends with the share
            if (here) {
                put(cr, s);
            } else {
#pragma unroll
                for (int t = 0; t < CPL; ++t) lead[g][t * LPR + j] = (double)s[t];
                if (j == 0) lead_row[g] = cr;
            }
            ++cr;
            if (g == NG - 1)
                while (cr < r1) put(cr++, zero);
        } else if (here) {                                  // continues into the next shares
#pragma unroll
            for (int t = 0; t < CPL; ++t) tail[g][t * LPR + j] = (double)s[t];
            if (j == 0) tail_row[g] = cr;
        } else {                                            // the whole share is inside one row
#pragma unroll
            for (int t = 0; t < CPL; ++t) lead[g][t * LPR + j] = (double)s[t];
            if (j == 0) lead_row[g] = cr;
        }
    }
    __syncthreads();
    const int32_t R = tail_row[g];
    if (R >= 0) {
        acc_t a[CPL];
#pragma unroll
        for (int t = 0; t < CPL; ++t) a[t] = (acc_t)tail[g][t * LPR + j];
        for (int q = g + 1; q < NG; ++q) {
            const bool empty = (int64_t)q * E / NG == (int64_t)(q + 1) * E / NG;
            if (empty) continue;
            if (lead_row[q] != R) break;
#pragma unroll
            for (int t = 0; t < CPL; ++t) a[t] += (acc_t)lead[q][t * LPR + j];
        }
        put(R, a);
    }
    if (ytile) {
        __syncthreads();
        const int32_t nr = r1 - r0;
        const int lane = g * LPR + j;
        for (int64_t q = lane; q < (int64_t)nr * k; q += NG * LPR) {
            const int32_t c = (int32_t)(q / nr), rr = (int32_t)(q % nr);
            write_y(Y + (int64_t)c * ldy, r0 + rr, ytile[q], alpha, beta);
        }
    }
}

// CRS, interleaved X.  One workgroup per plan block of nr rows: GPR groups
// per row (GPR = largest power of two <= NG/nr), the row's entries dealt to
// its groups with stride GPR; the GPR partials are added in group order.  A
// multi-row block first copies its val/col into LDS with coalesced loads
// (the groups of a wavefront work on different rows, so reading val/col
// straight from memory would touch one line per group per load).
template <int K2, int NT, typename VT, typename XT>
__global__ __launch_bounds__(NT) void spmm_crs_il_kernel(const int32_t *__restrict__ row_ptr,
                                                                 const int32_t *__restrict__ col,
                                                                 const VT *__restrict__ val,
                                                                 const XT *__restrict__ Xr, int32_t k,
                                                                 XT *__restrict__ Y, int64_t ldy,
                                                                 const int32_t *__restrict__ plan, int32_t block_nnz,
                                                                 double alpha, double beta)
{
    constexpr int LPR = mm_crs_lpr<K2, XT>();           // lanes per row group
    constexpr int CPL = K2 / LPR;                       // columns per lane
    constexpr int NG = NT / LPR;
    constexpr bool F64 = IsF64<VT>::value;
    __shared__ double part[NG][K2];
    __shared__ double tailp[sizeof(XT) == 8 ? NG : 1][K2];
    __shared__ int32_t lead_row[NG], tail_row[NG];
    // block_nnz cols, block_nnz values, then the block's row offsets
    extern __shared__ int32_t mm_stage[];
    int32_t *col_s = mm_stage;
    VT *val_s = reinterpret_cast<VT *>(mm_stage + ((block_nnz + 3) & ~3));
    int32_t *rp_s = reinterpret_cast<int32_t *>(val_s + ((block_nnz + 1) & ~1));
    const int64_t b = xcd_remap(blockIdx.x, gridDim.x);
    const int32_t r0 = plan[b], r1 = plan[b + 1];
    const int32_t nr = r1 - r0;
    const int t = (int)threadIdx.x;
    const int g = t / LPR, j = t % LPR;
    int GPR = 1;
    while (GPR * 2 * nr <= NG) GPR *= 2;
    const int sub = g % GPR;
    const int rows_per_round = NG / GPR;
    const bool wide = !F64 && nr == 1 && row_ptr[r1] - row_ptr[r0] > SPMV_WIDE_ROW_NNZ;
    const bool staged = nr > 1;                           // then ne <= block_nnz (plan contract)
    // with FP64 vectors the row offsets go to LDS too when the block has at
    // most mm_rp_lds(block_nnz) rows (the share search and the row ends are
    // then LDS reads, not dependent memory round trips: 1.15x at k = 8 and 32);
    // FP32 vectors keep them in memory (their one-wavefront workgroups need
    // the LDS for occupancy)
    const bool rp_lds = sizeof(XT) == 8 && staged && nr <= mm_rp_lds(block_nnz);
    int32_t be0 = 0;
    if (staged) {
        be0 = row_ptr[r0];
        const int32_t ne = row_ptr[r1] - be0;
        for (int32_t i = t; i < ne; i += NT) {
            col_s[i] = ld_stream(col + be0 + i);
            val_s[i] = ld_stream(val + be0 + i);
        }
        if (rp_lds)
            for (int32_t i = t; i <= nr; i += NT) rp_s[i] = row_ptr[r0 + i] - be0;
        __syncthreads();
        // FP64 vectors: entry-balanced shares (3-9% faster than rows in
        // rounds on the power-law matrix); FP32 vectors keep the rounds
        // (the shares were 1.3x slower at k = 32 with one-wavefront groups)
        if constexpr (sizeof(XT) == 8) {
            if (rp_lds) {
                // after the row offsets, rounded up to 16 bytes
                const uintptr_t tile_at = ((uintptr_t)(rp_s + mm_rp_lds(block_nnz) + 1) + 15) & ~(uintptr_t)15;
                double *ytile = K2 >= 16 && nr * K2 <= MM_YTILE_ELEMS ? reinterpret_cast<double *>(tile_at) : nullptr;
                mm_crs_balanced<LPR, CPL, NG, K2, F64, VT, XT>(rp_s, r0, r1, col_s, val_s, Xr, k, Y, ldy, alpha,
                                                               beta, g, j, part, tailp, lead_row, tail_row, ytile);
                return;
            }
        }
    }
    for (int32_t rbase = r0; rbase < r1; rbase += rows_per_round) {
        const int32_t row = rbase + g / GPR;
        double td[CPL];
#pragma unroll
        for (int q = 0; q < CPL; ++q) td[q] = 0.0;
        if (row < r1) {
            const int32_t e0 = rp_lds ? rp_s[row - r0] + be0 : row_ptr[row];
            const int32_t e1 = rp_lds ? rp_s[row + 1 - r0] + be0 : row_ptr[row + 1];
            if (staged) {
                if (F64) mm_group_sum<LPR, CPL, true, VT, XT>(col_s, val_s, Xr, k, j, e0 - be0 + sub, e1 - be0, GPR, td);
                else mm_group_sum<LPR, CPL, false, VT, XT>(col_s, val_s, Xr, k, j, e0 - be0 + sub, e1 - be0, GPR, td);
            } else if (F64 || wide) {
                mm_group_sum<LPR, CPL, true, VT, XT>(col, val, Xr, k, j, e0 + sub, e1, GPR, td);
            } else {
                mm_group_sum<LPR, CPL, false, VT, XT>(col, val, Xr, k, j, e0 + sub, e1, GPR, td);
            }
        }
        if (GPR > 1) {
#pragma unroll
            for (int q = 0; q < CPL; ++q) part[g][q * LPR + j] = td[q];
            __syncthreads();
            if (sub == 0 && row < r1) {
#pragma unroll
                for (int q = 0; q < CPL; ++q) {
                    if (F64 || wide) {
                        double t2 = 0.0;
                        for (int p = 0; p < GPR; ++p) t2 += part[g + p][q * LPR + j];
                        td[q] = t2;
                    } else {
                        float t2 = 0.0f;
                        for (int p = 0; p < GPR; ++p) t2 += (float)part[g + p][q * LPR + j];
                        td[q] = (double)t2;
                    }
                }
            }
            __syncthreads();
        }
        if (sub == 0 && row < r1) {
#pragma unroll
            for (int q = 0; q < CPL; ++q)
                if (q * LPR + j < k) write_y(Y + (int64_t)(q * LPR + j) * ldy, row, td[q], alpha, beta);
        }
    }
}

// JDS, interleaved X.  The host splits the permuted rows (longest first) into
// classes with GPR wavefronts per row set (enough that each handles at most
// about 32 of a row's diagonals, GPR <= wavefronts per workgroup); a
// workgroup holds NG/GPR rows of a class.
struct MmClass {
    int32_t wg_end, row_start, row_end, gpr;
    int32_t len0;       // diagonals of the class's first (longest) row
};
struct MmPlan {
    MmClass c[8];
    int32_t ncls;
};

// One lane's share of a JDS row for the interleaved multi-vector kernel:
// columns j, j + LPR, ..., j + (CPL-1)*LPR over diagonals sub, sub + GPR, ...
// of row r, U per trip, stopping (for the whole wavefront) where the
// wavefront's first and longest row r_first ends.  Column t*LPR + j of the
// row's LPR lanes is one contiguous run of LPR elements per load.
template <int LPR, int CPL, bool WIDE, typename VT, typename XT>
__device__ __forceinline__ void mm_jds_sum(const int32_t *__restrict__ jp, int32_t dlim,
                                           const int32_t *__restrict__ col, const VT *__restrict__ val,
                                           const XT *__restrict__ Xr, int32_t k, int j, int32_t r, bool ok,
                                           int32_t r_first, int sub, int GPR, double (&out)[CPL])
{
    typedef typename Acc<WIDE>::T acc_t;
    constexpr int U = 2;   // diagonals per trip (2 measured 1-2% faster than 4, 8 slower)
    acc_t s[CPL];
#pragma unroll
    for (int t = 0; t < CPL; ++t) s[t] = 0;
    for (int32_t base = 0; base < dlim; base += GPR * U) {
        if (jp[base + 1] - jp[base] <= r_first) break;
        int32_t c[U];
        VT v[U];
        bool act[U];
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const int32_t dd = base + sub + u * GPR;
            act[u] = false;
            if (ok && dd < dlim) {
                const int32_t off = jp[dd];
                if (r < jp[dd + 1] - off) {
                    act[u] = true;
                    c[u] = ld_stream(col + off + r);
                    v[u] = ld_stream(val + off + r);
                }
            }
        }
        XT xv[U][CPL];
#pragma unroll
        for (int u = 0; u < U; ++u)
#pragma unroll
            for (int t = 0; t < CPL; ++t)
                xv[u][t] = (act[u] && t * LPR + j < k) ? Xr[(int64_t)c[u] * k + t * LPR + j] : XT(0);
#pragma unroll
        for (int u = 0; u < U; ++u)
            if (act[u]) {
#pragma unroll
                for (int t = 0; t < CPL; ++t) s[t] = Acc<WIDE>::mac(s[t], v[u], xv[u][t]);
            }
    }
#pragma unroll
    for (int t = 0; t < CPL; ++t) out[t] = (double)s[t];
}

template <int K2, int NT, typename VT, typename XT>
__global__ __launch_bounds__(NT) void spmm_jds_il_kernel(int32_t ndiag, const int32_t *__restrict__ jp,
                                                                 const int32_t *__restrict__ perm, int symperm,
                                                                 const int32_t *__restrict__ col,
                                                                 const VT *__restrict__ val,
                                                                 const XT *__restrict__ Xr, int32_t k,
                                                                 XT *__restrict__ Y, int64_t ldy, MmPlan P,
                                                                 double alpha, double beta)
{
    // a row is handled by a group of LPR <= 8 lanes, lane j owning columns
    // j, j + LPR, ..., so a wavefront holds at least 8 rows for any k
    constexpr int LPR = mm_jds_lpr<K2, XT>();
    constexpr int CPL = K2 / LPR;
    constexpr int NG = NT / LPR;
    constexpr int GPW = WAVE / LPR;            // rows per wavefront
    constexpr bool F64 = IsF64<VT>::value;
    __shared__ double part[NG][K2];
    const int64_t wg = blockIdx.x;
    int ci = 0;
    while (ci < P.ncls - 1 && wg >= P.c[ci].wg_end) ++ci;
    const MmClass K = P.c[ci];
    const int64_t wg0 = ci ? P.c[ci - 1].wg_end : 0;
    // a wavefront always holds GPW consecutive rows, so every val/col load
    // of one diagonal covers GPW consecutive entries; a row set's diagonals
    // are shared by GPR wavefronts (sub = 0..GPR-1, every GPR-th diagonal)
    const int GPR = K.gpr;
    const int g = (int)threadIdx.x / LPR, j = (int)threadIdx.x % LPR;
    const int w = (int)threadIdx.x / WAVE, gl = g % GPW;
    const int sub = w % GPR, rs = w / GPR;
    const int64_t rs0 = (int64_t)K.row_start + (wg - wg0) * (NG / GPR) + (int64_t)rs * GPW;
    const int64_t row64 = rs0 + gl;
    const bool ok = row64 < K.row_end;
    const int32_t r = (int32_t)(ok ? row64 : 0);
    // the wavefront's first row is its longest (rows are in JDS order): the
    // diagonal loop ends, for the whole wavefront, where that row ends
    const int32_t r_first = (int32_t)(rs0 < K.row_end ? rs0 : K.row_end);
    // the row's length decides the accumulator only for reduced-precision values
    bool wide = false;
    if (!F64 && ok && ndiag > SPMV_WIDE_ROW_NNZ) wide = jp[SPMV_WIDE_ROW_NNZ + 1] - jp[SPMV_WIDE_ROW_NNZ] > r;
    // no row of the class has more than len0 diagonals: the part of jd_ptr
    // this workgroup reads, jd_ptr[0 .. dlim], is staged in LDS when it fits
    const int32_t dlim = K.len0 < ndiag ? K.len0 : ndiag;
    extern __shared__ int32_t jp_s[];
    const bool jp_lds = dlim + 1 <= MM_JP_LDS;
    if (jp_lds) {
        for (int32_t i = (int32_t)threadIdx.x; i <= dlim; i += NT) jp_s[i] = jp[i];
        __syncthreads();
    }
    double td[CPL];
    if (jp_lds) {
        if (F64 || wide) mm_jds_sum<LPR, CPL, true, VT, XT>(jp_s, dlim, col, val, Xr, k, j, r, ok, r_first, sub, GPR, td);
        else mm_jds_sum<LPR, CPL, false, VT, XT>(jp_s, dlim, col, val, Xr, k, j, r, ok, r_first, sub, GPR, td);
    } else {
        if (F64 || wide) mm_jds_sum<LPR, CPL, true, VT, XT>(jp, dlim, col, val, Xr, k, j, r, ok, r_first, sub, GPR, td);
        else mm_jds_sum<LPR, CPL, false, VT, XT>(jp, dlim, col, val, Xr, k, j, r, ok, r_first, sub, GPR, td);
    }
    if (GPR > 1) {
#pragma unroll
        for (int t = 0; t < CPL; ++t) part[g][t * LPR + j] = td[t];
        __syncthreads();
        if (sub == 0 && ok) {
            // the row's GPR partial sums sit in wavefronts rs*GPR .. rs*GPR+GPR-1, same lane group
            const int g0 = rs * GPR * GPW + gl;
#pragma unroll
            for (int t = 0; t < CPL; ++t) {
                if (F64 || wide) {
                    double a = 0.0;
                    for (int q = 0; q < GPR; ++q) a += part[g0 + q * GPW][t * LPR + j];
                    td[t] = a;
                } else {
                    float a = 0.0f;
                    for (int q = 0; q < GPR; ++q) a += (float)part[g0 + q * GPW][t * LPR + j];
                    td[t] = (double)a;
                }
            }
        }
    }
    if (sub == 0 && ok) {
        const int32_t yi = symperm ? r : perm[r];
#pragma unroll
        for (int t = 0; t < CPL; ++t)
            if (t * LPR + j < k) write_y(Y + (int64_t)(t * LPR + j) * ldy, yi, td[t], alpha, beta);
    }
}

// Blocked JDS (RBJDS slices, in the global or the windowed row order),
// interleaved X.  A workgroup of MM_BLK_THREADS lanes is one plan record
// (first row, S, D).  A row is served by D groups of LPR lanes (lane j of a
// group owns columns j, j + LPR, ...; the D groups take every D-th diagonal),
// so a wavefront holds RW = 64 / (LPR * D) consecutive rows (RW divides the
// slice height: a wavefront's rows share a slice); the workgroup's (8/S) row
// sets each get S wavefronts, which cut the slice's diagonals into S
// contiguous ranges.  Partial sums meet by a fixed shuffle tree over the D
// groups, then in LDS in range order.  Rows of a slice are sorted by
// decreasing length, so a wavefront stops, as a whole, where its first row's
// entries end (padding has col = -1).  Deep slices get larger D and S, so no
// lane walks more than about MM_BLK_DIAGS diagonals.
constexpr int MM_BLK_THREADS = 512;
constexpr int MM_BLK_WAVES = MM_BLK_THREADS / WAVE;
constexpr int MM_BLK_DIAGS = 32;           // target diagonals per lane
constexpr int MM_BLK_MAX_D = 8;
constexpr int MM_BLK_XCDS = 8;             // MI355X: workgroup b runs on XCD b % 8

template <int K2, typename VT, typename XT>
__global__ __launch_bounds__(MM_BLK_THREADS) void spmm_blk_il_kernel(
    int32_t n, const int32_t *__restrict__ perm, int32_t C, const int64_t *__restrict__ slice_ptr,
    const int32_t *__restrict__ slice_nd, const int32_t *__restrict__ col, const VT *__restrict__ val,
    const XT *__restrict__ Xr, int32_t k, XT *__restrict__ Y, int64_t ldy, const int32_t *__restrict__ recs,
    double alpha, double beta)
{
    constexpr int LPR = mm_jds_lpr<K2, XT>();
    constexpr int CPL = K2 / LPR;
    constexpr bool F64 = IsF64<VT>::value;
    constexpr int U = CPL == 1 ? 4 : 2;     // diagonals per trip: 4 measured 5-14% faster at k <= 8, 2 at k = 32
    __shared__ double part[MM_BLK_WAVES][CPL][WAVE];
    // ranged plan (recs[0] >= 0): workgroup b runs on XCD b % 8 and takes
    // the (b / 8)-th record of that XCD's range (ranges of equal stored work,
    // in row order); otherwise workgroup b takes record b (the hardware deals
    // consecutive workgroups to the XCDs in turn)
    int64_t ri = blockIdx.x;
    if (recs[0] >= 0) {
        const int xcd = (int)(blockIdx.x % MM_BLK_XCDS);
        const int32_t lo = recs[xcd], hi = recs[xcd + 1];
        ri = (int64_t)lo + blockIdx.x / MM_BLK_XCDS;
        if (ri >= hi) return;                      // the whole workgroup: no barrier is reached
    }
    const int32_t *rec = recs + (MM_BLK_XCDS + 1) + 3 * ri;
    const int32_t first = rec[0], last = rec[1], sd = rec[2];
    const int S = sd & 0xff, D = sd >> 8;
    const int RW = WAVE / (LPR * D);
    const int w = (int)threadIdx.x / WAVE, lane = lane_id();
    const int g = w / S, p = w % S;
    const int j = lane % LPR, dl = (lane / LPR) % D, gl = lane / (LPR * D);
    const int64_t row0l = (int64_t)first + (int64_t)g * RW;
    const bool valid = row0l < last;
    const int32_t row0 = valid ? (int32_t)row0l : 0;
    const int32_t r = row0 + gl;
    const bool ok = valid && r < last;
    const int32_t sl = row0 / C;
    const int64_t sp = slice_ptr[sl];
    const int32_t nd = valid ? slice_nd[sl] : 0;
    const int32_t rs = r - sl * C;
    // rows of more than SPMV_WIDE_ROW_NNZ entries accumulate in FP64 (their
    // length found by a binary search of the padding, only in such slices)
    bool wide = false;
    if (!F64 && ok && nd > SPMV_WIDE_ROW_NNZ) {
        int32_t lo = 0, hi = nd;
        while (lo < hi) {
            const int32_t mid = (lo + hi) >> 1;
            if (col[sp + (int64_t)mid * C + rs] >= 0) lo = mid + 1;
            else hi = mid;
        }
        wide = lo > SPMV_WIDE_ROW_NNZ;
    }
    const int32_t dA = (int32_t)((int64_t)p * nd / S), dB = (int32_t)((int64_t)(p + 1) * nd / S);
    double td[CPL];
    auto walk = [&](auto acc_tag) {
        typedef decltype(acc_tag) acc_t;
        constexpr bool WD = sizeof(acc_t) == 8;
        acc_t sacc[CPL];
#pragma unroll
        for (int t = 0; t < CPL; ++t) sacc[t] = 0;
        for (int32_t d0 = dA; d0 < dB; d0 += U * D) {
            int32_t c[U];
            VT v[U];
#pragma unroll
            for (int u = 0; u < U; ++u) {
                // in bounds for every lane of a wavefront that runs the loop:
                // d < nd and 0 <= rs < C address its slice's storage
                const int32_t du = d0 + u * D + dl;
                const int32_t d = min(du, dB - 1);
                const int64_t e = sp + (int64_t)d * C + rs;
                c[u] = ld_stream(col + e);
                v[u] = ld_stream(val + e);
                c[u] = (ok && du < dB) ? c[u] : -1;
            }
            // the first row of the wavefront is its longest: once it has no
            // entry at d0 (lane 0's first load), no row of the wavefront has
            // one at any later diagonal
            if (__builtin_amdgcn_readfirstlane(c[0]) < 0) break;
            XT xv[U][CPL];
#pragma unroll
            for (int u = 0; u < U; ++u)
#pragma unroll
                for (int t = 0; t < CPL; ++t)
                    xv[u][t] = (c[u] >= 0 && t * LPR + j < k) ? Xr[(int64_t)c[u] * k + t * LPR + j] : XT(0);
#pragma unroll
            for (int u = 0; u < U; ++u)
                if (c[u] >= 0) {
#pragma unroll
                    for (int t = 0; t < CPL; ++t) sacc[t] = Acc<WD>::mac(sacc[t], v[u], xv[u][t]);
                }
        }
        // the D groups of a row: fixed xor tree over the group index
        for (int off = LPR; off < LPR * D; off <<= 1)
#pragma unroll
            for (int t = 0; t < CPL; ++t) sacc[t] += __shfl_xor(sacc[t], off, WAVE);
#pragma unroll
        for (int t = 0; t < CPL; ++t) td[t] = (double)sacc[t];
    };
    if (F64 || wide) walk(0.0);
    else walk(0.0f);
    if (S > 1) {
#pragma unroll
        for (int t = 0; t < CPL; ++t) part[w][t][lane] = td[t];
        __syncthreads();
        if (p == 0 && ok && dl == 0) {
#pragma unroll
            for (int t = 0; t < CPL; ++t) {
                if (F64 || wide) {
                    double a = 0.0;
                    for (int q = 0; q < S; ++q) a += part[w + q][t][lane];
                    td[t] = a;
                } else {
                    float a = 0.0f;
                    for (int q = 0; q < S; ++q) a += (float)part[w + q][t][lane];
                    td[t] = (double)a;
                }
            }
        }
    }
    if (p == 0 && ok && dl == 0) {
        const int32_t yi = perm[r];
#pragma unroll
        for (int t = 0; t < CPL; ++t)
            if (t * LPR + j < k) write_y(Y + (int64_t)(t * LPR + j) * ldy, yi, td[t], alpha, beta);
    }
}

// Records (first row, end row, S | D << 8).  Each slice's depth sets its
// (D, S): D doubles up to min(MM_BLK_MAX_D, 64 / LPR), then S up to 8, until
// D * S * MM_BLK_DIAGS reaches the depth.  A run of consecutive slices with
// the same (D, S) is cut into records of (8/S) * 64 / (LPR * D) rows from the
// run's first row (a slice start), so every wavefront's rows start at a
// multiple of its row count and stay inside one slice; the run's last record
// ends with the run.
static void plan_mm_blk(int32_t n, int32_t C, int32_t n_slices, const int32_t *h_slice_nd, int LPR, int max_groups,
                        std::vector<int32_t> &out)
{
    const int dmax = std::min(max_groups, WAVE / LPR);
    auto ds_of = [&](int32_t nd) {
        int D = 1, S = 1;
        while ((int64_t)D * S * MM_BLK_DIAGS < nd) {
            if (D < dmax) D *= 2;
            else if (S < MM_BLK_WAVES) S *= 2;
            else break;
        }
        return S | (D << 8);
    };
    out.clear();
    for (int32_t s0 = 0; s0 < n_slices;) {
        const int sd = ds_of(h_slice_nd[s0]);
        int32_t s1 = s0 + 1;
        while (s1 < n_slices && ds_of(h_slice_nd[s1]) == sd) ++s1;
        const int S = sd & 0xff, D = sd >> 8;
        const int64_t rows = (int64_t)(MM_BLK_WAVES / S) * (WAVE / (LPR * D));
        const int64_t end = std::min<int64_t>(n, (int64_t)s1 * C);
        for (int64_t row = (int64_t)s0 * C; row < end; row += rows) {
            out.push_back((int32_t)row);
            out.push_back((int32_t)std::min<int64_t>(end, row + rows));
            out.push_back(sd);
        }
        s0 = s1;
    }
}

// Plan words: MM_BLK_XCDS + 1 range bounds, then the records.  Ranged: the
// bounds are record indices, range x (run on XCD x) holding about an eighth
// of the stored work (rows times their slice's depth), and the grid is
// MM_BLK_XCDS times the longest range.  Not ranged: the bounds are -1 and
// the grid is the record count.
static int64_t plan_mm_blk_words(int32_t n, int32_t C, int32_t n_slices, const int32_t *h_slice_nd, int LPR,
                                 int max_groups, bool ranged, std::vector<int32_t> &words)
{
    std::vector<int32_t> recs;
    plan_mm_blk(n, C, n_slices, h_slice_nd, LPR, max_groups, recs);
    const int64_t nr = (int64_t)recs.size() / 3;
    if (!ranged) {
        words.assign(MM_BLK_XCDS + 1, -1);
        words.insert(words.end(), recs.begin(), recs.end());
        return nr;
    }
    std::vector<int64_t> pre((size_t)nr + 1, 0);
    for (int64_t i = 0; i < nr; ++i) {
        const int64_t rows = recs[3 * i + 1] - recs[3 * i];
        pre[i + 1] = pre[i] + rows * std::max<int64_t>(1, h_slice_nd[recs[3 * i] / C]);
    }
    words.assign(MM_BLK_XCDS + 1, 0);
    int64_t longest = 0;
    for (int x = 1; x <= MM_BLK_XCDS; ++x) {
        const int64_t target = (pre[nr] * x + MM_BLK_XCDS - 1) / MM_BLK_XCDS;
        words[x] = x == MM_BLK_XCDS ? (int32_t)nr
                                    : (int32_t)(std::lower_bound(pre.begin(), pre.end(), target) - pre.begin());
        words[x] = std::max(words[x], words[x - 1]);
        longest = std::max<int64_t>(longest, words[x] - words[x - 1]);
    }
    words.insert(words.end(), recs.begin(), recs.end());
    return longest * MM_BLK_XCDS;
}

static int k2_for(int32_t k)
{
    int K2 = 1;
    while (K2 < k && K2 < MM_MAX_K2) K2 *= 2;
    return K2;
}

// NG row groups per workgroup, NW wavefronts per workgroup: a class's rows
// get GPR = 1, 2, ..., NW wavefronts each (a power of two), NG / GPR rows per
// workgroup.
static MmPlan plan_mm_jds(int32_t n, const int32_t *h_jd_ptr, int32_t ndiag, int NG, int NW)
{
    constexpr int64_t LT = 32;   // target diagonals per group
    MmPlan P{};
    auto len_of = [&](int64_t row) -> int64_t {
        int32_t lo = 0, hi = ndiag;
        while (lo < hi) {
            int32_t mid = (lo + hi) >> 1;
            if (h_jd_ptr[mid + 1] - h_jd_ptr[mid] > row) lo = mid + 1;
            else hi = mid;
        }
        return lo;
    };
    auto gpr_of = [&](int64_t L) {
        int gpr = 1;
        while (gpr < NW && gpr * LT < L) gpr *= 2;
        return gpr;
    };
    int64_t row = 0, wgs = 0;
    int cls = 0;
    while (row < n && cls < 8) {
        const int gpr = gpr_of(len_of(row));
        int64_t end = n;
        if (cls < 7 && gpr > 1) {
            // rows needing this many groups: length > (gpr/2)*LT; lengths never increase
            const int64_t lower = (int64_t)(gpr / 2) * LT;
            int64_t lo = row + 1, hi = n;
            while (lo < hi) {
                const int64_t mid = (lo + hi) >> 1;
                if (len_of(mid) > lower) lo = mid + 1;
                else hi = mid;
            }
            end = lo;
        }
        MmClass &K = P.c[cls++];
        K.row_start = (int32_t)row;
        K.row_end = (int32_t)end;
        K.gpr = gpr;
        K.len0 = (int32_t)len_of(row);
        wgs += ceil_div(end - row, NG / gpr);
        K.wg_end = (int32_t)wgs;
        row = end;
    }
    P.ncls = cls;
    return P;
}

// The row-major block the interleaved kernels read: X itself for k = 1,
// otherwise Xr in the workspace, filled here.
template <typename T>
static spmv_status stage(int64_t n, int32_t k, const void *X, int64_t ldx, void *ws, const void **Xr, hipStream_t s)
{
    if (k == 1) {
        *Xr = X;
        return SPMV_OK;
    }
    *Xr = ws;
    if (n == 0) return SPMV_OK;
    const int64_t rows = STAGE_ELEMS / k;              // 2 <= k <= MM_MAX_K2 = 64
    stage_rowmajor_kernel<T><<<(unsigned)ceil_div(n, rows), STAGE_THREADS, 0, s>>>(n, k, (const T *)X, ldx, (T *)ws);
    SPMV_CHECK_LAUNCH("spmm staging");
    return SPMV_OK;
}

template <int K2, typename VT, typename XT>
static void launch_crs_il(const int32_t *row_ptr, const int32_t *col, const void *val, const void *Xr, int32_t k,
                          void *Y, int64_t ldy, const int32_t *plan, int32_t nb, int32_t block_nnz, double alpha,
                          double beta, hipStream_t s)
{
    const size_t lds = (size_t)((block_nnz + 3) & ~3) * 4 + (size_t)((block_nnz + 1) & ~1) * sizeof(VT) +
                       (sizeof(XT) == 8 ? sizeof(int32_t) * ((size_t)mm_rp_lds(block_nnz) + 1) + mm_ytile_bytes<K2>()
                                        : 0);
    constexpr int NT = mm_crs_threads<K2, XT>();
    spmm_crs_il_kernel<K2, NT, VT, XT><<<nb, NT, lds, s>>>(row_ptr, col, (const VT *)val, (const XT *)Xr, k,
                                                          (XT *)Y, ldy, plan, block_nnz, alpha, beta);
}

template <int K2, typename VT, typename XT>
static void launch_jds_il(int32_t n, const int32_t *h_jd_ptr, int32_t ndiag, const int32_t *jp, const int32_t *perm,
                          int symperm, const int32_t *col, const void *val, const void *Xr, int32_t k, void *Y,
                          int64_t ldy, double alpha, double beta, hipStream_t s)
{
    constexpr int NT = MM_JDS_THREADS;
    const MmPlan P = plan_mm_jds(n, h_jd_ptr, ndiag, NT / mm_jds_lpr<K2, XT>(), NT / WAVE);
    if (P.ncls == 0) return;
    // room for the longest jd_ptr prefix a class stages (dlim + 1 <= min(ndiag + 1, MM_JP_LDS))
    const size_t lds = sizeof(int32_t) * (size_t)std::min<int64_t>((int64_t)ndiag + 1, MM_JP_LDS);
    spmm_jds_il_kernel<K2, NT, VT, XT><<<(unsigned)P.c[P.ncls - 1].wg_end, NT, lds, s>>>(
        ndiag, jp, perm, symperm, col, (const VT *)val, (const XT *)Xr, k, (XT *)Y, ldy, P, alpha, beta);
}

template <int K2, typename VT, typename XT>
static void launch_blk_il(int32_t n, const int32_t *perm, int32_t C, const int64_t *slice_ptr,
                          const int32_t *slice_nd, const int32_t *col, const void *val, const void *Xr, int32_t k,
                          void *Y, int64_t ldy, const int32_t *recs, int32_t grid, double alpha, double beta,
                          hipStream_t s)
{
    spmm_blk_il_kernel<K2, VT, XT><<<(unsigned)grid, MM_BLK_THREADS, 0, s>>>(
        n, perm, C, slice_ptr, slice_nd, col, (const VT *)val, (const XT *)Xr, k, (XT *)Y, ldy, recs, alpha, beta);
}

#define K2_SWITCH(K2VAR, CALL)          \
    switch (K2VAR) {                    \
    case 1: { constexpr int K2 = 1; CALL; } break;   \
    case 2: { constexpr int K2 = 2; CALL; } break;   \
    case 4: { constexpr int K2 = 4; CALL; } break;   \
    case 8: { constexpr int K2 = 8; CALL; } break;   \
    case 16: { constexpr int K2 = 16; CALL; } break; \
    case 32: { constexpr int K2 = 32; CALL; } break; \
    default: { constexpr int K2 = 64; CALL; } break; \
    }

}  // namespace spmv

using namespace spmv;

extern "C" {

size_t spmm_workspace_size(int32_t n_cols, int32_t k, spmv_dtype vec_dt)
{
    if (n_cols < 0 || k < 0) return 0;
    return align_up((size_t)n_cols * (size_t)k * dtype_size(vec_dt), 256) + 256;
}

spmv_status spmm_crs(int32_t n_rows, int32_t n_cols, const int32_t *row_ptr, const int32_t *col_idx, const void *val,
                     spmv_dtype val_dt, int32_t k, const void *X, int64_t ldx, void *Y, int64_t ldy,
                     spmv_dtype vec_dt, double alpha, double beta, const int32_t *plan, int32_t n_blocks,
                     int32_t block_nnz, void *ws, size_t ws_bytes, void *stream)
{
    SPMV_REQUIRE(n_rows >= 0 && n_cols >= 0 && k >= 0, "spmm_crs: negative size");
    if (block_nnz == 0) block_nnz = crs_default_block_nnz();
    SPMV_REQUIRE(block_nnz >= 256 && block_nnz <= 4096, "spmm_crs: block_nnz must be in [256, 4096]");
    SPMV_REQUIRE(valid_dtype(val_dt) && valid_vec_dtype(vec_dt), "spmm_crs: bad dtype");
    if (n_rows == 0 || k == 0) return SPMV_OK;
    SPMV_REQUIRE(plan && n_blocks >= 0, "spmm_crs: needs a plan from spmv_crs_plan");
    SPMV_REQUIRE(ldx >= n_cols && ldy >= n_rows, "spmm_crs: leading dimension too small");
    SPMV_REQUIRE(row_ptr && Y, "spmm_crs: null row_ptr or Y");
    hipStream_t s = as_stream(stream);
    if (!ws || k > MM_MAX_K2)
        return spmm_crs_colmajor(n_rows, n_cols, row_ptr, col_idx, val, val_dt, k, X, ldx, Y, ldy, vec_dt, alpha,
                                 beta, plan, n_blocks, s);
    SPMV_REQUIRE(ws_bytes >= spmm_workspace_size(n_cols, k, vec_dt), "spmm_crs: workspace too small");
    if (n_blocks == 0) return SPMV_OK;
    const void *Xr = nullptr;
    spmv_status st = vec_dt == SPMV_F64 ? stage<double>(n_cols, k, X, ldx, ws, &Xr, s)
                                        : stage<float>(n_cols, k, X, ldx, ws, &Xr, s);
    if (st != SPMV_OK) return st;
    const int K2v = k2_for(k);
#define CRS_IL(VDT, VT, XDT, XT)                                                                              \
    if (val_dt == VDT && vec_dt == XDT) {                                                                     \
        K2_SWITCH(K2v, (launch_crs_il<K2, VT, XT>(row_ptr, col_idx, val, Xr, k, Y, ldy, plan, n_blocks,        \
                                                  block_nnz, alpha, beta, s)));                               \
        SPMV_CHECK_LAUNCH("spmm_crs");                                                                        \
        return SPMV_OK;                                                                                       \
    }
    CRS_IL(SPMV_F64, double, SPMV_F64, double)
    CRS_IL(SPMV_F32, float, SPMV_F32, float)
    CRS_IL(SPMV_F32, float, SPMV_F64, double)
    CRS_IL(SPMV_BF16, bf16, SPMV_F32, float)
    CRS_IL(SPMV_BF16, bf16, SPMV_F64, double)
    CRS_IL(SPMV_F64, double, SPMV_F32, float)
#undef CRS_IL
    return fail(SPMV_ERR_UNSUPPORTED, "spmm_crs: dtype combination");
}

spmv_status spmm_jds(int32_t n, int32_t n_cols, const int32_t *perm, const int32_t *jd_ptr, const int32_t *h_jd_ptr,
                     int32_t ndiag, const int32_t *jd_col, const void *jd_val, spmv_dtype val_dt, int32_t k,
                     const void *X, int64_t ldx, void *Y, int64_t ldy, spmv_dtype vec_dt, double alpha, double beta,
                     unsigned flags, void *ws, size_t ws_bytes, void *stream)
{
    SPMV_REQUIRE(n >= 0 && n_cols >= 0 && ndiag >= 0 && k >= 0, "spmm_jds: negative size");
    SPMV_REQUIRE(ldx >= n_cols, "spmm_jds: ldx < n_cols");
    SPMV_REQUIRE(valid_dtype(val_dt) && valid_vec_dtype(vec_dt), "spmm_jds: bad dtype");
    SPMV_REQUIRE((flags & ~SPMV_SYMPERM) == 0, "spmm_jds: unknown flag");
    if (n == 0 || k == 0) return SPMV_OK;
    SPMV_REQUIRE(ldy >= n, "spmm_jds: ldy < n");
    SPMV_REQUIRE(Y && jd_ptr, "spmm_jds: null Y or jd_ptr");
    SPMV_REQUIRE((flags & SPMV_SYMPERM) || perm, "spmm_jds: null perm");
    SPMV_REQUIRE(ndiag == 0 || (jd_col && jd_val && X), "spmm_jds: null input");
    hipStream_t s = as_stream(stream);
    if (!ws || k > MM_MAX_K2)
        return spmm_jds_colmajor(n, perm, jd_ptr, ndiag, jd_col, jd_val, val_dt, k, X, ldx, Y, ldy, vec_dt, alpha,
                                 beta, flags, s);
    SPMV_REQUIRE(h_jd_ptr, "spmm_jds: the interleaved path needs h_jd_ptr");
    SPMV_REQUIRE(ws_bytes >= spmm_workspace_size(n_cols, k, vec_dt), "spmm_jds: workspace too small");
    const void *Xr = nullptr;
    spmv_status st = vec_dt == SPMV_F64 ? stage<double>(n_cols, k, X, ldx, ws, &Xr, s)
                                        : stage<float>(n_cols, k, X, ldx, ws, &Xr, s);
    if (st != SPMV_OK) return st;
    const int K2v = k2_for(k);
    const int sym = (flags & SPMV_SYMPERM) ? 1 : 0;
#define JDS_IL(VDT, VT, XDT, XT)                                                                                 \
    if (val_dt == VDT && vec_dt == XDT) {                                                                        \
        K2_SWITCH(K2v, (launch_jds_il<K2, VT, XT>(n, h_jd_ptr, ndiag, jd_ptr, perm, sym, jd_col, jd_val, Xr, k, Y, \
                                                  ldy, alpha, beta, s)));                                        \
        SPMV_CHECK_LAUNCH("spmm_jds");                                                                           \
        return SPMV_OK;                                                                                          \
    }
    JDS_IL(SPMV_F64, double, SPMV_F64, double)
    JDS_IL(SPMV_F32, float, SPMV_F32, float)
    JDS_IL(SPMV_F32, float, SPMV_F64, double)
    JDS_IL(SPMV_BF16, bf16, SPMV_F32, float)
    JDS_IL(SPMV_BF16, bf16, SPMV_F64, double)
    JDS_IL(SPMV_F64, double, SPMV_F32, float)
#undef JDS_IL
    return fail(SPMV_ERR_UNSUPPORTED, "spmm_jds: dtype combination");
}

spmv_status spmm_jds_blocked_plan(int32_t n, int32_t C, int32_t n_slices, const int32_t *h_slice_nd, int32_t k,
                                  int32_t max_groups, int32_t xcd_ranges, int32_t *plan, int32_t plan_cap,
                                  int32_t *h_plan_words, int32_t *h_grid, void *stream)
{
    SPMV_REQUIRE(n >= 0 && k >= 1 && k <= MM_MAX_K2, "spmm_jds_blocked_plan: n < 0 or k outside [1, 64]");
    if (max_groups == 0) max_groups = 1;
    SPMV_REQUIRE(max_groups == 1 || max_groups == 2 || max_groups == 4 || max_groups == 8,
                 "spmm_jds_blocked_plan: max_groups must be 1, 2, 4 or 8");
    SPMV_REQUIRE(C >= WAVE && C % WAVE == 0, "spmm_jds_blocked_plan: C must be a positive multiple of 64");
    SPMV_REQUIRE(n_slices == (int32_t)ceil_div(n, C), "spmm_jds_blocked_plan: n_slices != ceil(n / C)");
    SPMV_REQUIRE(h_plan_words && h_grid && (n == 0 || h_slice_nd), "spmm_jds_blocked_plan: null pointer");
    const int K2v = k2_for(k);
    const int LPR = K2v <= 8 ? K2v : 8;             // mm_jds_lpr
    std::vector<int32_t> words;
    const int64_t grid = plan_mm_blk_words(n, C, n_slices, h_slice_nd, LPR, max_groups, xcd_ranges != 0, words);
    SPMV_REQUIRE(grid <= INT32_MAX, "spmm_jds_blocked_plan: too many records");
    *h_plan_words = (int32_t)words.size();
    *h_grid = (int32_t)grid;
    if (!plan || plan_cap < (int32_t)words.size())
        return fail(SPMV_ERR_CAPACITY, "spmm_jds_blocked_plan: plan capacity < *h_plan_words");
    hipStream_t s = as_stream(stream);
    SPMV_HIP(hipMemcpyAsync(plan, words.data(), sizeof(int32_t) * words.size(), hipMemcpyHostToDevice, s));
    SPMV_HIP(hipStreamSynchronize(s));
    return SPMV_OK;
}

spmv_status spmm_jds_blocked(int32_t n, int32_t n_cols, const int32_t *perm, int32_t C, int32_t n_slices,
                             const int64_t *slice_ptr, const int32_t *slice_nd, const int32_t *bl_col,
                             const void *bl_val, spmv_dtype val_dt, int32_t k, const void *X, int64_t ldx, void *Y,
                             int64_t ldy, spmv_dtype vec_dt, double alpha, double beta, const int32_t *plan,
                             int32_t grid, void *ws, size_t ws_bytes, void *stream)
{
    SPMV_REQUIRE(n >= 0 && n_cols >= 0 && k >= 0 && grid >= 0, "spmm_jds_blocked: negative size");
    SPMV_REQUIRE(k <= MM_MAX_K2, "spmm_jds_blocked: k > 64");
    SPMV_REQUIRE(C >= WAVE && C % WAVE == 0, "spmm_jds_blocked: C must be a positive multiple of 64");
    SPMV_REQUIRE(valid_dtype(val_dt) && valid_vec_dtype(vec_dt), "spmm_jds_blocked: bad dtype");
    if (n == 0 || k == 0) return SPMV_OK;
    SPMV_REQUIRE(ldx >= n_cols && ldy >= n, "spmm_jds_blocked: leading dimension too small");
    SPMV_REQUIRE(n_slices == (int32_t)ceil_div(n, C), "spmm_jds_blocked: n_slices != ceil(n / C)");
    SPMV_REQUIRE(perm && slice_ptr && slice_nd && Y && plan && X, "spmm_jds_blocked: null pointer");
    SPMV_REQUIRE(ws && ws_bytes >= spmm_workspace_size(n_cols, k, vec_dt), "spmm_jds_blocked: workspace too small");
    hipStream_t s = as_stream(stream);
    const void *Xr = nullptr;
    spmv_status st = vec_dt == SPMV_F64 ? stage<double>(n_cols, k, X, ldx, ws, &Xr, s)
                                        : stage<float>(n_cols, k, X, ldx, ws, &Xr, s);
    if (st != SPMV_OK) return st;
    if (grid == 0) return SPMV_OK;
    const int K2v = k2_for(k);
#define BLK_IL(VDT, VT, XDT, XT)                                                                                 \
    if (val_dt == VDT && vec_dt == XDT) {                                                                        \
        K2_SWITCH(K2v, (launch_blk_il<K2, VT, XT>(n, perm, C, slice_ptr, slice_nd, bl_col, bl_val, Xr, k, Y, ldy,  \
                                                  plan, grid, alpha, beta, s)));                                 \
        SPMV_CHECK_LAUNCH("spmm_jds_blocked");                                                                   \
        return SPMV_OK;                                                                                          \
    }
    BLK_IL(SPMV_F64, double, SPMV_F64, double)
    BLK_IL(SPMV_F32, float, SPMV_F32, float)
    BLK_IL(SPMV_F32, float, SPMV_F64, double)
    BLK_IL(SPMV_BF16, bf16, SPMV_F32, float)
    BLK_IL(SPMV_BF16, bf16, SPMV_F64, double)
    BLK_IL(SPMV_F64, double, SPMV_F32, float)
#undef BLK_IL
    return fail(SPMV_ERR_UNSUPPORTED, "spmm_jds_blocked: dtype combination");
}

}  // extern "C"
