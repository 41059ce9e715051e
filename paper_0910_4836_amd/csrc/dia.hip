// DIA + CRS hybrid product (the dense storage of heavily filled diagonals that
// the paper's Section 4.2 suggests for its Hamiltonian, with the other
// entries in CRS).
//
// gfx950 design.  One lane per row, consecutive lanes on consecutive rows:
// for every stored diagonal the wavefront reads 64 consecutive values and 64
// consecutive x entries (no index array, no gather), then each lane adds its
// row's remainder entries.  The offsets travel in the kernel arguments
// (scalar registers); the diagonal loop is unrolled so that several value
// and x loads are in flight per lane.  Workgroups are remapped so that each
// XCD walks a contiguous range of rows and keeps its x windows in its L2.
// Every row is summed in FP64 in a fixed order and y is written once.
//
// Symmetric storage (the paper notes its Hamiltonian is symmetric): only the
// diagonals with offset >= 0 are stored and each also stands for its mirror,
// whose entry a(i, i - o) = dia[k][i - o] is the same diagonal read o rows
// earlier: another contiguous stream, so every lane still writes only its own
// row of y.
//
// Remainder in window-sorted slices: the rows of a workgroup's window are
// ordered by remainder length and cut into slices of 16, the RBJDS layout
// with the sort kept inside the workgroup.  The diagonal sums meet the
// remainder sums in LDS, so the row order, the sums and y's coalesced writes
// stay those of the CRS-remainder kernel while the remainder loads become
// contiguous and the padding small.
#include "common.hpp"

namespace spmv {

constexpr int DIA_THREADS = 256;

struct DiaArgs {
    int32_t n_rows, n_cols, ndia;
    int32_t off[SPMV_DIA_MAX];
    const void *dia;
    const int32_t *rem_rp;      // CRS remainder, or
    const int64_t *rem_sp;      // window-sorted slices (slice pointers, depths, window-local rows)
    const int32_t *rem_nd;
    const uint8_t *rem_slot_row;
    const int32_t *rem_col;
    const void *rem_val;
    const void *x;
    void *y;
    double alpha, beta;
};

// SYM: the stored offsets are >= 0 and diagonal k (offset o > 0) also holds
// the mirrored entries a(i, i - o) = a(i - o, i) = dia[k][i - o]; the row adds
// its upper terms in offset order, then its mirrored terms in offset order.
template <typename VT, typename XT, bool SYM>
__device__ __forceinline__ double dia_row_sum(const DiaArgs &a, int64_t i)
{
    const VT *__restrict__ dia = (const VT *)a.dia + i;
    const XT *__restrict__ x = (const XT *)a.x;
    // U diagonals per trip, the last trip masked (diagonals past ndia are
    // not loaded), so that every trip has all its loads in flight at once
    constexpr int U = 8;
    double s = 0.0;
    for (int k = 0; k < a.ndia; k += U) {
        VT v[U];
        XT xv[U];
        bool in[U];
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const bool live = k + u < a.ndia;
            const int64_t j = i + a.off[live ? k + u : 0];
            in[u] = live && j >= 0 && j < a.n_cols;
            if (in[u]) {
                v[u] = ld_stream(dia + (int64_t)(k + u) * a.n_rows);
                xv[u] = x[j];
            }
        }
#pragma unroll
        for (int u = 0; u < U; ++u)
            if (in[u]) s = fma(to_f64(v[u]), to_f64(xv[u]), s);
    }
    if (SYM) {
        for (int k = 0; k < a.ndia; k += U) {
            VT v[U];
            XT xv[U];
            bool in[U];
#pragma unroll
            for (int u = 0; u < U; ++u) {
                const bool live = k + u < a.ndia;
                const int32_t o = a.off[live ? k + u : 0];
                const int64_t j = i - o;
                in[u] = live && o > 0 && j >= 0;
                if (in[u]) {
                    v[u] = ld_stream((const VT *)a.dia + (int64_t)(k + u) * a.n_rows + j);
                    xv[u] = x[j];
                }
            }
#pragma unroll
            for (int u = 0; u < U; ++u)
                if (in[u]) s = fma(to_f64(v[u]), to_f64(xv[u]), s);
        }
    }
    return s;
}

// Remainder in CRS: the lane adds its own row's entries.
template <typename VT, typename XT, bool SYM>
__global__ __launch_bounds__(DIA_THREADS) void dia_kernel(DiaArgs a)
{
    const int64_t i = xcd_remap(blockIdx.x, gridDim.x) * DIA_THREADS + threadIdx.x;
    if (i >= a.n_rows) return;
    double s = dia_row_sum<VT, XT, SYM>(a, i);
    if (a.rem_rp) {
        const VT *__restrict__ rv = (const VT *)a.rem_val;
        const XT *__restrict__ x = (const XT *)a.x;
        for (int32_t e = a.rem_rp[i]; e < a.rem_rp[i + 1]; ++e) s = fma(to_f64(rv[e]), to_f64(x[a.rem_col[e]]), s);
    }
    write_y((XT *)a.y, i, s, a.alpha, a.beta);
}

// Remainder in window-sorted slices: the workgroup owns one window of
// SPMV_REM_WINDOW rows.  Lane t sums row base + t's diagonals into LDS; after
// a barrier the lane at sorted position base + t continues the sum of the
// window's row slot_row[base + t] with its remainder (the d-th entries of 16
// consecutive positions are 16 consecutive slots) and puts it back; after a
// second barrier lane t writes y for row base + t.  Each LDS slot is touched
// by one lane between the barriers (slot_row is a permutation of the window).
template <typename VT, typename XT, bool SYM>
__global__ __launch_bounds__(DIA_THREADS) void dia_sliced_kernel(DiaArgs a)
{
    static_assert(DIA_THREADS == SPMV_REM_WINDOW, "one workgroup per remainder window");
    __shared__ double part[DIA_THREADS];
    const int64_t base = xcd_remap(blockIdx.x, gridDim.x) * DIA_THREADS;
    const int64_t i = base + threadIdx.x;
    const bool row = i < a.n_rows;
    part[threadIdx.x] = row ? dia_row_sum<VT, XT, SYM>(a, i) : 0.0;
    if (a.rem_sp) {
        __syncthreads();
        if (row) {
            const int lr = a.rem_slot_row[i];
            const int64_t sp = a.rem_sp[i / SPMV_REM_SLICE] + i % SPMV_REM_SLICE;
            const int32_t nd = a.rem_nd[i / SPMV_REM_SLICE];
            const VT *__restrict__ rv = (const VT *)a.rem_val;
            const XT *__restrict__ x = (const XT *)a.x;
            double s = part[lr];
            // UR entries per trip, the last trip masked like the diagonals'
            // (8 takes most rows of a banded remainder in one trip: 3.7%
            // faster than 4 on the Hamiltonian-shaped matrix, 16 no faster)
            constexpr int UR = 8;
            for (int32_t d = 0; d < nd; d += UR) {
                int32_t c[UR];
                VT v[UR];
                XT xv[UR];
#pragma unroll
                for (int u = 0; u < UR; ++u) {
                    c[u] = -1;
                    if (d + u < nd) {
                        c[u] = ld_stream(a.rem_col + sp + (int64_t)(d + u) * SPMV_REM_SLICE);
                        v[u] = ld_stream(rv + sp + (int64_t)(d + u) * SPMV_REM_SLICE);
                    }
                }
#pragma unroll
                for (int u = 0; u < UR; ++u)
                    if (c[u] >= 0) xv[u] = x[c[u]];
#pragma unroll
                for (int u = 0; u < UR; ++u)
                    if (c[u] >= 0) s = fma(to_f64(v[u]), to_f64(xv[u]), s);
            }
            part[lr] = s;
        }
        __syncthreads();
    }
    if (row) write_y((XT *)a.y, i, part[threadIdx.x], a.alpha, a.beta);
}

template <bool SYM, bool SLICED = false>
static spmv_status dia_product(int32_t n_rows, int32_t n_cols, int32_t ndia, const int32_t *h_offsets,
                               const void *dia_val, spmv_dtype val_dt, const int32_t *rem_row_ptr,
                               const int32_t *rem_col, const void *rem_val, const void *x, void *y, spmv_dtype vec_dt,
                               double alpha, double beta, void *stream, const int64_t *rem_sp = nullptr,
                               const int32_t *rem_nd = nullptr, const uint8_t *rem_slot_row = nullptr)
{
    SPMV_REQUIRE(n_rows >= 0 && n_cols >= 0, "spmv_dia: negative size");
    SPMV_REQUIRE(ndia >= 0 && ndia <= SPMV_DIA_MAX, "spmv_dia: ndia must be 0..SPMV_DIA_MAX");
    SPMV_REQUIRE(valid_dtype(val_dt) && valid_vec_dtype(vec_dt), "spmv_dia: bad dtype");
    if (n_rows == 0) return SPMV_OK;
    SPMV_REQUIRE(y, "spmv_dia: null y");
    SPMV_REQUIRE(ndia == 0 || (h_offsets && dia_val && x), "spmv_dia: null offsets, values or x");
    SPMV_REQUIRE(!rem_row_ptr || x, "spmv_dia: null x");
    SPMV_REQUIRE(!rem_sp || (x && rem_nd && rem_slot_row && rem_col && rem_val),
                 "spmv_dia_sliced: null remainder slices or x");
    DiaArgs a{};
    a.n_rows = n_rows;
    a.n_cols = n_cols;
    a.ndia = ndia;
    for (int k = 0; k < ndia; ++k) {
        SPMV_REQUIRE(h_offsets[k] > -n_rows && h_offsets[k] < n_cols, "spmv_dia: offset outside the matrix");
        SPMV_REQUIRE(!SYM || h_offsets[k] >= 0, "spmv_dia_sym: offsets must be >= 0 (upper diagonals)");
        SPMV_REQUIRE(k == 0 || h_offsets[k] > h_offsets[k - 1], "spmv_dia: offsets must increase");
        a.off[k] = h_offsets[k];
    }
    a.dia = dia_val;
    a.rem_rp = rem_row_ptr;
    a.rem_sp = rem_sp;
    a.rem_nd = rem_nd;
    a.rem_slot_row = rem_slot_row;
    a.rem_col = rem_col;
    a.rem_val = rem_val;
    a.x = x;
    a.y = y;
    a.alpha = alpha;
    a.beta = beta;
    hipStream_t s = as_stream(stream);
    const unsigned grid = (unsigned)ceil_div(n_rows, DIA_THREADS);
#define DIA_CASE(VDT, VT, XDT, XT)                                          \
    if (val_dt == VDT && vec_dt == XDT) {                                   \
        if (SLICED) dia_sliced_kernel<VT, XT, SYM><<<grid, DIA_THREADS, 0, s>>>(a); \
        else dia_kernel<VT, XT, SYM><<<grid, DIA_THREADS, 0, s>>>(a);       \
        SPMV_CHECK_LAUNCH("spmv_dia");                                      \
        return SPMV_OK;                                                     \
    }
    DIA_CASE(SPMV_F64, double, SPMV_F64, double)
    DIA_CASE(SPMV_F32, float, SPMV_F64, double)
    DIA_CASE(SPMV_BF16, bf16, SPMV_F64, double)
    DIA_CASE(SPMV_F32, float, SPMV_F32, float)
    DIA_CASE(SPMV_BF16, bf16, SPMV_F32, float)
    DIA_CASE(SPMV_F64, double, SPMV_F32, float)
#undef DIA_CASE
    return fail(SPMV_ERR_UNSUPPORTED, "spmv_dia: dtype combination");
}

}  // namespace spmv

using namespace spmv;

extern "C" {

spmv_status spmv_dia(int32_t n_rows, int32_t n_cols, int32_t ndia, const int32_t *h_offsets, const void *dia_val,
                     spmv_dtype val_dt, const int32_t *rem_row_ptr, const int32_t *rem_col, const void *rem_val,
                     const void *x, void *y, spmv_dtype vec_dt, double alpha, double beta, void *stream)
{
    return dia_product<false>(n_rows, n_cols, ndia, h_offsets, dia_val, val_dt, rem_row_ptr, rem_col, rem_val, x, y,
                              vec_dt, alpha, beta, stream);
}

spmv_status spmv_dia_sym(int32_t n, int32_t ndia, const int32_t *h_offsets, const void *dia_val, spmv_dtype val_dt,
                         const int32_t *rem_row_ptr, const int32_t *rem_col, const void *rem_val, const void *x,
                         void *y, spmv_dtype vec_dt, double alpha, double beta, void *stream)
{
    return dia_product<true>(n, n, ndia, h_offsets, dia_val, val_dt, rem_row_ptr, rem_col, rem_val, x, y, vec_dt,
                             alpha, beta, stream);
}

spmv_status spmv_dia_sliced(int32_t n_rows, int32_t n_cols, int32_t ndia, const int32_t *h_offsets,
                            const void *dia_val, spmv_dtype val_dt, const int64_t *rem_slice_ptr,
                            const int32_t *rem_slice_nd, const uint8_t *rem_slot_row, const int32_t *rem_col,
                            const void *rem_val, const void *x, void *y, spmv_dtype vec_dt, double alpha, double beta,
                            int symmetric, void *stream)
{
    if (symmetric) {
        SPMV_REQUIRE(n_rows == n_cols, "spmv_dia_sliced: symmetric storage needs a square matrix");
        return dia_product<true, true>(n_rows, n_cols, ndia, h_offsets, dia_val, val_dt, nullptr, rem_col, rem_val, x,
                                       y, vec_dt, alpha, beta, stream, rem_slice_ptr, rem_slice_nd, rem_slot_row);
    }
    return dia_product<false, true>(n_rows, n_cols, ndia, h_offsets, dia_val, val_dt, nullptr, rem_col, rem_val, x, y,
                                    vec_dt, alpha, beta, stream, rem_slice_ptr, rem_slice_nd, rem_slot_row);
}

}  // extern "C"
