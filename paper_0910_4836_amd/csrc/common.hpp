// Shared device helpers and host error plumbing for the gfx950 SpMV library.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <string>

#include "spmv.h"

namespace spmv {

// ---------------------------------------------------------------- host errors

void set_error(const std::string &msg);
spmv_status fail(spmv_status s, const std::string &msg);
spmv_status hip_fail(hipError_t e, const char *what);

#define SPMV_HIP(call)                                   \
    do {                                                 \
        hipError_t e__ = (call);                         \
        if (e__ != hipSuccess) return hip_fail(e__, #call); \
    } while (0)

#define SPMV_CHECK_LAUNCH(name)                                   \
    do {                                                          \
        hipError_t e__ = hipGetLastError();                       \
        if (e__ != hipSuccess) return hip_fail(e__, name);        \
    } while (0)

#define SPMV_REQUIRE(cond, msg)                                    \
    do {                                                           \
        if (!(cond)) return fail(SPMV_ERR_INVALID_ARG, msg);       \
    } while (0)

inline hipStream_t as_stream(void *s) { return reinterpret_cast<hipStream_t>(s); }

// y_i = alpha * sum of slots[slot_ptr[i] .. slot_ptr[i+1]) (in slot order,
// FP64) + beta * y_i: the last step of the column-split products (util.hip).
spmv_status launch_combine(int32_t n, const int32_t *slot_ptr, const double *slots, void *y, spmv_dtype vec_dt,
                           double alpha, double beta, hipStream_t s);

// Compute units of the current device (queried once per device, util.hip);
// 256 if the query fails.
int device_cus();

// Default rows-block size of the CRS plans (crs.hip).
int32_t crs_default_block_nnz();

// Column-major multi-vector kernels (crs.hip, jds.hip), the no-workspace path
// of spmm_crs / spmm_jds (spmm.hip).
spmv_status spmm_crs_colmajor(int32_t n_rows, int32_t n_cols, const int32_t *row_ptr, const int32_t *col_idx,
                              const void *val, spmv_dtype val_dt, int32_t k, const void *X, int64_t ldx, void *Y,
                              int64_t ldy, spmv_dtype vec_dt, double alpha, double beta, const int32_t *plan,
                              int32_t n_blocks, hipStream_t s);
spmv_status spmm_jds_colmajor(int32_t n, const int32_t *perm, const int32_t *jd_ptr, int32_t ndiag,
                              const int32_t *jd_col, const void *jd_val, spmv_dtype val_dt, int32_t k, const void *X,
                              int64_t ldx, void *Y, int64_t ldy, spmv_dtype vec_dt, double alpha, double beta,
                              unsigned flags, hipStream_t s);

inline size_t dtype_size(spmv_dtype dt)
{
    return dt == SPMV_F64 ? 8 : (dt == SPMV_F32 || dt == SPMV_I32) ? 4 : 2;
}

inline bool valid_dtype(spmv_dtype dt) { return dt == SPMV_F64 || dt == SPMV_F32 || dt == SPMV_BF16; }
// Element types of the calls that only move values (bit-for-bit copies).
inline bool valid_payload_dtype(spmv_dtype dt) { return valid_dtype(dt) || dt == SPMV_I32; }
inline bool valid_vec_dtype(spmv_dtype dt) { return dt == SPMV_F64 || dt == SPMV_F32; }

inline int64_t ceil_div(int64_t a, int64_t b) { return (a + b - 1) / b; }
inline size_t align_up(size_t v, size_t a) { return (v + a - 1) / a * a; }

// Carves a caller workspace into aligned pieces.
struct WsCarver {
    char *base;
    size_t used = 0;
    size_t cap;
    WsCarver(void *b, size_t c) : base(static_cast<char *>(b)), cap(c) {}
    template <typename T>
    T *take(size_t count)
    {
        used = align_up(used, 256);
        T *p = reinterpret_cast<T *>(base ? base + used : nullptr);
        used += count * sizeof(T);
        return p;
    }
    bool ok() const { return used <= cap; }
};

// ---------------------------------------------------------------- device types

struct bf16 {
    uint16_t bits;
};

__device__ __forceinline__ float to_f32(float v) { return v; }
__device__ __forceinline__ float to_f32(double v) { return (float)v; }
__device__ __forceinline__ float to_f32(bf16 v) { return __uint_as_float((uint32_t)v.bits << 16); }
__device__ __forceinline__ double to_f64(float v) { return (double)v; }
__device__ __forceinline__ double to_f64(double v) { return v; }
__device__ __forceinline__ double to_f64(bf16 v) { return (double)to_f32(v); }

template <typename T>
__device__ __forceinline__ void store_from_f64(T *p, double v);
template <>
__device__ __forceinline__ void store_from_f64<double>(double *p, double v) { *p = v; }
template <>
__device__ __forceinline__ void store_from_f64<float>(float *p, double v) { *p = (float)v; }

// Non-temporal streaming loads for the matrix arrays, which are read once per
// product and should not evict the gathered vector from the caches.
template <typename T>
__device__ __forceinline__ T ld_stream(const T *p) { return __builtin_nontemporal_load(p); }
template <>
__device__ __forceinline__ bf16 ld_stream<bf16>(const bf16 *p)
{
    bf16 r;
    r.bits = __builtin_nontemporal_load(reinterpret_cast<const uint16_t *>(p));
    return r;
}

// Accumulator for one row: FP64 when WIDE (FP64 values, or long rows with
// reduced-precision values), otherwise FP32 with x rounded to FP32.
template <bool WIDE>
struct Acc;
template <>
struct Acc<true> {
    typedef double T;
    template <typename VT, typename XT>
    __device__ __forceinline__ static double mac(double a, VT v, XT x) { return fma(to_f64(v), to_f64(x), a); }
};
template <>
struct Acc<false> {
    typedef float T;
    template <typename VT, typename XT>
    __device__ __forceinline__ static float mac(float a, VT v, XT x) { return fmaf(to_f32(v), to_f32(x), a); }
};

template <typename VT>
struct IsF64 { static constexpr bool value = false; };
template <>
struct IsF64<double> { static constexpr bool value = true; };

// y = alpha*acc + beta*y in FP64, one rounding to the vector type.
template <typename XT>
__device__ __forceinline__ void write_y(XT *y, int64_t i, double acc, double alpha, double beta)
{
    double r = alpha * acc;
    if (beta != 0.0) r = fma(beta, to_f64(y[i]), r);
    store_from_f64(&y[i], r);
}

// ---------------------------------------------------------------- wave helpers

constexpr int WAVE = 64;

// Column-split products: one part per XCD (MI355X has 8; workgroup b runs on
// XCD b % 8).
constexpr int SPLIT_PARTS = SPMV_SPLIT_PARTS;

__device__ __forceinline__ int lane_id() { return (int)(threadIdx.x & (WAVE - 1)); }

template <typename T>
__device__ __forceinline__ T shfl_xor(T v, int mask) { return __shfl_xor(v, mask, WAVE); }

// Sum over aligned groups of G lanes (G power of two <= 64), fixed tree.
template <typename T>
__device__ __forceinline__ T group_sum(T v, int G)
{
    for (int off = G >> 1; off > 0; off >>= 1) v += __shfl_xor(v, off, WAVE);
    return v;
}

// Workgroup index remapped so that each XCD (8 per MI355X, workgroups are
// dealt to them round-robin) processes a contiguous range of logical blocks:
// neighbouring rows, and so neighbouring x windows, share one L2.
__device__ __forceinline__ int64_t xcd_remap(int64_t bid, int64_t nblk)
{
    constexpr int64_t NX = 8;
    if (nblk < NX * 2) return bid;
    int64_t q = nblk / NX, r = nblk % NX;
    int64_t xcd = bid % NX, local = bid / NX;
    return xcd < r ? xcd * (q + 1) + local : r * (q + 1) + (xcd - r) * q + local;
}

}  // namespace spmv
