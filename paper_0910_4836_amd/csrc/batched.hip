// Many independent SpMVs y_m = A_m x_m in one persistent launch.
//
// Every matrix is in blocked-JDS storage (its own slice height C_m) inside
// shared arrays.  The host cuts all matrices into tiles of R consecutive
// permuted rows and writes a tile table: matrices largest first, each
// matrix's tiles together and in row order.  A grid sized to the GPU walks
// the table: each XCD takes one contiguous eighth of it and its wavefronts
// step through that range with a fixed stride.  No atomics, no queue to
// reset, so the result does not depend on timing and the launch can be
// captured in a HIP graph and replayed.  This is the paper's
// static-versus-dynamic scheduling question (Section 5) answered for a GPU:
// static assignment, as the paper found best, with locality (one matrix's x
// per L2 at a time) taking the place of first-touch page placement.
#include <algorithm>
#include <numeric>
#include <vector>

#include "common.hpp"

namespace spmv {

struct BTile {
    int64_t base;      // bl_col/bl_val offset of the tile's first row, diagonal 0
    int64_t row_base;  // matrix offset into y and perm
    int64_t col_base;  // matrix offset into x
    int32_t r0;        // first local (permuted) row of the tile
    int32_t nrows;     // valid rows (<= R)
    int32_t C;         // slice height: stride between diagonals
    int32_t nd;        // diagonals of the tile's slice
    int32_t rlog;      // R = 1 << rlog rows per wavefront
    int32_t pad;
};
static_assert(sizeof(BTile) == SPMV_BATCHED_PLAN_WORDS * sizeof(int32_t), "tile record size");

constexpr int B_THREADS = 256;
constexpr int B_WAVES = B_THREADS / WAVE;

template <int U, bool WIDE>
__device__ __forceinline__ typename Acc<WIDE>::T batched_lane_sum(const BTile &T, const int32_t *__restrict__ col,
                                                                  const float *__restrict__ val,
                                                                  const float *__restrict__ x, int rl, int kk, int G,
                                                                  bool r_ok)
{
    typename Acc<WIDE>::T s = 0;
    for (int32_t base = 0; base < T.nd; base += G * U) {
        int32_t c[U];
        float v[U];
        bool act[U];
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const int32_t dd = base + kk + u * G;
            act[u] = false;
            if (r_ok && dd < T.nd) {
                const int64_t e = T.base + (int64_t)dd * T.C + rl;
                c[u] = ld_stream(col + e);
                v[u] = ld_stream(val + e);
                act[u] = c[u] >= 0;
            }
        }
        float xv[U];
#pragma unroll
        for (int u = 0; u < U; ++u)
            if (act[u]) xv[u] = x[T.col_base + c[u]];
#pragma unroll
        for (int u = 0; u < U; ++u)
            if (act[u]) s = Acc<WIDE>::mac(s, v[u], xv[u]);
    }
    return s;
}

template <int U>
__global__ __launch_bounds__(B_THREADS) void batched_kernel(int64_t n_tiles, const BTile *__restrict__ tiles,
                                                            const int32_t *__restrict__ perm,
                                                            const int32_t *__restrict__ col,
                                                            const float *__restrict__ val,
                                                            const float *__restrict__ x, float *__restrict__ y)
{
    // Workgroups are dealt to the 8 XCDs round-robin (the host launches a
    // multiple of 8).  Each XCD owns one contiguous eighth of the tile table, so
    // its L2 holds the x of the one or two matrices it is working on; inside
    // that range its wavefronts take tiles with a fixed stride.
    constexpr int NX = 8;
    const int w = (int)threadIdx.x / WAVE, lane = lane_id();
    const int xcd = (int)(blockIdx.x % NX);
    const int64_t local = blockIdx.x / NX;
    const int64_t waves_per_xcd = (int64_t)(gridDim.x / NX) * B_WAVES;
    const int64_t t_begin = n_tiles * xcd / NX, t_end = n_tiles * (xcd + 1) / NX;
    for (int64_t t = t_begin + local * B_WAVES + w; t < t_end; t += waves_per_xcd) {
        const BTile T = tiles[t];
        const int R = 1 << T.rlog, G = WAVE >> T.rlog;
        const int rl = lane & (R - 1), kk = lane >> T.rlog;
        const bool r_ok = rl < T.nrows;
        double td;
        if (T.nd > SPMV_WIDE_ROW_NNZ) {
            double s = batched_lane_sum<U, true>(T, col, val, x, rl, kk, G, r_ok);
            for (int off = 32; off >= R; off >>= 1) s += __shfl_xor(s, off, WAVE);
            td = s;
        } else {
            float s = batched_lane_sum<U, false>(T, col, val, x, rl, kk, G, r_ok);
            for (int off = 32; off >= R; off >>= 1) s += __shfl_xor(s, off, WAVE);
            td = (double)s;
        }
        if (r_ok && kk == 0) {
            const int64_t pr = T.row_base + T.r0 + rl;
            y[T.row_base + perm[pr]] = (float)td;
        }
    }
}

}  // namespace spmv

using namespace spmv;

extern "C" {

spmv_status spmv_batched_plan(int32_t n_mat, const int32_t *h_n_rows, const int32_t *h_C, const int64_t *h_slice_base,
                              const int64_t *h_row_base, const int64_t *h_col_base, const int64_t *h_slice_ptr,
                              const int32_t *h_slice_nd, int32_t rows_per_wave, int32_t *plan, int64_t plan_cap,
                              int64_t *h_n_tiles, void *stream)
{
    SPMV_REQUIRE(n_mat >= 0, "spmv_batched_plan: n_mat < 0");
    SPMV_REQUIRE(h_n_tiles, "spmv_batched_plan: null h_n_tiles");
    if (rows_per_wave == 0) rows_per_wave = 64;
    SPMV_REQUIRE(rows_per_wave == 8 || rows_per_wave == 16 || rows_per_wave == 32 || rows_per_wave == 64,
                 "spmv_batched_plan: rows_per_wave must be 8, 16, 32 or 64");
    SPMV_REQUIRE(n_mat == 0 || (h_n_rows && h_C && h_slice_base && h_row_base && h_col_base && h_slice_ptr &&
                                h_slice_nd),
                 "spmv_batched_plan: null descriptor");
    int rlog = 0;
    while ((1 << rlog) < rows_per_wave) ++rlog;
    // matrices ordered by stored slots, largest first (stable); each matrix's
    // tiles stay together in row order so that the wavefronts working at one
    // time share that matrix's x in L2
    std::vector<int64_t> work(n_mat, 0);
    for (int32_t m = 0; m < n_mat; ++m) {
        const int32_t n = h_n_rows[m], C = h_C[m];
        SPMV_REQUIRE(n >= 0 && C > 0 && C % 64 == 0, "spmv_batched_plan: bad n_rows or C");
        for (int64_t s = 0; s < ceil_div(n, C); ++s) work[m] += (int64_t)h_slice_nd[h_slice_base[m] + s] * C;
    }
    std::vector<int32_t> order(n_mat);
    std::iota(order.begin(), order.end(), 0);
    std::stable_sort(order.begin(), order.end(), [&](int32_t a, int32_t b) { return work[a] > work[b]; });
    std::vector<BTile> tiles;
    for (int32_t m : order) {
        const int32_t n = h_n_rows[m], C = h_C[m];
        const int64_t ns = ceil_div(n, C);
        for (int64_t s = 0; s < ns; ++s) {
            const int64_t sp = h_slice_ptr[h_slice_base[m] + s];
            const int32_t nd = h_slice_nd[h_slice_base[m] + s];
            for (int32_t g = 0; g < C; g += rows_per_wave) {
                const int64_t r0 = s * C + g;
                if (r0 >= n) break;
                BTile t{};
                t.base = sp + g;
                t.row_base = h_row_base[m];
                t.col_base = h_col_base[m];
                t.r0 = (int32_t)r0;
                t.nrows = (int32_t)std::min<int64_t>(rows_per_wave, n - r0);
                t.C = C;
                t.nd = nd;
                t.rlog = rlog;
                tiles.push_back(t);
            }
        }
    }
    *h_n_tiles = (int64_t)tiles.size();
    const int64_t words = (int64_t)tiles.size() * SPMV_BATCHED_PLAN_WORDS;
    if (!plan || plan_cap < words) return fail(SPMV_ERR_CAPACITY, "spmv_batched_plan: plan capacity too small");
    if (!tiles.empty()) {
        hipStream_t s = as_stream(stream);
        SPMV_HIP(hipMemcpyAsync(plan, tiles.data(), sizeof(BTile) * tiles.size(), hipMemcpyHostToDevice, s));
        SPMV_HIP(hipStreamSynchronize(s));
    }
    return SPMV_OK;
}

spmv_status spmv_batched(int64_t n_tiles, const int32_t *plan, const int32_t *perm, const int32_t *bl_col,
                         const float *bl_val, const float *x, float *y, int32_t unroll, int32_t n_workgroups,
                         void *stream)
{
    SPMV_REQUIRE(n_tiles >= 0 && n_workgroups >= 0, "spmv_batched: negative size");
    SPMV_REQUIRE(unroll == 0 || unroll == 2 || unroll == 4 || unroll == 8, "spmv_batched: unroll must be 0, 2, 4 or 8");
    if (n_tiles == 0) return SPMV_OK;
    SPMV_REQUIRE(plan && perm && bl_col && bl_val && x && y, "spmv_batched: null pointer");
    if (n_workgroups == 0) {
        int dev = 0, cus = 0;
        SPMV_HIP(hipGetDevice(&dev));
        SPMV_HIP(hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev));
        n_workgroups = cus * 8;
    }
    // a multiple of 8 workgroups: every XCD gets the same number
    const int64_t need = ceil_div(n_tiles, B_WAVES);
    int64_t g = std::min<int64_t>(n_workgroups, need);
    g = std::max<int64_t>(8, g / 8 * 8);
    const unsigned grid = (unsigned)g;
    const BTile *tiles = reinterpret_cast<const BTile *>(plan);
    hipStream_t s = as_stream(stream);
    switch (unroll) {
    case 2: batched_kernel<2><<<grid, B_THREADS, 0, s>>>(n_tiles, tiles, perm, bl_col, bl_val, x, y); break;
    case 8: batched_kernel<8><<<grid, B_THREADS, 0, s>>>(n_tiles, tiles, perm, bl_col, bl_val, x, y); break;
    default: batched_kernel<4><<<grid, B_THREADS, 0, s>>>(n_tiles, tiles, perm, bl_col, bl_val, x, y); break;
    }
    SPMV_CHECK_LAUNCH("spmv_batched");
    return SPMV_OK;
}

}  // extern "C"
