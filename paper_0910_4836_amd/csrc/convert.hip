// Format construction on the GPU (paper Section 2): COO -> CRS, CRS checks,
// CRS -> JDS (row permutation by decreasing length, jagged diagonals), JDS ->
// CRS, JDS -> blocked JDS (RBJDS, optionally SOJDS), CRS transpose, value
// rounding, vector permutation and gathers.
//
// All orderings are produced by a stable least-significant-digit radix sort
// written here (8-bit digits, wave ballots for the in-tile ranks), so every
// permutation is unique and reproducible; counts use integer atomics only.
#include <algorithm>
#include <vector>

#include "common.hpp"

namespace spmv {

// ======================================================================= scan
// Exclusive prefix sum out[i] = sum_{j<i} in[j], out[n] = total.  Three
// phases: tile sums, (recursive) scan of the tile sums, tile scans.

constexpr int SCAN_THREADS = 256;
constexpr int SCAN_ITEMS = 8;
constexpr int SCAN_TILE = SCAN_THREADS * SCAN_ITEMS;

template <typename T>
__device__ __forceinline__ T block_exclusive_scan(T v, T *wave_tot, T *total)
{
    const int lane = lane_id(), w = (int)threadIdx.x / WAVE;
    T inc = v;
    for (int off = 1; off < WAVE; off <<= 1) {
        T o = __shfl_up(inc, off, WAVE);
        if (lane >= off) inc += o;
    }
    if (lane == WAVE - 1) wave_tot[w] = inc;
    __syncthreads();
    T wbase = 0, all = 0;
    for (int i = 0; i < SCAN_THREADS / WAVE; ++i) {
        if (i < w) wbase += wave_tot[i];
        all += wave_tot[i];
    }
    if (total) *total = all;
    __syncthreads();
    return wbase + inc - v;
}

template <typename TI, typename TO>
__global__ __launch_bounds__(SCAN_THREADS) void scan_tile_sums(const TI *__restrict__ in, int64_t n,
                                                               TO *__restrict__ sums)
{
    __shared__ TO wt[SCAN_THREADS / WAVE];
    const int64_t base = (int64_t)blockIdx.x * SCAN_TILE;
    TO s = 0;
    for (int j = 0; j < SCAN_ITEMS; ++j) {
        int64_t i = base + (int64_t)j * SCAN_THREADS + threadIdx.x;
        if (i < n) s += (TO)in[i];
    }
    TO tot;
    block_exclusive_scan<TO>(s, wt, &tot);
    if (threadIdx.x == 0) sums[blockIdx.x] = tot;
}

template <typename TI, typename TO>
__global__ __launch_bounds__(SCAN_THREADS) void scan_tiles(const TI *__restrict__ in, int64_t n,
                                                           const TO *__restrict__ tile_base, TO *__restrict__ out,
                                                           bool write_total)
{
    __shared__ TO wt[SCAN_THREADS / WAVE];
    const int64_t base = (int64_t)blockIdx.x * SCAN_TILE + (int64_t)threadIdx.x * SCAN_ITEMS;
    TO v[SCAN_ITEMS];
    TO s = 0;
#pragma unroll
    for (int j = 0; j < SCAN_ITEMS; ++j) {
        int64_t i = base + j;
        v[j] = i < n ? (TO)in[i] : (TO)0;
        s += v[j];
    }
    TO tot;
    TO run = block_exclusive_scan<TO>(s, wt, &tot) + (tile_base ? tile_base[blockIdx.x] : (TO)0);
#pragma unroll
    for (int j = 0; j < SCAN_ITEMS; ++j) {
        int64_t i = base + j;
        if (i < n) out[i] = run;
        run += v[j];
    }
    if (write_total && blockIdx.x == gridDim.x - 1 && threadIdx.x == 0)
        out[n] = (tile_base ? tile_base[blockIdx.x] : (TO)0) + tot;
}

static size_t scan_ws_elems(int64_t n)
{
    size_t total = 0;
    int64_t tiles = ceil_div(n, SCAN_TILE);
    while (tiles > 1) {
        total += (size_t)tiles + 1;
        tiles = ceil_div(tiles, SCAN_TILE);
    }
    return total + 1;
}

// out has n+1 entries; ws holds scan_ws_elems(n) TO values.
template <typename TI, typename TO>
static spmv_status exclusive_scan(const TI *in, int64_t n, TO *out, TO *ws, hipStream_t s)
{
    if (n == 0) {
        SPMV_HIP(hipMemsetAsync(out, 0, sizeof(TO), s));
        return SPMV_OK;
    }
    int64_t tiles = ceil_div(n, SCAN_TILE);
    if (tiles == 1) {
        scan_tiles<TI, TO><<<1, SCAN_THREADS, 0, s>>>(in, n, (const TO *)nullptr, out, true);
        SPMV_CHECK_LAUNCH("scan");
        return SPMV_OK;
    }
    TO *sums = ws;                    // tiles + 1 entries
    TO *rest = ws + tiles + 1;
    scan_tile_sums<TI, TO><<<(unsigned)tiles, SCAN_THREADS, 0, s>>>(in, n, sums);
    SPMV_CHECK_LAUNCH("scan tile sums");
    spmv_status st = exclusive_scan<TO, TO>(sums, tiles, sums, rest, s);   // in place is safe per tile
    if (st != SPMV_OK) return st;
    scan_tiles<TI, TO><<<(unsigned)tiles, SCAN_THREADS, 0, s>>>(in, n, sums, out, true);
    SPMV_CHECK_LAUNCH("scan tiles");
    return SPMV_OK;
}

// ================================================================ radix sort
// Stable LSD radix sort of (uint32 key, int32 value) pairs, 8 bits per pass.

constexpr int RS_THREADS = 256;
constexpr int RS_WAVES = RS_THREADS / WAVE;
constexpr int RS_ITEMS = 16;                       // per lane
constexpr int RS_TILE = RS_THREADS * RS_ITEMS;     // 4096 keys per tile
constexpr int RS_BINS = 256;

__global__ __launch_bounds__(RS_THREADS) void radix_hist_kernel(const uint32_t *__restrict__ keys, int64_t n,
                                                                int shift, int32_t *__restrict__ counts,
                                                                int64_t ntiles)
{
    __shared__ int32_t h[RS_BINS];
    for (int i = threadIdx.x; i < RS_BINS; i += RS_THREADS) h[i] = 0;
    __syncthreads();
    const int64_t base = (int64_t)blockIdx.x * RS_TILE;
    for (int j = 0; j < RS_ITEMS; ++j) {
        int64_t i = base + (int64_t)j * RS_THREADS + threadIdx.x;
        if (i < n) atomicAdd(&h[(keys[i] >> shift) & 0xff], 1);
    }
    __syncthreads();
    for (int i = threadIdx.x; i < RS_BINS; i += RS_THREADS) counts[(int64_t)i * ntiles + blockIdx.x] = h[i];
}

__global__ __launch_bounds__(RS_THREADS) void radix_scatter_kernel(const uint32_t *__restrict__ kin,
                                                                   const int32_t *__restrict__ vin, int64_t n,
                                                                   int shift, const int32_t *__restrict__ offs,
                                                                   int64_t ntiles, uint32_t *__restrict__ kout,
                                                                   int32_t *__restrict__ vout)
{
    __shared__ int32_t cnt[RS_WAVES][RS_BINS];
    for (int i = threadIdx.x; i < RS_WAVES * RS_BINS; i += RS_THREADS) (&cnt[0][0])[i] = 0;
    __syncthreads();
    const int w = (int)threadIdx.x / WAVE, lane = lane_id();
    const uint64_t lt_mask = (lane == 0) ? 0ull : (~0ull >> (WAVE - lane));
    // wave w owns keys [base_w, base_w + 64*RS_ITEMS), in rounds of 64 in order
    const int64_t base_w = (int64_t)blockIdx.x * RS_TILE + (int64_t)w * WAVE * RS_ITEMS;
    uint32_t k[RS_ITEMS];
    int32_t v[RS_ITEMS];
    int32_t rank[RS_ITEMS];
#pragma unroll
    for (int j = 0; j < RS_ITEMS; ++j) {
        const int64_t i = base_w + (int64_t)j * WAVE + lane;
        const bool in = i < n;
        k[j] = in ? kin[i] : 0u;
        v[j] = in ? vin[i] : 0;
        const uint32_t dg = (k[j] >> shift) & 0xff;
        uint64_t peers = __ballot(in);
#pragma unroll
        for (int b = 0; b < 8; ++b) {
            const uint64_t m = __ballot((dg >> b) & 1u);
            peers &= ((dg >> b) & 1u) ? m : ~m;
        }
        const int before = __popcll(peers & lt_mask);
        const int32_t start = cnt[w][dg];
        rank[j] = start + before;
        // the first lane of each digit group advances the wave's counter
        if (in && before == 0) cnt[w][dg] = start + __popcll(peers);
        __builtin_amdgcn_wave_barrier();
    }
    __syncthreads();
    // per digit: exclusive prefix over the waves (tile order = wave order)
    for (int dg = threadIdx.x; dg < RS_BINS; dg += RS_THREADS) {
        int32_t run = 0;
        for (int q = 0; q < RS_WAVES; ++q) {
            int32_t c = cnt[q][dg];
            cnt[q][dg] = run;
            run += c;
        }
    }
    __syncthreads();
#pragma unroll
    for (int j = 0; j < RS_ITEMS; ++j) {
        const int64_t i = base_w + (int64_t)j * WAVE + lane;
        if (i < n) {
            const uint32_t dg = (k[j] >> shift) & 0xff;
            const int64_t pos = (int64_t)offs[(int64_t)dg * ntiles + blockIdx.x] + cnt[w][dg] + rank[j];
            kout[pos] = k[j];
            vout[pos] = v[j];
        }
    }
}

static size_t radix_ws_bytes(int64_t n)
{
    int64_t ntiles = n > 0 ? ceil_div(n, RS_TILE) : 1;
    size_t cells = (size_t)ntiles * RS_BINS;
    size_t b = 0;
    b += align_up(sizeof(int32_t) * cells, 256);                 // counts
    b += align_up(sizeof(int32_t) * (cells + 1), 256);           // offsets
    b += align_up(sizeof(int32_t) * scan_ws_elems((int64_t)cells), 256);
    b += 2 * align_up(sizeof(uint32_t) * (size_t)(n > 0 ? n : 1), 256);   // ping-pong keys/values
    return b + 256;
}

// Sorts (keys, vals) by the low `bits` bits of the keys, stably.  The result
// is left in (keys, vals); ws provides the ping-pong buffers.
static spmv_status radix_sort_pairs(uint32_t *keys, int32_t *vals, int64_t n, int bits, void *ws, size_t ws_bytes,
                                    hipStream_t s)
{
    if (n <= 1 || bits <= 0) return SPMV_OK;
    int64_t ntiles = ceil_div(n, RS_TILE);
    size_t cells = (size_t)ntiles * RS_BINS;
    WsCarver wc(ws, ws_bytes);
    int32_t *counts = wc.take<int32_t>(cells);
    int32_t *offs = wc.take<int32_t>(cells + 1);
    int32_t *sws = wc.take<int32_t>(scan_ws_elems((int64_t)cells));
    uint32_t *k2 = wc.take<uint32_t>((size_t)n);
    int32_t *v2 = wc.take<int32_t>((size_t)n);
    if (!wc.ok()) return fail(SPMV_ERR_INVALID_ARG, "radix sort: workspace too small");
    uint32_t *ka = keys, *kb = k2;
    int32_t *va = vals, *vb = v2;
    int passes = 0;
    for (int shift = 0; shift < bits; shift += 8) {
        radix_hist_kernel<<<(unsigned)ntiles, RS_THREADS, 0, s>>>(ka, n, shift, counts, ntiles);
        SPMV_CHECK_LAUNCH("radix hist");
        spmv_status st = exclusive_scan<int32_t, int32_t>(counts, (int64_t)cells, offs, sws, s);
        if (st != SPMV_OK) return st;
        radix_scatter_kernel<<<(unsigned)ntiles, RS_THREADS, 0, s>>>(ka, va, n, shift, offs, ntiles, kb, vb);
        SPMV_CHECK_LAUNCH("radix scatter");
        uint32_t *tk = ka; ka = kb; kb = tk;
        int32_t *tv = va; va = vb; vb = tv;
        ++passes;
    }
    if (passes & 1) {
        SPMV_HIP(hipMemcpyAsync(keys, ka, sizeof(uint32_t) * n, hipMemcpyDeviceToDevice, s));
        SPMV_HIP(hipMemcpyAsync(vals, va, sizeof(int32_t) * n, hipMemcpyDeviceToDevice, s));
    }
    return SPMV_OK;
}

static int bits_for(int64_t maxval)
{
    int b = 0;
    while (b < 32 && ((int64_t)1 << b) <= maxval) ++b;
    return b;
}

// ============================================================ small kernels

#define GRID_LOOP(i, n) \
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < (n); i += (int64_t)gridDim.x * blockDim.x)

static unsigned grid_for(int64_t n)
{
    int64_t g = ceil_div(n, 256);
    if (g > 65536) g = 65536;
    return (unsigned)(g < 1 ? 1 : g);
}

__global__ void iota_kernel(int32_t *out, int64_t n) { GRID_LOOP(i, n) out[i] = (int32_t)i; }

__global__ void copy_u32_kernel(const int32_t *__restrict__ in, uint32_t *__restrict__ out, int64_t n)
{
    GRID_LOOP(i, n) out[i] = (uint32_t)in[i];
}

__global__ void gather_u32_kernel(const int32_t *__restrict__ src, const int32_t *__restrict__ idx,
                                  uint32_t *__restrict__ out, int64_t n)
{
    GRID_LOOP(i, n) out[i] = (uint32_t)src[idx[i]];
}

__global__ void coo_check_kernel(const int32_t *__restrict__ row, const int32_t *__restrict__ col, int64_t n,
                                 int32_t n_rows, int32_t n_cols, int32_t *__restrict__ bad)
{
    GRID_LOOP(i, n)
    {
        if (row[i] < 0 || row[i] >= n_rows || col[i] < 0 || col[i] >= n_cols) atomicOr(bad, 1);
    }
}

// sorted (row, col) pairs -> 1 where a new (row, col) starts
__global__ void head_flags_kernel(const uint32_t *__restrict__ rk, const int32_t *__restrict__ idx,
                                  const int32_t *__restrict__ col, int64_t n, int32_t *__restrict__ flag)
{
    GRID_LOOP(i, n)
    {
        int32_t f = 1;
        if (i > 0 && rk[i] == rk[i - 1] && col[idx[i]] == col[idx[i - 1]]) f = 0;
        flag[i] = f;
    }
}

// one thread per run of equal (row, col): sums the run's values in input order
template <typename T>
__global__ void compact_kernel(const uint32_t *__restrict__ rk, const int32_t *__restrict__ idx,
                               const int32_t *__restrict__ col, const T *__restrict__ val,
                               const int32_t *__restrict__ flag, const int32_t *__restrict__ pos, int64_t n,
                               int32_t *__restrict__ col_out, T *__restrict__ val_out, int32_t *__restrict__ row_u)
{
    GRID_LOOP(i, n)
    {
        if (!flag[i]) continue;
        const int32_t p = pos[i];
        T s = val[idx[i]];
        for (int64_t j = i + 1; j < n && !flag[j]; ++j) s = s + val[idx[j]];
        col_out[p] = col[idx[i]];
        val_out[p] = s;
        row_u[p] = (int32_t)rk[i];
    }
}

// first index in sorted a[0..n) with a[idx] >= key
template <typename T, typename K>
__device__ __forceinline__ int64_t lower_bound_dev(const T *a, int64_t n, K key)
{
    int64_t lo = 0, hi = n;
    while (lo < hi) {
        int64_t mid = (lo + hi) >> 1;
        if ((K)a[mid] < key) lo = mid + 1;
        else hi = mid;
    }
    return lo;
}

template <typename T>
__global__ void ptr_from_sorted_kernel(const T *__restrict__ sorted, int64_t n, int32_t nseg,
                                       int32_t *__restrict__ ptr)
{
    GRID_LOOP(r, (int64_t)nseg + 1) ptr[r] = (int32_t)lower_bound_dev(sorted, n, (int64_t)r);
}

__global__ void validate_rows_kernel(const int32_t *__restrict__ rp, int32_t n_rows, int64_t nnz,
                                     int32_t *__restrict__ bad)
{
    GRID_LOOP(r, (int64_t)n_rows)
    {
        if (rp[r + 1] < rp[r]) atomicOr(bad, 1);
        if (r == 0 && rp[0] != 0) atomicOr(bad, 2);
        if (r == n_rows - 1 && (int64_t)rp[n_rows] != nnz) atomicOr(bad, 4);
    }
}

__global__ void validate_cols_kernel(const int32_t *__restrict__ col, int64_t nnz, int32_t n_cols,
                                     int32_t *__restrict__ bad)
{
    GRID_LOOP(k, nnz)
    {
        if (col[k] < 0 || col[k] >= n_cols) atomicOr(bad, 8);
    }
}

__global__ void row_len_kernel(const int32_t *__restrict__ rp, int32_t n, int32_t *__restrict__ len,
                               int32_t *__restrict__ maxlen)
{
    GRID_LOOP(r, (int64_t)n)
    {
        int32_t l = rp[r + 1] - rp[r];
        len[r] = l;
        atomicMax(maxlen, l);
    }
}

__global__ void desc_key_kernel(const int32_t *__restrict__ len, int32_t n, int32_t ndiag, uint32_t *__restrict__ key)
{
    GRID_LOOP(r, (int64_t)n) key[r] = (uint32_t)(ndiag - len[r]);
}

__global__ void inverse_perm_kernel(const int32_t *__restrict__ perm, int32_t n, int32_t *__restrict__ iperm)
{
    GRID_LOOP(r, (int64_t)n) iperm[perm[r]] = (int32_t)r;
}

// count[d] = rows longer than d = first permuted row whose length is <= d
__global__ void diag_count_kernel(const uint32_t *__restrict__ skey, int32_t n, int32_t ndiag,
                                  int32_t *__restrict__ count)
{
    GRID_LOOP(d, (int64_t)ndiag)
    {
        // lengths ndiag - skey[r] never increase; find first r with length <= d
        int64_t lo = 0, hi = n;
        while (lo < hi) {
            int64_t mid = (lo + hi) >> 1;
            if ((int64_t)ndiag - (int64_t)skey[mid] > d) lo = mid + 1;
            else hi = mid;
        }
        count[d] = (int32_t)lo;
    }
}

// row containing CRS entry j: last r with rp[r] <= j
__device__ __forceinline__ int32_t row_of(const int32_t *__restrict__ rp, int32_t n, int64_t j)
{
    int32_t lo = 0, hi = n - 1;
    while (lo < hi) {
        int32_t mid = (lo + hi + 1) >> 1;
        if ((int64_t)rp[mid] <= j) lo = mid;
        else hi = mid - 1;
    }
    return lo;
}

template <typename T>
__global__ void jds_scatter_kernel(const int32_t *__restrict__ rp, const int32_t *__restrict__ col,
                                   const T *__restrict__ val, int32_t n, int64_t nnz, const int32_t *__restrict__ iperm,
                                   const int32_t *__restrict__ jd_ptr, int symperm, int32_t *__restrict__ jd_col,
                                   T *__restrict__ jd_val)
{
    GRID_LOOP(j, nnz)
    {
        const int32_t i = row_of(rp, n, j);
        const int32_t d = (int32_t)(j - rp[i]);
        const int64_t dst = (int64_t)jd_ptr[d] + iperm[i];
        const int32_t c = col[j];
        jd_col[dst] = symperm ? iperm[c] : c;
        jd_val[dst] = val[j];
    }
}

// length of permuted row r from the diagonal lengths
__device__ __forceinline__ int32_t jds_len_of(const int32_t *__restrict__ jp, int32_t ndiag, int64_t r)
{
    int32_t lo = 0, hi = ndiag;
    while (lo < hi) {
        int32_t mid = (lo + hi) >> 1;
        if ((int64_t)(jp[mid + 1] - jp[mid]) > r) lo = mid + 1;
        else hi = mid;
    }
    return lo;
}

__global__ void jds_row_len_kernel(const int32_t *__restrict__ jp, int32_t ndiag, const int32_t *__restrict__ perm,
                                   int32_t n, int32_t *__restrict__ len)
{
    GRID_LOOP(r, (int64_t)n) len[perm[r]] = jds_len_of(jp, ndiag, r);
}

// diagonal holding JDS entry e: last d with jp[d] <= e
__device__ __forceinline__ int32_t diag_of(const int32_t *__restrict__ jp, int32_t ndiag, int64_t e)
{
    int32_t lo = 0, hi = ndiag - 1;
    while (lo < hi) {
        int32_t mid = (lo + hi + 1) >> 1;
        if ((int64_t)jp[mid] <= e) lo = mid;
        else hi = mid - 1;
    }
    return lo;
}

template <typename T>
__global__ void jds_to_csr_kernel(const int32_t *__restrict__ jp, int32_t ndiag, int64_t nnz,
                                  const int32_t *__restrict__ perm, const int32_t *__restrict__ jd_col,
                                  const T *__restrict__ jd_val, int symperm, const int32_t *__restrict__ rp,
                                  int32_t *__restrict__ col, T *__restrict__ val)
{
    GRID_LOOP(e, nnz)
    {
        const int32_t d = diag_of(jp, ndiag, e);
        const int32_t r = (int32_t)(e - jp[d]);
        const int32_t i = perm[r];
        const int64_t dst = (int64_t)rp[i] + d;
        const int32_t c = jd_col[e];
        col[dst] = symperm ? perm[c] : c;
        val[dst] = jd_val[e];
    }
}

__global__ void slice_nd_kernel(const int32_t *__restrict__ jp, int32_t ndiag, int32_t C, int32_t n_slices,
                                int32_t *__restrict__ nd, int64_t *__restrict__ sz)
{
    GRID_LOOP(s, (int64_t)n_slices)
    {
        int32_t l = jds_len_of(jp, ndiag, s * (int64_t)C);
        nd[s] = l;
        sz[s] = (int64_t)l * C;
    }
}

template <typename T>
__global__ void blocked_fill_kernel(const int32_t *__restrict__ jp, int32_t ndiag, const int32_t *__restrict__ jd_col,
                                    const T *__restrict__ jd_val, int32_t n, int32_t C,
                                    const int64_t *__restrict__ slice_ptr, int32_t n_slices, int64_t total,
                                    int32_t *__restrict__ bl_col, T *__restrict__ bl_val)
{
    GRID_LOOP(k, total)
    {
        int32_t lo = 0, hi = n_slices - 1;
        while (lo < hi) {
            int32_t mid = (lo + hi + 1) >> 1;
            if (slice_ptr[mid] <= k) lo = mid;
            else hi = mid - 1;
        }
        const int64_t local = k - slice_ptr[lo];
        const int32_t d = (int32_t)(local / C);
        const int32_t rl = (int32_t)(local - (int64_t)d * C);
        const int64_t r = (int64_t)lo * C + rl;
        if (r < n && (int64_t)(jp[d + 1] - jp[d]) > r) {
            bl_col[k] = jd_col[jp[d] + r];
            bl_val[k] = jd_val[jp[d] + r];
        } else {
            bl_col[k] = -1;
            bl_val[k] = T{};
        }
    }
}

// Windowed RBJDS (rows sorted by length inside windows of sigma rows):
// window of the row each permuted position holds, the sort key of the
// second, stable pass.
__global__ void window_key_kernel(const int32_t *__restrict__ perm, int32_t n, int32_t sigma,
                                  uint32_t *__restrict__ key)
{
    GRID_LOOP(r, (int64_t)n) key[r] = (uint32_t)(perm[r] / sigma);
}

// slice s's depth = length of its first row (the longest: slices never span
// two windows and rows are sorted inside a window)
__global__ void window_slice_nd_kernel(const int32_t *__restrict__ rp, const int32_t *__restrict__ perm,
                                       int32_t C, int32_t n_slices, int32_t *__restrict__ nd,
                                       int64_t *__restrict__ sz)
{
    GRID_LOOP(s, (int64_t)n_slices)
    {
        const int32_t row = perm[s * (int64_t)C];
        const int32_t l = rp[row + 1] - rp[row];
        nd[s] = l;
        sz[s] = (int64_t)l * C;
    }
}

// slices of C rows in row order: depth = the slice's longest row
// One workgroup per window of SPMV_REM_WINDOW rows: each row's rank in the
// window's decreasing-length order (ties: lower row first) by counting over
// the window's lengths in LDS; the sorted position's window-local row (uint8)
// and global row (for the fill), and the depth of every slice of
// SPMV_REM_SLICE positions (its first row's length).
__global__ __launch_bounds__(SPMV_REM_WINDOW) void rem_order_kernel(const int32_t *__restrict__ rp, int32_t n,
                                                                     uint8_t *__restrict__ slot_row,
                                                                     int32_t *__restrict__ perm,
                                                                     int32_t *__restrict__ nd, int64_t *__restrict__ sz)
{
    __shared__ int32_t len[SPMV_REM_WINDOW];
    __shared__ int32_t at[SPMV_REM_WINDOW];
    const int64_t base = (int64_t)blockIdx.x * SPMV_REM_WINDOW;
    const int t = threadIdx.x;
    const int cnt = n - base < SPMV_REM_WINDOW ? (int)(n - base) : SPMV_REM_WINDOW;
    len[t] = t < cnt ? rp[base + t + 1] - rp[base + t] : -1;
    __syncthreads();
    if (t < cnt) {
        const int32_t l = len[t];
        int rank = 0;
        for (int j = 0; j < cnt; ++j) {
            const int32_t lj = len[j];
            rank += (lj > l) | ((lj == l) & (j < t));
        }
        at[rank] = t;
        slot_row[base + rank] = (uint8_t)t;
        perm[base + rank] = (int32_t)(base + t);
    }
    __syncthreads();
    if (t < cnt && t % SPMV_REM_SLICE == 0) {
        const int64_t sl = (base + t) / SPMV_REM_SLICE;
        const int32_t d = len[at[t]];
        nd[sl] = d;
        sz[sl] = (int64_t)d * SPMV_REM_SLICE;
    }
}

// slot k of the padded storage: entry d of permuted row r, taken from CRS in
// its row order, or padding (col = -1, value 0)
template <typename T>
__global__ void window_fill_kernel(const int32_t *__restrict__ rp, const int32_t *__restrict__ col,
                                   const T *__restrict__ val, const int32_t *__restrict__ perm, int32_t n, int32_t C,
                                   const int64_t *__restrict__ slice_ptr, int32_t n_slices, int64_t total,
                                   int32_t *__restrict__ bl_col, T *__restrict__ bl_val)
{
    GRID_LOOP(k, total)
    {
        int32_t lo = 0, hi = n_slices - 1;
        while (lo < hi) {
            int32_t mid = (lo + hi + 1) >> 1;
            if (slice_ptr[mid] <= k) lo = mid;
            else hi = mid - 1;
        }
        const int64_t local = k - slice_ptr[lo];
        const int32_t d = (int32_t)(local / C);
        const int32_t rl = (int32_t)(local - (int64_t)d * C);
        const int64_t r = (int64_t)lo * C + rl;
        int32_t e = -1;
        if (r < n) {
            const int32_t row = perm[r];
            if (d < rp[row + 1] - rp[row]) e = rp[row] + d;
        }
        if (e >= 0) {
            bl_col[k] = col[e];
            bl_val[k] = val[e];
        } else {
            bl_col[k] = -1;
            bl_val[k] = T{};
        }
    }
}

// SOJDS: one thread per slice re-assigns each row's entries to diagonal slots
// (first row keeps CRS order; later rows take, slot by slot, the unused entry
// whose column is nearest to the previous row's column in that slot plus one,
// the smaller column on a tie).  `taken` holds one bit per entry of a row.
// A row whose columns strictly increase (CRS order of a matrix built by
// spmv_csr_from_coo) finds that entry in O(log L) loads: a binary search for
// the target column, then the nearest clear bit of `taken` on either side;
// any other row compares all of its unused entries.

// first clear bit at index >= from, or -1 if none below len
__device__ __forceinline__ int32_t next_clear(const uint32_t *taken, int32_t from, int32_t len)
{
    if (from >= len) return -1;
    int32_t w = from >> 5;
    uint32_t m = ~taken[w] & (0xffffffffu << (from & 31));
    const int32_t last = (len - 1) >> 5;
    while (m == 0) {
        if (++w > last) return -1;
        m = ~taken[w];
    }
    const int32_t e = (w << 5) + __ffs(m) - 1;
    return e < len ? e : -1;
}

// last clear bit at index < below, or -1 if none
__device__ __forceinline__ int32_t prev_clear(const uint32_t *taken, int32_t below)
{
    if (below <= 0) return -1;
    int32_t w = (below - 1) >> 5;
    uint32_t m = ~taken[w] & (0xffffffffu >> (31 - ((below - 1) & 31)));
    while (m == 0) {
        if (--w < 0) return -1;
        m = ~taken[w];
    }
    return (w << 5) + 31 - __clz(m);
}

// The same greedy rule with one wavefront per slice, for slices whose first
// row has at most SOJDS_LDS_CAP entries: the current row's columns (placed
// entries overwritten by a marker) and the previous row's slot columns live
// in LDS; for each slot the 64 lanes scan the row's unused entries (lane l:
// entries l, l+64, ...) for the one nearest to (previous row's column in that
// slot) + 1, smaller column on a tie, and a fixed shuffle tree picks the
// wavefront's best.  Columns of a row are distinct, so the pick is unique and
// matches the serial search whatever the entries' order.
constexpr int SOJDS_LDS_CAP = 4096;
constexpr int32_t SOJDS_TAKEN = INT32_MAX;    // no column reaches it (columns < n_cols <= INT32_MAX)

template <typename T>
__global__ __launch_bounds__(WAVE) void sojds_wave_kernel(const int32_t *__restrict__ jp, int32_t ndiag,
                                                          const int32_t *__restrict__ jd_col,
                                                          const T *__restrict__ jd_val, int32_t n, int32_t C,
                                                          const int64_t *__restrict__ slice_ptr,
                                                          int32_t *__restrict__ bl_col, T *__restrict__ bl_val)
{
    __shared__ int32_t cur[SOJDS_LDS_CAP];        // the row's columns; SOJDS_TAKEN once placed
    __shared__ int32_t prv[SOJDS_LDS_CAP];        // the previous row's column in each slot
    __shared__ int32_t pick[SOJDS_LDS_CAP];       // entry placed in each slot
    const int l = (int)threadIdx.x;
    const int64_t s = blockIdx.x;
    const int64_t r0 = s * (int64_t)C;
    const int32_t len0 = jds_len_of(jp, ndiag, r0);
    if (len0 > SOJDS_LDS_CAP || len0 == 0) return;       // whole wavefront: serial kernel's slice, or nothing to do
    const int64_t sp = slice_ptr[s];
    for (int32_t d = l; d < len0; d += WAVE) prv[d] = bl_col[sp + (int64_t)d * C];   // first row, CRS order
    __syncthreads();
    for (int32_t rl = 1; rl < C; ++rl) {
        const int64_t r = r0 + rl;
        if (r >= n) break;
        const int32_t len = jds_len_of(jp, ndiag, r);     // <= the previous row's length
        if (len == 0) break;                              // rows of the slice are sorted by length
        for (int32_t e = l; e < len; e += WAVE) cur[e] = jd_col[jp[e] + r];
        __syncthreads();
        for (int32_t d = 0; d < len; ++d) {
            // key = distance << 32 | column: the smallest key is the nearest
            // entry, the smaller column on a tie
            const uint32_t want = (uint32_t)prv[d] + 1u;
            uint64_t best = UINT64_MAX;
            int32_t be = -1;
            for (int32_t e = l; e < len; e += WAVE) {
                const int32_t c = cur[e];
                if (c == SOJDS_TAKEN) continue;
                const uint32_t uc = (uint32_t)c;
                const uint64_t key = ((uint64_t)(uc > want ? uc - want : want - uc) << 32) | uc;
                if (key < best) {
                    best = key;
                    be = e;
                }
            }
#pragma unroll
            for (int off = WAVE / 2; off > 0; off >>= 1) {
                const uint64_t ok = __shfl_xor(best, off, WAVE);
                const int32_t oe = __shfl_xor(be, off, WAVE);
                if (ok < best) {
                    best = ok;
                    be = oe;
                }
            }
            if (l == 0) {
                cur[be] = SOJDS_TAKEN;
                pick[d] = be;
                prv[d] = (int32_t)(uint32_t)best;        // the next row's target in this slot
            }
            __syncthreads();
        }
        for (int32_t d = l; d < len; d += WAVE) {
            const int32_t e = pick[d];
            bl_col[sp + (int64_t)d * C + rl] = prv[d];
            bl_val[sp + (int64_t)d * C + rl] = jd_val[jp[e] + r];
        }
        __syncthreads();
    }
}

template <typename T>
__global__ void sojds_kernel(const int32_t *__restrict__ jp, int32_t ndiag, const int32_t *__restrict__ jd_col,
                             const T *__restrict__ jd_val, int32_t n, int32_t C, const int64_t *__restrict__ slice_ptr,
                             int32_t n_slices, int32_t words, uint32_t *__restrict__ taken_all,
                             int32_t *__restrict__ bl_col, T *__restrict__ bl_val, int32_t min_len)
{
    GRID_LOOP(s, (int64_t)n_slices)
    {
        if (jds_len_of(jp, ndiag, s * (int64_t)C) <= min_len) continue;   // sojds_wave_kernel's slice
        uint32_t *taken = taken_all + s * (int64_t)words;
        const int64_t sp = slice_ptr[s];
        for (int32_t rl = 1; rl < C; ++rl) {
            const int64_t r = s * (int64_t)C + rl;
            if (r >= n) break;
            const int32_t len = jds_len_of(jp, ndiag, r);
            for (int32_t q = 0; q < (len + 31) / 32; ++q) taken[q] = 0;
            auto col_of = [&](int32_t e) -> int64_t { return jd_col[jp[e] + r]; };
            bool sorted = true;
            for (int32_t e = 1; e < len && sorted; ++e) sorted = col_of(e) > col_of(e - 1);
            for (int32_t d = 0; d < len; ++d) {
                const int64_t want = (int64_t)bl_col[sp + (int64_t)d * C + rl - 1] + 1;
                int32_t pick = -1;
                if (sorted) {
                    int32_t lo = 0, hi = len;                  // first entry with column >= want
                    while (lo < hi) {
                        const int32_t mid = (lo + hi) >> 1;
                        if (col_of(mid) < want) lo = mid + 1;
                        else hi = mid;
                    }
                    const int32_t right = next_clear(taken, lo, len), left = prev_clear(taken, lo);
                    if (left < 0) pick = right;
                    else if (right < 0) pick = left;
                    else pick = (col_of(right) - want < want - col_of(left)) ? right : left;   // tie: smaller column
                } else {
                    int64_t best = 0, bestc = 0;
                    for (int32_t e = 0; e < len; ++e) {
                        if (taken[e >> 5] & (1u << (e & 31))) continue;
                        const int64_t c = col_of(e);
                        const int64_t dist = c > want ? c - want : want - c;
                        if (pick < 0 || dist < best || (dist == best && c < bestc)) {
                            pick = e;
                            best = dist;
                            bestc = c;
                        }
                    }
                }
                taken[pick >> 5] |= 1u << (pick & 31);
                bl_col[sp + (int64_t)d * C + rl] = jd_col[jp[pick] + r];
                bl_val[sp + (int64_t)d * C + rl] = jd_val[jp[pick] + r];
            }
        }
    }
}

// ---- DIA + CRS hybrid: diagonals (offset col - row) stored densely, the rest in CRS

__global__ void diag_hist_kernel(const int32_t *__restrict__ rp, int32_t n_rows, const int32_t *__restrict__ col,
                                 int32_t *__restrict__ hist)
{
    GRID_LOOP(i, (int64_t)n_rows)
    {
        for (int32_t e = rp[i]; e < rp[i + 1]; ++e) atomicAdd(hist + ((int64_t)col[e] - i + n_rows - 1), 1);
    }
}

struct DiaOffsets {
    int32_t n;
    int32_t off[SPMV_DIA_MAX];
};

__global__ void dia_index_kernel(int64_t m, int32_t *__restrict__ oidx)
{
    GRID_LOOP(t, m) oidx[t] = -1;
}

// stored diagonal k: oidx = k; with `sym`, its mirror -off (off > 0) gets
// SPMV_DIA_MAX + k: covered by the stored diagonal, kept out of the remainder
__global__ void dia_index_set_kernel(int32_t n_rows, DiaOffsets D, int sym, int32_t *__restrict__ oidx)
{
    const int k = (int)threadIdx.x;
    if (k >= D.n) return;
    oidx[(int64_t)D.off[k] + n_rows - 1] = k;
    if (sym && D.off[k] > 0) oidx[(int64_t)n_rows - 1 - D.off[k]] = SPMV_DIA_MAX + k;
}

template <typename T>
__global__ void dia_zero_kernel(int64_t m, T *__restrict__ out)
{
    GRID_LOOP(t, m) out[t] = T{};
}

// entries on a stored diagonal go to dia[k * n_rows + row]; the others are
// counted per row for the remainder CRS
template <typename T>
__global__ void dia_scatter_kernel(const int32_t *__restrict__ rp, int32_t n_rows, const int32_t *__restrict__ col,
                                   const T *__restrict__ val, const int32_t *__restrict__ oidx, T *__restrict__ dia,
                                   int32_t *__restrict__ rem_cnt)
{
    GRID_LOOP(i, (int64_t)n_rows)
    {
        int32_t cnt = 0;
        for (int32_t e = rp[i]; e < rp[i + 1]; ++e) {
            const int32_t k = oidx[(int64_t)col[e] - i + n_rows - 1];
            if (k < 0) ++cnt;
            else if (k < SPMV_DIA_MAX) dia[(int64_t)k * n_rows + i] = val[e];
        }
        rem_cnt[i] = cnt;
    }
}

// remainder entries of each row, in CRS order
template <typename T>
__global__ void dia_rem_kernel(const int32_t *__restrict__ rp, int32_t n_rows, const int32_t *__restrict__ col,
                               const T *__restrict__ val, const int32_t *__restrict__ oidx,
                               const int32_t *__restrict__ rem_rp, int32_t *__restrict__ rem_col,
                               T *__restrict__ rem_val)
{
    GRID_LOOP(i, (int64_t)n_rows)
    {
        int32_t p = rem_rp[i];
        for (int32_t e = rp[i]; e < rp[i + 1]; ++e) {
            if (oidx[(int64_t)col[e] - i + n_rows - 1] >= 0) continue;
            rem_col[p] = col[e];
            rem_val[p] = val[e];
            ++p;
        }
    }
}

// ---- row split: part k = rows [b_k, b_{k+1}), cut so each holds about nnz/8 entries

__global__ void row_bounds_kernel(const int32_t *__restrict__ rp, int32_t n_rows, int64_t nnz,
                                  int64_t *__restrict__ bounds, int64_t *__restrict__ entry_bounds)
{
    const int k = (int)threadIdx.x;
    if (k > SPLIT_PARTS) return;
    int64_t b;
    if (k == 0) b = 0;
    else if (k == SPLIT_PARTS) b = n_rows;
    else if (nnz == 0) b = (int64_t)k * n_rows / SPLIT_PARTS;
    else b = lower_bound_dev(rp, (int64_t)n_rows + 1, (k * nnz + SPLIT_PARTS - 1) / SPLIT_PARTS);
    if (b > n_rows) b = n_rows;     // only if row_ptr[n_rows] < nnz, which the host reports
    bounds[k] = b;
    entry_bounds[k] = rp[b];
}

// part k's rebased row pointer at row_ptr_parts[b_k + k .. b_{k+1} + k]
__global__ void row_split_ptr_kernel(const int32_t *__restrict__ rp, int32_t n_rows,
                                     const int64_t *__restrict__ bounds, int32_t *__restrict__ out)
{
    GRID_LOOP(j, (int64_t)n_rows + SPLIT_PARTS)
    {
        int k = 0;
        while (k < SPLIT_PARTS - 1 && j > bounds[k + 1] + k) ++k;
        const int64_t row = bounds[k] + (j - bounds[k] - k);
        out[j] = rp[row] - rp[bounds[k]];
    }
}

// ---- column split: part k = entries whose column lies in [k*width, (k+1)*width)

__global__ void row_of_entries_kernel(const int32_t *__restrict__ rp, int32_t n, int64_t nnz, int32_t *__restrict__ rowid)
{
    GRID_LOOP(j, nnz) rowid[j] = row_of(rp, n, j);
}

__global__ void part_key_kernel(const int32_t *__restrict__ col, int64_t nnz, int32_t width, uint32_t *__restrict__ key)
{
    GRID_LOOP(j, nnz) key[j] = (uint32_t)(col[j] / width);
}

template <typename T>
__global__ void gather_split_kernel(const int32_t *__restrict__ perm, int64_t nnz, const int32_t *__restrict__ col,
                                    const T *__restrict__ val, const int32_t *__restrict__ rowid,
                                    int32_t *__restrict__ col_out, T *__restrict__ val_out,
                                    int32_t *__restrict__ rowid_out)
{
    GRID_LOOP(i, nnz)
    {
        const int32_t j = perm[i];
        col_out[i] = col[j];
        val_out[i] = val[j];
        rowid_out[i] = rowid[j];
    }
}

__global__ void part_bounds_kernel(const uint32_t *__restrict__ skey, int64_t nnz, int64_t *__restrict__ bounds)
{
    GRID_LOOP(p, (int64_t)SPLIT_PARTS + 1) bounds[p] = lower_bound_dev(skey, nnz, (int64_t)p);
}

// Compressed rows: a part keeps only the rows holding at least one of its
// entries.  head[i] = 1 where entry i (part-major order) opens a (row, part)
// group; the exclusive scan of head numbers the compressed rows.
__global__ void split_head_kernel(const uint32_t *__restrict__ skey, const int32_t *__restrict__ rowid_s, int64_t nnz,
                                  int32_t *__restrict__ head)
{
    GRID_LOOP(i, nnz) head[i] = (i == 0 || skey[i] != skey[i - 1] || rowid_s[i] != rowid_s[i - 1]) ? 1 : 0;
}

// row pointer of each compressed row (relative to its part's first entry) and
// the parts present in each original row (bit k of mask[row])
__global__ void split_rows_kernel(const uint32_t *__restrict__ skey, const int32_t *__restrict__ rowid_s,
                                  const int32_t *__restrict__ head, const int32_t *__restrict__ qidx, int64_t nnz,
                                  const int64_t *__restrict__ bounds, int32_t *__restrict__ row_ptr_all,
                                  uint32_t *__restrict__ mask)
{
    GRID_LOOP(i, nnz)
    {
        if (!head[i]) continue;
        const uint32_t k = skey[i];
        row_ptr_all[qidx[i] + k] = (int32_t)(i - bounds[k]);
        atomicOr(mask + rowid_s[i], 1u << k);
    }
}

__global__ void split_terminators_kernel(const int64_t *__restrict__ bounds, const int32_t *__restrict__ qidx,
                                         int32_t *__restrict__ row_ptr_all, int64_t *__restrict__ row_off)
{
    const int k = (int)threadIdx.x;
    if (k <= SPLIT_PARTS) row_off[k] = qidx[bounds[k]];
    if (k < SPLIT_PARTS) row_ptr_all[qidx[bounds[k + 1]] + k] = (int32_t)(bounds[k + 1] - bounds[k]);
}

__global__ void popcount_kernel(const uint32_t *__restrict__ mask, int32_t n, int32_t *__restrict__ cnt)
{
    GRID_LOOP(i, (int64_t)n) cnt[i] = __popc(mask[i]);
}

// slot of compressed row (row, k): row's slots are ordered by part
__global__ void split_dest_kernel(const uint32_t *__restrict__ skey, const int32_t *__restrict__ rowid_s,
                                  const int32_t *__restrict__ head, const int32_t *__restrict__ qidx, int64_t nnz,
                                  const uint32_t *__restrict__ mask, const int32_t *__restrict__ slot_ptr,
                                  int32_t *__restrict__ dest_all)
{
    GRID_LOOP(i, nnz)
    {
        if (!head[i]) continue;
        const uint32_t k = skey[i];
        const int32_t r = rowid_s[i];
        dest_all[qidx[i]] = slot_ptr[r] + __popc(mask[r] & ((1u << k) - 1u));
    }
}

__global__ void transpose_cols_kernel(const int32_t *__restrict__ rp, int32_t n_rows, const int32_t *__restrict__ tmap,
                                      int64_t nnz, int32_t *__restrict__ colT)
{
    GRID_LOOP(t, nnz) colT[t] = row_of(rp, n_rows, tmap[t]);
}

// one round-to-nearest-even step from double to bfloat16
__device__ __forceinline__ uint16_t f64_to_bf16_rne(double d)
{
    const uint64_t b = (uint64_t)__double_as_longlong(d);
    const uint16_t sign = (uint16_t)((b >> 48) & 0x8000u);
    const uint64_t a = b & 0x7fffffffffffffffull;
    if (a > 0x7ff0000000000000ull) return (uint16_t)(sign | 0x7fc0u);        // NaN
    if (a == 0x7ff0000000000000ull) return (uint16_t)(sign | 0x7f80u);       // inf
    const int e = (int)(a >> 52) - 1023;
    if (e >= -126) {
        uint64_t q = a >> 45;                        // exponent + 7 mantissa bits
        const uint64_t rem = a & ((1ull << 45) - 1);
        const uint64_t half = 1ull << 44;
        if (rem > half || (rem == half && (q & 1))) ++q;
        int64_t bits = (int64_t)q - ((int64_t)(1023 - 127) << 7);
        if (bits >= 0x7f80) bits = 0x7f80;            // overflow to infinity
        return (uint16_t)(sign | (uint16_t)bits);
    }
    // below the smallest normal: multiples of 2^-133, ties to even
    const double m = rint(__longlong_as_double((long long)a) * 0x1p133);
    return (uint16_t)(sign | (uint16_t)m);
}

__device__ __forceinline__ uint16_t f32_to_bf16_rne(float f)
{
    const uint32_t u = __float_as_uint(f);
    if ((u & 0x7fffffffu) > 0x7f800000u) return (uint16_t)((u >> 16) | 0x40u);
    const uint32_t lsb = (u >> 16) & 1u;
    return (uint16_t)((u + 0x7fffu + lsb) >> 16);
}

__global__ void convert_kernel(int64_t n, const void *__restrict__ in, int in_dt, void *__restrict__ out, int out_dt)
{
    GRID_LOOP(i, n)
    {
        if (in_dt == SPMV_F64) {
            const double v = ((const double *)in)[i];
            if (out_dt == SPMV_F32) ((float *)out)[i] = (float)v;
            else if (out_dt == SPMV_BF16) ((uint16_t *)out)[i] = f64_to_bf16_rne(v);
            else ((double *)out)[i] = v;
        } else if (in_dt == SPMV_F32) {
            const float v = ((const float *)in)[i];
            if (out_dt == SPMV_F64) ((double *)out)[i] = (double)v;
            else if (out_dt == SPMV_BF16) ((uint16_t *)out)[i] = f32_to_bf16_rne(v);
            else ((float *)out)[i] = v;
        } else {
            const float v = __uint_as_float((uint32_t)((const uint16_t *)in)[i] << 16);
            if (out_dt == SPMV_F64) ((double *)out)[i] = (double)v;
            else if (out_dt == SPMV_F32) ((float *)out)[i] = v;
            else ((uint16_t *)out)[i] = ((const uint16_t *)in)[i];
        }
    }
}

template <typename T>
__global__ void permute_kernel(int32_t n, const int32_t *__restrict__ perm, const T *__restrict__ in,
                               T *__restrict__ out, int inverse)
{
    GRID_LOOP(r, (int64_t)n)
    {
        if (inverse) out[perm[r]] = in[r];
        else out[r] = in[perm[r]];
    }
}

template <typename T>
__global__ void gather_kernel(int64_t n, const int32_t *__restrict__ map, const T *__restrict__ in, T *__restrict__ out)
{
    GRID_LOOP(i, n) out[i] = in[map[i]];
}

// dtype-dispatched launch of a kernel templated on the element type
template <template <typename> class K>
struct DtDispatch;

// ============================================================ host helpers

static spmv_status read_flag(const int32_t *dev, int32_t *host, hipStream_t s)
{
    SPMV_HIP(hipMemcpyAsync(host, dev, sizeof(int32_t), hipMemcpyDeviceToHost, s));
    SPMV_HIP(hipStreamSynchronize(s));
    return SPMV_OK;
}

static size_t coo_ws_bytes(int32_t n_rows, int32_t n_cols, int64_t nnz)
{
    (void)n_rows;
    (void)n_cols;
    size_t n = (size_t)(nnz > 0 ? nnz : 1);
    size_t b = 0;
    b += align_up(sizeof(int32_t), 256);            // flag
    b += align_up(sizeof(uint32_t) * n, 256);        // keys
    b += align_up(sizeof(int32_t) * n, 256);         // idx
    b += align_up(sizeof(int32_t) * n, 256);         // head flags
    b += align_up(sizeof(int32_t) * (n + 1), 256);   // positions
    b += align_up(sizeof(int32_t) * n, 256);         // unique rows
    b += align_up(sizeof(int32_t) * scan_ws_elems((int64_t)n), 256);
    b += radix_ws_bytes((int64_t)n);
    return b + 1024;
}

}  // namespace spmv

using namespace spmv;

extern "C" {

size_t spmv_csr_from_coo_workspace_size(int32_t n_rows, int32_t n_cols, int64_t nnz)
{
    return coo_ws_bytes(n_rows, n_cols, nnz);
}

spmv_status spmv_csr_from_coo(int32_t n_rows, int32_t n_cols, int64_t nnz, const int32_t *row, const int32_t *col,
                              const void *val, spmv_dtype dt, int32_t *row_ptr, int32_t *col_idx, void *val_out,
                              int64_t *h_nnz_out, void *ws, size_t ws_bytes, void *stream)
{
    SPMV_REQUIRE(n_rows >= 0 && n_cols >= 0 && nnz >= 0, "spmv_csr_from_coo: negative size");
    if (nnz >= ((int64_t)1 << 31)) return fail(SPMV_ERR_UNSUPPORTED, "spmv_csr_from_coo: nnz >= 2^31");
    SPMV_REQUIRE(dt == SPMV_F64 || dt == SPMV_F32, "spmv_csr_from_coo: dtype must be F64 or F32");
    SPMV_REQUIRE(row_ptr && h_nnz_out, "spmv_csr_from_coo: null row_ptr or h_nnz_out");
    SPMV_REQUIRE(nnz == 0 || (row && col && val && col_idx && val_out), "spmv_csr_from_coo: null pointer");
    SPMV_REQUIRE(ws && ws_bytes >= coo_ws_bytes(n_rows, n_cols, nnz), "spmv_csr_from_coo: workspace too small");
    hipStream_t s = as_stream(stream);
    WsCarver wc(ws, ws_bytes);
    int32_t *flag_dev = wc.take<int32_t>(1);
    uint32_t *keys = wc.take<uint32_t>((size_t)(nnz > 0 ? nnz : 1));
    int32_t *idx = wc.take<int32_t>((size_t)(nnz > 0 ? nnz : 1));
    int32_t *head = wc.take<int32_t>((size_t)(nnz > 0 ? nnz : 1));
    int32_t *pos = wc.take<int32_t>((size_t)nnz + 1);
    int32_t *row_u = wc.take<int32_t>((size_t)(nnz > 0 ? nnz : 1));
    int32_t *sws = wc.take<int32_t>(scan_ws_elems(nnz > 0 ? nnz : 1));
    size_t rws_bytes = radix_ws_bytes(nnz);
    void *rws = wc.take<char>(rws_bytes);
    if (!wc.ok()) return fail(SPMV_ERR_INVALID_ARG, "spmv_csr_from_coo: workspace too small");

    if (nnz == 0) {
        SPMV_HIP(hipMemsetAsync(row_ptr, 0, sizeof(int32_t) * ((size_t)n_rows + 1), s));
        SPMV_HIP(hipStreamSynchronize(s));
        *h_nnz_out = 0;
        return SPMV_OK;
    }
    SPMV_HIP(hipMemsetAsync(flag_dev, 0, sizeof(int32_t), s));
    coo_check_kernel<<<grid_for(nnz), 256, 0, s>>>(row, col, nnz, n_rows, n_cols, flag_dev);
    SPMV_CHECK_LAUNCH("coo check");
    int32_t bad = 0;
    if (read_flag(flag_dev, &bad, s) != SPMV_OK) return SPMV_ERR_HIP;
    if (bad) return fail(SPMV_ERR_BAD_FORMAT, "spmv_csr_from_coo: row or column index out of range");

    // stable sort by column, then stably by row: order (row, col, input index)
    copy_u32_kernel<<<grid_for(nnz), 256, 0, s>>>(col, keys, nnz);
    iota_kernel<<<grid_for(nnz), 256, 0, s>>>(idx, nnz);
    SPMV_CHECK_LAUNCH("coo init");
    spmv_status st = radix_sort_pairs(keys, idx, nnz, bits_for(n_cols > 0 ? n_cols - 1 : 0), rws, rws_bytes, s);
    if (st != SPMV_OK) return st;
    gather_u32_kernel<<<grid_for(nnz), 256, 0, s>>>(row, idx, keys, nnz);
    SPMV_CHECK_LAUNCH("coo gather rows");
    st = radix_sort_pairs(keys, idx, nnz, bits_for(n_rows > 0 ? n_rows - 1 : 0), rws, rws_bytes, s);
    if (st != SPMV_OK) return st;

    head_flags_kernel<<<grid_for(nnz), 256, 0, s>>>(keys, idx, col, nnz, head);
    SPMV_CHECK_LAUNCH("coo heads");
    st = exclusive_scan<int32_t, int32_t>(head, nnz, pos, sws, s);
    if (st != SPMV_OK) return st;
    int32_t nout = 0;
    if (read_flag(pos + nnz, &nout, s) != SPMV_OK) return SPMV_ERR_HIP;
    if (dt == SPMV_F64)
        compact_kernel<double><<<grid_for(nnz), 256, 0, s>>>(keys, idx, col, (const double *)val, head, pos, nnz,
                                                             col_idx, (double *)val_out, row_u);
    else
        compact_kernel<float><<<grid_for(nnz), 256, 0, s>>>(keys, idx, col, (const float *)val, head, pos, nnz,
                                                            col_idx, (float *)val_out, row_u);
    SPMV_CHECK_LAUNCH("coo compact");
    ptr_from_sorted_kernel<int32_t><<<grid_for((int64_t)n_rows + 1), 256, 0, s>>>(row_u, nout, n_rows, row_ptr);
    SPMV_CHECK_LAUNCH("coo row_ptr");
    SPMV_HIP(hipStreamSynchronize(s));
    *h_nnz_out = nout;
    return SPMV_OK;
}

size_t spmv_csr_validate_workspace_size(void) { return 256; }

spmv_status spmv_csr_validate(int32_t n_rows, int32_t n_cols, int64_t nnz, const int32_t *row_ptr,
                              const int32_t *col_idx, int32_t *h_ok, void *ws, size_t ws_bytes, void *stream)
{
    SPMV_REQUIRE(n_rows >= 0 && n_cols >= 0 && nnz >= 0, "spmv_csr_validate: negative size");
    SPMV_REQUIRE(h_ok && row_ptr && ws && ws_bytes >= 4, "spmv_csr_validate: null pointer");
    SPMV_REQUIRE(nnz == 0 || col_idx, "spmv_csr_validate: null col_idx");
    hipStream_t s = as_stream(stream);
    int32_t *bad = (int32_t *)ws;
    SPMV_HIP(hipMemsetAsync(bad, 0, sizeof(int32_t), s));
    if (n_rows > 0) validate_rows_kernel<<<grid_for(n_rows), 256, 0, s>>>(row_ptr, n_rows, nnz, bad);
    if (nnz > 0) validate_cols_kernel<<<grid_for(nnz), 256, 0, s>>>(col_idx, nnz, n_cols, bad);
    SPMV_CHECK_LAUNCH("spmv_csr_validate");
    int32_t b = 0;
    if (read_flag(bad, &b, s) != SPMV_OK) return SPMV_ERR_HIP;
    if (n_rows == 0) {
        int32_t first = 0;
        if (read_flag(row_ptr, &first, s) != SPMV_OK) return SPMV_ERR_HIP;
        if (first != 0 || nnz != 0) b |= 2;
    }
    *h_ok = b == 0 ? 1 : 0;
    return SPMV_OK;
}

size_t spmv_jds_from_csr_workspace_size(int32_t n, int64_t nnz)
{
    size_t m = (size_t)(n > 0 ? n : 1);
    size_t b = 0;
    b += 256;                                       // max length
    b += align_up(sizeof(int32_t) * m, 256);        // lengths
    b += align_up(sizeof(uint32_t) * m, 256);       // keys
    b += align_up(sizeof(int32_t) * scan_ws_elems((int64_t)(m > (size_t)nnz ? m : (size_t)nnz)), 256);
    b += radix_ws_bytes((int64_t)m);
    return b + 1024;
}

spmv_status spmv_jds_from_csr(int32_t n, int64_t nnz, const int32_t *row_ptr, const int32_t *col_idx,
                              const void *val, spmv_dtype dt, unsigned flags, int32_t *perm, int32_t *iperm,
                              int32_t *jd_ptr, int32_t jd_ptr_cap, int32_t *jd_col, void *jd_val, int32_t *h_ndiag,
                              int32_t *h_jd_ptr, void *ws, size_t ws_bytes, void *stream)
{
    SPMV_REQUIRE(n >= 0 && nnz >= 0, "spmv_jds_from_csr: negative size");
    if (nnz >= ((int64_t)1 << 31)) return fail(SPMV_ERR_UNSUPPORTED, "spmv_jds_from_csr: nnz >= 2^31");
    SPMV_REQUIRE(valid_payload_dtype(dt), "spmv_jds_from_csr: bad dtype");
    SPMV_REQUIRE((flags & ~SPMV_SYMPERM) == 0, "spmv_jds_from_csr: unknown flag");
    SPMV_REQUIRE(h_ndiag && row_ptr && (jd_ptr || jd_ptr_cap == 0), "spmv_jds_from_csr: null pointer");
    SPMV_REQUIRE(n == 0 || (perm && iperm), "spmv_jds_from_csr: null perm");
    SPMV_REQUIRE(nnz == 0 || (col_idx && val && jd_col && jd_val), "spmv_jds_from_csr: null arrays");
    SPMV_REQUIRE(ws && ws_bytes >= spmv_jds_from_csr_workspace_size(n, nnz), "spmv_jds_from_csr: workspace too small");
    hipStream_t s = as_stream(stream);
    WsCarver wc(ws, ws_bytes);
    int32_t *maxlen = wc.take<int32_t>(1);
    int32_t *len = wc.take<int32_t>((size_t)(n > 0 ? n : 1));
    uint32_t *keys = wc.take<uint32_t>((size_t)(n > 0 ? n : 1));
    int32_t *sws = wc.take<int32_t>(scan_ws_elems((int64_t)n > nnz ? (int64_t)n : (nnz > 0 ? nnz : 1)));
    size_t rws_bytes = radix_ws_bytes(n);
    void *rws = wc.take<char>(rws_bytes);
    if (!wc.ok()) return fail(SPMV_ERR_INVALID_ARG, "spmv_jds_from_csr: workspace too small");

    int32_t ndiag = 0;
    if (n > 0) {
        SPMV_HIP(hipMemsetAsync(maxlen, 0, sizeof(int32_t), s));
        row_len_kernel<<<grid_for(n), 256, 0, s>>>(row_ptr, n, len, maxlen);
        SPMV_CHECK_LAUNCH("jds lengths");
        if (read_flag(maxlen, &ndiag, s) != SPMV_OK) return SPMV_ERR_HIP;
    }
    *h_ndiag = ndiag;
    if (jd_ptr_cap < ndiag + 1) return fail(SPMV_ERR_CAPACITY, "spmv_jds_from_csr: jd_ptr capacity < ndiag+1");
    if (n == 0) {
        SPMV_HIP(hipMemsetAsync(jd_ptr, 0, sizeof(int32_t), s));
        SPMV_HIP(hipStreamSynchronize(s));
        if (h_jd_ptr) h_jd_ptr[0] = 0;
        return SPMV_OK;
    }
    // stable sort of the rows by decreasing length: key = ndiag - length
    desc_key_kernel<<<grid_for(n), 256, 0, s>>>(len, n, ndiag, keys);
    iota_kernel<<<grid_for(n), 256, 0, s>>>(perm, n);
    SPMV_CHECK_LAUNCH("jds keys");
    spmv_status st = radix_sort_pairs(keys, perm, n, bits_for(ndiag), rws, rws_bytes, s);
    if (st != SPMV_OK) return st;
    inverse_perm_kernel<<<grid_for(n), 256, 0, s>>>(perm, n, iperm);
    SPMV_CHECK_LAUNCH("jds iperm");
    if (ndiag > 0) {
        // diagonal lengths go into jd_ptr itself, then an in-place scan
        diag_count_kernel<<<grid_for(ndiag), 256, 0, s>>>(keys, n, ndiag, jd_ptr);
        SPMV_CHECK_LAUNCH("jds diagonal counts");
        st = exclusive_scan<int32_t, int32_t>(jd_ptr, ndiag, jd_ptr, sws, s);
        if (st != SPMV_OK) return st;
    } else {
        SPMV_HIP(hipMemsetAsync(jd_ptr, 0, sizeof(int32_t), s));
    }
    const int sym = (flags & SPMV_SYMPERM) ? 1 : 0;
    if (nnz > 0) {
        if (dt == SPMV_F64)
            jds_scatter_kernel<uint64_t><<<grid_for(nnz), 256, 0, s>>>(row_ptr, col_idx, (const uint64_t *)val, n, nnz,
                                                                     iperm, jd_ptr, sym, jd_col, (uint64_t *)jd_val);
        else if (dt == SPMV_F32 || dt == SPMV_I32)
            jds_scatter_kernel<uint32_t><<<grid_for(nnz), 256, 0, s>>>(row_ptr, col_idx, (const uint32_t *)val, n, nnz,
                                                                    iperm, jd_ptr, sym, jd_col, (uint32_t *)jd_val);
        else
            jds_scatter_kernel<uint16_t><<<grid_for(nnz), 256, 0, s>>>(row_ptr, col_idx, (const uint16_t *)val, n,
                                                                       nnz, iperm, jd_ptr, sym, jd_col,
                                                                       (uint16_t *)jd_val);
        SPMV_CHECK_LAUNCH("jds scatter");
    }
    if (h_jd_ptr)
        SPMV_HIP(hipMemcpyAsync(h_jd_ptr, jd_ptr, sizeof(int32_t) * ((size_t)ndiag + 1), hipMemcpyDeviceToHost, s));
    SPMV_HIP(hipStreamSynchronize(s));
    return SPMV_OK;
}

size_t spmv_jds_to_csr_workspace_size(int32_t n)
{
    size_t m = (size_t)(n > 0 ? n : 1);
    return align_up(sizeof(int32_t) * m, 256) + align_up(sizeof(int32_t) * scan_ws_elems((int64_t)m), 256) + 512;
}

spmv_status spmv_jds_to_csr(int32_t n, const int32_t *perm, const int32_t *jd_ptr, int32_t ndiag, const int32_t *jd_col,
                            const void *jd_val, spmv_dtype dt, unsigned flags, int32_t *row_ptr, int32_t *col_idx,
                            void *val, void *ws, size_t ws_bytes, void *stream)
{
    SPMV_REQUIRE(n >= 0 && ndiag >= 0, "spmv_jds_to_csr: negative size");
    SPMV_REQUIRE(valid_payload_dtype(dt), "spmv_jds_to_csr: bad dtype");
    SPMV_REQUIRE((flags & ~SPMV_SYMPERM) == 0, "spmv_jds_to_csr: unknown flag");
    SPMV_REQUIRE(row_ptr && jd_ptr, "spmv_jds_to_csr: null pointer");
    SPMV_REQUIRE(ws && ws_bytes >= spmv_jds_to_csr_workspace_size(n), "spmv_jds_to_csr: workspace too small");
    hipStream_t s = as_stream(stream);
    WsCarver wc(ws, ws_bytes);
    int32_t *len = wc.take<int32_t>((size_t)(n > 0 ? n : 1));
    int32_t *sws = wc.take<int32_t>(scan_ws_elems(n > 0 ? n : 1));
    if (n == 0) {
        SPMV_HIP(hipMemsetAsync(row_ptr, 0, sizeof(int32_t), s));
        return SPMV_OK;
    }
    SPMV_REQUIRE(perm, "spmv_jds_to_csr: null perm");
    jds_row_len_kernel<<<grid_for(n), 256, 0, s>>>(jd_ptr, ndiag, perm, n, len);
    SPMV_CHECK_LAUNCH("jds_to_csr lengths");
    spmv_status st = exclusive_scan<int32_t, int32_t>(len, n, row_ptr, sws, s);
    if (st != SPMV_OK) return st;
    int32_t nnz = 0;
    SPMV_HIP(hipMemcpyAsync(&nnz, row_ptr + n, sizeof(int32_t), hipMemcpyDeviceToHost, s));
    SPMV_HIP(hipStreamSynchronize(s));
    if (nnz == 0) return SPMV_OK;
    SPMV_REQUIRE(jd_col && jd_val && col_idx && val, "spmv_jds_to_csr: null arrays");
    const int sym = (flags & SPMV_SYMPERM) ? 1 : 0;
    if (dt == SPMV_F64)
        jds_to_csr_kernel<uint64_t><<<grid_for(nnz), 256, 0, s>>>(jd_ptr, ndiag, nnz, perm, jd_col,
                                                                (const uint64_t *)jd_val, sym, row_ptr, col_idx,
                                                                (uint64_t *)val);
    else if (dt == SPMV_F32 || dt == SPMV_I32)
        jds_to_csr_kernel<uint32_t><<<grid_for(nnz), 256, 0, s>>>(jd_ptr, ndiag, nnz, perm, jd_col, (const uint32_t *)jd_val,
                                                               sym, row_ptr, col_idx, (uint32_t *)val);
    else
        jds_to_csr_kernel<uint16_t><<<grid_for(nnz), 256, 0, s>>>(jd_ptr, ndiag, nnz, perm, jd_col,
                                                                  (const uint16_t *)jd_val, sym, row_ptr, col_idx,
                                                                  (uint16_t *)val);
    SPMV_CHECK_LAUNCH("jds_to_csr scatter");
    return SPMV_OK;
}

size_t spmv_jds_blocked_windowed_workspace_size(int32_t n)
{
    size_t m = (size_t)(n > 0 ? n : 1);
    size_t b = 256;                                              // longest row
    b += align_up(sizeof(int32_t) * m, 256);                     // lengths
    b += align_up(sizeof(uint32_t) * m, 256);                    // sort keys
    b += radix_ws_bytes((int64_t)m);
    b += align_up(sizeof(int64_t) * m, 256);                     // slice sizes (at most n slices)
    b += align_up(sizeof(int64_t) * scan_ws_elems((int64_t)m), 256);
    return b + 1024;
}

size_t spmv_jds_blocked_workspace_size(int32_t n, int32_t ndiag, int32_t C, unsigned flags)
{
    if (C <= 0) return 0;
    size_t ns = (size_t)ceil_div(n > 0 ? n : 1, C);
    size_t b = align_up(sizeof(int64_t) * ns, 256) + align_up(sizeof(int64_t) * scan_ws_elems((int64_t)ns), 256);
    if (flags & SPMV_SOJDS) b += align_up(sizeof(uint32_t) * ns * (size_t)ceil_div(ndiag > 0 ? ndiag : 1, 32), 256);
    return b + 1024;
}

spmv_status spmv_jds_blocked_from_jds(int32_t n, const int32_t *jd_ptr, int32_t ndiag, const int32_t *jd_col,
                                      const void *jd_val, spmv_dtype dt, int32_t C, unsigned flags, int64_t *slice_ptr,
                                      int32_t *slice_nd, int32_t *bl_col, void *bl_val, int64_t bl_cap,
                                      int64_t *h_padded, int32_t *h_slice_nd, void *ws, size_t ws_bytes, void *stream)
{
    SPMV_REQUIRE(n >= 0 && ndiag >= 0, "spmv_jds_blocked_from_jds: negative size");
    SPMV_REQUIRE(C > 0 && C % 64 == 0, "spmv_jds_blocked_from_jds: C must be a positive multiple of 64");
    SPMV_REQUIRE(valid_payload_dtype(dt), "spmv_jds_blocked_from_jds: bad dtype");
    SPMV_REQUIRE((flags & ~SPMV_SOJDS) == 0, "spmv_jds_blocked_from_jds: unknown flag");
    SPMV_REQUIRE(jd_ptr && slice_ptr && h_padded, "spmv_jds_blocked_from_jds: null pointer");
    SPMV_REQUIRE(ws && ws_bytes >= spmv_jds_blocked_workspace_size(n, ndiag, C, flags),
                 "spmv_jds_blocked_from_jds: workspace too small");
    hipStream_t s = as_stream(stream);
    const int32_t ns = (int32_t)ceil_div(n, C);
    WsCarver wc(ws, ws_bytes);
    int64_t *sz = wc.take<int64_t>((size_t)(ns > 0 ? ns : 1));
    int64_t *sws = wc.take<int64_t>(scan_ws_elems(ns > 0 ? ns : 1));
    uint32_t *taken = (flags & SPMV_SOJDS) ? wc.take<uint32_t>((size_t)(ns > 0 ? ns : 1) *
                                                               (size_t)ceil_div(ndiag > 0 ? ndiag : 1, 32))
                                           : nullptr;
    if (ns == 0) {
        SPMV_HIP(hipMemsetAsync(slice_ptr, 0, sizeof(int64_t), s));
        SPMV_HIP(hipStreamSynchronize(s));
        *h_padded = 0;
        return SPMV_OK;
    }
    SPMV_REQUIRE(slice_nd, "spmv_jds_blocked_from_jds: null slice_nd");
    slice_nd_kernel<<<grid_for(ns), 256, 0, s>>>(jd_ptr, ndiag, C, ns, slice_nd, sz);
    SPMV_CHECK_LAUNCH("blocked slice sizes");
    spmv_status st = exclusive_scan<int64_t, int64_t>(sz, ns, slice_ptr, sws, s);
    if (st != SPMV_OK) return st;
    int64_t total = 0;
    SPMV_HIP(hipMemcpyAsync(&total, slice_ptr + ns, sizeof(int64_t), hipMemcpyDeviceToHost, s));
    if (h_slice_nd) SPMV_HIP(hipMemcpyAsync(h_slice_nd, slice_nd, sizeof(int32_t) * ns, hipMemcpyDeviceToHost, s));
    SPMV_HIP(hipStreamSynchronize(s));
    *h_padded = total;
    if (bl_cap < total) return fail(SPMV_ERR_CAPACITY, "spmv_jds_blocked_from_jds: capacity < padded size");
    if (total == 0) return SPMV_OK;
    SPMV_REQUIRE(jd_col && jd_val && bl_col && bl_val, "spmv_jds_blocked_from_jds: null arrays");
    const int32_t words = (int32_t)ceil_div(ndiag > 0 ? ndiag : 1, 32);
#define BLK_CASE(DT, T)                                                                                             \
    if (dt == DT) {                                                                                                 \
        blocked_fill_kernel<T><<<grid_for(total), 256, 0, s>>>(jd_ptr, ndiag, jd_col, (const T *)jd_val, n, C,      \
                                                               slice_ptr, ns, total, bl_col, (T *)bl_val);          \
        SPMV_CHECK_LAUNCH("blocked fill");                                                                          \
        if (flags & SPMV_SOJDS) {                                                                                   \
            sojds_wave_kernel<T><<<(unsigned)ns, WAVE, 0, s>>>(jd_ptr, ndiag, jd_col, (const T *)jd_val, n, C,       \
                                                               slice_ptr, bl_col, (T *)bl_val);                     \
            SPMV_CHECK_LAUNCH("sojds (wavefront per slice)");                                                       \
            if (ndiag > SOJDS_LDS_CAP) {                                                                            \
                sojds_kernel<T><<<grid_for(ns), 64, 0, s>>>(jd_ptr, ndiag, jd_col, (const T *)jd_val, n, C,         \
                                                            slice_ptr, ns, words, taken, bl_col, (T *)bl_val,       \
                                                            SOJDS_LDS_CAP);                                         \
                SPMV_CHECK_LAUNCH("sojds (long rows)");                                                             \
            }                                                                                                       \
        }                                                                                                           \
    }
    BLK_CASE(SPMV_F64, uint64_t)
    BLK_CASE(SPMV_F32, uint32_t)
    BLK_CASE(SPMV_I32, uint32_t)
    BLK_CASE(SPMV_BF16, uint16_t)
#undef BLK_CASE
    SPMV_HIP(hipStreamSynchronize(s));
    return SPMV_OK;
}

spmv_status spmv_jds_blocked_windowed_from_csr(int32_t n, int64_t nnz, const int32_t *row_ptr, const int32_t *col_idx,
                                               const void *val, spmv_dtype dt, int32_t C, int32_t sigma,
                                               int32_t *perm, int64_t *slice_ptr, int32_t *slice_nd,
                                               int32_t *bl_col, void *bl_val, int64_t bl_cap, int64_t *h_padded,
                                               int32_t *h_slice_nd, void *ws, size_t ws_bytes, void *stream)
{
    SPMV_REQUIRE(n >= 0 && nnz >= 0, "spmv_jds_blocked_windowed_from_csr: negative size");
    if (nnz >= ((int64_t)1 << 31)) return fail(SPMV_ERR_UNSUPPORTED, "spmv_jds_blocked_windowed_from_csr: nnz >= 2^31");
    SPMV_REQUIRE(C > 0 && C % 64 == 0, "spmv_jds_blocked_windowed_from_csr: C must be a positive multiple of 64");
    SPMV_REQUIRE(sigma > 0 && sigma % C == 0, "spmv_jds_blocked_windowed_from_csr: sigma must be a positive multiple of C");
    SPMV_REQUIRE(valid_payload_dtype(dt), "spmv_jds_blocked_windowed_from_csr: bad dtype");
    SPMV_REQUIRE(row_ptr && slice_ptr && h_padded, "spmv_jds_blocked_windowed_from_csr: null pointer");
    SPMV_REQUIRE(ws && ws_bytes >= spmv_jds_blocked_windowed_workspace_size(n),
                 "spmv_jds_blocked_windowed_from_csr: workspace too small");
    hipStream_t s = as_stream(stream);
    const int32_t ns = (int32_t)ceil_div(n, C);
    if (ns == 0) {
        SPMV_HIP(hipMemsetAsync(slice_ptr, 0, sizeof(int64_t), s));
        SPMV_HIP(hipStreamSynchronize(s));
        *h_padded = 0;
        return SPMV_OK;
    }
    SPMV_REQUIRE(perm && slice_nd, "spmv_jds_blocked_windowed_from_csr: null perm or slice_nd");
    const size_t m = (size_t)n;
    WsCarver wc(ws, ws_bytes);
    int32_t *maxlen = wc.take<int32_t>(1);
    int32_t *len = wc.take<int32_t>(m);
    uint32_t *keys = wc.take<uint32_t>(m);
    const size_t rws_bytes = radix_ws_bytes((int64_t)m);
    void *rws = wc.take<char>(rws_bytes);
    int64_t *sz = wc.take<int64_t>(m);
    int64_t *sws = wc.take<int64_t>(scan_ws_elems((int64_t)m));
    if (!wc.ok()) return fail(SPMV_ERR_INVALID_ARG, "spmv_jds_blocked_windowed_from_csr: workspace too small");
    int32_t ndiag = 0;
    SPMV_HIP(hipMemsetAsync(maxlen, 0, sizeof(int32_t), s));
    row_len_kernel<<<grid_for(n), 256, 0, s>>>(row_ptr, n, len, maxlen);
    SPMV_CHECK_LAUNCH("windowed lengths");
    if (read_flag(maxlen, &ndiag, s) != SPMV_OK) return SPMV_ERR_HIP;
    // rows by decreasing length (stable), then by window (stable): window-major,
    // longest first inside a window, ties in original order
    desc_key_kernel<<<grid_for(n), 256, 0, s>>>(len, n, ndiag, keys);
    iota_kernel<<<grid_for(n), 256, 0, s>>>(perm, n);
    SPMV_CHECK_LAUNCH("windowed keys");
    spmv_status st = radix_sort_pairs(keys, perm, n, bits_for(ndiag), rws, rws_bytes, s);
    if (st != SPMV_OK) return st;
    window_key_kernel<<<grid_for(n), 256, 0, s>>>(perm, n, sigma, keys);
    SPMV_CHECK_LAUNCH("windowed window keys");
    st = radix_sort_pairs(keys, perm, n, bits_for((int64_t)(n - 1) / sigma), rws, rws_bytes, s);
    if (st != SPMV_OK) return st;
    window_slice_nd_kernel<<<grid_for(ns), 256, 0, s>>>(row_ptr, perm, C, ns, slice_nd, sz);
    SPMV_CHECK_LAUNCH("windowed slice sizes");
    st = exclusive_scan<int64_t, int64_t>(sz, ns, slice_ptr, sws, s);
    if (st != SPMV_OK) return st;
    int64_t total = 0;
    SPMV_HIP(hipMemcpyAsync(&total, slice_ptr + ns, sizeof(int64_t), hipMemcpyDeviceToHost, s));
    if (h_slice_nd) SPMV_HIP(hipMemcpyAsync(h_slice_nd, slice_nd, sizeof(int32_t) * ns, hipMemcpyDeviceToHost, s));
    SPMV_HIP(hipStreamSynchronize(s));
    *h_padded = total;
    if (bl_cap < total) return fail(SPMV_ERR_CAPACITY, "spmv_jds_blocked_windowed_from_csr: capacity < padded size");
    if (total == 0) return SPMV_OK;
    SPMV_REQUIRE(col_idx && val && bl_col && bl_val, "spmv_jds_blocked_windowed_from_csr: null arrays");
#define WFILL_CASE(T)                                                                                              \
    window_fill_kernel<T><<<grid_for(total), 256, 0, s>>>(row_ptr, col_idx, (const T *)val, perm, n, C, slice_ptr, \
                                                          ns, total, bl_col, (T *)bl_val)
    if (dt == SPMV_F64) WFILL_CASE(uint64_t);
    else if (dt == SPMV_F32 || dt == SPMV_I32) WFILL_CASE(uint32_t);
    else WFILL_CASE(uint16_t);
#undef WFILL_CASE
    SPMV_CHECK_LAUNCH("windowed fill");
    SPMV_HIP(hipStreamSynchronize(s));
    return SPMV_OK;
}

size_t spmv_csr_slices_workspace_size(int32_t n_rows)
{
    const int64_t n = n_rows > 0 ? n_rows : 1;
    const int64_t ns = ceil_div(n, SPMV_REM_SLICE);
    return align_up(sizeof(int32_t) * (size_t)n, 256) + align_up(sizeof(int64_t) * (size_t)ns, 256) +
           align_up(sizeof(int64_t) * scan_ws_elems(ns), 256) + 512;
}

spmv_status spmv_csr_to_slices(int32_t n_rows, const int32_t *row_ptr, const int32_t *col_idx, const void *val,
                               spmv_dtype dt, int64_t *slice_ptr, int32_t *slice_nd, uint8_t *slot_row,
                               int32_t *bl_col, void *bl_val, int64_t bl_cap, int64_t *h_padded, void *ws,
                               size_t ws_bytes, void *stream)
{
    SPMV_REQUIRE(n_rows >= 0, "spmv_csr_to_slices: n_rows < 0");
    SPMV_REQUIRE(valid_payload_dtype(dt), "spmv_csr_to_slices: bad dtype");
    SPMV_REQUIRE(slice_ptr && h_padded, "spmv_csr_to_slices: null pointer");
    SPMV_REQUIRE(ws && ws_bytes >= spmv_csr_slices_workspace_size(n_rows), "spmv_csr_to_slices: workspace too small");
    hipStream_t s = as_stream(stream);
    const int32_t ns = (int32_t)ceil_div(n_rows, SPMV_REM_SLICE);
    if (ns == 0) {
        SPMV_HIP(hipMemsetAsync(slice_ptr, 0, sizeof(int64_t), s));
        SPMV_HIP(hipStreamSynchronize(s));
        *h_padded = 0;
        return SPMV_OK;
    }
    SPMV_REQUIRE(row_ptr && slice_nd && slot_row, "spmv_csr_to_slices: null row_ptr, slice_nd or slot_row");
    WsCarver wc(ws, ws_bytes);
    int32_t *perm = wc.take<int32_t>((size_t)n_rows);
    int64_t *sz = wc.take<int64_t>((size_t)ns);
    int64_t *sws = wc.take<int64_t>(scan_ws_elems(ns));
    if (!wc.ok()) return fail(SPMV_ERR_INVALID_ARG, "spmv_csr_to_slices: workspace too small");
    rem_order_kernel<<<(unsigned)ceil_div(n_rows, SPMV_REM_WINDOW), SPMV_REM_WINDOW, 0, s>>>(row_ptr, n_rows,
                                                                                          slot_row, perm, slice_nd, sz);
    SPMV_CHECK_LAUNCH("slice order");
    spmv_status st = exclusive_scan<int64_t, int64_t>(sz, ns, slice_ptr, sws, s);
    if (st != SPMV_OK) return st;
    int64_t total = 0;
    SPMV_HIP(hipMemcpyAsync(&total, slice_ptr + ns, sizeof(int64_t), hipMemcpyDeviceToHost, s));
    SPMV_HIP(hipStreamSynchronize(s));
    *h_padded = total;
    if (!bl_col) return SPMV_OK;                                   // sizes only
    if (bl_cap < total) return fail(SPMV_ERR_CAPACITY, "spmv_csr_to_slices: capacity < padded size");
    if (total == 0) return SPMV_OK;
    SPMV_REQUIRE(col_idx && val && bl_val, "spmv_csr_to_slices: null arrays");
#define SFILL_CASE(T)                                                                                                \
    window_fill_kernel<T><<<grid_for(total), 256, 0, s>>>(row_ptr, col_idx, (const T *)val, perm, n_rows,            \
                                                          SPMV_REM_SLICE, slice_ptr, ns, total, bl_col, (T *)bl_val)
    if (dt == SPMV_F64) SFILL_CASE(uint64_t);
    else if (dt == SPMV_F32 || dt == SPMV_I32) SFILL_CASE(uint32_t);
    else SFILL_CASE(uint16_t);
#undef SFILL_CASE
    SPMV_CHECK_LAUNCH("slice fill");
    SPMV_HIP(hipStreamSynchronize(s));
    return SPMV_OK;
}

size_t spmv_split_columns_workspace_size(int32_t n_rows, int64_t nnz)
{
    const size_t m = (size_t)(nnz > 0 ? nnz : 1);
    const size_t n = (size_t)(n_rows > 0 ? n_rows : 1);
    const size_t sc = scan_ws_elems((int64_t)std::max(m + 1, n + 1));
    return 5 * align_up(sizeof(int32_t) * m, 256) + align_up(sizeof(int32_t) * (m + 1), 256) +
           2 * align_up(sizeof(int32_t) * n, 256) + 2 * align_up(sizeof(int64_t) * (SPLIT_PARTS + 1), 256) +
           align_up(sizeof(int32_t) * sc, 256) + radix_ws_bytes((int64_t)m) + 2048;
}

spmv_status spmv_split_columns(int32_t n_rows, int32_t n_cols, int64_t nnz, const int32_t *row_ptr,
                               const int32_t *col_idx, const void *val, spmv_dtype dt, int32_t width,
                               int32_t *row_ptr_all, int32_t *dest_all, int32_t *slot_ptr, int32_t *col_out,
                               void *val_out, int64_t *h_bounds, int64_t *h_row_off, void *ws, size_t ws_bytes,
                               void *stream)
{
    SPMV_REQUIRE(n_rows >= 0 && n_cols >= 0 && nnz >= 0, "spmv_split_columns: negative size");
    if (nnz >= ((int64_t)1 << 31)) return fail(SPMV_ERR_UNSUPPORTED, "spmv_split_columns: nnz >= 2^31");
    SPMV_REQUIRE(valid_dtype(dt), "spmv_split_columns: bad dtype");
    if (width == 0) width = (int32_t)(ceil_div(ceil_div(n_cols > 0 ? n_cols : 1, SPLIT_PARTS), 64) * 64);
    SPMV_REQUIRE(width > 0 && (int64_t)width * SPLIT_PARTS >= n_cols,
                 "spmv_split_columns: width * SPMV_SPLIT_PARTS must cover the columns");
    SPMV_REQUIRE(row_ptr && row_ptr_all && slot_ptr && h_bounds && h_row_off, "spmv_split_columns: null pointer");
    SPMV_REQUIRE(nnz == 0 || (col_idx && val && col_out && val_out && dest_all), "spmv_split_columns: null arrays");
    SPMV_REQUIRE(ws && ws_bytes >= spmv_split_columns_workspace_size(n_rows, nnz),
                 "spmv_split_columns: workspace too small");
    hipStream_t s = as_stream(stream);
    WsCarver wc(ws, ws_bytes);
    const size_t m = (size_t)(nnz > 0 ? nnz : 1);
    const size_t nn = (size_t)(n_rows > 0 ? n_rows : 1);
    int32_t *rowid = wc.take<int32_t>(m);
    int32_t *rowid_s = wc.take<int32_t>(m);
    uint32_t *keys = wc.take<uint32_t>(m);
    int32_t *perm = wc.take<int32_t>(m);
    int32_t *head = wc.take<int32_t>(m);
    int32_t *qidx = wc.take<int32_t>(m + 1);
    uint32_t *mask = wc.take<uint32_t>(nn);
    int32_t *cnt = wc.take<int32_t>(nn);
    int64_t *bounds = wc.take<int64_t>(SPLIT_PARTS + 1);
    int64_t *row_off = wc.take<int64_t>(SPLIT_PARTS + 1);
    int32_t *scan_ws = wc.take<int32_t>(scan_ws_elems((int64_t)std::max(m + 1, nn + 1)));
    const size_t rws_bytes = radix_ws_bytes((int64_t)m);
    void *rws = wc.take<char>(rws_bytes);
    if (!wc.ok()) return fail(SPMV_ERR_INVALID_ARG, "spmv_split_columns: workspace too small");
    if (n_rows > 0) SPMV_HIP(hipMemsetAsync(mask, 0, sizeof(uint32_t) * n_rows, s));
    if (nnz > 0) {
        row_of_entries_kernel<<<grid_for(nnz), 256, 0, s>>>(row_ptr, n_rows, nnz, rowid);
        part_key_kernel<<<grid_for(nnz), 256, 0, s>>>(col_idx, nnz, width, keys);
        iota_kernel<<<grid_for(nnz), 256, 0, s>>>(perm, nnz);
        SPMV_CHECK_LAUNCH("split keys");
        // stable: each part keeps the row-major order of its entries
        spmv_status st = radix_sort_pairs(keys, perm, nnz, bits_for(SPLIT_PARTS - 1), rws, rws_bytes, s);
        if (st != SPMV_OK) return st;
        if (dt == SPMV_F64)
            gather_split_kernel<uint64_t><<<grid_for(nnz), 256, 0, s>>>(perm, nnz, col_idx, (const uint64_t *)val, rowid,
                                                                         col_out, (uint64_t *)val_out, rowid_s);
        else if (dt == SPMV_F32)
            gather_split_kernel<uint32_t><<<grid_for(nnz), 256, 0, s>>>(perm, nnz, col_idx, (const uint32_t *)val, rowid,
                                                                         col_out, (uint32_t *)val_out, rowid_s);
        else
            gather_split_kernel<uint16_t><<<grid_for(nnz), 256, 0, s>>>(perm, nnz, col_idx, (const uint16_t *)val, rowid,
                                                                         col_out, (uint16_t *)val_out, rowid_s);
        SPMV_CHECK_LAUNCH("split gather");
        split_head_kernel<<<grid_for(nnz), 256, 0, s>>>(keys, rowid_s, nnz, head);
        SPMV_CHECK_LAUNCH("split heads");
    }
    spmv_status st = exclusive_scan<int32_t, int32_t>(head, nnz, qidx, scan_ws, s);
    if (st != SPMV_OK) return st;
    part_bounds_kernel<<<1, 64, 0, s>>>(keys, nnz, bounds);
    SPMV_CHECK_LAUNCH("split bounds");
    if (nnz > 0) {
        split_rows_kernel<<<grid_for(nnz), 256, 0, s>>>(keys, rowid_s, head, qidx, nnz, bounds, row_ptr_all, mask);
        SPMV_CHECK_LAUNCH("split rows");
    }
    split_terminators_kernel<<<1, 64, 0, s>>>(bounds, qidx, row_ptr_all, row_off);
    popcount_kernel<<<grid_for(n_rows), 256, 0, s>>>(mask, n_rows, cnt);
    SPMV_CHECK_LAUNCH("split slots");
    st = exclusive_scan<int32_t, int32_t>(cnt, n_rows, slot_ptr, scan_ws, s);
    if (st != SPMV_OK) return st;
    if (nnz > 0) {
        split_dest_kernel<<<grid_for(nnz), 256, 0, s>>>(keys, rowid_s, head, qidx, nnz, mask, slot_ptr, dest_all);
        SPMV_CHECK_LAUNCH("split dest");
    }
    SPMV_HIP(hipMemcpyAsync(h_bounds, bounds, sizeof(int64_t) * (SPLIT_PARTS + 1), hipMemcpyDeviceToHost, s));
    SPMV_HIP(hipMemcpyAsync(h_row_off, row_off, sizeof(int64_t) * (SPLIT_PARTS + 1), hipMemcpyDeviceToHost, s));
    SPMV_HIP(hipStreamSynchronize(s));
    return SPMV_OK;
}

size_t spmv_dia_workspace_size(int32_t n_rows, int32_t n_cols)
{
    const int64_t m = (int64_t)(n_rows > 0 ? n_rows : 1) + (n_cols > 0 ? n_cols : 1) - 1;
    const size_t nn = (size_t)(n_rows > 0 ? n_rows : 1);
    return align_up(sizeof(int32_t) * (size_t)m, 256) + align_up(sizeof(int32_t) * nn, 256) +
           align_up(sizeof(int32_t) * scan_ws_elems((int64_t)nn), 256) + 1024;
}

}  // extern "C"

namespace spmv {
// ---- upper triangle of a symmetric matrix: entries with col >= row

__global__ void upper_count_kernel(const int32_t *__restrict__ rp, int32_t n, const int32_t *__restrict__ col,
                                   int32_t *__restrict__ cnt)
{
    GRID_LOOP(i, (int64_t)n)
    {
        int32_t c = 0;
        for (int32_t e = rp[i]; e < rp[i + 1]; ++e) c += col[e] >= i;
        cnt[i] = c;
    }
}

template <typename T>
__global__ void upper_fill_kernel(const int32_t *__restrict__ rp, int32_t n, const int32_t *__restrict__ col,
                                  const T *__restrict__ val, const int32_t *__restrict__ up_rp,
                                  int32_t *__restrict__ up_col, T *__restrict__ up_val)
{
    GRID_LOOP(i, (int64_t)n)
    {
        int32_t p = up_rp[i];
        for (int32_t e = rp[i]; e < rp[i + 1]; ++e) {
            if (col[e] < i) continue;
            up_col[p] = col[e];
            up_val[p] = val[e];
            ++p;
        }
    }
}

static spmv_status dia_from_csr_impl(bool sym, int32_t n_rows, int32_t n_cols, int64_t nnz, const int32_t *row_ptr,
                                     const int32_t *col_idx, const void *val, spmv_dtype dt, int32_t max_diags,
                                     int32_t *h_offsets, int32_t *h_ndia, int64_t *h_rem_nnz, void *dia_val,
                                     int32_t *rem_row_ptr, int32_t *rem_col, void *rem_val, void *ws, size_t ws_bytes,
                                     void *stream)
{
    SPMV_REQUIRE(n_rows >= 0 && n_cols >= 0 && nnz >= 0, "spmv_dia[_sym]_from_csr: negative size");
    if (nnz >= ((int64_t)1 << 31)) return fail(SPMV_ERR_UNSUPPORTED, "spmv_dia[_sym]_from_csr: nnz >= 2^31");
    SPMV_REQUIRE(valid_dtype(dt), "spmv_dia[_sym]_from_csr: bad dtype");
    if (max_diags == 0) max_diags = SPMV_DIA_MAX;
    SPMV_REQUIRE(max_diags > 0 && max_diags <= SPMV_DIA_MAX, "spmv_dia[_sym]_from_csr: max_diags must be 0..SPMV_DIA_MAX");
    SPMV_REQUIRE(h_offsets && h_ndia && h_rem_nnz, "spmv_dia[_sym]_from_csr: null host output");
    SPMV_REQUIRE(n_rows == 0 || row_ptr, "spmv_dia[_sym]_from_csr: null row_ptr");
    SPMV_REQUIRE(nnz == 0 || (col_idx && val), "spmv_dia[_sym]_from_csr: null col_idx or val");
    SPMV_REQUIRE(ws && ws_bytes >= spmv_dia_workspace_size(n_rows, n_cols), "spmv_dia[_sym]_from_csr: workspace too small");
    hipStream_t s = as_stream(stream);
    const int64_t m = (int64_t)(n_rows > 0 ? n_rows : 1) + (n_cols > 0 ? n_cols : 1) - 1;
    const size_t nn = (size_t)(n_rows > 0 ? n_rows : 1);
    WsCarver wc(ws, ws_bytes);
    int32_t *hist = wc.take<int32_t>((size_t)m);           // later: offset -> stored diagonal index
    int32_t *cnt = wc.take<int32_t>(nn);
    int32_t *scan_ws = wc.take<int32_t>(scan_ws_elems((int64_t)nn));
    if (!wc.ok()) return fail(SPMV_ERR_INVALID_ARG, "spmv_dia[_sym]_from_csr: workspace too small");

    // entries per offset
    std::vector<int32_t> h_hist((size_t)m, 0);
    if (nnz > 0 && n_rows > 0) {
        SPMV_HIP(hipMemsetAsync(hist, 0, sizeof(int32_t) * (size_t)m, s));
        diag_hist_kernel<<<grid_for(n_rows), 256, 0, s>>>(row_ptr, n_rows, col_idx, hist);
        SPMV_CHECK_LAUNCH("dia histogram");
        SPMV_HIP(hipMemcpyAsync(h_hist.data(), hist, sizeof(int32_t) * (size_t)m, hipMemcpyDeviceToHost, s));
        SPMV_HIP(hipStreamSynchronize(s));
    }
    // a diagonal is stored densely when its dense span costs no more bytes
    // than its entries do in CRS (value + 4-byte index); the fullest first.
    // Symmetric: only offsets >= 0 are stored, each also serving its mirror,
    // so its entries are those of offset o and -o
    const int64_t sv = (int64_t)dtype_size(dt);
    std::vector<std::pair<int32_t, int64_t>> cand;            // (count, offset)
    for (int64_t t = 0; t < m; ++t) {
        const int64_t o = t - (n_rows - 1);
        if (sym && o < 0) continue;
        int64_t c = h_hist[(size_t)t];
        if (sym && o > 0) c += h_hist[(size_t)(n_rows - 1 - o)];
        if (c == 0) continue;
        const int64_t span = std::min<int64_t>(n_rows, (int64_t)n_cols - o) - std::max<int64_t>(0, -o);
        if (c * (sv + 4) >= span * sv) cand.push_back({(int32_t)c, o});
    }
    std::sort(cand.begin(), cand.end(), [](const std::pair<int32_t, int64_t> &a, const std::pair<int32_t, int64_t> &b) {
        return a.first != b.first ? a.first > b.first : a.second < b.second;
    });
    if ((int64_t)cand.size() > max_diags) cand.resize((size_t)max_diags);
    DiaOffsets D{};
    D.n = (int32_t)cand.size();
    int64_t on_dia = 0;
    for (int k = 0; k < D.n; ++k) {
        D.off[k] = (int32_t)cand[(size_t)k].second;
        on_dia += cand[(size_t)k].first;
    }
    std::sort(D.off, D.off + D.n);
    *h_ndia = D.n;
    for (int k = 0; k < D.n; ++k) h_offsets[k] = D.off[k];
    *h_rem_nnz = nnz - on_dia;
    if (!dia_val) return SPMV_OK;                            // sizes only

    SPMV_REQUIRE(rem_row_ptr && (*h_rem_nnz == 0 || (rem_col && rem_val)), "spmv_dia[_sym]_from_csr: null output");
    if (n_rows > 0) {
        dia_index_kernel<<<grid_for(m), 256, 0, s>>>(m, hist);
        dia_index_set_kernel<<<1, SPMV_DIA_MAX, 0, s>>>(n_rows, D, sym ? 1 : 0, hist);
        SPMV_CHECK_LAUNCH("dia index");
    }
    const int64_t ndv = (int64_t)D.n * n_rows;
#define DIA_CASE(DT, T)                                                                                          \
    if (dt == DT) {                                                                                              \
        if (ndv > 0) dia_zero_kernel<T><<<grid_for(ndv), 256, 0, s>>>(ndv, (T *)dia_val);                       \
        if (n_rows > 0)                                                                                          \
            dia_scatter_kernel<T><<<grid_for(n_rows), 256, 0, s>>>(row_ptr, n_rows, col_idx, (const T *)val,     \
                                                                   hist, (T *)dia_val, cnt);                    \
        SPMV_CHECK_LAUNCH("dia scatter");                                                                        \
        spmv_status st = exclusive_scan<int32_t, int32_t>(cnt, n_rows, rem_row_ptr, scan_ws, s);                \
        if (st != SPMV_OK) return st;                                                                            \
        if (*h_rem_nnz > 0)                                                                                      \
            dia_rem_kernel<T><<<grid_for(n_rows), 256, 0, s>>>(row_ptr, n_rows, col_idx, (const T *)val, hist,  \
                                                               rem_row_ptr, rem_col, (T *)rem_val);             \
        SPMV_CHECK_LAUNCH("dia remainder");                                                                      \
    }
    DIA_CASE(SPMV_F64, uint64_t)
    DIA_CASE(SPMV_F32, uint32_t)
    DIA_CASE(SPMV_BF16, uint16_t)
#undef DIA_CASE
    SPMV_HIP(hipStreamSynchronize(s));
    return SPMV_OK;
}

}  // namespace spmv

extern "C" {

spmv_status spmv_dia_from_csr(int32_t n_rows, int32_t n_cols, int64_t nnz, const int32_t *row_ptr,
                              const int32_t *col_idx, const void *val, spmv_dtype dt, int32_t max_diags,
                              int32_t *h_offsets, int32_t *h_ndia, int64_t *h_rem_nnz, void *dia_val,
                              int32_t *rem_row_ptr, int32_t *rem_col, void *rem_val, void *ws, size_t ws_bytes,
                              void *stream)
{
    return dia_from_csr_impl(false, n_rows, n_cols, nnz, row_ptr, col_idx, val, dt, max_diags, h_offsets, h_ndia,
                             h_rem_nnz, dia_val, rem_row_ptr, rem_col, rem_val, ws, ws_bytes, stream);
}

spmv_status spmv_dia_sym_from_csr(int32_t n, int64_t nnz, const int32_t *row_ptr, const int32_t *col_idx,
                                  const void *val, spmv_dtype dt, int32_t max_diags, int32_t *h_offsets,
                                  int32_t *h_ndia, int64_t *h_rem_nnz, void *dia_val, int32_t *rem_row_ptr,
                                  int32_t *rem_col, void *rem_val, void *ws, size_t ws_bytes, void *stream)
{
    return dia_from_csr_impl(true, n, n, nnz, row_ptr, col_idx, val, dt, max_diags, h_offsets, h_ndia, h_rem_nnz,
                             dia_val, rem_row_ptr, rem_col, rem_val, ws, ws_bytes, stream);
}

size_t spmv_csr_upper_workspace_size(int32_t n)
{
    const size_t nn = (size_t)(n > 0 ? n : 1);
    return align_up(sizeof(int32_t) * nn, 256) + align_up(sizeof(int32_t) * (nn + 1), 256) +
           align_up(sizeof(int32_t) * scan_ws_elems((int64_t)nn), 256) + 512;
}

spmv_status spmv_csr_upper_from_csr(int32_t n, int64_t nnz, const int32_t *row_ptr, const int32_t *col_idx,
                                    const void *val, spmv_dtype dt, int64_t *h_nnz_upper, int32_t *up_row_ptr,
                                    int32_t *up_col, void *up_val, void *ws, size_t ws_bytes, void *stream)
{
    SPMV_REQUIRE(n >= 0 && nnz >= 0, "spmv_csr_upper_from_csr: negative size");
    if (nnz >= ((int64_t)1 << 31)) return fail(SPMV_ERR_UNSUPPORTED, "spmv_csr_upper_from_csr: nnz >= 2^31");
    SPMV_REQUIRE(valid_payload_dtype(dt), "spmv_csr_upper_from_csr: bad dtype");
    SPMV_REQUIRE(h_nnz_upper, "spmv_csr_upper_from_csr: null h_nnz_upper");
    SPMV_REQUIRE(n == 0 || row_ptr, "spmv_csr_upper_from_csr: null row_ptr");
    SPMV_REQUIRE(nnz == 0 || (col_idx && val), "spmv_csr_upper_from_csr: null col_idx or val");
    SPMV_REQUIRE(ws && ws_bytes >= spmv_csr_upper_workspace_size(n), "spmv_csr_upper_from_csr: workspace too small");
    hipStream_t s = as_stream(stream);
    const size_t nn = (size_t)(n > 0 ? n : 1);
    WsCarver wc(ws, ws_bytes);
    int32_t *cnt = wc.take<int32_t>(nn);
    int32_t *rp = wc.take<int32_t>(nn + 1);
    int32_t *sws = wc.take<int32_t>(scan_ws_elems((int64_t)nn));
    if (!wc.ok()) return fail(SPMV_ERR_INVALID_ARG, "spmv_csr_upper_from_csr: workspace too small");
    int32_t total = 0;
    if (n > 0) {
        upper_count_kernel<<<grid_for(n), 256, 0, s>>>(row_ptr, n, col_idx, cnt);
        SPMV_CHECK_LAUNCH("upper count");
        spmv_status st = exclusive_scan<int32_t, int32_t>(cnt, n, rp, sws, s);
        if (st != SPMV_OK) return st;
        SPMV_HIP(hipMemcpyAsync(&total, rp + n, sizeof(int32_t), hipMemcpyDeviceToHost, s));
        SPMV_HIP(hipStreamSynchronize(s));
    }
    *h_nnz_upper = total;
    if (!up_row_ptr) return SPMV_OK;                          // size only
    SPMV_REQUIRE(total == 0 || (up_col && up_val), "spmv_csr_upper_from_csr: null output");
    if (n == 0) {
        SPMV_HIP(hipMemsetAsync(up_row_ptr, 0, sizeof(int32_t), s));
        SPMV_HIP(hipStreamSynchronize(s));
        return SPMV_OK;
    }
    SPMV_HIP(hipMemcpyAsync(up_row_ptr, rp, sizeof(int32_t) * ((size_t)n + 1), hipMemcpyDeviceToDevice, s));
    if (total > 0) {
#define UP_CASE(DT, T)                                                                                          \
        if (dt == DT)                                                                                           \
            upper_fill_kernel<T><<<grid_for(n), 256, 0, s>>>(row_ptr, n, col_idx, (const T *)val, rp, up_col,   \
                                                             (T *)up_val);
        UP_CASE(SPMV_F64, uint64_t)
        UP_CASE(SPMV_F32, uint32_t)
        UP_CASE(SPMV_BF16, uint16_t)
        UP_CASE(SPMV_I32, uint32_t)
#undef UP_CASE
        SPMV_CHECK_LAUNCH("upper fill");
    }
    SPMV_HIP(hipStreamSynchronize(s));
    return SPMV_OK;
}

size_t spmv_split_rows_workspace_size(void) { return 2 * align_up(sizeof(int64_t) * (SPLIT_PARTS + 1), 256); }

spmv_status spmv_split_rows(int32_t n_rows, int64_t nnz, const int32_t *row_ptr, int32_t *row_ptr_parts,
                            int64_t *h_bounds, int64_t *h_entry_bounds, void *ws, size_t ws_bytes, void *stream)
{
    SPMV_REQUIRE(n_rows >= 0 && nnz >= 0, "spmv_split_rows: negative size");
    if (nnz >= ((int64_t)1 << 31)) return fail(SPMV_ERR_UNSUPPORTED, "spmv_split_rows: nnz >= 2^31");
    SPMV_REQUIRE(row_ptr && row_ptr_parts && h_bounds && h_entry_bounds, "spmv_split_rows: null pointer");
    SPMV_REQUIRE(ws && ws_bytes >= spmv_split_rows_workspace_size(), "spmv_split_rows: workspace too small");
    hipStream_t s = as_stream(stream);
    WsCarver wc(ws, ws_bytes);
    int64_t *bounds = wc.take<int64_t>(SPLIT_PARTS + 1);
    int64_t *entry_bounds = wc.take<int64_t>(SPLIT_PARTS + 1);
    row_bounds_kernel<<<1, 64, 0, s>>>(row_ptr, n_rows, nnz, bounds, entry_bounds);
    row_split_ptr_kernel<<<grid_for((int64_t)n_rows + SPLIT_PARTS), 256, 0, s>>>(row_ptr, n_rows, bounds,
                                                                                 row_ptr_parts);
    SPMV_CHECK_LAUNCH("spmv_split_rows");
    SPMV_HIP(hipMemcpyAsync(h_bounds, bounds, sizeof(int64_t) * (SPLIT_PARTS + 1), hipMemcpyDeviceToHost, s));
    SPMV_HIP(hipMemcpyAsync(h_entry_bounds, entry_bounds, sizeof(int64_t) * (SPLIT_PARTS + 1), hipMemcpyDeviceToHost,
                            s));
    SPMV_HIP(hipStreamSynchronize(s));
    if (h_entry_bounds[SPLIT_PARTS] != nnz)
        return fail(SPMV_ERR_BAD_FORMAT, "spmv_split_rows: row_ptr[n_rows] != nnz");
    return SPMV_OK;
}

size_t spmv_transpose_workspace_size(int32_t n_rows, int32_t n_cols, int64_t nnz)
{
    (void)n_rows;
    (void)n_cols;
    size_t n = (size_t)(nnz > 0 ? nnz : 1);
    return align_up(sizeof(uint32_t) * n, 256) + radix_ws_bytes((int64_t)n) + 512;
}

spmv_status spmv_transpose_csr(int32_t n_rows, int32_t n_cols, int64_t nnz, const int32_t *row_ptr,
                               const int32_t *col_idx, int32_t *rowT_ptr, int32_t *colT, int32_t *tmap, void *ws,
                               size_t ws_bytes, void *stream)
{
    SPMV_REQUIRE(n_rows >= 0 && n_cols >= 0 && nnz >= 0, "spmv_transpose_csr: negative size");
    if (nnz >= ((int64_t)1 << 31)) return fail(SPMV_ERR_UNSUPPORTED, "spmv_transpose_csr: nnz >= 2^31");
    SPMV_REQUIRE(rowT_ptr && row_ptr, "spmv_transpose_csr: null pointer");
    SPMV_REQUIRE(nnz == 0 || (col_idx && colT && tmap), "spmv_transpose_csr: null arrays");
    SPMV_REQUIRE(ws && ws_bytes >= spmv_transpose_workspace_size(n_rows, n_cols, nnz),
                 "spmv_transpose_csr: workspace too small");
    hipStream_t s = as_stream(stream);
    WsCarver wc(ws, ws_bytes);
    uint32_t *keys = wc.take<uint32_t>((size_t)(nnz > 0 ? nnz : 1));
    size_t rws_bytes = radix_ws_bytes(nnz);
    void *rws = wc.take<char>(rws_bytes);
    if (nnz == 0) {
        SPMV_HIP(hipMemsetAsync(rowT_ptr, 0, sizeof(int32_t) * ((size_t)n_cols + 1), s));
        SPMV_HIP(hipStreamSynchronize(s));
        return SPMV_OK;
    }
    // entries are in row order, so a stable sort by column lists each column's
    // entries by ascending row
    copy_u32_kernel<<<grid_for(nnz), 256, 0, s>>>(col_idx, keys, nnz);
    iota_kernel<<<grid_for(nnz), 256, 0, s>>>(tmap, nnz);
    SPMV_CHECK_LAUNCH("transpose init");
    spmv_status st = radix_sort_pairs(keys, tmap, nnz, bits_for(n_cols > 0 ? n_cols - 1 : 0), rws, rws_bytes, s);
    if (st != SPMV_OK) return st;
    transpose_cols_kernel<<<grid_for(nnz), 256, 0, s>>>(row_ptr, n_rows, tmap, nnz, colT);
    ptr_from_sorted_kernel<uint32_t><<<grid_for((int64_t)n_cols + 1), 256, 0, s>>>(keys, nnz, n_cols, rowT_ptr);
    SPMV_CHECK_LAUNCH("transpose structure");
    SPMV_HIP(hipStreamSynchronize(s));
    return SPMV_OK;
}

spmv_status spmv_convert_values(int64_t n, const void *in, spmv_dtype in_dt, void *out, spmv_dtype out_dt, void *stream)
{
    SPMV_REQUIRE(n >= 0, "spmv_convert_values: n < 0");
    SPMV_REQUIRE(valid_dtype(in_dt) && valid_dtype(out_dt), "spmv_convert_values: bad dtype");
    if (n == 0) return SPMV_OK;
    SPMV_REQUIRE(in && out, "spmv_convert_values: null pointer");
    convert_kernel<<<grid_for(n), 256, 0, as_stream(stream)>>>(n, in, (int)in_dt, out, (int)out_dt);
    SPMV_CHECK_LAUNCH("spmv_convert_values");
    return SPMV_OK;
}

spmv_status spmv_permute_vec(int32_t n, const int32_t *perm, const void *in, void *out, spmv_dtype dt, int inverse,
                             void *stream)
{
    SPMV_REQUIRE(n >= 0, "spmv_permute_vec: n < 0");
    SPMV_REQUIRE(valid_vec_dtype(dt) || dt == SPMV_I32, "spmv_permute_vec: dtype must be F64, F32 or I32");
    if (n == 0) return SPMV_OK;
    SPMV_REQUIRE(perm && in && out && in != out, "spmv_permute_vec: null or aliased pointer");
    hipStream_t s = as_stream(stream);
    if (dt == SPMV_F64)
        permute_kernel<uint64_t><<<grid_for(n), 256, 0, s>>>(n, perm, (const uint64_t *)in, (uint64_t *)out, inverse);
    else
        permute_kernel<uint32_t><<<grid_for(n), 256, 0, s>>>(n, perm, (const uint32_t *)in, (uint32_t *)out, inverse);
    SPMV_CHECK_LAUNCH("spmv_permute_vec");
    return SPMV_OK;
}

spmv_status spmv_gather_values(int64_t n, const int32_t *map, const void *in, void *out, spmv_dtype dt, void *stream)
{
    SPMV_REQUIRE(n >= 0, "spmv_gather_values: n < 0");
    SPMV_REQUIRE(valid_payload_dtype(dt), "spmv_gather_values: bad dtype");
    if (n == 0) return SPMV_OK;
    SPMV_REQUIRE(map && in && out && in != out, "spmv_gather_values: null or aliased pointer");
    hipStream_t s = as_stream(stream);
    if (dt == SPMV_F64)
        gather_kernel<uint64_t><<<grid_for(n), 256, 0, s>>>(n, map, (const uint64_t *)in, (uint64_t *)out);
    else if (dt == SPMV_F32 || dt == SPMV_I32)
        gather_kernel<uint32_t><<<grid_for(n), 256, 0, s>>>(n, map, (const uint32_t *)in, (uint32_t *)out);
    else
        gather_kernel<uint16_t><<<grid_for(n), 256, 0, s>>>(n, map, (const uint16_t *)in, (uint16_t *)out);
    SPMV_CHECK_LAUNCH("spmv_gather_values");
    return SPMV_OK;
}

}  // extern "C"
