// JDS and blocked-JDS sparse matrix-vector products (paper Section 2: the JDS
// kernel and its NBJDS / NUJDS / RBJDS refinements), plus the multi-vector form
// and the value gradient in JDS order.
//
// gfx950 design.  Rows are in the JDS permuted order, longest first.  A
// wavefront owns R consecutive permuted rows (R = 64: one row per lane); its
// lanes walk the jagged diagonals that reach their rows, U diagonals per trip
// (the NUJDS idea: more independent loads in flight per row).  Consecutive
// lanes read consecutive entries of one diagonal, so val/col loads are fully
// coalesced; the row's partial result stays in a register for all diagonals
// (NBJDS with the block held in registers: no result-vector traffic per
// diagonal).  Long rows would serialise one lane over thousands of diagonals,
// so the host splits the rows into classes by length: a class has R rows per
// wavefront (64/R lanes share a row and stride over its diagonals) and S
// wavefronts per row group (each takes a contiguous range of diagonals; the S
// partial sums meet in LDS and are added in a fixed order).  A workgroup holds
// 4, 8 or 16 wavefronts (launch parameter).  Every y element is written by one
// lane; no atomics.
//
// The same kernel runs on both storages:
//   JDS:     entry (d, r) at jd_ptr[d] + r, diagonal d reaches rows r < len_d
//   blocked: entry (d, r) at slice_ptr[s] + d*C + (r - s*C), s = r / C, padded
//            slots (col = -1) skipped.
#include <algorithm>
#include <vector>

#include "common.hpp"

namespace spmv {

constexpr int JDS_WAVES = 16;                 // wavefronts per workgroup: the most, and the default
constexpr int JDS_THREADS = JDS_WAVES * WAVE;
constexpr int JDS_MAX_CLASSES = 8;
constexpr int JDS_DEFAULT_MAX_ITERS = 32;

struct JdsClass {
    int32_t wg_end;     // cumulative workgroup count up to and including this class
    int32_t row_start;  // permuted rows [row_start, row_end)
    int32_t row_end;
    int32_t rlog;       // R = 1 << rlog rows per wavefront
    int32_t slog;       // S = 1 << slog wavefronts per row group
};

// No XCD-aware dealing of workgroups: a class holds rows of many lengths, so
// contiguous per-XCD chunks of a class would give the XCDs very unequal work;
// the hardware's round-robin spreads every class evenly.
struct JdsPlan {
    JdsClass c[JDS_MAX_CLASSES];
    int32_t ncls;
    int32_t waves;      // wavefronts per workgroup (4, 8 or 16)
};

struct JdsArgs {
    int32_t n;
    const int32_t *perm;
    const int32_t *jd_ptr;  // JDS storage
    int32_t ndiag;
    int32_t C;              // blocked storage
    const int64_t *slice_ptr;
    const int32_t *slice_nd;
    const int32_t *col;
    const void *val;
    const void *x;
    void *y;
    int64_t ldx, ldy;       // multi-vector forms
    int32_t k;
    double alpha, beta;
    int symperm;
    const void *g;          // value gradient: dL/dy
    void *dval;             // value gradient output (JDS order)
};

enum { FMT_JDS = 0, FMT_BLOCKED = 1 };

// Number of diagonals of permuted row `row` in JDS storage: the first d whose
// diagonal is too short to reach the row (diagonal lengths never increase).
__device__ __forceinline__ int32_t jds_row_len(const int32_t *__restrict__ jp, int32_t ndiag, int32_t row)
{
    int32_t lo = 0, hi = ndiag;
    while (lo < hi) {
        int32_t mid = (lo + hi) >> 1;
        if (jp[mid + 1] - jp[mid] > row) lo = mid + 1;
        else hi = mid;
    }
    return lo;
}

// JDS storage: partial sum of one lane over its diagonals in [dA, dB), d =
// base + kk + G*u.  The U diagonal offsets of a trip are fetched first, all
// at once (clamped to the last diagonal of the range, so every fetch is in
// bounds), and only then the entries and the x elements: no load waits on
// another inside a trip except the gathers on their column.  UNI (G == 1,
// one lane per row): every lane walks the same diagonals, so base, the
// offsets and the stop test are wave-uniform and use scalar loads.
// `bounded` false: stop as soon as the group's first row has no diagonal
// (used by unsplit groups, which then never search for their length).
template <bool UNI, int U, bool WIDE, typename VT, typename XT>
__device__ __forceinline__ typename Acc<WIDE>::T jds_diag_sum(const JdsArgs &a, int32_t row0, int32_t r,
                                                              bool row_ok, int kk, int G, int32_t dA,
                                                              int32_t dB, bool bounded, int64_t xoff)
{
    typedef typename Acc<WIDE>::T acc_t;
    const VT *__restrict__ val = (const VT *)a.val;
    const XT *__restrict__ x = (const XT *)a.x + xoff;
    const int32_t *__restrict__ col = a.col;
    const int32_t *__restrict__ jp = a.jd_ptr;
    if (UNI) {
        dA = __builtin_amdgcn_readfirstlane(dA);
        dB = __builtin_amdgcn_readfirstlane(dB);
        row0 = __builtin_amdgcn_readfirstlane(row0);
        kk = 0;
        G = 1;
    }
    acc_t s = 0;
    for (int32_t base = dA; base < dB; base += G * U) {
        if (!bounded && jp[base + 1] - jp[base] <= row0) break;
        int32_t off[U], len[U];
#pragma unroll
        for (int u = 0; u < U; ++u) {
            int32_t dd = base + kk + u * G;
            dd = dd < dB ? dd : dB - 1;
            off[u] = jp[dd];
            len[u] = jp[dd + 1] - off[u];
        }
        int32_t c[U];
        VT v[U];
        bool act[U];
#pragma unroll
        for (int u = 0; u < U; ++u) {
            act[u] = row_ok && base + kk + u * G < dB && r < len[u];
            if (act[u]) {
                c[u] = ld_stream(col + off[u] + r);
                v[u] = ld_stream(val + off[u] + r);
            }
        }
        XT xv[U];
#pragma unroll
        for (int u = 0; u < U; ++u)
            if (act[u]) xv[u] = x[c[u]];
#pragma unroll
        for (int u = 0; u < U; ++u)
            if (act[u]) s = Acc<WIDE>::mac(s, v[u], xv[u]);
    }
    return s;
}

// Partial sum of one lane over its diagonals in [dA, dB): d = base + kk + G*u.
template <int FMT, int U, bool WIDE, typename VT, typename XT>
__device__ __forceinline__ typename Acc<WIDE>::T jds_lane_sum(const JdsArgs &a, int32_t row0, int32_t r,
                                                              bool row_ok, int kk, int G, int32_t dA,
                                                              int32_t dB, bool bounded, int64_t xoff)
{
    typedef typename Acc<WIDE>::T acc_t;
    const VT *__restrict__ val = (const VT *)a.val;
    const XT *__restrict__ x = (const XT *)a.x + xoff;
    const int32_t *__restrict__ col = a.col;
    acc_t s = 0;
    if (FMT == FMT_JDS) {
        if (G == 1) return jds_diag_sum<true, U, WIDE, VT, XT>(a, row0, r, row_ok, kk, G, dA, dB, bounded, xoff);
        return jds_diag_sum<false, U, WIDE, VT, XT>(a, row0, r, row_ok, kk, G, dA, dB, bounded, xoff);
    } else {
        const int32_t sl = row0 / a.C;
        const int64_t sp = a.slice_ptr[sl];
        const int32_t nd = a.slice_nd[sl];
        const int32_t rs = r - sl * a.C;
        if (dB > nd) dB = nd;
        for (int32_t base = dA; base < dB; base += G * U) {
            int32_t c[U];
            VT v[U];
            bool act[U];
#pragma unroll
            for (int u = 0; u < U; ++u) {
                const int32_t dd = base + kk + u * G;
                act[u] = false;
                if (row_ok && dd < dB) {
                    const int64_t e = sp + (int64_t)dd * a.C + rs;
                    c[u] = ld_stream(col + e);
                    v[u] = ld_stream(val + e);
                    act[u] = c[u] >= 0;
                }
            }
            XT xv[U];
#pragma unroll
            for (int u = 0; u < U; ++u)
                if (act[u]) xv[u] = x[c[u]];
#pragma unroll
            for (int u = 0; u < U; ++u)
                if (act[u]) s = Acc<WIDE>::mac(s, v[u], xv[u]);
        }
    }
    return s;
}

// Lanes rl + R*kk (kk < G) hold partials of one row: fixed xor tree over kk.
template <typename T>
__device__ __forceinline__ T reduce_over_kk(T v, int rlog)
{
    for (int off = 32; off >= (1 << rlog); off >>= 1) v += __shfl_xor(v, off, WAVE);
    return v;
}

// What one wavefront does: R rows starting at row0 (lane = rl + R*kk owns row
// row0 + rl and every G-th diagonal from dA + kk), diagonals [dA, dB) of
// part p of S.
struct WaveTask {
    bool valid, row_ok, bounded, wide;
    int32_t row0, r, dA, dB;
    int w, rl, kk, G, S, p, rlog;
};

template <int FMT>
__device__ __forceinline__ WaveTask wave_task(const JdsArgs &a, const JdsPlan &P, bool reduced_values, int64_t wg)
{
    WaveTask t;
    int ci = 0;
    while (ci < P.ncls - 1 && wg >= P.c[ci].wg_end) ++ci;
    const JdsClass K = P.c[ci];
    const int64_t wg0 = ci ? P.c[ci - 1].wg_end : 0;
    t.w = (int)threadIdx.x / WAVE;
    const int lane = lane_id();
    t.rlog = K.rlog;
    t.S = 1 << K.slog;
    const int R = 1 << K.rlog;
    t.G = WAVE >> K.rlog;
    const int64_t slot = (wg - wg0) * P.waves + t.w;
    const int64_t grp = slot >> K.slog;
    t.p = (int)(slot & (t.S - 1));
    const int64_t row0l = (int64_t)K.row_start + grp * R;
    t.valid = row0l < K.row_end;
    t.row0 = t.valid ? (int32_t)row0l : K.row_start;
    t.rl = lane & (R - 1);
    t.kk = lane >> K.rlog;
    t.r = t.row0 + t.rl;
    t.row_ok = t.valid && t.r < K.row_end;

    // length of the group's first (longest) row: only split groups need it
    int32_t Lmax = 0;
    t.wide = false;
    if (t.valid) {
        if (FMT == FMT_JDS) {
            if (t.S > 1) Lmax = jds_row_len(a.jd_ptr, a.ndiag, t.row0);
            if (reduced_values)
                t.wide = a.ndiag > SPMV_WIDE_ROW_NNZ &&
                         a.jd_ptr[SPMV_WIDE_ROW_NNZ + 1] - a.jd_ptr[SPMV_WIDE_ROW_NNZ] > t.row0;
        } else {
            Lmax = a.slice_nd[t.row0 / a.C];
            if (reduced_values) t.wide = Lmax > SPMV_WIDE_ROW_NNZ;
        }
    }
    t.dA = 0;
    t.dB = (FMT == FMT_JDS) ? a.ndiag : Lmax;
    if (t.S > 1) {
        const int64_t SG = (int64_t)t.S * t.G;
        const int32_t per = (int32_t)(((int64_t)Lmax + SG - 1) / SG * t.G);
        t.dA = t.p * per;
        t.dB = t.dA + per < Lmax ? t.dA + per : Lmax;
        if (t.dA > t.dB) t.dA = t.dB;
    }
    t.bounded = (FMT == FMT_BLOCKED) || t.S > 1;
    return t;
}

// Workgroup wg of plan P: y (or a partial result of type OT) for its rows.
// WIDE_ALL: accumulate every row in FP64 (the column-split parts, whose rows
// are pieces of rows whose full length the workgroup does not see).
template <int FMT, int U, typename VT, typename XT, typename OT, bool WIDE_ALL = false>
__device__ __forceinline__ void jds_body_task(const JdsArgs &a, const WaveTask &t, double (*part)[WAVE])
{
    constexpr bool F64 = IsF64<VT>::value || WIDE_ALL;
    const bool valid = t.valid, row_ok = t.row_ok, wide = t.wide, bounded = t.bounded;
    const int32_t row0 = t.row0, r = t.r, dA = t.dA, dB = t.dB;
    const int w = t.w, rl = t.rl, kk = t.kk, G = t.G, S = t.S, p = t.p;
    const JdsClass K{0, 0, 0, t.rlog, 0};

    double td = 0.0;
    if (valid) {
        if (F64 || wide) {
            double s = jds_lane_sum<FMT, U, true, VT, XT>(a, row0, r, row_ok, kk, G, dA, dB, bounded, 0);
            td = reduce_over_kk(s, K.rlog);
        } else {
            float s = jds_lane_sum<FMT, U, false, VT, XT>(a, row0, r, row_ok, kk, G, dA, dB, bounded, 0);
            td = (double)reduce_over_kk(s, K.rlog);
        }
    }
    if (S > 1) {
        if (kk == 0) part[w][rl] = td;
        __syncthreads();
        if (p != 0) return;
        if (F64 || wide) {
            double t = 0.0;
            for (int q = 0; q < S; ++q) t += part[w + q][rl];
            td = t;
        } else {
            float t = 0.0f;
            for (int q = 0; q < S; ++q) t += (float)part[w + q][rl];
            td = (double)t;
        }
    }
    if (row_ok && kk == 0) {
        const int32_t yi = a.symperm ? r : a.perm[r];
        write_y((OT *)a.y, yi, td, a.alpha, a.beta);
    }
}

template <int FMT, int U, typename VT, typename XT, typename OT, bool WIDE_ALL = false>
__device__ __forceinline__ void jds_body(const JdsArgs &a, const JdsPlan &P, int64_t wg,
                                         double (*part)[WAVE])
{
    constexpr bool F64 = IsF64<VT>::value || WIDE_ALL;
    jds_body_task<FMT, U, VT, XT, OT, WIDE_ALL>(a, wave_task<FMT>(a, P, !F64, wg), part);
}

// Tile plans (JDS storage, or blocked storage in any row order): workgroup
// record (row0, code) covers permuted rows [row0, row0 + nrows) with R =
// 2^rlog rows per wave group and S = 2^slog waves per group, code = rlog |
// slog << 4 | nrows << 8 (a blocked record stays inside one slice).  The
// records form 8 ranges, range k for the workgroups on XCD k (workgroup b
// runs on XCD b % 8): contiguous ranges of equal work for a windowed order,
// XCD-local pieces of the long equal-length runs plus records dealt for
// equal cost for a globally sorted order.
struct TileBounds {
    int64_t b[9];
};

template <int FMT>
__device__ __forceinline__ WaveTask tile_task(const JdsArgs &a, int32_t row0, int32_t nrows, int rlog, int slog,
                                              bool reduced_values)
{
    WaveTask t;
    t.w = (int)threadIdx.x / WAVE;
    const int lane = lane_id();
    t.rlog = rlog;
    t.S = 1 << slog;
    const int R = 1 << rlog;
    t.G = WAVE >> rlog;
    const int64_t row_end = min((int64_t)row0 + nrows, (int64_t)a.n);
    const int64_t grp = t.w >> slog;
    t.p = t.w & (t.S - 1);
    const int64_t row0l = (int64_t)row0 + grp * R;
    t.valid = row0l < row_end;
    t.row0 = t.valid ? (int32_t)row0l : row0;
    t.rl = lane & (R - 1);
    t.kk = lane >> rlog;
    t.r = t.row0 + t.rl;
    t.row_ok = t.valid && t.r < row_end;
    // length of the group's first (longest) row, as in wave_task
    int32_t Lmax = 0;
    t.wide = false;
    if (t.valid) {
        if (FMT == FMT_JDS) {
            if (t.S > 1) Lmax = jds_row_len(a.jd_ptr, a.ndiag, t.row0);
            if (reduced_values)
                t.wide = a.ndiag > SPMV_WIDE_ROW_NNZ &&
                         a.jd_ptr[SPMV_WIDE_ROW_NNZ + 1] - a.jd_ptr[SPMV_WIDE_ROW_NNZ] > t.row0;
        } else {
            Lmax = a.slice_nd[t.row0 / a.C];
            t.wide = reduced_values && Lmax > SPMV_WIDE_ROW_NNZ;
        }
    }
    t.dA = 0;
    t.dB = (FMT == FMT_JDS) ? a.ndiag : Lmax;
    if (t.S > 1) {
        const int64_t SG = (int64_t)t.S * t.G;
        const int32_t per = (int32_t)(((int64_t)Lmax + SG - 1) / SG * t.G);
        t.dA = t.p * per;
        t.dB = t.dA + per < Lmax ? t.dA + per : Lmax;
        if (t.dA > t.dB) t.dA = t.dB;
    }
    t.bounded = (FMT == FMT_BLOCKED) || t.S > 1;
    return t;
}

template <int FMT, int U, typename VT, typename XT>
__global__ __launch_bounds__(JDS_THREADS) void jds_tiles_kernel(JdsArgs a, const int32_t *__restrict__ tiles,
                                                                TileBounds xb)
{
    __shared__ double part[JDS_WAVES][WAVE];
    constexpr bool F64 = IsF64<VT>::value;
    const int x = (int)(blockIdx.x % 8);
    const int64_t idx = xb.b[x] + blockIdx.x / 8;
    if (idx >= xb.b[x + 1]) return;
    const int32_t row0 = tiles[2 * idx], code = tiles[2 * idx + 1];
    jds_body_task<FMT, U, VT, XT, XT>(a, tile_task<FMT>(a, row0, code >> 8, code & 15, (code >> 4) & 15, !F64),
                                      part);
}

template <int FMT, int U, typename VT, typename XT>
__global__ __launch_bounds__(JDS_THREADS) void jds_kernel(JdsArgs a, JdsPlan P)
{
    __shared__ double part[JDS_WAVES][WAVE];
    jds_body<FMT, U, VT, XT, XT>(a, P, blockIdx.x, part);
}

// Column-split JDS / blocked JDS: part k (the matrix restricted to the k-th
// eighth of the columns and to the rows holding one of its entries, with its
// own permutation) runs on XCD k (workgroup b -> part b % 8).  Its perm maps
// each permuted row straight to the row's slot in a[k].y, which receives the
// FP64 partial result.  All rows accumulate in FP64, reduced-precision values
// included.
struct JdsSplitArgs {
    JdsArgs a[SPLIT_PARTS];
    JdsPlan P[SPLIT_PARTS];
};

template <int FMT, int U, typename VT, typename XT>
__global__ __launch_bounds__(JDS_THREADS) void jds_split_kernel(JdsSplitArgs S)
{
    __shared__ double part[JDS_WAVES][WAVE];
    const int k = (int)(blockIdx.x % SPLIT_PARTS);
    const int64_t wg = blockIdx.x / SPLIT_PARTS;
    const JdsPlan &P = S.P[k];
    if (P.ncls == 0 || wg >= P.c[P.ncls - 1].wg_end) return;
    jds_body<FMT, U, VT, XT, double, true>(S.a[k], P, wg, part);
}

// Row-split JDS / blocked JDS: part k (a contiguous block of rows with its own
// JDS or blocked-JDS storage and local permutation) runs on XCD k; a[k].y
// points at the part's first row of y, which receives complete results.
template <int FMT, int U, typename VT, typename XT>
__global__ __launch_bounds__(JDS_THREADS) void jds_rows_kernel(JdsSplitArgs S)
{
    __shared__ double part[JDS_WAVES][WAVE];
    const int k = (int)(blockIdx.x % SPLIT_PARTS);
    const int64_t wg = blockIdx.x / SPLIT_PARTS;
    const JdsPlan &P = S.P[k];
    if (P.ncls == 0 || wg >= P.c[P.ncls - 1].wg_end) return;
    jds_body<FMT, U, VT, XT, XT>(S.a[k], P, wg, part);
}

// Multi-vector JDS: each lane owns one row (R = 64) and keeps k accumulators;
// the row's entries are read once for all k columns of X.  Rows longer than
// SPMV_WIDE_ROW_NNZ entries with reduced-precision values accumulate in FP64.
template <int KB, bool WIDE, typename VT, typename XT>
__device__ __forceinline__ void spmm_jds_row(const JdsArgs &a, int32_t r, int32_t row0, int col0, int kb)
{
    typedef typename Acc<WIDE>::T acc_t;
    const int32_t *__restrict__ jp = a.jd_ptr;
    const VT *__restrict__ val = (const VT *)a.val;
    const XT *__restrict__ X = (const XT *)a.x + (int64_t)col0 * a.ldx;
    acc_t acc[KB];
#pragma unroll
    for (int j = 0; j < KB; ++j) acc[j] = 0;
    for (int32_t d = 0; d < a.ndiag; ++d) {
        const int32_t off = jp[d], len = jp[d + 1] - off;
        if (len <= row0) break;
        if (r < len) {
            const int32_t c = ld_stream(a.col + off + r);
            const VT v = ld_stream(val + off + r);
#pragma unroll
            for (int j = 0; j < KB; ++j)
                if (j < kb) acc[j] = Acc<WIDE>::mac(acc[j], v, X[c + (int64_t)j * a.ldx]);
        }
    }
    const int32_t yi = a.symperm ? r : a.perm[r];
    XT *Y = (XT *)a.y + (int64_t)col0 * a.ldy;
#pragma unroll
    for (int j = 0; j < KB; ++j)
        if (j < kb) write_y(Y + (int64_t)j * a.ldy, yi, (double)acc[j], a.alpha, a.beta);
}

template <int KB, typename VT, typename XT>
__global__ __launch_bounds__(256) void spmm_jds_kernel(JdsArgs a)
{
    constexpr bool F64 = IsF64<VT>::value;
    const int64_t r64 = (int64_t)blockIdx.x * 256 + threadIdx.x;
    const int col0 = blockIdx.y * KB;
    const int kb = a.k - col0 < KB ? a.k - col0 : KB;
    if (r64 >= a.n) return;
    const int32_t r = (int32_t)r64;
    const int32_t row0 = (int32_t)(r64 & ~(int64_t)(WAVE - 1));
    // row r has more than SPMV_WIDE_ROW_NNZ entries iff diagonal 4096 reaches it
    const bool wide = !F64 && a.ndiag > SPMV_WIDE_ROW_NNZ &&
                      a.jd_ptr[SPMV_WIDE_ROW_NNZ + 1] - a.jd_ptr[SPMV_WIDE_ROW_NNZ] > r;
    if (F64 || wide) spmm_jds_row<KB, true, VT, XT>(a, r, row0, col0, kb);
    else spmm_jds_row<KB, false, VT, XT>(a, r, row0, col0, kb);
}

// Value gradient in JDS storage order: dval[e] = alpha*g[row]*x[col[e]] +
// beta*dval[e], computed in FP64 and rounded once.  Same wavefront layout as
// the product (each lane walks its row's diagonals; writes of consecutive lanes
// are consecutive), with no reduction: every entry is its own output.
template <bool UNI, int U, typename T>
__device__ __forceinline__ void jds_grad_lane(const JdsArgs &a, const WaveTask &t)
{
    const int32_t *__restrict__ jp = a.jd_ptr;
    const int32_t *__restrict__ col = a.col;
    const T *__restrict__ x = (const T *)a.x;
    T *__restrict__ dval = (T *)a.dval;
    const int32_t row = a.symperm ? t.r : a.perm[t.r];
    const double gv = a.alpha * to_f64(((const T *)a.g)[row]);
    int32_t dA = t.dA, dB = t.dB, row0 = t.row0, kk = t.kk, G = t.G;
    if (UNI) {                                 // see jds_diag_sum
        dA = __builtin_amdgcn_readfirstlane(dA);
        dB = __builtin_amdgcn_readfirstlane(dB);
        row0 = __builtin_amdgcn_readfirstlane(row0);
        kk = 0;
        G = 1;
    }
    for (int32_t base = dA; base < dB; base += G * U) {
        if (!t.bounded && jp[base + 1] - jp[base] <= row0) break;
        int32_t off[U], len[U];
#pragma unroll
        for (int u = 0; u < U; ++u) {
            int32_t dd = base + kk + u * G;
            dd = dd < dB ? dd : dB - 1;
            off[u] = jp[dd];
            len[u] = jp[dd + 1] - off[u];
        }
        int32_t c[U];
        bool act[U];
#pragma unroll
        for (int u = 0; u < U; ++u) {
            act[u] = base + kk + u * G < dB && t.r < len[u];
            if (act[u]) c[u] = ld_stream(col + off[u] + t.r);
        }
#pragma unroll
        for (int u = 0; u < U; ++u) {
            if (!act[u]) continue;
            const int64_t e = (int64_t)off[u] + t.r;
            double v = gv * to_f64(x[c[u]]);
            if (a.beta != 0.0) v = fma(a.beta, to_f64(dval[e]), v);
            store_from_f64(&dval[e], v);
        }
    }
}

template <int U, typename T>
__global__ __launch_bounds__(JDS_THREADS) void jds_grad_kernel(JdsArgs a, JdsPlan P)
{
    const WaveTask t = wave_task<FMT_JDS>(a, P, false, blockIdx.x);
    if (!t.row_ok) return;
    if (t.G == 1) jds_grad_lane<true, U, T>(a, t);
    else jds_grad_lane<false, U, T>(a, t);
}

// ---------------------------------------------------------------- host planning

// W wavefronts per 64-row chunk, split into (R rows per wave, S waves per
// group); a group's S waves share a workgroup of `waves` wavefronts.
static void split_for(int W, int forced_rlog, int waves, int &rlog, int &slog)
{
    if (forced_rlog >= 0) {
        int G = 1 << (6 - forced_rlog);
        int S = W / G;
        if (S < 1) S = 1;
        if (S > waves) S = waves;
        rlog = forced_rlog;
        slog = 0;
        while ((1 << slog) < S) ++slog;
        return;
    }
    switch (W) {
    case 1: rlog = 6; slog = 0; break;
    case 2: rlog = 5; slog = 0; break;
    case 4: rlog = 4; slog = 0; break;
    case 8: rlog = 4; slog = 1; break;
    case 16: rlog = 4; slog = 2; break;
    case 32: rlog = 4; slog = 3; break;
    case 64: rlog = 4; slog = 4; break;
    default: rlog = 3; slog = 4; break;   // 128
    }
    while ((1 << slog) > waves) --slog;   // then each wave takes more diagonals
}

// chunk_len(i) = length of the first row of 64-row chunk i (non-increasing).
template <typename F>
static JdsPlan build_plan(int32_t n, int32_t max_iters, int forced_rlog, int waves, F chunk_len)
{
    JdsPlan P{};
    P.waves = waves;
    int64_t nchunks = ceil_div(n, 64);
    int cls = 0;
    int64_t wg_total = 0;
    int64_t i = 0;
    while (i < nchunks && cls < JDS_MAX_CLASSES) {
        int64_t L = chunk_len(i);
        int W = 1;
        while (W < 128 && (int64_t)W * max_iters < L) W <<= 1;
        int rlog, slog;
        split_for(W, forced_rlog, waves, rlog, slog);
        // extend the class while the chunks want the same split
        int64_t j = i + 1;
        if (cls == JDS_MAX_CLASSES - 1) {
            j = nchunks;
        } else {
            // binary search the last chunk with the same W (lengths never increase)
            int64_t lo = i + 1, hi = nchunks;
            int64_t lower = (W > 1) ? (int64_t)(W / 2) * max_iters : -1;   // L > lower keeps W
            while (lo < hi) {
                int64_t mid = (lo + hi) >> 1;
                if (chunk_len(mid) > lower) lo = mid + 1;
                else hi = mid;
            }
            j = lo;
        }
        JdsClass &K = P.c[cls];
        K.row_start = (int32_t)(i * 64);
        K.row_end = (int32_t)(j * 64 < n ? j * 64 : n);
        K.rlog = rlog;
        K.slog = slog;
        int64_t groups = ceil_div(K.row_end - K.row_start, (int64_t)1 << rlog);
        wg_total += ceil_div(groups << slog, waves);
        K.wg_end = (int32_t)wg_total;
        ++cls;
        i = j;
    }
    P.ncls = cls;
    return P;
}

static JdsPlan plan_jds(int32_t n, const int32_t *h_jd_ptr, int32_t ndiag, int32_t max_iters, int forced_rlog,
                        int waves = JDS_WAVES)
{
    // rows longer than d are the first (jd_ptr[d+1]-jd_ptr[d]) permuted rows
    auto chunk_len = [&](int64_t i) -> int64_t {
        int64_t row = i * 64;
        int32_t lo = 0, hi = ndiag;
        while (lo < hi) {
            int32_t mid = (lo + hi) >> 1;
            if (h_jd_ptr[mid + 1] - h_jd_ptr[mid] > row) lo = mid + 1;
            else hi = mid;
        }
        return lo;
    };
    return build_plan(n, max_iters, forced_rlog, waves, chunk_len);
}

static JdsPlan plan_blocked(int32_t n, int32_t C, const int32_t *h_slice_nd, int32_t max_iters, int forced_rlog,
                            int waves = JDS_WAVES)
{
    auto chunk_len = [&](int64_t i) -> int64_t { return h_slice_nd[(i * 64) / C]; };
    return build_plan(n, max_iters, forced_rlog, waves, chunk_len);
}

// Tile plan of blocked storage whose slice depths need not decrease: each run
// of slices that wants the same (R, S) is covered by workgroups of
// (waves / S) * R rows; the record list is cut into 8 ranges of about equal
// cost (padded slots covered plus a fixed cost per wavefront).
static void plan_tiles(int32_t n, int32_t C, const int32_t *h_slice_nd, int32_t max_iters, int forced_rlog, int waves,
                       std::vector<int32_t> &rec, int64_t bounds[9])
{
    rec.clear();
    std::vector<double> cost;
    const int32_t ns = (int32_t)ceil_div(n, C);
    auto split_of = [&](int32_t sl, int &rlog, int &slog) {
        const int64_t L = h_slice_nd[sl];
        int W = 1;
        while (W < 128 && (int64_t)W * max_iters < L) W <<= 1;
        split_for(W, forced_rlog, waves, rlog, slog);
    };
    int32_t sl = 0;
    while (sl < ns) {
        int rlog, slog;
        split_of(sl, rlog, slog);
        int32_t e = sl + 1;
        for (; e < ns; ++e) {
            int r2, s2;
            split_of(e, r2, s2);
            if (r2 != rlog || s2 != slog) break;
        }
        const int64_t a0 = (int64_t)sl * C, a1 = std::min<int64_t>((int64_t)e * C, n);
        const int64_t rpw = (int64_t)(waves >> slog) << rlog;
        for (int64_t r = a0; r < a1; r += rpw) {
            const int64_t nr = std::min<int64_t>(rpw, a1 - r);
            rec.push_back((int32_t)r);
            rec.push_back(rlog | (slog << 4) | (int32_t)(nr << 8));
            cost.push_back((double)nr * h_slice_nd[r / C] + 64.0 * waves);
        }
        sl = e;
    }
    const int64_t nt = (int64_t)cost.size();
    double total = 0;
    for (double c : cost) total += c;
    bounds[0] = 0;
    double acc = 0;
    int64_t i = 0;
    for (int k = 1; k < 8; ++k) {
        while (i < nt && acc + cost[i] / 2 < total * k / 8) acc += cost[i++];
        bounds[k] = i;
    }
    bounds[8] = nt;
}

template <int FMT, typename VT, typename XT>
static spmv_status launch_jds_t(const JdsArgs &a, const JdsPlan &P, int unroll, hipStream_t s)
{
    if (P.ncls == 0) return SPMV_OK;
    unsigned grid = (unsigned)P.c[P.ncls - 1].wg_end;
    if (grid == 0) return SPMV_OK;
    switch (unroll) {
    case 2: jds_kernel<FMT, 2, VT, XT><<<grid, P.waves * WAVE, 0, s>>>(a, P); break;
    case 8: jds_kernel<FMT, 8, VT, XT><<<grid, P.waves * WAVE, 0, s>>>(a, P); break;
    default: jds_kernel<FMT, 4, VT, XT><<<grid, P.waves * WAVE, 0, s>>>(a, P); break;
    }
    SPMV_CHECK_LAUNCH(FMT == FMT_JDS ? "spmv_jds" : "spmv_jds_blocked");
    return SPMV_OK;
}

// XCD-local tile plan of a globally length-sorted storage (JDS rows, or
// the slices of a blocked JDS whose depths never increase).  A length class
// holds rows from all over the matrix, so dealing workgroups round robin (or
// in contiguous ranges of the sorted order) spreads the rows of one region
// of the original matrix over all XCDs, each fetching the same x lines of
// that region's band.  Here every long run of equal length (in original row
// order, since the sort is stable) is cut into 8 contiguous pieces, piece k
// to XCD k, so each XCD's short rows come from one eighth of the original
// rows; the remaining records (long rows, short runs) are dealt to the XCDs
// for equal cost, longest first.  Each XCD walks its dealt records (in
// sorted order), then its pieces ordered by their place inside their runs
// (all lengths side by side), so that it moves through its eighth of the
// original rows once instead of once per length.
//   unit_len(u): length of unit u (a row, or a slice's depth); units are
//     non-increasing in length; unit u spans rows [u*U, min((u+1)*U, n)).
//   U: rows per unit (1 for JDS rows, C for slices); chunk: rows per split
//     decision (64 for JDS, C for slices: a record never crosses a slice).
// Runs of at least this many rows of one length are cut into 8 XCD pieces
// (JDS on the power-law matrix: 512 and 1,024 rows 342 µs, 2,048 and 4,096
// rows 348 µs, 16,384 rows 353 µs, the class plan 360 µs).
constexpr int64_t TILE_LOCAL_MIN_RUN = 1024;

template <typename F>
static void plan_tiles_local(int32_t n, int32_t U, int64_t n_units, F unit_len, int32_t max_iters, int forced_rlog,
                             int waves, int64_t min_run_rows, std::vector<int32_t> &rec, int64_t bounds[9])
{
    struct Rec {
        int32_t row0, code;
        double cost, pos;   // pos: place of the record's first unit inside its length run, in [0, 1)
    };
    auto split_of = [&](int64_t L, int &rlog, int &slog) {
        int W = 1;
        while (W < 128 && (int64_t)W * max_iters < L) W <<= 1;
        split_for(W, forced_rlog, waves, rlog, slog);
    };
    auto records = [&](int64_t a0, int64_t a1, int rlog, int slog, int64_t L, std::vector<Rec> &out,
                       double pos = 0.0) {
        const int64_t rpw = (int64_t)(waves >> slog) << rlog;
        for (int64_t r = a0; r < a1; r += rpw) {
            const int64_t nr = std::min<int64_t>(rpw, a1 - r);
            out.push_back({(int32_t)r, rlog | (slog << 4) | (int32_t)(nr << 8), (double)nr * L + 64.0 * waves, pos});
        }
    };
    auto row_end = [&](int64_t u) { return std::min<int64_t>(u * U, n); };
    // first unit of length <= max_iters: one lane per row from there on
    int64_t q = 0, hi = n_units;
    while (q < hi) {
        const int64_t mid = (q + hi) >> 1;
        if (unit_len(mid) > max_iters) q = mid + 1;
        else hi = mid;
    }
    std::vector<Rec> others, pieces[8];
    // long units: runs of 64-row (JDS) or one-slice (blocked) steps wanting the same split
    const int64_t step = U == 1 ? 64 : 1;
    for (int64_t i = 0; i < q;) {
        int rlog, slog;
        split_of(unit_len(i), rlog, slog);
        int64_t j = std::min(i + step, q);
        for (; j < q; j = std::min(j + step, q)) {
            int r2, s2;
            split_of(unit_len(j), r2, s2);
            if (r2 != rlog || s2 != slog) break;
        }
        if (U == 1) {
            records(i, j, rlog, slog, unit_len(i), others);
        } else {
            for (int64_t u = i; u < j; ++u) records(u * U, row_end(u + 1), rlog, slog, unit_len(u), others);
        }
        i = j;
    }
    // short units: runs of equal length
    for (int64_t i = q; i < n_units;) {
        const int64_t L = unit_len(i);
        int64_t lo = i + 1, h2 = n_units;
        while (lo < h2) {
            const int64_t mid = (lo + h2) >> 1;
            if (unit_len(mid) == L) lo = mid + 1;
            else h2 = mid;
        }
        const int64_t j = lo;
        int rlog, slog;
        split_of(L, rlog, slog);
        if (row_end(j) - i * U >= min_run_rows) {
            for (int k = 0; k < 8; ++k) {
                const int64_t u0 = i + (j - i) * k / 8, u1 = i + (j - i) * (k + 1) / 8;
                const size_t first = pieces[k].size();
                if (U == 1) records(u0, u1, rlog, slog, L, pieces[k]);
                else
                    for (int64_t u = u0; u < u1; ++u) records(u * U, row_end(u + 1), rlog, slog, L, pieces[k]);
                for (size_t t = first; t < pieces[k].size(); ++t)
                    pieces[k][t].pos = (double)(pieces[k][t].row0 / U - i) / (double)(j - i);
            }
        } else if (U == 1) {
            records(i, j, rlog, slog, L, others);
        } else {
            for (int64_t u = i; u < j; ++u) records(u * U, row_end(u + 1), rlog, slog, L, others);
        }
        i = j;
    }
    // pieces at one place of their runs come from the same stretch of
    // original rows, so their band gathers meet in L2
    double load[8];
    for (int k = 0; k < 8; ++k) {
        std::stable_sort(pieces[k].begin(), pieces[k].end(), [](const Rec &a, const Rec &b) { return a.pos < b.pos; });
        load[k] = 0;
        for (const Rec &r : pieces[k]) load[k] += r.cost;
    }
    std::vector<int64_t> order(others.size());
    for (size_t t = 0; t < order.size(); ++t) order[t] = (int64_t)t;
    std::stable_sort(order.begin(), order.end(), [&](int64_t a, int64_t b) { return others[a].cost > others[b].cost; });
    std::vector<int64_t> dealt[8];
    for (int64_t t : order) {
        int k = 0;
        for (int m = 1; m < 8; ++m)
            if (load[m] < load[k]) k = m;
        dealt[k].push_back(t);
        load[k] += others[t].cost;
    }
    rec.clear();
    bounds[0] = 0;
    for (int k = 0; k < 8; ++k) {
        std::sort(dealt[k].begin(), dealt[k].end());
        for (int64_t t : dealt[k]) {
            rec.push_back(others[t].row0);
            rec.push_back(others[t].code);
        }
        for (const Rec &r : pieces[k]) {
            rec.push_back(r.row0);
            rec.push_back(r.code);
        }
        bounds[k + 1] = (int64_t)rec.size() / 2;
    }
}

template <int FMT>
static spmv_status launch_jds(const JdsArgs &a, const JdsPlan &P, int unroll, spmv_dtype vdt, spmv_dtype xdt,
                              hipStream_t s)
{
#define JDS_CASE(VDT, VT, XDT, XT) \
    if (vdt == VDT && xdt == XDT) return launch_jds_t<FMT, VT, XT>(a, P, unroll, s);
    JDS_CASE(SPMV_F64, double, SPMV_F64, double)
    JDS_CASE(SPMV_F32, float, SPMV_F64, double)
    JDS_CASE(SPMV_BF16, bf16, SPMV_F64, double)
    JDS_CASE(SPMV_F32, float, SPMV_F32, float)
    JDS_CASE(SPMV_BF16, bf16, SPMV_F32, float)
    JDS_CASE(SPMV_F64, double, SPMV_F32, float)
#undef JDS_CASE
    return fail(SPMV_ERR_UNSUPPORTED, "jds: dtype combination");
}

static int unroll_ok(int32_t u) { return u == 0 || u == 2 || u == 4 || u == 8; }
static int waves_ok(int32_t w) { return w == 0 || w == 4 || w == 8 || w == 16; }
static int waves_or_default(int32_t w) { return w ? w : JDS_WAVES; }

// Row bounds of the row-split parts: 0 = b_0 <= b_1 <= ... <= b_8 = n.
static spmv_status row_bounds_ok(int32_t n, const int64_t *h_bounds, const char *who)
{
    if (!h_bounds) return fail(SPMV_ERR_INVALID_ARG, std::string(who) + ": null h_bounds");
    if (h_bounds[0] != 0 || h_bounds[SPLIT_PARTS] != n)
        return fail(SPMV_ERR_INVALID_ARG, std::string(who) + ": h_bounds must run from 0 to n");
    for (int k = 0; k < SPLIT_PARTS; ++k)
        if (h_bounds[k + 1] < h_bounds[k]) return fail(SPMV_ERR_INVALID_ARG, std::string(who) + ": h_bounds decrease");
    return SPMV_OK;
}

template <int FMT>
static spmv_status launch_rows(const JdsSplitArgs &S, int64_t max_wg, int32_t unroll, int waves, spmv_dtype val_dt,
                               spmv_dtype vec_dt, hipStream_t s, const char *who)
{
    const unsigned grid = (unsigned)(max_wg * SPLIT_PARTS);
    const unsigned threads = (unsigned)(waves * WAVE);
    if (grid == 0) return SPMV_OK;
    const int u = unroll ? unroll : 4;
#define JROWS_CASE(VDT, VT, XDT, XT)                                                       \
    if (val_dt == VDT && vec_dt == XDT) {                                                  \
        if (u == 2) jds_rows_kernel<FMT, 2, VT, XT><<<grid, threads, 0, s>>>(S);       \
        else if (u == 8) jds_rows_kernel<FMT, 8, VT, XT><<<grid, threads, 0, s>>>(S);  \
        else jds_rows_kernel<FMT, 4, VT, XT><<<grid, threads, 0, s>>>(S);              \
    } else
    JROWS_CASE(SPMV_F64, double, SPMV_F64, double)
    JROWS_CASE(SPMV_F32, float, SPMV_F64, double)
    JROWS_CASE(SPMV_BF16, bf16, SPMV_F64, double)
    JROWS_CASE(SPMV_F32, float, SPMV_F32, float)
    JROWS_CASE(SPMV_BF16, bf16, SPMV_F32, float)
    JROWS_CASE(SPMV_F64, double, SPMV_F32, float)
    return fail(SPMV_ERR_UNSUPPORTED, std::string(who) + ": dtype combination");
#undef JROWS_CASE
    SPMV_CHECK_LAUNCH(who);
    return SPMV_OK;
}

}  // namespace spmv

using namespace spmv;

// Checks a tile plan's 8 range bounds (h_plan[0..8]) and wavefront count
// (h_plan[9]); returns the widest range through *widest.
static spmv_status check_tile_plan(const int64_t *h_plan, int64_t n_tiles, TileBounds &xb, int64_t *widest,
                                   const char *who)
{
    if (!h_plan) return fail(SPMV_ERR_INVALID_ARG, who);
    for (int k = 0; k < 9; ++k) xb.b[k] = h_plan[k];
    if (xb.b[0] != 0 || xb.b[8] != n_tiles) return fail(SPMV_ERR_INVALID_ARG, who);
    *widest = 0;
    for (int k = 0; k < 8; ++k) {
        if (xb.b[k + 1] < xb.b[k]) return fail(SPMV_ERR_INVALID_ARG, who);
        *widest = std::max<int64_t>(*widest, xb.b[k + 1] - xb.b[k]);
    }
    if (!waves_ok((int32_t)h_plan[9]) || h_plan[9] == 0) return fail(SPMV_ERR_INVALID_ARG, who);
    return SPMV_OK;
}

template <int FMT>
static spmv_status launch_tiles(const JdsArgs &a, const int32_t *tiles, const TileBounds &xb, int64_t widest,
                                int64_t waves, int32_t unroll, spmv_dtype val_dt, spmv_dtype vec_dt, hipStream_t s,
                                const char *who)
{
    const unsigned grid = (unsigned)(8 * widest), threads = (unsigned)(waves * WAVE);
    const int u = unroll ? unroll : 4;
#define JTILE_CASE(VDT, VT, XDT, XT)                                                                         \
    if (val_dt == VDT && vec_dt == XDT) {                                                                    \
        if (u == 2) jds_tiles_kernel<FMT, 2, VT, XT><<<grid, threads, 0, s>>>(a, tiles, xb);              \
        else if (u == 8) jds_tiles_kernel<FMT, 8, VT, XT><<<grid, threads, 0, s>>>(a, tiles, xb);         \
        else jds_tiles_kernel<FMT, 4, VT, XT><<<grid, threads, 0, s>>>(a, tiles, xb);                     \
    } else
    JTILE_CASE(SPMV_F64, double, SPMV_F64, double)
    JTILE_CASE(SPMV_F32, float, SPMV_F64, double)
    JTILE_CASE(SPMV_BF16, bf16, SPMV_F64, double)
    JTILE_CASE(SPMV_F32, float, SPMV_F32, float)
    JTILE_CASE(SPMV_BF16, bf16, SPMV_F32, float)
    JTILE_CASE(SPMV_F64, double, SPMV_F32, float)
    return fail(SPMV_ERR_UNSUPPORTED, who);
#undef JTILE_CASE
    SPMV_CHECK_LAUNCH(who);
    return SPMV_OK;
}

extern "C" {

spmv_status spmv_jds(int32_t n, const int32_t *perm, const int32_t *jd_ptr, const int32_t *h_jd_ptr, int32_t ndiag,
                     const int32_t *jd_col, const void *jd_val, spmv_dtype val_dt, const void *x, void *y,
                     spmv_dtype vec_dt, double alpha, double beta, int32_t unroll, int32_t max_iters,
                     int32_t wg_waves, unsigned flags, void *stream)
{
    SPMV_REQUIRE(n >= 0 && ndiag >= 0, "spmv_jds: negative size");
    SPMV_REQUIRE(waves_ok(wg_waves), "spmv_jds: wg_waves must be 0, 4, 8 or 16");
    SPMV_REQUIRE(valid_dtype(val_dt) && valid_vec_dtype(vec_dt), "spmv_jds: bad dtype");
    SPMV_REQUIRE(unroll_ok(unroll), "spmv_jds: unroll must be 0, 2, 4 or 8");
    SPMV_REQUIRE(max_iters >= 0, "spmv_jds: max_iters < 0");
    SPMV_REQUIRE((flags & ~SPMV_SYMPERM) == 0, "spmv_jds: unknown flag");
    if (n == 0) return SPMV_OK;
    SPMV_REQUIRE(y && jd_ptr && h_jd_ptr, "spmv_jds: null y, jd_ptr or h_jd_ptr");
    SPMV_REQUIRE((flags & SPMV_SYMPERM) || perm, "spmv_jds: null perm");
    SPMV_REQUIRE(ndiag == 0 || (jd_col && jd_val && x), "spmv_jds: null col, val or x");
    SPMV_REQUIRE(ndiag == 0 || h_jd_ptr[0] == 0, "spmv_jds: h_jd_ptr[0] != 0");
    JdsArgs a{};
    a.n = n;
    a.perm = perm;
    a.jd_ptr = jd_ptr;
    a.ndiag = ndiag;
    a.C = 64;
    a.col = jd_col;
    a.val = jd_val;
    a.x = x;
    a.y = y;
    a.alpha = alpha;
    a.beta = beta;
    a.symperm = (flags & SPMV_SYMPERM) ? 1 : 0;
    JdsPlan P = plan_jds(n, h_jd_ptr, ndiag, max_iters ? max_iters : JDS_DEFAULT_MAX_ITERS, -1,
                         waves_or_default(wg_waves));
    return launch_jds<FMT_JDS>(a, P, unroll ? unroll : 4, val_dt, vec_dt, as_stream(stream));
}

spmv_status spmv_jds_blocked(int32_t n, const int32_t *perm, int32_t C, int32_t n_slices, const int64_t *slice_ptr,
                             const int32_t *slice_nd, const int32_t *h_slice_nd, const int32_t *bl_col,
                             const void *bl_val, spmv_dtype val_dt, const void *x, void *y, spmv_dtype vec_dt,
                             double alpha, double beta, int32_t rows_per_wave, int32_t unroll, int32_t max_iters,
                             int32_t wg_waves, unsigned flags, void *stream)
{
    SPMV_REQUIRE(n >= 0, "spmv_jds_blocked: n < 0");
    SPMV_REQUIRE(waves_ok(wg_waves), "spmv_jds_blocked: wg_waves must be 0, 4, 8 or 16");
    SPMV_REQUIRE(C > 0 && C % 64 == 0, "spmv_jds_blocked: C must be a positive multiple of 64");
    SPMV_REQUIRE(n_slices == (int32_t)ceil_div(n, C), "spmv_jds_blocked: n_slices != ceil(n / C)");
    SPMV_REQUIRE(valid_dtype(val_dt) && valid_vec_dtype(vec_dt), "spmv_jds_blocked: bad dtype");
    SPMV_REQUIRE(unroll_ok(unroll), "spmv_jds_blocked: unroll must be 0, 2, 4 or 8");
    SPMV_REQUIRE(rows_per_wave == 0 || rows_per_wave == 8 || rows_per_wave == 16 || rows_per_wave == 32 ||
                     rows_per_wave == 64,
                 "spmv_jds_blocked: rows_per_wave must be 0, 8, 16, 32 or 64");
    SPMV_REQUIRE(max_iters >= 0, "spmv_jds_blocked: max_iters < 0");
    SPMV_REQUIRE((flags & ~(SPMV_SYMPERM | SPMV_SOJDS)) == 0, "spmv_jds_blocked: unknown flag");
    if (n == 0) return SPMV_OK;
    SPMV_REQUIRE(y && slice_ptr && slice_nd && h_slice_nd, "spmv_jds_blocked: null pointer");
    SPMV_REQUIRE(h_slice_nd[0] == 0 || (bl_col && bl_val && x), "spmv_jds_blocked: null col, val or x");
    SPMV_REQUIRE((flags & SPMV_SYMPERM) || perm, "spmv_jds_blocked: null perm");
    JdsArgs a{};
    a.n = n;
    a.perm = perm;
    a.C = C;
    a.slice_ptr = slice_ptr;
    a.slice_nd = slice_nd;
    a.col = bl_col;
    a.val = bl_val;
    a.x = x;
    a.y = y;
    a.alpha = alpha;
    a.beta = beta;
    a.symperm = (flags & SPMV_SYMPERM) ? 1 : 0;
    int forced = -1;
    if (rows_per_wave) {
        forced = 0;
        while ((1 << forced) < rows_per_wave) ++forced;
    }
    JdsPlan P = plan_blocked(n, C, h_slice_nd, max_iters ? max_iters : JDS_DEFAULT_MAX_ITERS, forced,
                             waves_or_default(wg_waves));
    return launch_jds<FMT_BLOCKED>(a, P, unroll ? unroll : 4, val_dt, vec_dt, as_stream(stream));
}

spmv_status spmv_jds_blocked_tiles(int32_t n, int32_t C, int32_t n_slices, const int32_t *h_slice_nd,
                                   int32_t max_iters, int32_t rows_per_wave, int32_t wg_waves, int32_t *tiles,
                                   int64_t tiles_cap, int64_t *h_n_tiles, int64_t *h_plan, void *stream)
{
    SPMV_REQUIRE(n >= 0, "spmv_jds_blocked_tiles: n < 0");
    SPMV_REQUIRE(C > 0 && C % 64 == 0, "spmv_jds_blocked_tiles: C must be a positive multiple of 64");
    SPMV_REQUIRE(n_slices == (int32_t)ceil_div(n, C), "spmv_jds_blocked_tiles: n_slices != ceil(n / C)");
    SPMV_REQUIRE(waves_ok(wg_waves), "spmv_jds_blocked_tiles: wg_waves must be 0, 4, 8 or 16");
    SPMV_REQUIRE(max_iters >= 0, "spmv_jds_blocked_tiles: max_iters < 0");
    SPMV_REQUIRE(rows_per_wave == 0 || rows_per_wave == 8 || rows_per_wave == 16 || rows_per_wave == 32 ||
                     rows_per_wave == 64,
                 "spmv_jds_blocked_tiles: rows_per_wave must be 0, 8, 16, 32 or 64");
    SPMV_REQUIRE(h_n_tiles && h_plan && (n_slices == 0 || h_slice_nd), "spmv_jds_blocked_tiles: null pointer");
    int forced = -1;
    if (rows_per_wave) {
        forced = 0;
        while ((1 << forced) < rows_per_wave) ++forced;
    }
    const int waves = waves_or_default(wg_waves);
    const int32_t mi = max_iters ? max_iters : JDS_DEFAULT_MAX_ITERS;
    std::vector<int32_t> rec;
    int64_t bounds[9];
    bool sorted = true;                       // the globally sorted order: depths never increase
    for (int32_t sl = 1; sl < n_slices && sorted; ++sl) sorted = h_slice_nd[sl] <= h_slice_nd[sl - 1];
    if (sorted)
        plan_tiles_local(n, C, n_slices, [&](int64_t u) -> int64_t { return h_slice_nd[u]; }, mi, forced, waves,
                         TILE_LOCAL_MIN_RUN, rec, bounds);
    else
        plan_tiles(n, C, h_slice_nd, mi, forced, waves, rec, bounds);
    const int64_t nt = (int64_t)rec.size() / 2;
    *h_n_tiles = nt;
    for (int k = 0; k < 9; ++k) h_plan[k] = bounds[k];
    h_plan[9] = waves;
    if (!tiles || tiles_cap < 2 * nt) return fail(SPMV_ERR_CAPACITY, "spmv_jds_blocked_tiles: tiles capacity < 2 * n_tiles");
    if (nt == 0) return SPMV_OK;
    hipStream_t s = as_stream(stream);
    SPMV_HIP(hipMemcpyAsync(tiles, rec.data(), sizeof(int32_t) * rec.size(), hipMemcpyHostToDevice, s));
    SPMV_HIP(hipStreamSynchronize(s));
    return SPMV_OK;
}

spmv_status spmv_jds_tiles(int32_t n, const int32_t *h_jd_ptr, int32_t ndiag, int32_t max_iters, int32_t rows_per_wave,
                           int32_t wg_waves, int32_t *tiles, int64_t tiles_cap, int64_t *h_n_tiles, int64_t *h_plan,
                           void *stream)
{
    SPMV_REQUIRE(n >= 0 && ndiag >= 0, "spmv_jds_tiles: negative size");
    SPMV_REQUIRE(waves_ok(wg_waves), "spmv_jds_tiles: wg_waves must be 0, 4, 8 or 16");
    SPMV_REQUIRE(max_iters >= 0, "spmv_jds_tiles: max_iters < 0");
    SPMV_REQUIRE(rows_per_wave == 0 || rows_per_wave == 8 || rows_per_wave == 16 || rows_per_wave == 32 ||
                     rows_per_wave == 64,
                 "spmv_jds_tiles: rows_per_wave must be 0, 8, 16, 32 or 64");
    SPMV_REQUIRE(h_n_tiles && h_plan && (ndiag == 0 || h_jd_ptr), "spmv_jds_tiles: null pointer");
    SPMV_REQUIRE(ndiag == 0 || (h_jd_ptr[0] == 0 && h_jd_ptr[1] <= n), "spmv_jds_tiles: h_jd_ptr inconsistent with n");
    int forced = -1;
    if (rows_per_wave) {
        forced = 0;
        while ((1 << forced) < rows_per_wave) ++forced;
    }
    const int waves = waves_or_default(wg_waves);
    // length of permuted row r: the diagonals longer than r
    auto row_len = [&](int64_t r) -> int64_t {
        int32_t lo = 0, hi = ndiag;
        while (lo < hi) {
            const int32_t mid = (lo + hi) >> 1;
            if (h_jd_ptr[mid + 1] - h_jd_ptr[mid] > r) lo = mid + 1;
            else hi = mid;
        }
        return lo;
    };
    std::vector<int32_t> rec;
    int64_t bounds[9];
    plan_tiles_local(n, 1, n, row_len, max_iters ? max_iters : JDS_DEFAULT_MAX_ITERS, forced, waves,
                     TILE_LOCAL_MIN_RUN, rec, bounds);
    const int64_t nt = (int64_t)rec.size() / 2;
    *h_n_tiles = nt;
    for (int k = 0; k < 9; ++k) h_plan[k] = bounds[k];
    h_plan[9] = waves;
    if (!tiles || tiles_cap < 2 * nt) return fail(SPMV_ERR_CAPACITY, "spmv_jds_tiles: tiles capacity < 2 * n_tiles");
    if (nt == 0) return SPMV_OK;
    hipStream_t s = as_stream(stream);
    SPMV_HIP(hipMemcpyAsync(tiles, rec.data(), sizeof(int32_t) * rec.size(), hipMemcpyHostToDevice, s));
    SPMV_HIP(hipStreamSynchronize(s));
    return SPMV_OK;
}

spmv_status spmv_jds_blocked_tiled(int32_t n, const int32_t *perm, int32_t C, int32_t n_slices,
                                   const int64_t *slice_ptr, const int32_t *slice_nd, const int32_t *bl_col,
                                   const void *bl_val, spmv_dtype val_dt, const void *x, void *y, spmv_dtype vec_dt,
                                   double alpha, double beta, const int32_t *tiles, int64_t n_tiles,
                                   const int64_t *h_plan, int32_t unroll, unsigned flags, void *stream)
{
    SPMV_REQUIRE(n >= 0 && n_tiles >= 0, "spmv_jds_blocked_tiled: negative size");
    SPMV_REQUIRE(C > 0 && C % 64 == 0, "spmv_jds_blocked_tiled: C must be a positive multiple of 64");
    SPMV_REQUIRE(n_slices == (int32_t)ceil_div(n, C), "spmv_jds_blocked_tiled: n_slices != ceil(n / C)");
    SPMV_REQUIRE(valid_dtype(val_dt) && valid_vec_dtype(vec_dt), "spmv_jds_blocked_tiled: bad dtype");
    SPMV_REQUIRE(unroll_ok(unroll), "spmv_jds_blocked_tiled: unroll must be 0, 2, 4 or 8");
    SPMV_REQUIRE((flags & ~(SPMV_SYMPERM | SPMV_SOJDS)) == 0, "spmv_jds_blocked_tiled: unknown flag");
    TileBounds xb;
    int64_t widest = 0;
    spmv_status st = check_tile_plan(h_plan, n_tiles, xb, &widest,
                                     "spmv_jds_blocked_tiled: h_plan bounds or wavefront count invalid");
    if (st != SPMV_OK) return st;
    if (n == 0 || n_tiles == 0) return SPMV_OK;
    // bl_col, bl_val and x are read only where a slice has diagonals (they may
    // be null for storage without entries)
    SPMV_REQUIRE(y && slice_ptr && slice_nd && tiles, "spmv_jds_blocked_tiled: null pointer");
    SPMV_REQUIRE((flags & SPMV_SYMPERM) || perm, "spmv_jds_blocked_tiled: null perm");
    JdsArgs a{};
    a.n = n;
    a.perm = perm;
    a.C = C;
    a.slice_ptr = slice_ptr;
    a.slice_nd = slice_nd;
    a.col = bl_col;
    a.val = bl_val;
    a.x = x;
    a.y = y;
    a.alpha = alpha;
    a.beta = beta;
    a.symperm = (flags & SPMV_SYMPERM) ? 1 : 0;
    return launch_tiles<FMT_BLOCKED>(a, tiles, xb, widest, h_plan[9], unroll, val_dt, vec_dt, as_stream(stream),
                                     "spmv_jds_blocked_tiled");
}

spmv_status spmv_jds_tiled(int32_t n, const int32_t *perm, const int32_t *jd_ptr, int32_t ndiag, const int32_t *jd_col,
                           const void *jd_val, spmv_dtype val_dt, const void *x, void *y, spmv_dtype vec_dt,
                           double alpha, double beta, const int32_t *tiles, int64_t n_tiles, const int64_t *h_plan,
                           int32_t unroll, unsigned flags, void *stream)
{
    SPMV_REQUIRE(n >= 0 && ndiag >= 0 && n_tiles >= 0, "spmv_jds_tiled: negative size");
    SPMV_REQUIRE(valid_dtype(val_dt) && valid_vec_dtype(vec_dt), "spmv_jds_tiled: bad dtype");
    SPMV_REQUIRE(unroll_ok(unroll), "spmv_jds_tiled: unroll must be 0, 2, 4 or 8");
    SPMV_REQUIRE((flags & ~SPMV_SYMPERM) == 0, "spmv_jds_tiled: unknown flag");
    TileBounds xb;
    int64_t widest = 0;
    spmv_status st = check_tile_plan(h_plan, n_tiles, xb, &widest,
                                     "spmv_jds_tiled: h_plan bounds or wavefront count invalid");
    if (st != SPMV_OK) return st;
    if (n == 0 || n_tiles == 0) return SPMV_OK;
    SPMV_REQUIRE(y && jd_ptr && tiles, "spmv_jds_tiled: null y, jd_ptr or tiles");
    SPMV_REQUIRE((flags & SPMV_SYMPERM) || perm, "spmv_jds_tiled: null perm");
    SPMV_REQUIRE(ndiag == 0 || (jd_col && jd_val && x), "spmv_jds_tiled: null col, val or x");
    JdsArgs a{};
    a.n = n;
    a.perm = perm;
    a.jd_ptr = jd_ptr;
    a.ndiag = ndiag;
    a.C = 64;
    a.col = jd_col;
    a.val = jd_val;
    a.x = x;
    a.y = y;
    a.alpha = alpha;
    a.beta = beta;
    a.symperm = (flags & SPMV_SYMPERM) ? 1 : 0;
    return launch_tiles<FMT_JDS>(a, tiles, xb, widest, h_plan[9], unroll, val_dt, vec_dt, as_stream(stream),
                                 "spmv_jds_tiled");
}

}  // extern "C"

// Multi-vector JDS straight from the column-major X (no workspace); called by
// spmm_jds, which validated the arguments.
spmv_status spmv::spmm_jds_colmajor(int32_t n, const int32_t *perm, const int32_t *jd_ptr, int32_t ndiag,
                                    const int32_t *jd_col, const void *jd_val, spmv_dtype val_dt, int32_t k,
                                    const void *X, int64_t ldx, void *Y, int64_t ldy, spmv_dtype vec_dt,
                                    double alpha, double beta, unsigned flags, hipStream_t s)
{
    JdsArgs a{};
    a.n = n;
    a.perm = perm;
    a.jd_ptr = jd_ptr;
    a.ndiag = ndiag;
    a.col = jd_col;
    a.val = jd_val;
    a.x = X;
    a.y = Y;
    a.ldx = ldx;
    a.ldy = ldy;
    a.k = k;
    a.alpha = alpha;
    a.beta = beta;
    a.symperm = (flags & SPMV_SYMPERM) ? 1 : 0;
    constexpr int KB = 8;
    dim3 grid((unsigned)ceil_div(n, 256), (unsigned)ceil_div(k, KB));
#define SPMM_CASE(VDT, VT, XDT, XT)                                           \
    if (val_dt == VDT && vec_dt == XDT) {                                     \
        spmm_jds_kernel<KB, VT, XT><<<grid, 256, 0, s>>>(a);                  \
        SPMV_CHECK_LAUNCH("spmm_jds");                                        \
        return SPMV_OK;                                                       \
    }
    SPMM_CASE(SPMV_F64, double, SPMV_F64, double)
    SPMM_CASE(SPMV_F32, float, SPMV_F32, float)
    SPMM_CASE(SPMV_F32, float, SPMV_F64, double)
    SPMM_CASE(SPMV_BF16, bf16, SPMV_F32, float)
    SPMM_CASE(SPMV_BF16, bf16, SPMV_F64, double)
    SPMM_CASE(SPMV_F64, double, SPMV_F32, float)
#undef SPMM_CASE
    return fail(SPMV_ERR_UNSUPPORTED, "spmm_jds: dtype combination");
}

extern "C" {

spmv_status spmv_grad_vals_jds(int32_t n, const int32_t *perm, const int32_t *jd_ptr, const int32_t *h_jd_ptr,
                               int32_t ndiag, int64_t nnz, const int32_t *jd_col, const void *g, const void *x,
                               void *dval, spmv_dtype dt, double alpha, double beta, unsigned flags, void *stream)
{
    SPMV_REQUIRE(n >= 0 && ndiag >= 0 && nnz >= 0, "spmv_grad_vals_jds: negative size");
    SPMV_REQUIRE(valid_vec_dtype(dt), "spmv_grad_vals_jds: dtype must be F64 or F32");
    SPMV_REQUIRE((flags & ~SPMV_SYMPERM) == 0, "spmv_grad_vals_jds: unknown flag");
    if (nnz == 0) return SPMV_OK;
    SPMV_REQUIRE(ndiag > 0 && jd_ptr && h_jd_ptr && jd_col && g && x && dval, "spmv_grad_vals_jds: null pointer");
    SPMV_REQUIRE((flags & SPMV_SYMPERM) || perm, "spmv_grad_vals_jds: null perm");
    SPMV_REQUIRE(h_jd_ptr[0] == 0 && (int64_t)h_jd_ptr[ndiag] == nnz, "spmv_grad_vals_jds: nnz != jd_ptr[ndiag]");
    JdsArgs a{};
    a.n = n;
    a.perm = perm;
    a.jd_ptr = jd_ptr;
    a.ndiag = ndiag;
    a.col = jd_col;
    a.x = x;
    a.g = g;
    a.dval = dval;
    a.alpha = alpha;
    a.beta = beta;
    a.symperm = (flags & SPMV_SYMPERM) ? 1 : 0;
    const JdsPlan P = plan_jds(n, h_jd_ptr, ndiag, JDS_DEFAULT_MAX_ITERS, -1);
    if (P.ncls == 0) return SPMV_OK;
    const unsigned grid = (unsigned)P.c[P.ncls - 1].wg_end;
    hipStream_t s = as_stream(stream);
    if (dt == SPMV_F64)
        jds_grad_kernel<4, double><<<grid, P.waves * WAVE, 0, s>>>(a, P);
    else
        jds_grad_kernel<4, float><<<grid, P.waves * WAVE, 0, s>>>(a, P);
    SPMV_CHECK_LAUNCH("spmv_grad_vals_jds");
    return SPMV_OK;
}

// Rows of part k: h_row_off[k+1] - h_row_off[k]; the slots hold h_row_off[8].
static spmv_status split_rows_ok(int32_t n, const int32_t *slot_ptr, const int64_t *h_row_off, const char *who)
{
    if (!slot_ptr || !h_row_off) return fail(SPMV_ERR_INVALID_ARG, std::string(who) + ": null slot_ptr or h_row_off");
    for (int k = 0; k < SPLIT_PARTS; ++k)
        if (h_row_off[k] < 0 || h_row_off[k + 1] < h_row_off[k] || h_row_off[k + 1] - h_row_off[k] > n)
            return fail(SPMV_ERR_INVALID_ARG, std::string(who) + ": bad h_row_off");
    if (h_row_off[SPLIT_PARTS] > (int64_t)SPLIT_PARTS * n)
        return fail(SPMV_ERR_INVALID_ARG, std::string(who) + ": bad h_row_off");
    return SPMV_OK;
}

spmv_status spmv_jds_split(int32_t n, const int32_t *slot_ptr, const int64_t *h_row_off, const int32_t *const *h_perm,
                           const int32_t *const *h_jd_ptr, const int32_t *const *h_jd_ptr_host, const int32_t *h_ndiag,
                           const int32_t *const *h_jd_col, const void *const *h_jd_val, spmv_dtype val_dt,
                           const void *x, void *y, spmv_dtype vec_dt, double alpha, double beta, int32_t unroll,
                           int32_t max_iters, int32_t wg_waves, void *ws, size_t ws_bytes, void *stream)
{
    SPMV_REQUIRE(n >= 0, "spmv_jds_split: n < 0");
    SPMV_REQUIRE(waves_ok(wg_waves), "spmv_jds_split: wg_waves must be 0, 4, 8 or 16");
    const int waves = waves_or_default(wg_waves);
    SPMV_REQUIRE(valid_dtype(val_dt) && valid_vec_dtype(vec_dt), "spmv_jds_split: bad dtype");
    SPMV_REQUIRE(unroll_ok(unroll) && max_iters >= 0, "spmv_jds_split: bad unroll or max_iters");
    if (n == 0) return SPMV_OK;
    SPMV_REQUIRE(h_perm && h_jd_ptr && h_jd_ptr_host && h_ndiag && h_jd_col && h_jd_val && y,
                 "spmv_jds_split: null pointer");
    spmv_status st = split_rows_ok(n, slot_ptr, h_row_off, "spmv_jds_split");
    if (st != SPMV_OK) return st;
    SPMV_REQUIRE(ws && ws_bytes >= spmv_split_workspace_size(h_row_off[SPLIT_PARTS]),
                 "spmv_jds_split: workspace too small");
    JdsSplitArgs S{};
    double *slots = (double *)ws;
    int64_t max_wg = 0;
    for (int k = 0; k < SPLIT_PARTS; ++k) {
        const int32_t nk = (int32_t)(h_row_off[k + 1] - h_row_off[k]);
        JdsArgs &a = S.a[k];
        if (nk == 0) continue;                 // S.P[k].ncls == 0: no workgroup of part k does anything
        SPMV_REQUIRE(x, "spmv_jds_split: null x");
        SPMV_REQUIRE(h_perm[k] && h_jd_ptr[k] && h_jd_ptr_host[k] && h_ndiag[k] >= 0, "spmv_jds_split: null part");
        SPMV_REQUIRE(h_ndiag[k] == 0 || (h_jd_col[k] && h_jd_val[k]), "spmv_jds_split: null part arrays");
        a.n = nk;
        a.perm = h_perm[k];
        a.jd_ptr = h_jd_ptr[k];
        a.ndiag = h_ndiag[k];
        a.C = 64;
        a.col = h_jd_col[k];
        a.val = h_jd_val[k];
        a.x = x;
        a.y = slots;                           // perm maps part rows to their slots
        a.alpha = 1.0;
        a.beta = 0.0;
        S.P[k] = plan_jds(nk, h_jd_ptr_host[k], h_ndiag[k], max_iters ? max_iters : JDS_DEFAULT_MAX_ITERS, -1,
                          waves);
        if (S.P[k].ncls) max_wg = std::max<int64_t>(max_wg, S.P[k].c[S.P[k].ncls - 1].wg_end);
    }
    hipStream_t s = as_stream(stream);
    const unsigned grid = (unsigned)(max_wg * SPLIT_PARTS);
    const unsigned threads = (unsigned)(waves * WAVE);
    if (grid) {
        const int u = unroll ? unroll : 4;
#define JSPLIT_CASE(VDT, VT, XDT, XT)                                                              \
    if (val_dt == VDT && vec_dt == XDT) {                                                          \
        if (u == 2) jds_split_kernel<FMT_JDS, 2, VT, XT><<<grid, threads, 0, s>>>(S);          \
        else if (u == 8) jds_split_kernel<FMT_JDS, 8, VT, XT><<<grid, threads, 0, s>>>(S);     \
        else jds_split_kernel<FMT_JDS, 4, VT, XT><<<grid, threads, 0, s>>>(S);                 \
    } else
        JSPLIT_CASE(SPMV_F64, double, SPMV_F64, double)
        JSPLIT_CASE(SPMV_F32, float, SPMV_F64, double)
        JSPLIT_CASE(SPMV_BF16, bf16, SPMV_F64, double)
        JSPLIT_CASE(SPMV_F32, float, SPMV_F32, float)
        JSPLIT_CASE(SPMV_BF16, bf16, SPMV_F32, float)
        JSPLIT_CASE(SPMV_F64, double, SPMV_F32, float)
        return fail(SPMV_ERR_UNSUPPORTED, "spmv_jds_split: dtype combination");
#undef JSPLIT_CASE
        SPMV_CHECK_LAUNCH("spmv_jds_split");
    }
    return launch_combine(n, slot_ptr, slots, y, vec_dt, alpha, beta, s);
}

spmv_status spmv_jds_blocked_split(int32_t n, int32_t C, const int32_t *slot_ptr, const int64_t *h_row_off,
                                   const int32_t *const *h_perm, const int64_t *const *h_slice_ptr,
                                   const int32_t *const *h_slice_nd, const int32_t *const *h_slice_nd_host,
                                   const int32_t *const *h_bl_col, const void *const *h_bl_val, spmv_dtype val_dt,
                                   const void *x, void *y, spmv_dtype vec_dt, double alpha, double beta,
                                   int32_t rows_per_wave, int32_t unroll, int32_t max_iters, int32_t wg_waves,
                                   void *ws, size_t ws_bytes, void *stream)
{
    SPMV_REQUIRE(n >= 0, "spmv_jds_blocked_split: n < 0");
    SPMV_REQUIRE(waves_ok(wg_waves), "spmv_jds_blocked_split: wg_waves must be 0, 4, 8 or 16");
    const int waves = waves_or_default(wg_waves);
    SPMV_REQUIRE(C > 0 && C % 64 == 0, "spmv_jds_blocked_split: C must be a positive multiple of 64");
    SPMV_REQUIRE(valid_dtype(val_dt) && valid_vec_dtype(vec_dt), "spmv_jds_blocked_split: bad dtype");
    SPMV_REQUIRE(unroll_ok(unroll) && max_iters >= 0, "spmv_jds_blocked_split: bad unroll or max_iters");
    SPMV_REQUIRE(rows_per_wave == 0 || rows_per_wave == 8 || rows_per_wave == 16 || rows_per_wave == 32 ||
                     rows_per_wave == 64,
                 "spmv_jds_blocked_split: rows_per_wave must be 0, 8, 16, 32 or 64");
    if (n == 0) return SPMV_OK;
    SPMV_REQUIRE(h_perm && h_slice_ptr && h_slice_nd && h_slice_nd_host && h_bl_col && h_bl_val && y,
                 "spmv_jds_blocked_split: null pointer");
    spmv_status st = split_rows_ok(n, slot_ptr, h_row_off, "spmv_jds_blocked_split");
    if (st != SPMV_OK) return st;
    SPMV_REQUIRE(ws && ws_bytes >= spmv_split_workspace_size(h_row_off[SPLIT_PARTS]),
                 "spmv_jds_blocked_split: workspace too small");
    int forced = -1;
    if (rows_per_wave) {
        forced = 0;
        while ((1 << forced) < rows_per_wave) ++forced;
    }
    JdsSplitArgs S{};
    double *slots = (double *)ws;
    int64_t max_wg = 0;
    for (int k = 0; k < SPLIT_PARTS; ++k) {
        const int32_t nk = (int32_t)(h_row_off[k + 1] - h_row_off[k]);
        JdsArgs &a = S.a[k];
        if (nk == 0) continue;                 // S.P[k].ncls == 0: no workgroup of part k does anything
        SPMV_REQUIRE(x, "spmv_jds_blocked_split: null x");
        SPMV_REQUIRE(h_perm[k] && h_slice_ptr[k] && h_slice_nd[k] && h_slice_nd_host[k],
                     "spmv_jds_blocked_split: null part");
        SPMV_REQUIRE(h_slice_nd_host[k][0] == 0 || (h_bl_col[k] && h_bl_val[k]),
                     "spmv_jds_blocked_split: null part arrays");
        a.n = nk;
        a.perm = h_perm[k];
        a.C = C;
        a.slice_ptr = h_slice_ptr[k];
        a.slice_nd = h_slice_nd[k];
        a.col = h_bl_col[k];
        a.val = h_bl_val[k];
        a.x = x;
        a.y = slots;                           // perm maps part rows to their slots
        a.alpha = 1.0;
        a.beta = 0.0;
        S.P[k] = plan_blocked(nk, C, h_slice_nd_host[k], max_iters ? max_iters : JDS_DEFAULT_MAX_ITERS, forced,
                              waves);
        if (S.P[k].ncls) max_wg = std::max<int64_t>(max_wg, S.P[k].c[S.P[k].ncls - 1].wg_end);
    }
    hipStream_t s = as_stream(stream);
    const unsigned grid = (unsigned)(max_wg * SPLIT_PARTS);
    const unsigned threads = (unsigned)(waves * WAVE);
    if (grid) {
        const int u = unroll ? unroll : 4;
#define BSPLIT_CASE(VDT, VT, XDT, XT)                                                                  \
    if (val_dt == VDT && vec_dt == XDT) {                                                              \
        if (u == 2) jds_split_kernel<FMT_BLOCKED, 2, VT, XT><<<grid, threads, 0, s>>>(S);          \
        else if (u == 8) jds_split_kernel<FMT_BLOCKED, 8, VT, XT><<<grid, threads, 0, s>>>(S);     \
        else jds_split_kernel<FMT_BLOCKED, 4, VT, XT><<<grid, threads, 0, s>>>(S);                 \
    } else
        BSPLIT_CASE(SPMV_F64, double, SPMV_F64, double)
        BSPLIT_CASE(SPMV_F32, float, SPMV_F64, double)
        BSPLIT_CASE(SPMV_BF16, bf16, SPMV_F64, double)
        BSPLIT_CASE(SPMV_F32, float, SPMV_F32, float)
        BSPLIT_CASE(SPMV_BF16, bf16, SPMV_F32, float)
        BSPLIT_CASE(SPMV_F64, double, SPMV_F32, float)
        return fail(SPMV_ERR_UNSUPPORTED, "spmv_jds_blocked_split: dtype combination");
#undef BSPLIT_CASE
        SPMV_CHECK_LAUNCH("spmv_jds_blocked_split");
    }
    return launch_combine(n, slot_ptr, slots, y, vec_dt, alpha, beta, s);
}

spmv_status spmv_jds_row_split(int32_t n, const int64_t *h_bounds, const int32_t *const *h_perm,
                               const int32_t *const *h_jd_ptr, const int32_t *const *h_jd_ptr_host,
                               const int32_t *h_ndiag, const int32_t *const *h_jd_col, const void *const *h_jd_val,
                               spmv_dtype val_dt, const void *x, void *y, spmv_dtype vec_dt, double alpha,
                               double beta, int32_t unroll, int32_t max_iters, int32_t wg_waves, void *stream)
{
    SPMV_REQUIRE(n >= 0, "spmv_jds_row_split: n < 0");
    SPMV_REQUIRE(waves_ok(wg_waves), "spmv_jds_row_split: wg_waves must be 0, 4, 8 or 16");
    const int waves = waves_or_default(wg_waves);
    SPMV_REQUIRE(valid_dtype(val_dt) && valid_vec_dtype(vec_dt), "spmv_jds_row_split: bad dtype");
    SPMV_REQUIRE(unroll_ok(unroll) && max_iters >= 0, "spmv_jds_row_split: bad unroll or max_iters");
    spmv_status st = row_bounds_ok(n, h_bounds, "spmv_jds_row_split");
    if (st != SPMV_OK) return st;
    if (n == 0) return SPMV_OK;
    SPMV_REQUIRE(h_perm && h_jd_ptr && h_jd_ptr_host && h_ndiag && h_jd_col && h_jd_val && y,
                 "spmv_jds_row_split: null pointer");
    const size_t ysz = dtype_size(vec_dt);
    JdsSplitArgs S{};
    int64_t max_wg = 0;
    for (int k = 0; k < SPLIT_PARTS; ++k) {
        const int32_t nk = (int32_t)(h_bounds[k + 1] - h_bounds[k]);
        if (nk == 0) continue;                 // S.P[k].ncls == 0: no workgroup of part k does anything
        SPMV_REQUIRE(h_perm[k] && h_jd_ptr[k] && h_jd_ptr_host[k] && h_ndiag[k] >= 0,
                     "spmv_jds_row_split: null part");
        SPMV_REQUIRE(h_ndiag[k] == 0 || (h_jd_col[k] && h_jd_val[k] && x), "spmv_jds_row_split: null part arrays");
        JdsArgs &a = S.a[k];
        a.n = nk;
        a.perm = h_perm[k];
        a.jd_ptr = h_jd_ptr[k];
        a.ndiag = h_ndiag[k];
        a.C = 64;
        a.col = h_jd_col[k];
        a.val = h_jd_val[k];
        a.x = x;
        a.y = (char *)y + h_bounds[k] * ysz;
        a.alpha = alpha;
        a.beta = beta;
        S.P[k] = plan_jds(nk, h_jd_ptr_host[k], h_ndiag[k], max_iters ? max_iters : JDS_DEFAULT_MAX_ITERS, -1,
                          waves);
        if (S.P[k].ncls) max_wg = std::max<int64_t>(max_wg, S.P[k].c[S.P[k].ncls - 1].wg_end);
    }
    return launch_rows<FMT_JDS>(S, max_wg, unroll, waves, val_dt, vec_dt, as_stream(stream), "spmv_jds_row_split");
}

spmv_status spmv_jds_blocked_row_split(int32_t n, int32_t C, const int64_t *h_bounds, const int32_t *const *h_perm,
                                       const int64_t *const *h_slice_ptr, const int32_t *const *h_slice_nd,
                                       const int32_t *const *h_slice_nd_host, const int32_t *const *h_bl_col,
                                       const void *const *h_bl_val, spmv_dtype val_dt, const void *x, void *y,
                                       spmv_dtype vec_dt, double alpha, double beta, int32_t rows_per_wave,
                                       int32_t unroll, int32_t max_iters, int32_t wg_waves, void *stream)
{
    SPMV_REQUIRE(n >= 0, "spmv_jds_blocked_row_split: n < 0");
    SPMV_REQUIRE(waves_ok(wg_waves), "spmv_jds_blocked_row_split: wg_waves must be 0, 4, 8 or 16");
    const int waves = waves_or_default(wg_waves);
    SPMV_REQUIRE(C > 0 && C % 64 == 0, "spmv_jds_blocked_row_split: C must be a positive multiple of 64");
    SPMV_REQUIRE(valid_dtype(val_dt) && valid_vec_dtype(vec_dt), "spmv_jds_blocked_row_split: bad dtype");
    SPMV_REQUIRE(unroll_ok(unroll) && max_iters >= 0, "spmv_jds_blocked_row_split: bad unroll or max_iters");
    SPMV_REQUIRE(rows_per_wave == 0 || rows_per_wave == 8 || rows_per_wave == 16 || rows_per_wave == 32 ||
                     rows_per_wave == 64,
                 "spmv_jds_blocked_row_split: rows_per_wave must be 0, 8, 16, 32 or 64");
    spmv_status st = row_bounds_ok(n, h_bounds, "spmv_jds_blocked_row_split");
    if (st != SPMV_OK) return st;
    if (n == 0) return SPMV_OK;
    SPMV_REQUIRE(h_perm && h_slice_ptr && h_slice_nd && h_slice_nd_host && h_bl_col && h_bl_val && y,
                 "spmv_jds_blocked_row_split: null pointer");
    int forced = -1;
    if (rows_per_wave) {
        forced = 0;
        while ((1 << forced) < rows_per_wave) ++forced;
    }
    const size_t ysz = dtype_size(vec_dt);
    JdsSplitArgs S{};
    int64_t max_wg = 0;
    for (int k = 0; k < SPLIT_PARTS; ++k) {
        const int32_t nk = (int32_t)(h_bounds[k + 1] - h_bounds[k]);
        if (nk == 0) continue;                 // S.P[k].ncls == 0: no workgroup of part k does anything
        SPMV_REQUIRE(h_perm[k] && h_slice_ptr[k] && h_slice_nd[k] && h_slice_nd_host[k],
                     "spmv_jds_blocked_row_split: null part");
        SPMV_REQUIRE(h_slice_nd_host[k][0] == 0 || (h_bl_col[k] && h_bl_val[k] && x),
                     "spmv_jds_blocked_row_split: null part arrays");
        JdsArgs &a = S.a[k];
        a.n = nk;
        a.perm = h_perm[k];
        a.C = C;
        a.slice_ptr = h_slice_ptr[k];
        a.slice_nd = h_slice_nd[k];
        a.col = h_bl_col[k];
        a.val = h_bl_val[k];
        a.x = x;
        a.y = (char *)y + h_bounds[k] * ysz;
        a.alpha = alpha;
        a.beta = beta;
        S.P[k] = plan_blocked(nk, C, h_slice_nd_host[k], max_iters ? max_iters : JDS_DEFAULT_MAX_ITERS, forced,
                              waves);
        if (S.P[k].ncls) max_wg = std::max<int64_t>(max_wg, S.P[k].c[S.P[k].ncls - 1].wg_end);
    }
    return launch_rows<FMT_BLOCKED>(S, max_wg, unroll, waves, val_dt, vec_dt, as_stream(stream),
                                    "spmv_jds_blocked_row_split");
}

}  // extern "C"
