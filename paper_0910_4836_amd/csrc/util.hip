// Status strings, error plumbing, small vector kernels, HIP graph helpers and
// bandwidth probes.
#include <mutex>
#include <string>

#include "common.hpp"

namespace spmv {

static thread_local std::string g_last_error;

void set_error(const std::string &msg) { g_last_error = msg; }

spmv_status fail(spmv_status s, const std::string &msg)
{
    g_last_error = msg;
    return s;
}

spmv_status hip_fail(hipError_t e, const char *what)
{
    g_last_error = std::string(what) + ": " + hipGetErrorString(e);
    return SPMV_ERR_HIP;
}

int device_cus()
{
    static std::mutex mu;
    static int cached[64] = {};
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= 64) return 256;
    std::lock_guard<std::mutex> lock(mu);
    if (cached[dev] == 0) {
        int cus = 0;
        if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || cus <= 0)
            cus = 256;
        cached[dev] = cus;
    }
    return cached[dev];
}

// ---------------------------------------------------------------- kernels

template <typename T>
__global__ void axpby_kernel(int64_t n, double alpha, const T *__restrict__ x, double beta, T *__restrict__ y)
{
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (; i < n; i += stride) {
        double r = alpha != 0.0 ? alpha * to_f64(x[i]) : 0.0;   // alpha == 0 never reads x
        if (beta != 0.0) r = fma(beta, to_f64(y[i]), r);
        store_from_f64(&y[i], r);
    }
}

// Dot product in FP64: each block reduces a fixed contiguous chunk with a
// fixed tree, then one block adds the block partials in order.
constexpr int DOT_THREADS = 256;
constexpr int DOT_CHUNK = DOT_THREADS * 16;

template <typename T>
__global__ __launch_bounds__(DOT_THREADS) void dot_partial_kernel(int64_t n, const T *__restrict__ x,
                                                                  const T *__restrict__ y,
                                                                  double *__restrict__ part)
{
    __shared__ double red[DOT_THREADS / WAVE];
    int64_t base = (int64_t)blockIdx.x * DOT_CHUNK;
    double s = 0.0;
    for (int k = 0; k < DOT_CHUNK / DOT_THREADS; ++k) {
        int64_t i = base + (int64_t)k * DOT_THREADS + threadIdx.x;
        if (i < n) s = fma(to_f64(x[i]), to_f64(y[i]), s);
    }
    s = group_sum(s, WAVE);
    if (lane_id() == 0) red[threadIdx.x / WAVE] = s;
    __syncthreads();
    if (threadIdx.x == 0) {
        double t = 0.0;
        for (int w = 0; w < DOT_THREADS / WAVE; ++w) t += red[w];
        part[blockIdx.x] = t;
    }
}

__global__ __launch_bounds__(DOT_THREADS) void dot_final_kernel(int64_t nparts, const double *__restrict__ part,
                                                                double *__restrict__ out)
{
    __shared__ double red[DOT_THREADS / WAVE];
    double s = 0.0;
    for (int64_t i = threadIdx.x; i < nparts; i += DOT_THREADS) s += part[i];
    s = group_sum(s, WAVE);
    if (lane_id() == 0) red[threadIdx.x / WAVE] = s;
    __syncthreads();
    if (threadIdx.x == 0) {
        double t = 0.0;
        for (int w = 0; w < DOT_THREADS / WAVE; ++w) t += red[w];
        *out = t;
    }
}

// Bandwidth probes: 16-byte accesses, four independent ones in flight per
// lane, grid-stride over 16-byte units (the host checks that n is even and
// the arrays 16-byte aligned).
constexpr int PROBE_UNROLL = 4;
typedef double v2d __attribute__((ext_vector_type(2)));

__global__ void triad_kernel(int64_t n2, const v2d *__restrict__ b, const v2d *__restrict__ c,
                             v2d *__restrict__ a, double s)
{
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    for (; i + (PROBE_UNROLL - 1) * stride < n2; i += PROBE_UNROLL * stride) {
        v2d bb[PROBE_UNROLL], cc[PROBE_UNROLL];
#pragma unroll
        for (int u = 0; u < PROBE_UNROLL; ++u) {
            bb[u] = __builtin_nontemporal_load(b + i + u * stride);
            cc[u] = __builtin_nontemporal_load(c + i + u * stride);
        }
#pragma unroll
        for (int u = 0; u < PROBE_UNROLL; ++u) {
            const v2d r = {fma(s, cc[u].x, bb[u].x), fma(s, cc[u].y, bb[u].y)};
            __builtin_nontemporal_store(r, a + i + u * stride);
        }
    }
    for (; i < n2; i += stride) {
        const v2d r = {fma(s, c[i].x, b[i].x), fma(s, c[i].y, b[i].y)};
        a[i] = r;
    }
}

__global__ void copy_kernel(int64_t n2, const v2d *__restrict__ b, v2d *__restrict__ a)
{
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    for (; i + (PROBE_UNROLL - 1) * stride < n2; i += PROBE_UNROLL * stride) {
        v2d bb[PROBE_UNROLL];
#pragma unroll
        for (int u = 0; u < PROBE_UNROLL; ++u) bb[u] = __builtin_nontemporal_load(b + i + u * stride);
#pragma unroll
        for (int u = 0; u < PROBE_UNROLL; ++u) __builtin_nontemporal_store(bb[u], a + i + u * stride);
    }
    for (; i < n2; i += stride) a[i] = b[i];
}

// Read-only probe: per-block partial sums (keeps the loads alive).
__global__ __launch_bounds__(256) void read_kernel(int64_t n2, const v2d *__restrict__ b,
                                                   double *__restrict__ part)
{
    __shared__ double red[256 / WAVE];
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    double s = 0.0;
    for (; i + (PROBE_UNROLL - 1) * stride < n2; i += PROBE_UNROLL * stride) {
        v2d bb[PROBE_UNROLL];
#pragma unroll
        for (int u = 0; u < PROBE_UNROLL; ++u) bb[u] = __builtin_nontemporal_load(b + i + u * stride);
#pragma unroll
        for (int u = 0; u < PROBE_UNROLL; ++u) s += bb[u].x + bb[u].y;
    }
    for (; i < n2; i += stride) s += b[i].x + b[i].y;
    s = group_sum(s, WAVE);
    if (lane_id() == 0) red[threadIdx.x / WAVE] = s;
    __syncthreads();
    if (threadIdx.x == 0) part[blockIdx.x] = red[0] + red[1] + red[2] + red[3];
}

// Gather probe: part[w] = sum over the indices read by workgroup w of x[idx[i]]
// (idx streamed, x gathered one 8-byte element per lane).  Measures how many
// random gathers per second the memory system serves for an x of a given size.
__global__ __launch_bounds__(256) void gather_probe_kernel(int64_t n, const int32_t *__restrict__ idx,
                                                           const double *__restrict__ x, double *__restrict__ part)
{
    __shared__ double red[256 / WAVE];
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    double s = 0.0;
    for (; i + (PROBE_UNROLL - 1) * stride < n; i += PROBE_UNROLL * stride) {
        int32_t c[PROBE_UNROLL];
#pragma unroll
        for (int u = 0; u < PROBE_UNROLL; ++u) c[u] = __builtin_nontemporal_load(idx + i + u * stride);
        double v[PROBE_UNROLL];
#pragma unroll
        for (int u = 0; u < PROBE_UNROLL; ++u) v[u] = x[c[u]];
#pragma unroll
        for (int u = 0; u < PROBE_UNROLL; ++u) s += v[u];
    }
    for (; i < n; i += stride) s += x[idx[i]];
    s = group_sum(s, WAVE);
    if (lane_id() == 0) red[threadIdx.x / WAVE] = s;
    __syncthreads();
    if (threadIdx.x == 0) part[blockIdx.x] = red[0] + red[1] + red[2] + red[3];
}

static int probe_grid()
{
    int dev = 0, cus = 0;
    if (hipGetDevice(&dev) != hipSuccess ||
        hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || cus <= 0)
        cus = 256;
    return cus * 8;
}

static int stream_grid(int64_t n, int per_thread)
{
    int64_t blocks = ceil_div(n, (int64_t)256 * per_thread);
    if (blocks > 256 * 64) blocks = 256 * 64;
    if (blocks < 1) blocks = 1;
    return (int)blocks;
}

static bool aligned16(const void *p) { return ((uintptr_t)p & 15u) == 0; }

// y_i = alpha * (sum of row i's slots, in slot order) + beta * y_i
// Each wavefront takes 64 consecutive rows, whose slots are one contiguous
// run of at most SPLIT_PARTS * 64: it loads the run into LDS with coalesced
// loads (eight per lane, all in flight), then each lane adds its row's slots
// in order, starting from 0.
template <typename T>
__global__ __launch_bounds__(256) void combine_kernel(int32_t n, const int32_t *__restrict__ slot_ptr,
                                                     const double *__restrict__ slots, T *__restrict__ y,
                                                     double alpha, double beta)
{
    constexpr int WAVES = 256 / WAVE;
    __shared__ double buf[WAVES][SPLIT_PARTS * WAVE];
    const int w = (int)threadIdx.x / WAVE, l = lane_id();
    const int64_t r0 = ((int64_t)blockIdx.x * WAVES + w) * WAVE;
    const int64_t i = r0 + l;
    int32_t s0 = 0, s1 = 0, base = 0, cnt = 0;
    if (r0 < n) {
        if (i < n) {
            s0 = slot_ptr[i];
            s1 = slot_ptr[i + 1];
        }
        base = slot_ptr[r0];
        cnt = slot_ptr[min(r0 + WAVE, (int64_t)n)] - base;       // <= SPLIT_PARTS * 64
    }
    if (cnt > 0) {
        double v[SPLIT_PARTS];
#pragma unroll
        for (int q = 0; q < SPLIT_PARTS; ++q)
            v[q] = __builtin_nontemporal_load(slots + base + min(l + q * WAVE, cnt - 1));
#pragma unroll
        for (int q = 0; q < SPLIT_PARTS; ++q)
            if (l + q * WAVE < cnt) buf[w][l + q * WAVE] = v[q];
    }
    __syncthreads();
    if (i < n) {
        double s = 0.0;
        for (int32_t k = s0 - base; k < s1 - base; ++k) s += buf[w][k];
        write_y(y, i, s, alpha, beta);
    }
}

spmv_status launch_combine(int32_t n, const int32_t *slot_ptr, const double *slots, void *y, spmv_dtype vec_dt,
                           double alpha, double beta, hipStream_t s)
{
    if (n == 0) return SPMV_OK;
    const int64_t grid = ceil_div(n, 256);
    if (vec_dt == SPMV_F64)
        combine_kernel<double><<<(unsigned)grid, 256, 0, s>>>(n, slot_ptr, slots, (double *)y, alpha, beta);
    else
        combine_kernel<float><<<(unsigned)grid, 256, 0, s>>>(n, slot_ptr, slots, (float *)y, alpha, beta);
    SPMV_CHECK_LAUNCH("split combine");
    return SPMV_OK;
}

}  // namespace spmv

using namespace spmv;

extern "C" {

const char *spmv_status_string(spmv_status s)
{
    switch (s) {
    case SPMV_OK: return "ok";
    case SPMV_ERR_INVALID_ARG: return "invalid argument";
    case SPMV_ERR_BAD_FORMAT: return "bad matrix format";
    case SPMV_ERR_CAPACITY: return "output capacity too small";
    case SPMV_ERR_UNSUPPORTED: return "unsupported";
    case SPMV_ERR_HIP: return "HIP runtime error";
    }
    return "unknown status";
}

const char *spmv_last_error(void) { return g_last_error.c_str(); }

const char *spmv_version(void) { return "1.0.0"; }

spmv_status spmv_axpby(int64_t n, double alpha, const void *x, double beta, void *y, spmv_dtype dt, void *stream)
{
    SPMV_REQUIRE(n >= 0, "spmv_axpby: n < 0");
    SPMV_REQUIRE(valid_vec_dtype(dt), "spmv_axpby: dtype must be F64 or F32");
    if (n == 0) return SPMV_OK;
    SPMV_REQUIRE(x && y, "spmv_axpby: null pointer");
    int grid = stream_grid(n, 4);
    if (dt == SPMV_F64)
        axpby_kernel<double><<<grid, 256, 0, as_stream(stream)>>>(n, alpha, (const double *)x, beta, (double *)y);
    else
        axpby_kernel<float><<<grid, 256, 0, as_stream(stream)>>>(n, alpha, (const float *)x, beta, (float *)y);
    SPMV_CHECK_LAUNCH("spmv_axpby");
    return SPMV_OK;
}

size_t spmv_split_workspace_size(int64_t n_slots)
{
    return (size_t)(n_slots > 0 ? n_slots : 1) * sizeof(double) + 256;
}

size_t spmv_dot_workspace_size(int64_t n)
{
    int64_t parts = n > 0 ? ceil_div(n, DOT_CHUNK) : 1;
    return (size_t)parts * sizeof(double);
}

spmv_status spmv_dot(int64_t n, const void *x, const void *y, spmv_dtype dt, double *out, void *ws, size_t ws_bytes,
                     void *stream)
{
    SPMV_REQUIRE(n >= 0, "spmv_dot: n < 0");
    SPMV_REQUIRE(valid_vec_dtype(dt), "spmv_dot: dtype must be F64 or F32");
    SPMV_REQUIRE(out, "spmv_dot: null output");
    SPMV_REQUIRE(ws && ws_bytes >= spmv_dot_workspace_size(n), "spmv_dot: workspace too small");
    SPMV_REQUIRE(n == 0 || (x && y), "spmv_dot: null input");
    int64_t parts = n > 0 ? ceil_div(n, DOT_CHUNK) : 0;
    double *part = (double *)ws;
    hipStream_t s = as_stream(stream);
    if (parts > 0) {
        if (dt == SPMV_F64)
            dot_partial_kernel<double><<<(unsigned)parts, DOT_THREADS, 0, s>>>(n, (const double *)x, (const double *)y, part);
        else
            dot_partial_kernel<float><<<(unsigned)parts, DOT_THREADS, 0, s>>>(n, (const float *)x, (const float *)y, part);
        SPMV_CHECK_LAUNCH("spmv_dot partial");
    }
    dot_final_kernel<<<1, DOT_THREADS, 0, s>>>(parts, part, out);
    SPMV_CHECK_LAUNCH("spmv_dot final");
    return SPMV_OK;
}

}  // extern "C"

namespace spmv {

// Scratch of spmv_dot_noalloc: the block partials of the dot product, one
// array per GPU for the life of the process.  Host code never passes the
// name `scratch` to a kernel (on the host it is only a stand-in for the
// symbol); it looks up the device address once per device and uses that.
static __device__ __align__(256) double scratch[SPMV_DOT_NOALLOC_PARTS];

namespace {
constexpr int MAX_DEVICES = 64;
std::mutex g_scratch_mu;
double *g_scratch_ptr[MAX_DEVICES] = {};
}  // namespace

// Device address of the current device's scratch array, looked up on the
// first call on that device (with that device current).
static spmv_status scratch_for_current_device(double **out)
{
    int dev = 0;
    SPMV_HIP(hipGetDevice(&dev));
    if (dev < 0 || dev >= MAX_DEVICES) return fail(SPMV_ERR_UNSUPPORTED, "spmv_dot_noalloc: device index >= 64");
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void *p = nullptr;
        SPMV_HIP(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
        if (!p) return fail(SPMV_ERR_HIP, "spmv_dot_noalloc: no device address for the scratch array");
        g_scratch_ptr[dev] = static_cast<double *>(p);
    }
    *out = g_scratch_ptr[dev];
    return SPMV_OK;
}

}  // namespace spmv

extern "C" {

spmv_status spmv_dot_noalloc(int64_t n, const void *x, const void *y, spmv_dtype dt, double *out, void *stream)
{
    SPMV_REQUIRE(n >= 0, "spmv_dot_noalloc: n < 0");
    if (n > SPMV_DOT_NOALLOC_MAX_N)
        return fail(SPMV_ERR_CAPACITY, "spmv_dot_noalloc: n > SPMV_DOT_NOALLOC_MAX_N (134,217,728); use spmv_dot "
                                       "with a workspace");
    SPMV_REQUIRE(valid_vec_dtype(dt), "spmv_dot_noalloc: dtype must be F64 or F32");
    SPMV_REQUIRE(out, "spmv_dot_noalloc: null output");
    SPMV_REQUIRE(n == 0 || (x && y), "spmv_dot_noalloc: null input");
    static_assert((int64_t)SPMV_DOT_NOALLOC_PARTS * DOT_CHUNK == SPMV_DOT_NOALLOC_MAX_N,
                  "the scratch array holds one partial per chunk of the largest input");
    double *part = nullptr;
    spmv_status st = scratch_for_current_device(&part);
    if (st != SPMV_OK) return st;
    // every partial the final kernel reads is written by this call's first
    // kernel, so nothing left by an earlier call is read
    const int64_t parts = n > 0 ? ceil_div(n, DOT_CHUNK) : 0;
    hipStream_t s = as_stream(stream);
    if (parts > 0) {
        if (dt == SPMV_F64)
            dot_partial_kernel<double><<<(unsigned)parts, DOT_THREADS, 0, s>>>(n, (const double *)x, (const double *)y, part);
        else
            dot_partial_kernel<float><<<(unsigned)parts, DOT_THREADS, 0, s>>>(n, (const float *)x, (const float *)y, part);
        SPMV_CHECK_LAUNCH("spmv_dot_noalloc partial");
    }
    dot_final_kernel<<<1, DOT_THREADS, 0, s>>>(parts, part, out);
    SPMV_CHECK_LAUNCH("spmv_dot_noalloc final");
    return SPMV_OK;
}

spmv_status spmv_graph_begin(void *stream)
{
    SPMV_REQUIRE(stream, "spmv_graph_begin: capture needs a non-default stream");
    SPMV_HIP(hipStreamBeginCapture(as_stream(stream), hipStreamCaptureModeThreadLocal));
    return SPMV_OK;
}

spmv_status spmv_graph_end(void *stream, void **h_exec)
{
    SPMV_REQUIRE(stream && h_exec, "spmv_graph_end: null argument");
    hipGraph_t graph = nullptr;
    SPMV_HIP(hipStreamEndCapture(as_stream(stream), &graph));
    hipGraphExec_t exec = nullptr;
    hipError_t e = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0);
    (void)hipGraphDestroy(graph);
    if (e != hipSuccess) return hip_fail(e, "hipGraphInstantiate");
    *h_exec = (void *)exec;
    return SPMV_OK;
}

spmv_status spmv_graph_launch(void *exec, void *stream)
{
    SPMV_REQUIRE(exec, "spmv_graph_launch: null graph");
    SPMV_HIP(hipGraphLaunch((hipGraphExec_t)exec, as_stream(stream)));
    return SPMV_OK;
}

spmv_status spmv_graph_destroy(void *exec)
{
    if (exec) SPMV_HIP(hipGraphExecDestroy((hipGraphExec_t)exec));
    return SPMV_OK;
}

spmv_status spmv_stream_triad(int64_t n, const double *b, const double *c, double *a, double s, void *stream)
{
    SPMV_REQUIRE(n >= 0 && (n == 0 || (a && b && c)), "spmv_stream_triad: bad arguments");
    SPMV_REQUIRE(n % 2 == 0 && aligned16(a) && aligned16(b) && aligned16(c),
                 "spmv_stream_triad: n must be even and the arrays 16-byte aligned");
    if (n == 0) return SPMV_OK;
    triad_kernel<<<probe_grid(), 256, 0, as_stream(stream)>>>(n / 2, (const v2d *)b, (const v2d *)c,
                                                              (v2d *)a, s);
    SPMV_CHECK_LAUNCH("spmv_stream_triad");
    return SPMV_OK;
}

spmv_status spmv_stream_copy(int64_t n, const double *b, double *a, void *stream)
{
    SPMV_REQUIRE(n >= 0 && (n == 0 || (a && b)), "spmv_stream_copy: bad arguments");
    SPMV_REQUIRE(n % 2 == 0 && aligned16(a) && aligned16(b),
                 "spmv_stream_copy: n must be even and the arrays 16-byte aligned");
    if (n == 0) return SPMV_OK;
    copy_kernel<<<probe_grid(), 256, 0, as_stream(stream)>>>(n / 2, (const v2d *)b, (v2d *)a);
    SPMV_CHECK_LAUNCH("spmv_stream_copy");
    return SPMV_OK;
}

spmv_status spmv_stream_read(int64_t n, const double *b, double *part, int64_t part_cap, void *stream)
{
    SPMV_REQUIRE(n >= 0 && (n == 0 || (b && part)), "spmv_stream_read: bad arguments");
    SPMV_REQUIRE(n % 2 == 0 && aligned16(b), "spmv_stream_read: n must be even and b 16-byte aligned");
    if (n == 0) return SPMV_OK;
    const int grid = probe_grid();
    SPMV_REQUIRE(part_cap >= grid, "spmv_stream_read: part needs one double per workgroup (8 per CU)");
    read_kernel<<<grid, 256, 0, as_stream(stream)>>>(n / 2, (const v2d *)b, part);
    SPMV_CHECK_LAUNCH("spmv_stream_read");
    return SPMV_OK;
}

spmv_status spmv_gather_probe(int64_t n, const int32_t *idx, const double *x, double *part, int64_t part_cap,
                              void *stream)
{
    SPMV_REQUIRE(n >= 0 && (n == 0 || (idx && x && part)), "spmv_gather_probe: bad arguments");
    if (n == 0) return SPMV_OK;
    const int grid = probe_grid();
    SPMV_REQUIRE(part_cap >= grid, "spmv_gather_probe: part needs one double per workgroup (8 per CU)");
    gather_probe_kernel<<<grid, 256, 0, as_stream(stream)>>>(n, idx, x, part);
    SPMV_CHECK_LAUNCH("spmv_gather_probe");
    return SPMV_OK;
}

}  // extern "C"
