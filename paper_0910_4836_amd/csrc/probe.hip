// Access-pattern microbenchmark: the basic sparse vector operations of the
// paper's Section 4.1 (Table 1) on gfx950.  For i < n the kernel forms
//   ADD:  s += b[j(i)]            SCP:  s += a[i] * b[j(i)]
// with j(i) = k*i (k = 1: the dense PDADD / PDSCP; k > 1: constant stride,
// CSADD / CSSCP) or j(i) = ind[i] (indirect: constant stride ISADD / ISSCP,
// random strides IRADD / IRSCP, or any other index stream).  Every lane
// takes i, i + G, i + 2G, ... (G = the grid's lanes), so at k = 1 a wavefront
// reads 64 consecutive elements; eight updates per lane are in flight.  The
// sums end in part[w], one per workgroup, so nothing can be optimised away.
#include <algorithm>

#include "common.hpp"

namespace spmv {

constexpr int SP_THREADS = 256;
constexpr int SP_UNROLL = 8;

template <bool SCP, bool IND>
__global__ __launch_bounds__(SP_THREADS) void stride_probe_kernel(int64_t n, int64_t k, const double *__restrict__ a,
                                                                  const double *__restrict__ b,
                                                                  const int32_t *__restrict__ ind,
                                                                  double *__restrict__ part)
{
    __shared__ double red[SP_THREADS / WAVE];
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    double s = 0.0;
    for (; i + (SP_UNROLL - 1) * stride < n; i += SP_UNROLL * stride) {
        int64_t j[SP_UNROLL];
#pragma unroll
        for (int u = 0; u < SP_UNROLL; ++u)
            j[u] = IND ? (int64_t)__builtin_nontemporal_load(ind + i + u * stride) : (i + u * stride) * k;
        double v[SP_UNROLL], w[SP_UNROLL];
#pragma unroll
        for (int u = 0; u < SP_UNROLL; ++u) {
            v[u] = b[j[u]];
            w[u] = SCP ? __builtin_nontemporal_load(a + i + u * stride) : 1.0;
        }
#pragma unroll
        for (int u = 0; u < SP_UNROLL; ++u) s = SCP ? fma(w[u], v[u], s) : s + v[u];
    }
    for (; i < n; i += stride) {
        const int64_t j = IND ? (int64_t)ind[i] : i * k;
        s = SCP ? fma(a[i], b[j], s) : s + b[j];
    }
    s = group_sum(s, WAVE);
    if (lane_id() == 0) red[threadIdx.x / WAVE] = s;
    __syncthreads();
    if (threadIdx.x == 0) {
        double t = 0.0;
        for (int q = 0; q < SP_THREADS / WAVE; ++q) t += red[q];
        part[blockIdx.x] = t;
    }
}

}  // namespace spmv

using namespace spmv;

extern "C" {

spmv_status spmv_stride_probe(int64_t n, int32_t scp, const double *a, const double *b, const int32_t *ind, int64_t k,
                              double *part, int64_t part_cap, void *stream)
{
    SPMV_REQUIRE(n >= 0 && k >= 1, "spmv_stride_probe: n < 0 or k < 1");
    if (n == 0) return SPMV_OK;
    SPMV_REQUIRE(b && part && (!scp || a), "spmv_stride_probe: null array");
    int dev = 0, cus = 0;
    if (hipGetDevice(&dev) != hipSuccess ||
        hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || cus <= 0)
        cus = 256;
    const int64_t grid = std::min<int64_t>((int64_t)cus * 8, ceil_div(n, SP_THREADS));
    SPMV_REQUIRE(part_cap >= grid, "spmv_stride_probe: part needs one double per workgroup (8 per CU)");
    hipStream_t s = as_stream(stream);
    const unsigned g = (unsigned)grid;
    if (scp) {
        if (ind) stride_probe_kernel<true, true><<<g, SP_THREADS, 0, s>>>(n, k, a, b, ind, part);
        else stride_probe_kernel<true, false><<<g, SP_THREADS, 0, s>>>(n, k, a, b, ind, part);
    } else {
        if (ind) stride_probe_kernel<false, true><<<g, SP_THREADS, 0, s>>>(n, k, a, b, ind, part);
        else stride_probe_kernel<false, false><<<g, SP_THREADS, 0, s>>>(n, k, a, b, ind, part);
    }
    SPMV_CHECK_LAUNCH("spmv_stride_probe");
    return SPMV_OK;
}

}  // extern "C"
