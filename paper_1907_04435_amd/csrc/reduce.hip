// Region sums of per-point values (the shadow area of Sec. 7.2, with each
// point standing for area[p] square metres) and their bin-weighted form
// (the shadow score of Sec. 7.2), accumulated in FP64.
#include <hip/hip_runtime.h>

#include "sa_internal.h"

namespace sa {
namespace {

constexpr int kThreads = 256;
constexpr int kBlocksPerRegion = 128;

// Phase 1: block b of region r sums a strided share of the region into
// part[r * kBlocksPerRegion + b] (wave reductions with cross-lane moves,
// then LDS).  Phase 2 adds each region's partials in a fixed order, so the
// result does not depend on scheduling.  With bin weights, a point's value
// is the weighted sum of its bins' values (bin-major, stride n).
__global__ __launch_bounds__(kThreads) void k_region_part(const float *__restrict__ v, int n_bins, int64_t n,
                                                          const double *__restrict__ bin_w,
                                                          const int64_t *__restrict__ off,
                                                          const float *__restrict__ area, double *__restrict__ part)
{
    __shared__ double red[kThreads / 64];
    const int r = wg_id_y();
    const int64_t lo = off[r], hi = off[r + 1];
    double s = 0.0;
    for (int64_t i = lo + (int64_t)wg_id() * kThreads + tid(); i < hi;
         i += (int64_t)kBlocksPerRegion * kThreads) {
        double x;
        if (bin_w) {
            x = 0.0;
            for (int b = 0; b < n_bins; ++b) x += bin_w[b] * (double)v[(int64_t)b * n + i];
        } else {
            x = (double)v[i];
        }
        s += x * (area ? (double)area[i] : 1.0);
    }
    for (int o = 32; o > 0; o >>= 1) s += __shfl_down(s, o, 64);
    if ((tid() & 63) == 0) red[tid() >> 6] = s;
    __syncthreads();
    if (tid() == 0) {
        double t = 0.0;
        for (int w = 0; w < kThreads / 64; ++w) t += red[w];
        part[(int64_t)r * kBlocksPerRegion + wg_id()] = t;
    }
}

__global__ __launch_bounds__(64) void k_region_final(int n_reg, const double *__restrict__ part,
                                                     double *__restrict__ out)
{
    const int r = wg_id() * 64 + tid();
    if (r >= n_reg) return;
    double t = 0.0;
    for (int b = 0; b < kBlocksPerRegion; ++b) t += part[(int64_t)r * kBlocksPerRegion + b];
    out[r] = t;
}

}  // namespace

sa_status launch_region_sum(const float *v, int n_bins, int64_t n, const double *bin_w, const int64_t *off,
                            int32_t n_reg, const float *area, double *out, Scratch &scr, hipStream_t st,
                            std::string &err)
{
    const size_t need = sizeof(double) * (size_t)n_reg * kBlocksPerRegion;
    if (scr.bytes < need) {
        (void)hipStreamSynchronize(st);
        (void)hipFree(scr.ptr);
        scr.ptr = nullptr;
        scr.bytes = 0;
        if (hipMalloc(&scr.ptr, need) != hipSuccess) {
            err = "region sum scratch allocation failed";
            return SA_ERR_OOM;
        }
        scr.bytes = need;
    }
    double *part = (double *)scr.ptr;
    hipLaunchKernelGGL(k_region_part, dim3(kBlocksPerRegion, n_reg), dim3(kThreads), 0, st, v, n_bins, n, bin_w, off,
                       area, part);
    hipLaunchKernelGGL(k_region_final, dim3((n_reg + 63) / 64), dim3(64), 0, st, n_reg, (const double *)part, out);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) {
        err = std::string("region sum: ") + hipGetErrorString(e);
        return SA_ERR_DEVICE;
    }
    return SA_OK;
}

}  // namespace sa
