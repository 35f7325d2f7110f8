// Region sums of per-point values (the shadow area of Sec. 7.2, with each
// point standing for area[p] square metres), accumulated in FP64.
#include <hip/hip_runtime.h>

#include "sa_internal.h"

namespace sa {
namespace {

constexpr int kThreads = 256;

// One block per region; wave reductions with cross-lane moves, then LDS.
__global__ __launch_bounds__(kThreads) void k_region_sum(const float *__restrict__ v,
                                                         const int64_t *__restrict__ off,
                                                         const float *__restrict__ area, double *__restrict__ out)
{
    __shared__ double part[kThreads / 64];
    const int r = blockIdx.x;
    const int64_t lo = off[r], hi = off[r + 1];
    double s = 0.0;
    for (int64_t i = lo + threadIdx.x; i < hi; i += kThreads) s += (double)v[i] * (area ? (double)area[i] : 1.0);
    for (int o = 32; o > 0; o >>= 1) s += __shfl_down(s, o, 64);
    if ((threadIdx.x & 63) == 0) part[threadIdx.x >> 6] = s;
    __syncthreads();
    if (threadIdx.x == 0) {
        double t = 0.0;
        for (int w = 0; w < kThreads / 64; ++w) t += part[w];
        out[r] = t;
    }
}

}  // namespace

sa_status launch_region_sum(const float *v, int64_t n, const int64_t *off, int32_t n_reg, const float *area,
                            double *out, hipStream_t st, std::string &err)
{
    (void)n;
    hipLaunchKernelGGL(k_region_sum, dim3(n_reg), dim3(kThreads), 0, st, v, off, area, out);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) {
        err = std::string("region sum: ") + hipGetErrorString(e);
        return SA_ERR_DEVICE;
    }
    return SA_OK;
}

sa_status launch_grad(const DeviceScene &, const DevicePath &, const PointsView &, const float *, float *,
                      hipStream_t, std::string &err)
{
    err = "not built yet";
    return SA_ERR_UNSUPPORTED;
}

sa_status launch_batched(const DeviceScene &, const DevicePath &, int32_t, int32_t, const int32_t *, const float *,
                         const PointsView &, const int64_t *, float, int32_t *, float *, SpillQueue &, Scratch &,
                         hipStream_t, std::string &err)
{
    err = "not built yet";
    return SA_ERR_UNSUPPORTED;
}

}  // namespace sa
