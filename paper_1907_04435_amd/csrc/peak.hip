// Measurement aid for the roofline, not a step of the method: the vector
// ALU's lane-op rate on this device, from chains of FP32 fused multiply-adds
// that do not depend on each other (one VALU operation per lane each; this
// library is built without packed FP32, so none is fused in pairs).  The
// derived peak is 256 CU x 64 lanes x 2.4 GHz; this measures what the part
// sustains under load.
#include <hip/hip_runtime.h>

#include <algorithm>

#include "sa_internal.h"

namespace sa {
namespace {

constexpr int kPeakThreads = 256;
constexpr int kChains = 8;  // independent FMA chains per lane: enough to hide the FMA latency

__global__ __launch_bounds__(kPeakThreads) void k_valu_peak(float *sink, int iters, float a, float b)
{
    float x[kChains];
#pragma unroll
    for (int c = 0; c < kChains; ++c) x[c] = (float)(tid() + c) * 1e-3f;
    for (int i = 0; i < iters; ++i) {
#pragma unroll
        for (int c = 0; c < kChains; ++c) x[c] = fmaf(x[c], a, b);
    }
    float s = 0.f;
#pragma unroll
    for (int c = 0; c < kChains; ++c) s += x[c];
    // with 0 < a < 1 and b > 0 every chain stays positive: never stored,
    // but the compiler cannot drop the chains
    if (s < 0.f) sink[wg_id()] = s;
}

}  // namespace

sa_status measure_valu_peak(int n_cu, float *sink, int64_t sink_floats, hipStream_t st, double &lane_ops_per_s,
                            std::string &err)
{
    // 32 waves per CU at once (8 per SIMD), four rounds of them
    const int64_t blocks = (int64_t)std::max(n_cu, 1) * 8 * 4;
    const int iters = 4096;
    if (blocks > sink_floats) {
        err = "peak measurement: sink too small";
        return SA_ERR_INVALID_ARG;
    }
    hipEvent_t e0 = nullptr, e1 = nullptr;
    if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess) {
        (void)hipGetLastError();
        if (e0) (void)hipEventDestroy(e0);
        err = "peak measurement: event creation failed";
        return SA_ERR_DEVICE;
    }
    double best = 0.0;
    sa_status rc = SA_OK;
    for (int r = 0; r < 4 && rc == SA_OK; ++r) {  // the first run warms up
        hipLaunchKernelGGL(k_valu_peak, dim3((unsigned)blocks), dim3(kPeakThreads), 0, st, sink, iters, 0.999f, 1e-3f);
        if (hipGetLastError() != hipSuccess) {
            err = "peak measurement: launch failed";
            rc = SA_ERR_DEVICE;
            break;
        }
        (void)hipEventRecord(e0, st);
        hipLaunchKernelGGL(k_valu_peak, dim3((unsigned)blocks), dim3(kPeakThreads), 0, st, sink, iters, 0.999f, 1e-3f);
        (void)hipEventRecord(e1, st);
        float ms = 0.f;
        if (hipEventSynchronize(e1) != hipSuccess || hipEventElapsedTime(&ms, e0, e1) != hipSuccess || ms <= 0.f) {
            (void)hipGetLastError();
            err = "peak measurement: timing failed";
            rc = SA_ERR_DEVICE;
            break;
        }
        if (r > 0) best = std::max(best, (double)blocks * kPeakThreads * iters * kChains / (ms * 1e-3));
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    lane_ops_per_s = best;
    return rc;
}

}  // namespace sa
