// Device issue-rate probe: how fast the GPU completes fused multiply-adds
// in the accumulating two-operand form (d = a * b + d) that the evaluation's
// chains use, in FP64 and FP32.  The evaluation's efficiency is quoted
// against this measured ceiling beside the published peak (which assumes one
// FMA per lane per clock at 2.4 GHz).
//
// Each lane runs 16 independent dependent chains, x_k <- c_k a + x_k (the
// product is not hoisted: its rounding is fused with the sum), 16 FMAs per
// iteration, over 8192 workgroups of 256 lanes; the sums are written out so
// that no chain is dead.  Every operand is a per-lane register, as in the
// evaluation (an operand in a scalar register lowers the rate of the FP32
// form).  With a of order 1e-9 the values stay near their start (no
// overflow, no denormals).
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <algorithm>

#include "hermite.h"
#include "pair_chain.h"

namespace hermite {
namespace {

constexpr int kProbeThreads = 256;
constexpr int kProbeBlocks = 8192;
constexpr int kProbeChains = 16;

template <typename T>
__global__ __launch_bounds__(kProbeThreads) void fma_rate_kernel(T *__restrict__ out, int iters, T a)
{
    const T av = a * (T(1) + T(threadIdx.x & 7) * T(0.125));   // per lane
    T x[kProbeChains], c[kProbeChains];
#pragma unroll
    for (int k = 0; k < kProbeChains; ++k) {
        x[k] = T(1) + T(k) * T(0.125) + T(threadIdx.x) * T(1e-3);
        c[k] = T(2) - T(k) * T(0.0625) + T(blockIdx.x) * T(1e-6);
    }
    for (int i = 0; i < iters; ++i) {
#pragma unroll
        for (int k = 0; k < kProbeChains; ++k) x[k] = fma_t(c[k], av, x[k]);
    }
    T s = T(0);
#pragma unroll
    for (int k = 0; k < kProbeChains; ++k) s += x[k];
    out[(int64_t)blockIdx.x * kProbeThreads + threadIdx.x] = s;
}

template <typename T>
hipError_t time_fma(double *rate)
{
    const int64_t lanes = (int64_t)kProbeBlocks * kProbeThreads;
    const int iters = 2048;
    T *out = nullptr;
    hipStream_t st = nullptr;
    hipEvent_t e0 = nullptr, e1 = nullptr;
    hipError_t e = hipMalloc((void **)&out, lanes * sizeof(T));
    if (e == hipSuccess) e = hipStreamCreate(&st);
    if (e == hipSuccess) e = hipEventCreate(&e0);
    if (e == hipSuccess) e = hipEventCreate(&e1);
    if (e == hipSuccess) {
        // a warm-up launch
        hipLaunchKernelGGL(fma_rate_kernel<T>, dim3(kProbeBlocks), dim3(kProbeThreads), 0, st, out, iters,
                           T(1e-9));
        e = hipGetLastError();
    }
    // the best of three timed launches (the clock settles over the first)
    double best = 0.0;
    for (int rep = 0; rep < 3 && e == hipSuccess; ++rep) {
        e = hipEventRecord(e0, st);
        if (e == hipSuccess) {
            hipLaunchKernelGGL(fma_rate_kernel<T>, dim3(kProbeBlocks), dim3(kProbeThreads), 0, st, out, iters,
                               T(1e-9));
            e = hipGetLastError();
        }
        if (e == hipSuccess) e = hipEventRecord(e1, st);
        if (e == hipSuccess) e = hipEventSynchronize(e1);
        float ms = 0.0f;
        if (e == hipSuccess) e = hipEventElapsedTime(&ms, e0, e1);
        if (e == hipSuccess && ms > 0.0f)
            best = std::max(best, (double)lanes * iters * kProbeChains / (ms * 1e-3));
    }
    if (e == hipSuccess) *rate = best;
    // (release errors do not change the measured rate)
    if (e1) (void)hipEventDestroy(e1);
    if (e0) (void)hipEventDestroy(e0);
    if (st) (void)hipStreamDestroy(st);
    if (out) (void)hipFree(out);
    return e;
}

}  // namespace
}  // namespace hermite

extern "C" hermite_status hermite_fma_rate(int32_t precision, double *lane_fma_per_s)
{
    if (!lane_fma_per_s || (precision != HERMITE_FP64 && precision != HERMITE_MIXED)) return HERMITE_E_ARG;
    *lane_fma_per_s = 0.0;
    const hipError_t e = precision == HERMITE_FP64 ? hermite::time_fma<double>(lane_fma_per_s)
                                                   : hermite::time_fma<float>(lane_fma_per_s);
    return e == hipSuccess ? HERMITE_OK : HERMITE_E_HIP;
}
