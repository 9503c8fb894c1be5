// probe.hip -- peak-rate probe used to report measured rooflines beside the datasheet ones.
#include "../../include/apm.h"
#include <hip/hip_runtime.h>

namespace {

// kChains independent fp64 FMA chains per thread, `iters` steps each: issue-bound on the
// vector FMA pipe (no memory traffic inside the loop); one value per thread is stored so
// that the chains are not removed.
constexpr int kChains = 8;

__global__ __launch_bounds__(256) void fma64_probe_kernel(double* sink, int iters, double b, double c)
{
    double a[kChains];
#pragma unroll
    for (int k = 0; k < kChains; ++k) a[k] = (double)(threadIdx.x + k);
    for (int it = 0; it < iters; ++it) {
#pragma unroll
        for (int k = 0; k < kChains; ++k) a[k] = fma(a[k], b, c);
    }
    double s = 0.0;
#pragma unroll
    for (int k = 0; k < kChains; ++k) s += a[k];
    sink[(size_t)blockIdx.x * blockDim.x + threadIdx.x] = s;
}

}  // namespace

extern "C" apm_status apm_probe_fma64(double* sink, int32_t blocks, int32_t iters, int64_t* fmas, apm_stream stream)
{
    if (!sink || blocks < 1 || iters < 1) return APM_EINVAL;
    hipLaunchKernelGGL(fma64_probe_kernel, dim3((unsigned)blocks), dim3(256), 0, (hipStream_t)stream, sink, iters,
                       0.999999, 1e-7);
    if (fmas) *fmas = (int64_t)blocks * 256 * kChains * iters;
    return hipGetLastError() == hipSuccess ? APM_OK : APM_EDEVICE;
}
