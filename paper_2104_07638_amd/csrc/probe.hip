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

// Grid-stride copy of n16 16-byte values, four loads in flight per thread before the stores.
__global__ __launch_bounds__(256) void copy_probe_kernel(uint4* __restrict__ dst, const uint4* __restrict__ src,
                                                         int64_t n16)
{
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    for (; i + 3 * stride < n16; i += 4 * stride) {
        const uint4 a = src[i], b = src[i + stride], c = src[i + 2 * stride], d = src[i + 3 * stride];
        dst[i] = a;
        dst[i + stride] = b;
        dst[i + 2 * stride] = c;
        dst[i + 3 * stride] = d;
    }
    for (; i < n16; i += stride) dst[i] = src[i];
}

}  // namespace

extern "C" apm_status apm_probe_copy(void* dst, const void* src, int64_t bytes, int32_t blocks, apm_stream stream)
{
    if (!dst || !src || bytes < 16 || (bytes & 15) || blocks < 1) return APM_EINVAL;
    if ((reinterpret_cast<uintptr_t>(dst) | reinterpret_cast<uintptr_t>(src)) & 15) return APM_EINVAL;
    hipLaunchKernelGGL(copy_probe_kernel, dim3((unsigned)blocks), dim3(256), 0, (hipStream_t)stream,
                       static_cast<uint4*>(dst), static_cast<const uint4*>(src), bytes / 16);
    return hipGetLastError() == hipSuccess ? APM_OK : APM_EDEVICE;
}

extern "C" apm_status apm_probe_fma64(double* sink, int32_t blocks, int32_t iters, int64_t* fmas, apm_stream stream)
{
    if (!sink || blocks < 1 || iters < 1) return APM_EINVAL;
    hipLaunchKernelGGL(fma64_probe_kernel, dim3((unsigned)blocks), dim3(256), 0, (hipStream_t)stream, sink, iters,
                       0.999999, 1e-7);
    if (fmas) *fmas = (int64_t)blocks * 256 * kChains * iters;
    return hipGetLastError() == hipSuccess ? APM_OK : APM_EDEVICE;
}
