// fpm.hip -- dispatch of apm_all_minors to the per-type kernel instantiations, the queue
// preparation of mixed-order batches, and the table of autotuned lane-subtree orders.
#include <atomic>

#include "apm_kernels.h"

namespace apm {

namespace {
std::atomic<int> g_tuned[4][21];   // zero-initialised: nothing tuned
}

int tuned_k0(int dtype, int n)
{
    if (dtype < 0 || dtype > 3 || n < 0 || n > 20) return 0;
    return g_tuned[dtype][n].load(std::memory_order_relaxed);
}

void set_tuned_k0(int dtype, int n, int k0)
{
    if (dtype < 0 || dtype > 3 || n < 0 || n > 20) return;
    g_tuned[dtype][n].store(k0, std::memory_order_relaxed);
}

// the instantiated lane-subtree orders of each type (the K0Set of the kernels)
void k0_range(int dtype, int* lo, int* hi)
{
    static const int r[4][2] = {{3, 5}, {3, 5}, {2, 3}, {3, 4}};
    *lo = r[dtype & 3][0];
    *hi = r[dtype & 3][1];
}

// Synthetic tuning input: diagonally dominant matrices with entries from a hash of
// (matrix, row, column) in [-0.5, 0.5) plus n on the diagonal (no pivot shifts).
__global__ __launch_bounds__(256) void fill_tune_kernel(double* A, int comps, int n, int64_t total)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= total) return;
    uint64_t h = (uint64_t)i * 0x9E3779B97F4A7C15ull;
    h ^= h >> 31;
    h *= 0xBF58476D1CE4E5B9ull;
    h ^= h >> 29;
    double v = (double)(h >> 11) * 0x1p-53 - 0.5;
    const int64_t e = i / comps;               // element index within the batch
    const int64_t ij = e % ((int64_t)n * n);
    if (ij / n == ij % n && (i % comps) == 0) v += n;
    A[i] = v;
}

hipError_t fill_tune_input(void* A, int dtype, int n, int batch, hipStream_t st)
{
    const int comps = (dtype == 2 || dtype == 3) ? 2 : 1;
    const int64_t total = (int64_t)batch * n * n * comps;
    hipLaunchKernelGGL(fill_tune_kernel, dim3((unsigned)((total + 255) / 256)), dim3(256), 0, st,
                       static_cast<double*>(A), comps, n, total);
    return hipGetLastError();
}

// Queue preparation (one workgroup): bucket the matrices by order, largest first, so the
// persistent waves start with the longest work; packed default offsets; queue head = 0.
__global__ __launch_bounds__(1024) void fpm_prep_kernel(int32_t batch, const int32_t* __restrict__ nv, int32_t* order,
                                                        int32_t* counter, int64_t* ioff, int64_t* ooff)
{
    __shared__ int cnt[22];
    __shared__ int pos[22];
    __shared__ int64_t carry[2];
    __shared__ int64_t part[2][1024];
    const int t = threadIdx.x;
    if (t < 22) cnt[t] = 0;
    if (t < 2) carry[t] = 0;
    __syncthreads();
    // bucket 21 - n for valid orders (so that larger n come first), 21 for invalid ones
    for (int b = t; b < batch; b += 1024) {
        const int n = nv[b];
        atomicAdd(&cnt[(n >= 1 && n <= 20) ? 20 - n : 21], 1);
    }
    __syncthreads();
    if (t == 0) {
        int s = 0;
        for (int k = 0; k < 22; ++k) {
            pos[k] = s;
            counter[kBucketBase + k] = s;   // where the matrices of order 20 - k start
            s += cnt[k];
        }
        counter[kBucketBase + 22] = s;
        counter[0] = 0;
        counter[1] = 0;
    }
    __syncthreads();
    for (int b = t; b < batch; b += 1024) {
        const int n = nv[b];
        const int k = (n >= 1 && n <= 20) ? 20 - n : 21;
        order[atomicAdd(&pos[k], 1)] = b;
    }
    // exclusive prefix sums of n^2 and 2^n in matrix order (chunks of 1024)
    for (int b0 = 0; b0 < batch; b0 += 1024) {
        const int b = b0 + t;
        const int n = (b < batch) ? nv[b] : 0;
        const bool ok = n >= 1 && n <= 20;
        part[0][t] = ok ? (int64_t)n * n : 0;
        part[1][t] = ok ? (int64_t(1) << n) : 0;
        __syncthreads();
        for (int d = 1; d < 1024; d <<= 1) {
            int64_t a0 = 0, a1 = 0;
            if (t >= d) { a0 = part[0][t - d]; a1 = part[1][t - d]; }
            __syncthreads();
            part[0][t] += a0;
            part[1][t] += a1;
            __syncthreads();
        }
        if (b < batch) {
            ioff[b] = carry[0] + part[0][t] - (ok ? (int64_t)n * n : 0);
            ooff[b] = carry[1] + part[1][t] - (ok ? (int64_t(1) << n) : 0);
        }
        __syncthreads();
        if (t == 1023) { carry[0] += part[0][1023]; carry[1] += part[1][1023]; }
        __syncthreads();
    }
}

hipError_t fpm_prep_launch(const LaunchMinors& L, hipStream_t st)
{
    hipLaunchKernelGGL(fpm_prep_kernel, dim3(1), dim3(1024), 0, st, L.batch, L.n, L.order, L.counter, L.ioff_ws,
                       L.ooff_ws);
    return hipGetLastError();
}

hipError_t fpm_launch_r64(const LaunchMinors& L, hipStream_t st);
hipError_t fpm_launch_r32s(const LaunchMinors& L, hipStream_t st);
hipError_t fpm_launch_c128(const LaunchMinors& L, hipStream_t st);
hipError_t fpm_launch_c64s(const LaunchMinors& L, hipStream_t st);

hipError_t fpm_launch(const LaunchMinors& L, hipStream_t st)
{
    switch (L.dtype) {
    case 0: return fpm_launch_r64(L, st);
    case 1: return fpm_launch_r32s(L, st);
    case 2: return fpm_launch_c128(L, st);
    case 3: return fpm_launch_c64s(L, st);
    default: return hipErrorInvalidValue;
    }
}

}  // namespace apm
