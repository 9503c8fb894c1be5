// ppm.hip -- all permanent principal minors (Sec. IV) on gfx950.
//
//   per(A[S]) = sum_{T subset of S} (-1)^{|S|-|T|} prod_{i in S} r_i(T),   r_i(T) = sum_{j in T} A_ij
//
// (Ryser's formula per subset, with the (-1)^|S| factor that the printed formula drops.)
// The paper's O(3^n) organisation: the row sums r_i(T) are shared by every S containing T,
// and for a fixed T the products over all supersets S = T + U (U a subset of the other
// indices) are built without divisions, one factor r_i(T) per added index.
//
// One wavefront per matrix:
//   * T runs over all 2^n column sets in Gray-code order, so r(T) changes by one column per
//     step (n multiply-adds, kept in registers by every lane);
//   * for the complement C of T, the lowest min(6, |C|) indices of C are distributed over
//     the lanes (lane l takes the subset U_l they encode), the remaining h indices are
//     enumerated serially: their 2^h partial products are built by doubling in LDS;
//   * lane l adds (-1)^|U| r-products to per[T + U] in LDS (distinct S per lane, so no
//     conflicts); orders n <= 14 keep per[] in LDS, larger orders accumulate in the output.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "apm_device.h"
#include "apm_kernels.h"

namespace apm {
namespace {

constexpr int kPermLdsMax = 14;

__device__ __forceinline__ uint32_t pdep32(uint32_t k, uint32_t mask)
{
    uint32_t r = 0;
    for (uint32_t bit = 1; mask; bit <<= 1) {
        const uint32_t low = mask & (0u - mask);
        if (k & bit) r |= low;
        mask ^= low;
    }
    return r;
}

template <int N>
__device__ void ppm_wave(const double* __restrict__ A, double* __restrict__ out, double* lds)
{
    constexpr bool kInLds = N <= kPermLdsMax;
    constexpr int HMAX = N > 6 ? N - 6 : 0;
    const int lane = lane_id();
    double* Am = lds;                          // n x n matrix
    double* Hs = lds + N * N;                  // 2^HMAX partial products
    double* per = kInLds ? (lds + N * N + (1 << HMAX)) : out;
    const uint32_t full = (1u << N) - 1;

    for (int i = lane; i < N * N; i += kWave) Am[i] = A[i];
    for (uint32_t s = lane; s <= full; s += kWave) per[s] = 0.0;
    if constexpr (!kInLds) __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "workgroup");
    wave_sync();

    double r[N];
#pragma unroll
    for (int i = 0; i < N; ++i) r[i] = 0.0;
    uint32_t T = 0;
    for (uint32_t g = 0; g <= full; ++g) {
        if (g > 0) {
            const int j = __builtin_ctz(g);
            T ^= 1u << j;
            const double sg = (T >> j & 1u) ? 1.0 : -1.0;
#pragma unroll
            for (int i = 0; i < N; ++i) r[i] = fma(sg, Am[i * N + j], r[i]);
        }
        // product over T
        double base = 1.0;
#pragma unroll
        for (int i = 0; i < N; ++i)
            if (T >> i & 1u) base *= r[i];
        const uint32_t comp = full & ~T;
        const int c = __builtin_popcount(comp);
        const int lb = c < 6 ? c : 6;
        // split the complement: lowest lb indices to lanes, the rest serial
        uint32_t clow = 0, m = comp;
        for (int k = 0; k < lb; ++k) {
            const uint32_t low = m & (0u - m);
            clow |= low;
            m ^= low;
        }
        const uint32_t chigh = comp & ~clow;
        const int h = c - lb;
        // serial partial products H[e] = prod over pdep(e, chigh), built by doubling
        if (h > 0) {
            if (lane == 0) Hs[0] = 1.0;
            wave_sync();
            uint32_t mm = chigh;
            for (int k = 0; k < h; ++k) {
                const uint32_t low = mm & (0u - mm);
                mm ^= low;
                const int i = __builtin_ctz(low);
                double ri = 0.0;
#pragma unroll
                for (int q = 0; q < N; ++q) ri = (q == i) ? r[q] : ri;
                for (int e = lane; e < (1 << k); e += kWave) Hs[e + (1 << k)] = Hs[e] * ri;
                wave_sync();
            }
        }
        if (lane < (1 << lb)) {
            const uint32_t ul = pdep32((uint32_t)lane, clow);
            double L = base;
#pragma unroll
            for (int i = 0; i < N; ++i)
                if (ul >> i & 1u) L *= r[i];
            if (__builtin_popcount(ul) & 1) L = -L;
            const uint32_t s0 = T | ul;
            if (h == 0) {
                per[s0] += L;
            } else {
                // serial subsets of chigh in increasing order <-> e = 0, 1, 2, ...
                uint32_t sub = 0;
                for (int e = 0; e < (1 << h); ++e) {
                    const double v = L * Hs[e];
                    per[s0 | sub] += (__builtin_popcount(sub) & 1) ? -v : v;
                    sub = (sub - chigh) & chigh;
                }
            }
        }
        if constexpr (!kInLds) __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "workgroup");
        wave_sync();
    }
    if constexpr (kInLds) {
        for (uint32_t s = lane; s <= full; s += kWave) out[s] = per[s];
    }
}

template <int N>
constexpr size_t ppm_lds_bytes()
{
    return sizeof(double) * (N * N + (1 << (N > 6 ? N - 6 : 0)) + (N <= kPermLdsMax ? (1 << N) : 0));
}

template <int N>
__global__ __launch_bounds__(64) void ppm_kernel(const double* __restrict__ A, double* out, int32_t batch,
                                                 int n_uniform, const int32_t* nv, const int64_t* in_off,
                                                 const int64_t* out_off)
{
    extern __shared__ __align__(16) double lds_p[];
    const int b = blockIdx.x;
    if (b >= batch) return;
    const int n = n_uniform > 0 ? n_uniform : nv[b];
    if (n != N) return;
    const int64_t io = in_off ? in_off[b] : (int64_t)b * N * N;
    const int64_t oo = out_off ? out_off[b] : ((int64_t)b << N);
    ppm_wave<N>(A + io, out + oo, lds_p);
}

template <int N>
hipError_t launch_ppm(const LaunchPerm& L, hipStream_t st)
{
    constexpr size_t bytes = ppm_lds_bytes<N>();
    if (bytes > 65536) {
        hipError_t e = hipFuncSetAttribute((const void*)ppm_kernel<N>, hipFuncAttributeMaxDynamicSharedMemorySize,
                                           (int)bytes);
        if (e != hipSuccess) return e;
    }
    hipLaunchKernelGGL(ppm_kernel<N>, dim3((unsigned)L.batch), dim3(64), bytes, st, L.A, L.out, L.batch,
                       L.n_uniform, L.n, L.in_off, L.out_off);
    return hipGetLastError();
}

template <int N>
hipError_t launch_range(int lo, int hi, const LaunchPerm& L, hipStream_t st)
{
    if constexpr (N > 16) {
        return hipSuccess;
    } else {
        if (N >= lo && N <= hi) {
            hipError_t e = launch_ppm<N>(L, st);
            if (e != hipSuccess) return e;
        }
        return launch_range<N + 1>(lo, hi, L, st);
    }
}

}  // namespace

hipError_t perm_launch(const LaunchPerm& L, hipStream_t st)
{
    const int lo = L.n_uniform > 0 ? L.n_uniform : 1;
    const int hi = L.n_uniform > 0 ? L.n_uniform : L.n_max;
    return launch_range<1>(lo, hi, L, st);
}

}  // namespace apm
