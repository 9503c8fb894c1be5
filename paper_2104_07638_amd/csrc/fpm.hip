// fpm.hip -- dispatch of apm_all_minors to the per-type kernel instantiations, the queue
// preparation of mixed-order batches, and the table of autotuned lane-subtree orders.
#include <atomic>

#include "apm_device.h"
#include "apm_kernels.h"

namespace apm {

namespace {
std::atomic<int> g_tuned[4][21];   // zero-initialised: nothing tuned
std::atomic<int> g_tuned_mixed[4][2];
}

int tuned_mixed_k0(int dtype, int which)
{
    if (dtype < 0 || dtype > 3 || which < 0 || which > 1) return 0;
    return g_tuned_mixed[dtype][which].load(std::memory_order_relaxed);
}

void set_tuned_mixed_k0(int dtype, int which, int k0)
{
    if (dtype < 0 || dtype > 3 || which < 0 || which > 1) return;
    g_tuned_mixed[dtype][which].store(k0, std::memory_order_relaxed);
}

// the instantiated lane-subtree orders of the mixed-order kernels (RaggedK0 / BigK0) and
// their defaults
void mixed_k0_range(int dtype, int which, int* lo, int* hi, int* def)
{
    static const int r[4][2][3] = {{{3, 4, 4}, {4, 5, 5}},     // r64
                                   {{3, 4, 4}, {4, 5, 5}},     // r32s
                                   {{2, 2, 2}, {2, 3, 3}},     // c128
                                   {{3, 3, 3}, {3, 4, 4}}};    // c64s
    const int* v = r[dtype & 3][which & 1];
    *lo = v[0];
    *hi = v[1];
    *def = v[2];
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

// Mixed orders: one workgroup per matrix, the same entries plus n_b on the diagonal.
__global__ __launch_bounds__(256) void fill_tune_mixed_kernel(double* A, int comps, const int32_t* nv,
                                                              const int64_t* ioff)
{
    const int b = blockIdx.x;
    const int n = nv[b];
    const int64_t base = ioff[b] * comps;
    for (int i = threadIdx.x; i < n * n * comps; i += 256) {
        uint64_t h = (uint64_t)(base + i) * 0x9E3779B97F4A7C15ull;
        h ^= h >> 31;
        h *= 0xBF58476D1CE4E5B9ull;
        h ^= h >> 29;
        double v = (double)(h >> 11) * 0x1p-53 - 0.5;
        const int ij = i / comps;
        if (ij / n == ij % n && (i % comps) == 0) v += n;
        A[base + i] = v;
    }
}

hipError_t fill_tune_input_mixed(void* A, int dtype, const int32_t* nv, const int64_t* ioff, int batch,
                                 hipStream_t st)
{
    const int comps = (dtype == 2 || dtype == 3) ? 2 : 1;
    hipLaunchKernelGGL(fill_tune_mixed_kernel, dim3((unsigned)batch), dim3(256), 0, st, static_cast<double*>(A), comps,
                       nv, ioff);
    return hipGetLastError();
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
// persistent waves start with the longest work; packed default offsets; queue heads = 0.
// Wavefront w owns the segment [w S, (w + 1) S) of consecutive matrices, S = 64 per with
// per = ceil(B / 1024) rounds; in round i lane l takes matrix w S + 64 i + l, so every
// access of a round is one contiguous run.  The orders of the first kPrepCache rounds are
// kept in registers.  Counting sort without atomics: each wavefront counts its matrices per
// bucket with ballots, the counts of all wavefronts give every (bucket, wavefront) its first
// queue position, and each wavefront then places its matrices in the order it counted them
// (within a bucket: by matrix index).  The offsets are one scan per round over the lanes,
// carried from round to round, on top of the totals of the wavefronts before.
constexpr int kPrepCache = 16;
constexpr int kPrepBuckets = 22;   // bucket 20 - n for orders n = 1..20, 21 for invalid ones

__device__ __forceinline__ int prep_bucket(int n) { return (n >= 1 && n <= 20) ? 20 - n : 21; }

// x plus the int64 of its DPP source lane (0 where there is none or the row is masked off)
template <int CTRL, int RM, bool BC>
__device__ __forceinline__ int64_t dpp_add64(int64_t x)
{
    const int lo = __builtin_amdgcn_update_dpp(0, (int)(uint32_t)x, CTRL, RM, 0xF, BC);
    const int hi = __builtin_amdgcn_update_dpp(0, (int)(uint32_t)((uint64_t)x >> 32), CTRL, RM, 0xF, BC);
    return x + (int64_t)(((uint64_t)(uint32_t)hi << 32) | (uint32_t)lo);
}

// inclusive prefix sum over the 64 lanes by DPP: row_shr:1, 2, 4, 8 within rows of 16, then
// row_bcast:15 into rows 1 and 3 and row_bcast:31 into rows 2 and 3
__device__ __forceinline__ int64_t wave_scan64(int64_t v)
{
    v = dpp_add64<0x111, 0xF, true>(v);
    v = dpp_add64<0x112, 0xF, true>(v);
    v = dpp_add64<0x114, 0xF, true>(v);
    v = dpp_add64<0x118, 0xF, true>(v);
    v = dpp_add64<0x142, 0xA, false>(v);
    v = dpp_add64<0x143, 0xC, false>(v);
    return v;
}

// the int64 of lane 63 (uniform)
__device__ __forceinline__ int64_t lane63(int64_t v)
{
    const uint32_t lo = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)v, 63);
    const uint32_t hi = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)((uint64_t)v >> 32), 63);
    return (int64_t)(((uint64_t)hi << 32) | lo);
}

__global__ __launch_bounds__(1024) void fpm_prep_kernel(int32_t batch, const int32_t* __restrict__ nv, int32_t* order,
                                                        int32_t* counter, int64_t* ioff, int64_t* ooff)
{
    __shared__ int wcnt[16][kPrepBuckets];   // matrices per (wavefront, bucket), then first positions
    __shared__ int btot[kPrepBuckets];       // matrices per bucket
    __shared__ int64_t wtot[2][16];
    const int t = threadIdx.x, lane = t & 63, wv = t >> 6;
    const int per = (int)(((int64_t)batch + 1023) / 1024);
    const int64_t seg = (int64_t)wv * 64 * per + lane;   // this lane's matrix of round 0
    auto mat = [&](int i) { return seg + (int64_t)i * 64; };
    auto order_of = [&](int i) { return mat(i) < batch ? nv[mat(i)] : 0; };
    int nc[kPrepCache];
#pragma unroll
    for (int i = 0; i < kPrepCache; ++i) nc[i] = i < per ? order_of(i) : 0;
    // the buckets that occur in this wavefront (uniform): only those are counted and placed
    uint32_t seen = 0;
#pragma unroll
    for (int i = 0; i < kPrepCache; ++i)
        if (i < per && mat(i) < batch) seen |= 1u << prep_bucket(nc[i]);
    for (int i = kPrepCache; i < per; ++i)
        if (mat(i) < batch) seen |= 1u << prep_bucket(nv[mat(i)]);
    for (int o = 1; o < 64; o <<= 1) seen |= (uint32_t)__shfl_xor((int)seen, o);
    const uint32_t present = (uint32_t)__builtin_amdgcn_readfirstlane((int)seen);
    // round i: this lane's matrix (bucket -1 past the batch); the cached rounds unrolled.
    // Lane k of cw holds this wavefront's count of bucket k; the loops run over the present
    // buckets only (a scalar loop: present is uniform).
    int cw = 0;
    auto count_round = [&](int bk) {
        for (uint32_t pb = present; pb; pb &= pb - 1u) {
            const int k = __builtin_ctz(pb);
            const int c = __builtin_popcountll(ballot(bk == k));
            cw += lane == k ? c : 0;
        }
    };
#pragma unroll
    for (int i = 0; i < kPrepCache; ++i)
        if (i < per) count_round(mat(i) < batch ? prep_bucket(nc[i]) : -1);
    for (int i = kPrepCache; i < per; ++i) count_round(mat(i) < batch ? prep_bucket(nv[mat(i)]) : -1);
    if (lane < kPrepBuckets) wcnt[wv][lane] = cw;
    // this lane's sums of n^2 and 2^n over its rounds, for the wavefront totals
    auto sq = [](int n) { return (n >= 1 && n <= 20) ? (int64_t)n * n : (int64_t)0; };
    auto p2 = [](int n) { return (n >= 1 && n <= 20) ? (int64_t(1) << n) : (int64_t)0; };
    int64_t a0 = 0, a1 = 0;
#pragma unroll
    for (int i = 0; i < kPrepCache; ++i) {
        a0 += sq(nc[i]);
        a1 += p2(nc[i]);
    }
    for (int i = kPrepCache; i < per; ++i) {
        const int n = order_of(i);
        a0 += sq(n);
        a1 += p2(n);
    }
    a0 = wave_scan64(a0);
    a1 = wave_scan64(a1);
    if (lane == 63) {
        wtot[0][wv] = a0;
        wtot[1][wv] = a1;
    }
    __syncthreads();
    if (t < kPrepBuckets) {   // bucket totals
        int s = 0;
        for (int w = 0; w < 16; ++w) s += wcnt[w][t];
        btot[t] = s;
    }
    __syncthreads();
    if (t < kPrepBuckets) {   // first queue position of each (wavefront, bucket)
        int start = 0;
        for (int k = 0; k < t; ++k) start += btot[k];
        if (t == kPrepBuckets - 1) {
            counter[kBucketBase + kPrepBuckets] = start + btot[t];
            counter[0] = 0;
            counter[1] = 0;
            for (int h = 32; h < 64; ++h) counter[h] = 0;   // the persistent kernels' stream heads
        }
        counter[kBucketBase + t] = start;   // where the matrices of order 20 - t start
        for (int w = 0; w < 16; ++w) {
            const int c = wcnt[w][t];
            wcnt[w][t] = start;
            start += c;
        }
    }
    __syncthreads();
    cw = lane < kPrepBuckets ? wcnt[wv][lane] : 0;   // first positions
    const uint64_t below = (uint64_t(1) << lane) - 1;
    auto place_round = [&](int bk, int64_t b) {
        for (uint32_t pb = present; pb; pb &= pb - 1u) {
            const int k = __builtin_ctz(pb);
            const uint64_t m = ballot(bk == k);
            const int first = __builtin_amdgcn_readlane(cw, k);
            if (bk == k) order[first + __builtin_popcountll(m & below)] = (int32_t)b;
            cw += lane == k ? __builtin_popcountll(m) : 0;
        }
    };
#pragma unroll
    for (int i = 0; i < kPrepCache; ++i)
        if (i < per) place_round(mat(i) < batch ? prep_bucket(nc[i]) : -1, mat(i));
    for (int i = kPrepCache; i < per; ++i) place_round(mat(i) < batch ? prep_bucket(nv[mat(i)]) : -1, mat(i));
    // exclusive prefix sums of n^2 and 2^n in matrix order: the wavefronts before, then the
    // rounds before, then the lanes before
    int64_t e0 = 0, e1 = 0;
    for (int w = 0; w < wv; ++w) {
        e0 += wtot[0][w];
        e1 += wtot[1][w];
    }
    auto offsets_round = [&](int i, int n) {
        const int64_t v0 = sq(n), v1 = p2(n);
        const int64_t i0 = wave_scan64(v0), i1 = wave_scan64(v1);
        if (mat(i) < batch) {
            ioff[mat(i)] = e0 + i0 - v0;
            ooff[mat(i)] = e1 + i1 - v1;
        }
        e0 += lane63(i0);
        e1 += lane63(i1);
    };
#pragma unroll
    for (int i = 0; i < kPrepCache; ++i)
        if (i < per) offsets_round(i, nc[i]);
    for (int i = kPrepCache; i < per; ++i) offsets_round(i, order_of(i));
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
