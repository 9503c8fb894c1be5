// ppm.hip -- all permanent principal minors (Sec. IV) on gfx950.
//
//   per(A[S]) = sum_{T subset of S} (-1)^{|S|-|T|} prod_{i in S} r_i(T),   r_i(T) = sum_{j in T} A_ij
//
// (Ryser's formula per subset, with the (-1)^|S| factor that the printed formula drops.)
// As in the paper, the row sums r_i(T) are shared by every S containing T, and for a fixed
// T the products over the supersets S are built without divisions, one factor per added
// index, so the work is one multiply-add per (T, S) pair: 3^n per matrix.
//
// The n indices are split into three groups (low bits first):
//   H   (NH <= 6 bits)  the supersets Sh of Th are enumerated inside a lane, fully unrolled,
//                       into 2^NH register accumulators acc[Sh];
//   L1  (NL1 <= 6 bits) one lane per pair (Sl1, Tl1) with Tl1 subset of Sl1 (3^NL1 pairs);
//   L2  (NL2 = n - 12 bits, orders above 12) one workgroup per Sl2, looping over Tl2 in Sl2.
// (Orders below 12 use fewer L1 indices, see PermPlan.)
// A lane runs Th over all of H in Gray order (row sums updated one index at a time), and
// for each Th adds prod_{i in S} (+-r_i) into acc[Sh] for every Sh containing Th: the
// factor of the L1 and L2 indices is one product per Th, the H indices are a depth-first
// superset tree whose leaves are fused multiply-adds.  The lanes of one Sl1 (2^|Sl1| of
// them, aligned, never crossing a wavefront) are summed through LDS at the end, and every
// output is written exactly once: no atomics, no per-T LDS traffic.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "apm_device.h"
#include "apm_kernels.h"

namespace apm {
namespace {

#ifndef APM_PPM_SCHED_BARRIER
#define APM_PPM_SCHED_BARRIER 0   // 1: fence each Gray step off from the scheduler (measured slower)
#endif
#ifndef APM_PPM_NH
#define APM_PPM_NH 6   // largest H group: 2^NH fp64 accumulators per lane
#endif

// Lane-group size per order (measured): 3^4 pairs up to n = 10, then one more L1 index per
// order up to 6 at n = 12; H takes up to 6 of the rest, L2 what remains.
template <int N>
struct PermPlan {
    static constexpr int NL1 = N <= 4 ? N : (N <= 10 ? 4 : (N >= 12 ? 6 : N - 6));
    static constexpr int NH = N - NL1 > APM_PPM_NH ? APM_PPM_NH : N - NL1;
    static constexpr int NL2 = N - NH - NL1;
    static constexpr int PAIRS = [] { int p = 1; for (int i = 0; i < NL1; ++i) p *= 3; return p; }();
    static constexpr int NW = (PAIRS + kWave - 1) / kWave;   // wavefronts per (matrix, Sl2)
    static constexpr int CH = (1 << NH) < 32 ? (1 << NH) : 32; // accumulators per LDS pass
    static constexpr int RS = CH + 1;                          // odd row stride (doubles)
};

// Pair p of the L1 indices: groups of equal Sl1 ordered by descending |Sl1| (then by value),
// each group 2^|Sl1| consecutive lanes with Tl1 = the group-local index deposited into Sl1.
// A group of 2^k lanes starts at a multiple of 2^k (the groups before it all have sizes that
// are multiples of 2^(k+1) or of 2^k), so no group crosses a wavefront.
// Entry: Sl1 | Tl1 << 6 | |Sl1| << 12.
struct PairTable {
    uint16_t e[7][729];
};

constexpr uint32_t cx_pdep(uint32_t k, uint32_t mask)
{
    uint32_t r = 0, bit = 1;
    for (int i = 0; i < 32; ++i) {
        if ((mask >> i) & 1u) {
            if (k & bit) r |= 1u << i;
            bit <<= 1;
        }
    }
    return r;
}

constexpr int cx_popc(uint32_t m)
{
    int c = 0;
    for (; m; m &= m - 1) ++c;
    return c;
}

constexpr PairTable make_pairs()
{
    PairTable t{};
    for (int nl = 0; nl <= 6; ++nl) {
        int p = 0;
        for (int k = nl; k >= 0; --k)
            for (uint32_t m = 0; m < (1u << nl); ++m) {
                if (cx_popc(m) != k) continue;
                for (uint32_t w = 0; w < (1u << k); ++w)
                    t.e[nl][p++] = (uint16_t)(m | cx_pdep(w, m) << 6 | (uint32_t)k << 12);
            }
    }
    return t;
}

__constant__ PairTable kPairs = make_pairs();

// Superset tree of Th over the H indices.  Node S (a superset of TH) has the value
// parent * f with f = nr[b] = -r_b for the index b just added; a node with children forms its
// value, a leaf adds parent * f with one fused multiply-add (in place: no sign modifier).
template <int NH, int TH, int S, int B>
__device__ __forceinline__ void children(double (&acc)[1 << NH], const double* r, double v);

template <int NH, int TH, int S, int B>
constexpr bool has_children()
{
    for (int b = B; b < NH; ++b)
        if (!((TH >> b) & 1)) return true;
    return false;
}

template <int NH, int TH, int S, int B>
__device__ __forceinline__ void visit(double (&acc)[1 << NH], const double* r, double pv, double f)
{
    if constexpr (has_children<NH, TH, S, B>()) {
        const double v = pv * f;
        acc[S] += v;
        children<NH, TH, S, B>(acc, r, v);
    } else {
        acc[S] = fma(pv, f, acc[S]);
    }
}

template <int NH, int TH, int S, int B>
__device__ __forceinline__ void children(double (&acc)[1 << NH], const double* r, double v)
{
    if constexpr (B < NH) {
        if constexpr (!((TH >> B) & 1)) visit<NH, TH, (S | (1 << B)), B + 1>(acc, r, v, r[B]);
        children<NH, TH, S, B + 1>(acc, r, v);
    }
}

// Row j of A, read where it is used: the pointer passes through an empty asm so that the
// compiler cannot hoist the (wave-uniform, scalar) loads of every row to the kernel start,
// where they would not fit in scalar registers.
typedef const __attribute__((address_space(4))) double const_f64;

template <int N>
__device__ __forceinline__ void load_row(const double* __restrict__ Am, int j, double (&v)[N])
{
    const_f64* p = (const_f64*)(Am + j * N);
    asm volatile("" : "+s"(p));
#pragma unroll
    for (int i = 0; i < N; ++i) v[i] = p[i];
}

// Product of v[i] over the bits i of MASK, as a balanced tree (short dependency chains).
template <int MASK, int LO, int HI, int NV>
__device__ __forceinline__ double prod_bits(const double (&v)[NV])
{
    constexpr int sub = MASK & (((1 << HI) - 1) & ~((1 << LO) - 1));
    if constexpr (sub == 0) {
        return 1.0;
    } else if constexpr ((sub & (sub - 1)) == 0) {
        return v[__builtin_ctz(sub)];
    } else {
        constexpr int mid = (LO + HI) / 2;
        constexpr bool lo_any = (MASK & (((1 << mid) - 1) & ~((1 << LO) - 1))) != 0;
        constexpr bool hi_any = (MASK & (((1 << HI) - 1) & ~((1 << mid) - 1))) != 0;
        if constexpr (!lo_any) return prod_bits<MASK, mid, HI, NV>(v);
        else if constexpr (!hi_any) return prod_bits<MASK, LO, mid, NV>(v);
        else return prod_bits<MASK, LO, mid, NV>(v) * prod_bits<MASK, mid, HI, NV>(v);
    }
}

// Th = G ^ (G >> 1) for G = 0 .. 2^NH - 1.  The sums run over the transpose
// (r_i(T) = sum_{j in T} A_ji, and per(M) = per(M^T)), so a toggled index j adds one
// contiguous row of A.
//   nr[i]  -r_i(T) for the H indices (the tree's factors; the root's sign is compile-time);
//   q[i]   the factor of an L index i: s_i r_i(T) with s_i = +1 (i in T) or -1 (i in S \ T),
//          and 1 for i outside S.  With ms[i] = s_i (0 outside S) every update is the exact
//          fma(+-ms[i], a, q[i]), and the L part of the product is a plain product of q.
//          L1 indices (i < NL1) have per-lane ms, L2 indices the wavefront's.
template <int N, int NH, int NL, int G>
__device__ __forceinline__ void gray_steps(const double* __restrict__ Am, double (&nr)[NH > 0 ? NH : 1],
                                           double (&q)[NL > 0 ? NL : 1], double (&acc)[1 << NH],
                                           const double (&ms)[NL > 0 ? NL : 1])
{
    if constexpr (G < (1 << NH)) {
        constexpr int TH = G ^ (G >> 1);
#if APM_PPM_SCHED_BARRIER
        __builtin_amdgcn_sched_barrier(0);
#endif
        if constexpr (G > 0) {
            constexpr bool added = (TH >> __builtin_ctz(G)) & 1;
            double row[N];
            load_row<N>(Am, __builtin_ctz(G), row);
#pragma unroll
            for (int i = 0; i < NH; ++i) nr[i] = added ? nr[i] - row[i] : nr[i] + row[i];
#pragma unroll
            for (int i = 0; i < NL; ++i) q[i] = fma(added ? ms[i] : -ms[i], row[NH + i], q[i]);
        }
        constexpr int NLa = NL > 0 ? NL : 1;
        const double pl = NL > 0 ? prod_bits<(1 << NL) - 1, 0, NLa, NLa>(q) : 1.0;
        if constexpr (TH == 0) {
            acc[0] += pl;
            children<NH, 0, 0, 0>(acc, nr, pl);
        } else {
            // root = pl * prod_{i in TH} r_i = (-1)^|TH| pl * prod nr_i; the highest factor
            // goes through visit()
            constexpr int top = 31 - __builtin_clz(TH);
            constexpr int rest = TH & ~(1 << top);
            double pv = (__builtin_popcount(TH) & 1) ? -pl : pl;
            if constexpr (rest != 0) pv *= prod_bits<rest, 0, NH, NH>(nr);
            visit<NH, TH, TH, 0>(acc, nr, pv, nr[top]);
        }
        gray_steps<N, NH, NL, G + 1>(Am, nr, q, acc, ms);
    }
}

template <int N>
__global__ __launch_bounds__(64) void ppm_kernel(const double* __restrict__ A, double* __restrict__ out,
                                                 int32_t batch, int32_t b0, int n_uniform,
                                                 const int32_t* __restrict__ nv, const int64_t* __restrict__ in_off,
                                                 const int64_t* __restrict__ out_off)
{
    using P = PermPlan<N>;
    constexpr int NH = P::NH, NL1 = P::NL1, NL2 = P::NL2;
    __shared__ double red[kWave * P::RS];
    const int w = blockIdx.x % P::NW;
    const int rest = blockIdx.x / P::NW;
    const uint32_t sl2 = (uint32_t)rest & ((1u << NL2) - 1u);
    const int b = b0 + (rest >> NL2);
    if (b >= batch) return;
    const int n = n_uniform > 0 ? n_uniform : nv[b];
    if (n != N) return;
    const double* __restrict__ Am = A + (in_off ? in_off[b] : (int64_t)b * N * N);
    double* __restrict__ o = out + (out_off ? out_off[b] : ((int64_t)b << N));
    const int lane = (int)threadIdx.x;
    const int p = w * kWave + lane;
    const bool valid = p < P::PAIRS;
    const uint32_t e = valid ? kPairs.e[NL1][p] : 0u;
    const uint32_t sl1 = e & 63u, tl1 = (e >> 6) & 63u;
    const int k = (int)(e >> 12);

    constexpr int NL = NL1 + NL2;
    constexpr int NHa = NH > 0 ? NH : 1, NLa = NL > 0 ? NL : 1;
    // signed membership of the L1 indices (per lane) and the 0/1 membership of Tl1
    double ms[NLa], t1[NL1 > 0 ? NL1 : 1];
#pragma unroll
    for (int i = 0; i < NL1; ++i) {
        const bool in_s = (sl1 >> i) & 1u, in_t = (tl1 >> i) & 1u;
        ms[i] = in_s ? (in_t ? 1.0 : -1.0) : 0.0;
        t1[i] = in_t ? 1.0 : 0.0;
    }
    double acc[1 << NH];
#pragma unroll
    for (int s = 0; s < (1 << NH); ++s) acc[s] = 0.0;
    // The L2 loop stays a loop even with no L2 indices (sl2 = 0 is hidden from the compiler):
    // as straight-line code the row loads of the set-up and the steps get interleaved and
    // the register demand more than doubles.
    uint32_t sl2v = sl2;
    asm volatile("" : "+s"(sl2v));
    uint32_t tl2 = 0;
    do {
#pragma unroll
        for (int i = 0; i < NL2; ++i) {
            const bool in_s = (sl2 >> i) & 1u, in_t = (tl2 >> i) & 1u;
            ms[NL1 + i] = in_s ? (in_t ? 1.0 : -1.0) : 0.0;
        }
        // row sums of T = Tl1 + Tl2 (Th empty): 0/1 multiply-adds are exact
        double r[N];
#pragma unroll
        for (int i = 0; i < N; ++i) r[i] = 0.0;
#pragma unroll
        for (int j = 0; j < NL1; ++j) {
            double a[N];
            load_row<N>(Am, NH + j, a);
#pragma unroll
            for (int i = 0; i < N; ++i) r[i] = fma(t1[j], a[i], r[i]);
        }
#pragma unroll
        for (int j = 0; j < NL2; ++j) {
            if ((tl2 >> j) & 1u) {
                double a[N];
                load_row<N>(Am, NH + NL1 + j, a);
#pragma unroll
                for (int i = 0; i < N; ++i) r[i] += a[i];
            }
        }
        double nr[NHa], q[NLa];
#pragma unroll
        for (int i = 0; i < NHa; ++i) nr[i] = i < NH ? -r[i] : 0.0;
#pragma unroll
        for (int i = 0; i < NLa; ++i) q[i] = i < NL ? (ms[i] != 0.0 ? ms[i] * r[NH + i] : 1.0) : 1.0;
        gray_steps<N, NH, NL, 0>(Am, nr, q, acc, ms);
        tl2 = (tl2 - sl2v) & sl2v;
    } while (tl2 != 0u);

    // sum the lanes of each Sl1 group: lane t0 of a group of g lanes writes Sh = t0 + g u
    const int g = 1 << k;
    const int gl = lane & ~(g - 1);             // group's first lane in this wavefront
    const int t0 = lane - gl;
    const uint64_t obase = ((uint64_t)sl1 << NH) | ((uint64_t)sl2 << (NH + NL1));
#pragma unroll
    for (int c0 = 0; c0 < (1 << NH); c0 += P::CH) {
#pragma unroll
        for (int s = 0; s < P::CH; ++s) red[lane * P::RS + s] = acc[c0 + s];
        __syncthreads();
        if (valid) {
            for (int s = t0; s < P::CH; s += g) {
                double v = 0.0;
                for (int t = 0; t < g; ++t) v += red[(gl + t) * P::RS + s];
                o[obase | (uint64_t)(c0 + s)] = v;
            }
        }
        __syncthreads();
    }
}

template <int N>
hipError_t launch_ppm(const LaunchPerm& L, hipStream_t st)
{
    using P = PermPlan<N>;
    const int64_t per = (int64_t)P::NW << P::NL2;           // workgroups per matrix
    const int64_t chunk = ((int64_t)1 << 30) / per;         // matrices per launch
    for (int64_t b0 = 0; b0 < L.batch; b0 += chunk) {
        const int64_t nb = L.batch - b0 < chunk ? L.batch - b0 : chunk;
        hipLaunchKernelGGL(ppm_kernel<N>, dim3((unsigned)(nb * per)), dim3(kWave), 0, st, L.A, L.out, L.batch,
                           (int32_t)b0, L.n_uniform, L.n, L.in_off, L.out_off);
        const hipError_t e = hipGetLastError();
        if (e != hipSuccess) return e;
    }
    return hipSuccess;
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
