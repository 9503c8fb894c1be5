// xor.hip -- XOR principal minors of 2n x 2n block matrices (Sec. III, XOR case) on gfx950.
//
// A 2n x 2n matrix is read as n x n blocks of 2 x 2.  Its XOR minors keep exactly one
// row/column of every block; with the Keldysh block matrix of Sec. V.C they are the
// determinants of all 2^n branch assignments.  The binary tree of the XOR case: a node at
// depth d holds the matrix of the blocks not yet decided, as the Schur complement over the
// rows kept so far.  Each of its two children keeps one row of the next block as pivot,
// drops the other, and is the Schur complement over that pivot; the child's minor is the
// node's minor times the pivot (the ratio rule of Sec. II with a 1 x 1 pivot).  No pivot
// shift is made: its correction would need minors this tree never forms (the paper notes
// the same), so a zero pivot leaves its subtree non-finite and info = -3.
//
// Mapping (one wavefront per matrix):
//   * the last block is decided first, so a node's remaining blocks are the leading ones
//     and the pivot rows are the last two rows of its matrix; depth k of the output holds
//     the minors of the k trailing blocks, and every subtree's outputs are contiguous;
//   * top levels (d < T = n - Q): depth first over the 2^T depth-T nodes, the stack of
//     node matrices (orders 2(n-1) ... 2(n-T)) in a workspace in global memory, each child
//     computed by all lanes from the staged pivot row (scaled by 1/pivot) and column;
//   * the last Q = min(n, 6) levels of each depth-T node: breadth first in LDS, all the
//     children of a level computed by the lanes at once (at most 288 entries per level).
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "apm_device.h"
#include "apm_kernels.h"

namespace apm {
namespace {

constexpr int kXQ = 6;       // levels expanded breadth first in LDS
constexpr int kXBuf = 288;   // largest such level: 8 nodes of order 6 (orders 12, 10, 8, ...)

// Start of the depth-d node matrix (d >= 1) in a matrix's workspace, in elements.
__host__ __device__ inline int64_t xor_top_off(int n, int d)
{
    int64_t s = 0;
    for (int l = 1; l < d; ++l) s += (int64_t)(2 * (n - l)) * (2 * (n - l));
    return s;
}

template <class F>
__global__ __launch_bounds__(64) void xor_kernel(const typename F::E* __restrict__ A, typename F::E* __restrict__ out,
                                                 int32_t* __restrict__ info, int32_t batch, int n,
                                                 typename F::E* __restrict__ ws, int64_t ws_stride)
{
    using E = typename F::E;
    using R = typename F::R;
    __shared__ E buf[2][kXBuf];
    __shared__ E mn[2][1 << kXQ];   // minors of the nodes of the current and the next level
    __shared__ R rc[1 << kXQ];      // reciprocal pivots of the next level's nodes
    __shared__ E wv[32];            // top levels: pivot row times 1/pivot
    __shared__ E cv[32];            // and pivot column
    __shared__ E topm[17];          // minors along the top path
    const int b = blockIdx.x;
    if (b >= batch) return;
    const int lane = threadIdx.x;
    const int w = 2 * n;
    const E* A0 = A + (int64_t)b * w * w;
    E* ob = out + (int64_t)b * ((int64_t(2) << n) - 2);
    const int64_t nout = (int64_t(2) << n) - 2;

    bool fin = true;
    for (int e = lane; e < w * w; e += 64) fin = fin && F::in_finite(A0[e]);
    if (!__all(fin ? 1 : 0)) {
        for (int64_t i = lane; i < nout; i += 64) F::store_nan(ob, nullptr, i, false);
        if (info && lane == 0) info[b] = -2;
        return;
    }
    const int Q = n < kXQ ? n : kXQ;
    const int T = n - Q;
    E* st = ws + (int64_t)b * ws_stride;
    double chk = 0.0;
    if (lane == 0) topm[0] = F::one();

    for (int s = 0; s < (1 << T); ++s) {
        // top levels: redo the path below the first choice that changed from s - 1
        const int d0 = s ? T - 1 - (31 - __clz((unsigned)(s ^ (s - 1)))) : 0;
        for (int d = d0; d < T; ++d) {
            const int m = 2 * (n - d), mc = m - 2;
            const E* P = d == 0 ? A0 : st + xor_top_off(n, d);
            E* C = st + xor_top_off(n, d + 1);
            const int p = mc + ((s >> (T - 1 - d)) & 1);
            const E pv = P[p * m + p];
            const R r = F::recip(pv);
            if (lane < mc) {
                wv[lane] = F::rowscale(P[p * m + lane], r);
                cv[lane] = P[lane * m + p];
            }
            if (lane == 0) {
                const E mk = F::bmul(topm[d], pv, 0);
                topm[d + 1] = mk;
                ob[(int64_t(2) << d) - 2 + (s >> (T - 1 - d))] = mk;
                chk += F::fincheck(mk);
            }
            __syncthreads();
            for (int e = lane; e < mc * mc; e += 64) {
                const int i = e / mc, j = e - i * mc;
                C[e] = F::upd(P[i * m + j], cv[i], wv[j]);
            }
            __syncthreads();
        }
        // the subtree of depth-T node s, breadth first in LDS
        const int q = 2 * Q;
        const E* S0 = T == 0 ? A0 : st + xor_top_off(n, T);
        for (int e = lane; e < q * q; e += 64) buf[0][e] = S0[e];
        if (lane == 0) mn[0][0] = topm[T];
        __syncthreads();
        for (int j = 0; j < Q; ++j) {
            const int cur = j & 1, nxt = cur ^ 1;
            const int m = 2 * (Q - j), mc = m - 2;
            const int kids = 2 << j;
            // child k of node k/2 keeps row mc + (k & 1) of the node's last block
            if (lane < kids) {
                const int node = lane >> 1, p = mc + (lane & 1);
                const E pv = buf[cur][node * m * m + p * m + p];
                const E mk = F::bmul(mn[cur][node], pv, 0);
                mn[nxt][lane] = mk;
                rc[lane] = F::recip(pv);
                ob[(int64_t(2) << (T + j)) - 2 + ((int64_t)s << (j + 1)) + lane] = mk;
                chk += F::fincheck(mk);
            }
            __syncthreads();
            const int per = mc * mc;
            for (int e = lane; e < kids * per; e += 64) {
                const int k = e / per, rr = e - k * per, i = rr / mc, jj = rr - i * mc;
                const int p = mc + (k & 1);
                const E* P = &buf[cur][(k >> 1) * m * m];
                buf[nxt][e] = F::upd(P[i * m + jj], P[i * m + p], F::rowscale(P[p * m + jj], rc[k]));
            }
            __syncthreads();
        }
    }
    const bool bad = __any(chk == 0.0 ? 0 : 1);
    if (info && lane == 0) info[b] = bad ? -3 : 0;
}

}  // namespace

int64_t xor_ws_elems(int n)
{
    const int T = n > kXQ ? n - kXQ : 0;
    return T > 0 ? xor_top_off(n, T + 1) : 0;
}

hipError_t xor_launch(const LaunchXor& L, hipStream_t st)
{
    if (L.dtype == 0) {
        hipLaunchKernelGGL(xor_kernel<FR64>, dim3((unsigned)L.batch), dim3(64), 0, st,
                           static_cast<const double*>(L.A), static_cast<double*>(L.out), L.info, L.batch, L.n,
                           static_cast<double*>(L.ws), L.ws_stride);
    } else if (L.dtype == 2) {
        hipLaunchKernelGGL(xor_kernel<FC128>, dim3((unsigned)L.batch), dim3(64), 0, st,
                           static_cast<const cd*>(L.A), static_cast<cd*>(L.out), L.info, L.batch, L.n,
                           static_cast<cd*>(L.ws), L.ws_stride);
    } else {
        return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

}  // namespace apm
