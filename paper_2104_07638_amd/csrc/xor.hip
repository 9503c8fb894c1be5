// xor.hip -- XOR and XNOR principal minors of 2n x 2n block matrices (Sec. III) on gfx950.
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
// The XNOR case (Sec. III) keeps both or neither row of every block.  Its tree has the
// same shape: one child drops the last undecided block (the node's leading part, minor
// unchanged), the other keeps it (the Schur complement over the 2 x 2 pivot block, minor
// times the block's determinant).  Only the 2^n leaves are minors of distinct subsets;
// they are written in block-mask order (bit i <-> block i kept).
//
// Mapping (one wavefront per matrix; lanes exchange through LDS with wavefront syncs only,
// so the stores of the minors stay in flight):
//   * the last block is decided first, so a node's remaining blocks are the leading ones
//     and the pivot rows are the last two rows of its matrix; depth k of the output holds
//     the minors of the k trailing blocks, and every subtree's outputs are contiguous;
//   * top levels (d < T = n - Q): depth first over the 2^T depth-T nodes, the stack of
//     node matrices (orders 2(n-1) ... 2(n-T+1)) in a workspace in global memory (the
//     depth T-1 node in LDS), each row of the child split over as many lanes as the
//     wavefront allows, with the pivot row (scaled by 1/pivot) staged in LDS; the depth-T
//     node is written straight into LDS;
//   * the last Q = min(n, 6) levels of each depth-T node: breadth first in LDS, one row of
//     a child per lane (split over column groups where the rows leave lanes idle), so
//     each level is one pass (at most 64 rows);
//   * the LDS arrays are sized for the one tree a kernel runs (binary or ternary), which
//     sets how many wavefronts a compute unit holds;
//   * every size is a compile-time constant (one kernel per number of blocks), so no index
//     arithmetic divides at run time.
#include <hip/hip_runtime.h>
#include <stdint.h>
#include <type_traits>

#include "apm_device.h"
#include "apm_kernels.h"

namespace apm {
namespace {

#ifndef APM_XOR_Q
#define APM_XOR_Q 6
#endif
constexpr int kXQ = APM_XOR_Q;   // levels expanded breadth first in LDS (XOR, XNOR)
constexpr int kXQ3 = 4;      // the same for the ternary NAND tree
// modes: the XOR, XNOR and NAND cases of Sec. III
constexpr int kXor = 0, kXnor = 1, kNand = 2;
__host__ __device__ constexpr int xq(int mode) { return mode == kNand ? kXQ3 : kXQ; }
__host__ __device__ constexpr int64_t pow3(int k) { return k <= 0 ? 1 : 3 * pow3(k - 1); }
#ifndef APM_XOR_PAD
#define APM_XOR_PAD 1
#endif
// Row stride of an order-m node matrix in LDS: one element of padding, so that lanes
// reading the same column of different rows fall on different banks.
__host__ __device__ constexpr int xs(int m) { return m + APM_XOR_PAD; }
// Entries of the largest subtree level of one tree (mode) in LDS: the root, and every
// level's children with padded rows.
__host__ __device__ constexpr int xbuf_need(int mode)
{
    const int Q = xq(mode);
    int kids = 1, need = 2 * Q * xs(2 * Q);
    for (int J = 0; J < Q; ++J) {
        kids *= mode == kNand ? 3 : 2;
        const int mc = 2 * (Q - J) - 2;
        const int lvl = kids * mc * xs(mc);
        need = lvl > need ? lvl : need;
    }
    return need;
}
#ifndef APM_XOR_PRE
#define APM_XOR_PRE 1     // keep the depth T-1 node (order 2(Q + 1)) in LDS as well
#endif
__host__ __device__ constexpr int xpre_need(int mode)
{
    return APM_XOR_PRE ? 2 * (xq(mode) + 1) * xs(2 * (xq(mode) + 1)) : 1;
}
// Lanes per row in a subtree pass of `rows` rows of mc entries: the largest divisor of mc
// that keeps rows x H within the wavefront (1 when the rows fill it).
__host__ __device__ constexpr int col_groups(int rows, int mc)
{
    int h = 1;
    for (int c = 2; c <= mc && rows * c <= 64; ++c)
        if (mc % c == 0) h = c;
    return h;
}
// Columns per lane in a top-level pass over a child of order mc (mc rows): as few as the
// wavefront allows, with the column groups as even as that count permits.
__host__ __device__ constexpr int top_cols(int mc)
{
    const int hmax = 64 / mc < mc ? 64 / mc : mc;
    return (mc + hmax - 1) / hmax;
}
// Zero pivot rows of the widest subtree level (two rows of order 2Q - 2).
__host__ __device__ constexpr int xzero_need(int mode) { return xq(mode) > 1 ? 4 * xq(mode) - 4 : 1; }

// Start of the depth-d node matrix (d >= 1) in a matrix's workspace, in elements.
__host__ __device__ constexpr int64_t xor_top_off(int n, int d)
{
    int64_t s = 0;
    for (int l = 1; l < d; ++l) s += (int64_t)(2 * (n - l)) * (2 * (n - l));
    return s;
}

template <class F, int MODE>
struct XorLds {
    typename F::E buf[2][xbuf_need(MODE)];
    // minors of the nodes of the current and the next level (at most 2^Q, or 3^Q for NAND)
    typename F::E mn[2][MODE == kNand ? pow3(xq(MODE)) : (1 << xq(MODE))];
    typename F::E wk[64];            // subtree levels: each child's pivot row times 1/pivot
    typename F::E wv[32];            // top levels: pivot row times 1/pivot (XNOR: first row of
    typename F::E wv2[32];           // the pivot block's inverse times the pivot rows, and second)
    typename F::E topm[17];          // minors along the top path
    typename F::E pre[xpre_need(MODE)];     // the depth T-1 node
    // zeros: the pivot column and rows of a child that leaves its block out, so that it
    // runs the keeping children's code
    typename F::E wz[xzero_need(MODE)];
};

// Top level D of matrix order 2N: the child of the depth-D node on path s (a group of
// columns of a row of the child per lane), from the workspace (or the input at D = 0) to
// the workspace.
template <class F, int N, int T, int D, int MODE>
__device__ __forceinline__ void xor_top(int d0, int s, const typename F::E* A0, typename F::E* st,
                                        typename F::E* ob, XorLds<F, MODE>& sh, double& chk)
{
    if constexpr (D < T) {
        using E = typename F::E;
        constexpr int m = 2 * (N - D), mc = m - 2;
        if (D >= d0) {
            const int lane = threadIdx.x;
            // node and child: the input (D = 0), the workspace, or LDS for the depth T-1 node
            // (when kept there) and the depth-T node; LDS rows have stride xs(order)
            constexpr bool kPin = APM_XOR_PRE && T >= 2;
            constexpr bool kPinP = kPin && D == T - 1, kLdsC = D == T - 1 || (kPin && D == T - 2);
            constexpr int ps = kPinP ? xs(m) : m;
            constexpr int cs = kLdsC ? xs(mc) : mc;
            static_assert(!kLdsC || mc * xs(mc) <= (D == T - 1 ? xbuf_need(MODE) : xpre_need(MODE)),
                          "LDS node fits its buffer");
            const E* P;
            if constexpr (D == 0) {
                P = A0;
            } else if constexpr (kPinP) {
                P = sh.pre;
            } else {
                P = st + xor_top_off(N, D);
            }
            E* C;
            if constexpr (D == T - 1) {
                C = &sh.buf[0][0];
            } else if constexpr (kLdsC) {
                C = sh.pre;
            } else {
                C = st + xor_top_off(N, D + 1);
            }
            // this level's choice: a bit (XOR, XNOR) or a ternary digit (NAND: 0 leaves the
            // block out, 1 and 2 keep its first or second row)
            const int a = MODE == kNand ? (int)((s / pow3(T - 1 - D)) % 3) : (s >> (T - 1 - D)) & 1;
            // every load of the node first, then the arithmetic: one round trip per node.
            // Lane h mc + i takes columns [h cw, (h + 1) cw) of row i of the child.
            constexpr int cw = top_cols(mc), H = (mc + cw - 1) / cw;
            constexpr bool kEven = mc % cw == 0;
            const int i = lane % mc, h = lane / mc, h0 = h * cw;
            const bool act = h < H;
            E row[cw];
            if (act) {
#pragma unroll
                for (int j = 0; j < cw; ++j)
                    if (kEven || h0 + j < mc) row[j] = P[i * ps + h0 + j];
            }
            if (MODE == kXor || (MODE == kNand && a != 0)) {
                // child keeps row p of the last block: 1 x 1 pivot
                const int p = MODE == kNand ? mc + a - 1 : mc + a;
                const E pv = P[p * ps + p];
                E pc = F::zero(), pr = F::zero();
                if (act) pc = P[i * ps + p];
                if (lane < mc) pr = P[p * ps + lane];
                const typename F::R r = F::recip(pv);
                if (lane < mc) sh.wv[lane] = F::rowscale(pr, r);
                if (lane == 0) {
                    const E mk = F::bmul(sh.topm[D], pv, 0);
                    sh.topm[D + 1] = mk;
                    if constexpr (MODE == kXor) ob[(int64_t(2) << D) - 2 + (s >> (T - 1 - D))] = mk;
                    chk += F::fincheck(mk);
                }
                wave_sync();
                if (act) {
#pragma unroll
                    for (int j = 0; j < cw; ++j)
                        if (kEven || h0 + j < mc) C[i * cs + h0 + j] = F::upd(row[j], pc, sh.wv[h0 + j]);
                }
            } else if (a == 0) {
                // XNOR or NAND, the block left out: the leading part of the node, minor unchanged
                if (lane == 0) sh.topm[D + 1] = sh.topm[D];
                if (act) {
#pragma unroll
                    for (int j = 0; j < cw; ++j)
                        if (kEven || h0 + j < mc) C[i * cs + h0 + j] = row[j];
                }
            } else {
                // XNOR, the block kept: 2 x 2 pivot block, its inverse applied to the pivot rows
                const E a00 = P[mc * ps + mc], a01 = P[mc * ps + mc + 1];
                const E a10 = P[(mc + 1) * ps + mc], a11 = P[(mc + 1) * ps + mc + 1];
                E pc0 = F::zero(), pc1 = F::zero(), pr0 = F::zero(), pr1 = F::zero();
                if (act) {
                    pc0 = P[i * ps + mc];
                    pc1 = P[i * ps + mc + 1];
                }
                if (lane < mc) {
                    pr0 = P[mc * ps + lane];
                    pr1 = P[(mc + 1) * ps + lane];
                }
                const E det = F::det2(a00, a01, a10, a11);
                const typename F::R r = F::recip(det);
                if (lane < mc) {
                    sh.wv[lane] = F::rowscale(F::upd(F::bmul(pr0, a11, 0), a01, pr1), r);
                    sh.wv2[lane] = F::rowscale(F::upd(F::bmul(pr1, a00, 0), a10, pr0), r);
                }
                if (lane == 0) {
                    const E mk = F::bmul(sh.topm[D], det, 0);
                    sh.topm[D + 1] = mk;
                    chk += F::fincheck(mk);
                }
                wave_sync();
                if (act) {
#pragma unroll
                    for (int j = 0; j < cw; ++j)
                        if (kEven || h0 + j < mc)
                            C[i * cs + h0 + j] = F::upd(F::upd(row[j], pc0, sh.wv[h0 + j]), pc1, sh.wv2[h0 + j]);
                }
            }
            if constexpr (kLdsC) {
                wave_sync();
            } else {
                wave_mem_fence();   // the child is the next level's node (and wv is rewritten)
            }
        }
        xor_top<F, N, T, D + 1, MODE>(d0, s, A0, st, ob, sh, chk);
    }
}

// Subtree level J of a Q-level subtree: the children of the 2^J nodes in buf[J & 1]
// (order 2(Q - J)) into buf[(J + 1) & 1], one row (or column group) of a child per lane.
// base is where the children's depth T+J+1 starts in the output (2^(T+J+1) - 2; XOR
// only: the XNOR minors are the 2^N leaves, written at the last level in block-mask order).
template <class F, int Q, int J, int MODE>
__device__ __forceinline__ void xor_sub(int64_t base, int s, typename F::E* ob, XorLds<F, MODE>& sh, double& chk)
{
    if constexpr (J < Q) {
        using E = typename F::E;
        constexpr int cur = J & 1, nxt = cur ^ 1;
        constexpr int m = 2 * (Q - J), mc = m - 2;
        constexpr int kids = MODE == kNand ? (int)pow3(J + 1) : 2 << J;
        static_assert(kids * mc <= 64 && (MODE == kNand || kids <= 64), "one pass per level");
        static_assert(kids * mc * xs(mc) <= xbuf_need(MODE) &&
                          m * xs(m) * (kids / (MODE == kNand ? 3 : 2)) <= xbuf_need(MODE),
                      "a subtree level fits its LDS buffer");
        static_assert(2 * mc <= xzero_need(MODE), "zero pivot rows cover a level");
        static_assert(kids * sizeof(E) <= sizeof(XorLds<F, MODE>::mn[0]), "a level's minors fit");
        const int lane = threadIdx.x;
        if constexpr (MODE == kXor) {
            // child k of node k/2 keeps row mc + (k & 1) of the node's last block: its minor,
            // and the pivot row times 1/pivot (lane k mc + j holds entry j)
            if (lane < kids) {
                const int p = mc + (lane & 1);
                const E pv = sh.buf[cur][(lane >> 1) * m * xs(m) + p * xs(m) + p];
                const E mk = F::bmul(sh.mn[cur][lane >> 1], pv, 0);
                sh.mn[nxt][lane] = mk;
                ob[base + ((int64_t)s << (J + 1)) + lane] = mk;
                chk += F::fincheck(mk);
            }
            if constexpr (mc > 0) {
                if (lane < kids * mc) {
                    const int k = lane / mc, j = lane - k * mc, p = mc + (k & 1);
                    const E* P = &sh.buf[cur][(k >> 1) * m * xs(m)];
                    sh.wk[lane] = F::rowscale(P[p * xs(m) + j], F::recip(P[p * xs(m) + p]));
                }
            }
        } else if constexpr (MODE == kXnor) {
            // child 2v drops node v's last block (minor unchanged), child 2v+1 keeps it (minor
            // times the pivot block's determinant; the inverse times the two pivot rows go to
            // wk[v][0..1][...], lane 2 v mc + r mc + j holding entry j of row r)
            if (lane < kids) {
                const E* P = &sh.buf[cur][(lane >> 1) * m * xs(m)];
                E mk = sh.mn[cur][lane >> 1];
                if (lane & 1)
                    mk = F::bmul(mk, F::det2(P[mc * xs(m) + mc], P[mc * xs(m) + mc + 1], P[(mc + 1) * xs(m) + mc],
                                             P[(mc + 1) * xs(m) + mc + 1]), 0);
                sh.mn[nxt][lane] = mk;
                if constexpr (J == Q - 1) ob[((int64_t)s << Q) + lane] = mk;
                chk += F::fincheck(mk);
            }
            if constexpr (mc > 0) {
                if (lane < kids * mc) {
                    const int v = lane / (2 * mc), rr = lane - v * 2 * mc, r = rr / mc, j = rr - r * mc;
                    const E* P = &sh.buf[cur][v * m * xs(m)];
                    const E a00 = P[mc * xs(m) + mc], a01 = P[mc * xs(m) + mc + 1];
                    const E a10 = P[(mc + 1) * xs(m) + mc], a11 = P[(mc + 1) * xs(m) + mc + 1];
                    const typename F::R rd = F::recip(F::det2(a00, a01, a10, a11));
                    const E p0 = P[mc * xs(m) + j], p1 = P[(mc + 1) * xs(m) + j];
                    sh.wk[lane] = r == 0 ? F::rowscale(F::upd(F::bmul(p0, a11, 0), a01, p1), rd)
                                         : F::rowscale(F::upd(F::bmul(p1, a00, 0), a10, p0), rd);
                }
            }
        } else {
            // NAND: child 3v + c of node v leaves the last block out (c = 0, minor unchanged)
            // or keeps its row mc + c - 1; the kept rows' pivot rows times 1/pivot go to
            // wk[v][c - 1][...] (lane 2 v mc + r mc + j holds entry j of row mc + r)
            for (int t = lane; t < kids; t += 64) {
                const int v = t / 3, c = t - 3 * v;
                E mk = sh.mn[cur][v];
                if (c) {
                    const int p = mc + c - 1;
                    mk = F::bmul(mk, sh.buf[cur][v * m * xs(m) + p * xs(m) + p], 0);
                }
                sh.mn[nxt][t] = mk;
                if constexpr (J == Q - 1) ob[(int64_t)s * pow3(Q) + t] = mk;
                chk += F::fincheck(mk);
            }
            if constexpr (mc > 0) {
                if (lane < 2 * (kids / 3) * mc) {
                    const int v = lane / (2 * mc), rr = lane - v * 2 * mc, r = rr / mc, j = rr - r * mc;
                    const E* P = &sh.buf[cur][v * m * xs(m)];
                    const int p = mc + r;
                    sh.wk[lane] = F::rowscale(P[p * xs(m) + j], F::recip(P[p * xs(m) + p]));
                }
            }
        }
        wave_sync();
        if constexpr (mc > 0) {
            // lane (h, k, i) writes columns [h cw, (h + 1) cw) of row i of child k: where the
            // rows do not fill the wavefront, each row is split over H lanes
            constexpr int rows = kids * mc, H = col_groups(rows, mc), cw = mc / H;
            if (lane < rows * H) {
                const int r = lane % rows, h = lane / rows;
                const int k = r / mc, i = r - k * mc, j0 = h * cw;
                E* Cr = &sh.buf[nxt][k * mc * xs(mc) + i * xs(mc)] + j0;
                // the node's entries from column j0 on (two children per node, three for NAND)
                const E* P = &sh.buf[cur][(MODE == kNand ? k / 3 : k >> 1) * m * xs(m)] + j0;
                if constexpr (MODE == kNand) {
                    const int c = k % 3;
                    // one instruction stream for all three children (a copy branch beside the
                    // update would issue both): the one that leaves the block out subtracts
                    // zero times a zero row
                    const E ci = c ? P[i * xs(m) + mc - j0 + c - 1] : F::zero();
                    const E* wr = (c ? &sh.wk[(2 * (k / 3) + c - 1) * mc] : sh.wz) + j0;
#pragma unroll
                    for (int j = 0; j < cw; ++j) Cr[j] = F::upd(P[i * xs(m) + j], ci, wr[j]);
                } else if constexpr (MODE == kXor) {
                    const E ci = P[i * xs(m) + mc - j0 + (k & 1)];
                    const E* wr = &sh.wk[k * mc] + j0;
#pragma unroll
                    for (int j = 0; j < cw; ++j) Cr[j] = F::upd(P[i * xs(m) + j], ci, wr[j]);
                } else {
                    // both children in one instruction stream: the one that drops the block
                    // subtracts zero times zero rows
                    const bool keep = k & 1;
                    const E c0 = keep ? P[i * xs(m) + mc - j0] : F::zero();
                    const E c1 = keep ? P[i * xs(m) + mc - j0 + 1] : F::zero();
                    const E* w0 = (keep ? &sh.wk[(k >> 1) * 2 * mc] : sh.wz) + j0;
#pragma unroll
                    for (int j = 0; j < cw; ++j) Cr[j] = F::upd(F::upd(P[i * xs(m) + j], c0, w0[j]), c1, w0[mc + j]);
                }
            }
            wave_sync();
        }
        xor_sub<F, Q, J + 1, MODE>(2 * base + 2, s, ob, sh, chk);   // XOR depth T+J+2 starts at 2^(T+J+2) - 2
    }
}

// The block minors of matrix blockIdx.x (one wavefront).
template <class F, int N, int MODE>
__device__ __forceinline__ void xor_matrix(const typename F::E* __restrict__ A, typename F::E* __restrict__ out,
                                           int32_t* __restrict__ info, int32_t batch,
                                           typename F::E* __restrict__ ws, int64_t ws_stride)
{
    using E = typename F::E;
    constexpr int Q = N < xq(MODE) ? N : xq(MODE);
    constexpr int T = N - Q;
    constexpr int w = 2 * N;
    __shared__ XorLds<F, MODE> sh;
    const int b = blockIdx.x;
    if (b >= batch) return;
    const int lane = threadIdx.x;
    const E* A0 = A + (int64_t)b * w * w;
    constexpr int64_t nout = MODE == kNand ? pow3(N) : MODE == kXnor ? (int64_t(1) << N) : (int64_t(2) << N) - 2;
    E* ob = out + (int64_t)b * nout;

    bool fin = true;
    for (int e = lane; e < w * w; e += 64) fin = fin && F::in_finite(A0[e]);
    if (!__all(fin ? 1 : 0)) {
        for (int64_t i = lane; i < nout; i += 64) F::store_nan(ob, nullptr, i, false);
        if (info && lane == 0) info[b] = -2;
        return;
    }
    E* st = ws + (int64_t)b * ws_stride;
    double chk = 0.0;
    if (lane == 0) sh.topm[0] = F::one();
    for (int e = lane; e < xzero_need(MODE); e += 64) sh.wz[e] = F::zero();
    constexpr int ntop = MODE == kNand ? (int)pow3(T) : 1 << T;
    for (int s = 0; s < ntop; ++s) {
        // top levels: redo the path below the first choice that changed from s - 1 (the
        // number of trailing zero digits of s, binary or ternary)
        int d0 = 0;
        if (s) {
            if constexpr (MODE == kNand) {
                int tz = 0;
                for (int t = s; t % 3 == 0; t /= 3) ++tz;
                d0 = T - 1 - tz;
            } else {
                d0 = T - 1 - (31 - __clz((unsigned)(s ^ (s - 1))));
            }
        }
        xor_top<F, N, T, 0, MODE>(d0, s, A0, st, ob, sh, chk);
        // the subtree of depth-T node s, breadth first in LDS
        if constexpr (T == 0) {
            for (int e = lane; e < w * w; e += 64) sh.buf[0][(e / w) * xs(w) + e % w] = A0[e];
        }
        if (lane == 0) sh.mn[0][0] = sh.topm[T];
        wave_sync();
        xor_sub<F, Q, 0, MODE>((int64_t(2) << T) - 2, s, ob, sh, chk);
    }
    const bool bad = __any(chk == 0.0 ? 0 : 1);
    if (info && lane == 0) info[b] = bad ? -3 : 0;
}

template <class F, int N, int MODE>
__global__ __launch_bounds__(64) void xor_kernel(const typename F::E* __restrict__ A, typename F::E* __restrict__ out,
                                                 int32_t* __restrict__ info, int32_t batch,
                                                 typename F::E* __restrict__ ws, int64_t ws_stride)
{
    xor_matrix<F, N, MODE>(A, out, info, batch, ws, ws_stride);
}

// fp64: registers capped for four wavefronts per SIMD (the compiler's choice at 14 blocks,
// 140 registers, holds three); a few spilled registers cost less than the residency gains.
template <int N, int MODE>
__global__ __launch_bounds__(64) __attribute__((amdgpu_waves_per_eu(4))) void xor_kernel_r64(
    const double* __restrict__ A, double* __restrict__ out, int32_t* __restrict__ info, int32_t batch,
    double* __restrict__ ws, int64_t ws_stride)
{
    xor_matrix<FR64, N, MODE>(A, out, info, batch, ws, ws_stride);
}

template <class F, int N, int MODE>
constexpr auto xor_kernel_for()
{
    if constexpr (std::is_same_v<F, FR64>)
        return xor_kernel_r64<N, MODE>;
    else
        return xor_kernel<F, N, MODE>;
}

template <class F, int N>
hipError_t xor_launch_n(const LaunchXor& L, hipStream_t st)
{
    if constexpr (N > 16) {
        return hipErrorInvalidValue;
    } else {
        if (L.n != N) return xor_launch_n<F, N + 1>(L, st);
        auto go = [&](auto kern) {
            hipLaunchKernelGGL(kern, dim3((unsigned)L.batch), dim3(64), 0, st,
                               static_cast<const typename F::E*>(L.A), static_cast<typename F::E*>(L.out), L.info,
                               L.batch, static_cast<typename F::E*>(L.ws), L.ws_stride);
        };
        if (L.mode == kXnor) {
            go(xor_kernel_for<F, N, kXnor>());
        } else if (L.mode == kNand) {
            if constexpr (N <= 13) go(xor_kernel_for<F, N, kNand>());
            else return hipErrorInvalidValue;
        } else {
            go(xor_kernel_for<F, N, kXor>());
        }
        return hipGetLastError();
    }
}

}  // namespace

int64_t xor_ws_elems(int n, int mode)
{
    // depths 1 .. G live in the workspace, the deeper top nodes in LDS
    const int T = n > xq(mode) ? n - xq(mode) : 0;
    const int G = (APM_XOR_PRE && T >= 2) ? T - 2 : T - 1;
    return G >= 1 ? xor_top_off(n, G + 1) : 0;
}

hipError_t xor_launch(const LaunchXor& L, hipStream_t st)
{
    if (L.dtype == 0) return xor_launch_n<FR64, 1>(L, st);
    if (L.dtype == 2) return xor_launch_n<FC128, 1>(L, st);
    return hipErrorInvalidValue;
}

}  // namespace apm
