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
// The NAND case (Sec. III) keeps at most one row of every block: a ternary tree whose
// children leave the block out (minor unchanged) or keep one of its rows (1 x 1 pivot).
// Its left-out children are the minors that the pivot correction needs, so a small or zero
// pivot is shifted (the test and C of the minors tree) and the kept child's subtree is
// corrected once it is complete (see nand_top_fix).
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

// NAND subtree levels that can shift (child order >= 1): J <= kXQ3 - 2.  Kept-row pairs of
// the widest such level, and the shift codes of all their children.
__host__ __device__ constexpr int xsub_pairs_max() { return 2 * (int)pow3(kXQ3 - 2); }
__host__ __device__ constexpr int xsub_codes() { return ((int)pow3(kXQ3) - 3) / 2; }
__host__ __device__ constexpr int xsub_code_base(int J) { return ((int)pow3(J + 1) - 3) / 2; }

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
    // NAND pivot shifts: the (possibly shifted) pivots of a subtree level's kept rows (levels
    // with a small pivot only), the shift codes of the subtree's nodes (level J + 1 children
    // from xsub_code_base(J) on; valid for the levels in XPiv::sub_mask)
    typename F::E pvs[MODE == kNand ? xsub_pairs_max() : 1];
    int8_t scode[MODE == kNand ? xsub_codes() : 1];
    // a shifted child's own entry (no deeper row kept), with the true pivot: subtree
    // children by code index, and the top-level child of the current path
    typename F::E sown[MODE == kNand ? xsub_codes() : 1];
    typename F::E topown;
};

// Biased binary exponent of max(|Re v|, |Im v|) (0 for zero and subnormals), from the high
// words: the fast pivot-shift test compares exponents with integer operations.  The exact
// test can fail only with an entry above |p| / tau >= 2^9 |p| (tau = 1e-3 <= 2^-9), whose
// exponent is then at least kFastExp above p's; so "p normal and no entry kFastExp or more
// above it" passes the exact test.
__device__ __forceinline__ int xexp(double v) { return (__double2hiint(v) & 0x7FFFFFFF) >> 20; }
__device__ __forceinline__ int xexp(cd v) { return xexp(v.x) > xexp(v.y) ? xexp(v.x) : xexp(v.y); }
constexpr int kFastExp = 9;
static_assert(kDefaultPivTol <= 0x1p-9, "an entry above |p| / tau has an exponent >= kFastExp above p's");

// Matrix-wide state of the NAND pivot shifts: tau^2, the exponent of the largest input
// magnitude, the shifts made, and whether the current subtree made any.
struct XPiv {
    double tau2;
    int es;
    int nsh;
    int sub_mask;    // subtree levels of the current subtree with a shifted pivot (bit J)
    bool top_own;    // the current path's top-level child was shifted (own entry in topown)
    uint64_t tc0, tc1;   // shift code of the top path's child at depth D: byte D & 7 of tc0 (D < 8) or tc1
    __device__ int tcode(int D) const { return (int)(int8_t)((D < 8 ? tc0 : tc1) >> (8 * (D & 7))); }
    __device__ void set_tcode(int D, int code)
    {
        const int sh = 8 * (D & 7);
        const uint64_t v = (uint64_t)(uint8_t)code << sh, m = ~(0xFFull << sh);
        if (D < 8)
            tc0 = (tc0 & m) | v;
        else
            tc1 = (tc1 & m) | v;
    }
};

// Pivot of kept row p of an order-m subtree node P (rows of stride xs(m)), shifted if the
// test fails on the row and column entries that enter the child (the first mc = m - 2).
template <class F, int m>
__device__ __forceinline__ typename F::E nand_sub_pivot(const typename F::E* P, int p, const XPiv& xp, int8_t& code)
{
    constexpr int mc = m - 2;
    typename F::E pv = P[p * xs(m) + p];
    double rmax = 0.0, cmax = 0.0;
#pragma unroll
    for (int j = 0; j < mc; ++j) {
        rmax = fmax(rmax, F::mag(P[p * xs(m) + j]));
        cmax = fmax(cmax, F::mag(P[j * xs(m) + p]));
    }
    const double pm = F::mag(pv);
    code = kNoEv;
    if (pm == 0.0 || pm * pm < xp.tau2 * rmax * cmax) {
        code = shift_code(rmax, cmax, xp.es, F::re(pv) < 0.0);
        pv = F::shift(pv, shift_value(xp.es, code));
    }
    return pv;
}

// NAND top level D whose fast pivot test failed (rare, out of line): the test on the row and
// column maxima of kept row p of node P (row stride ps); if the pivot is shifted, the child C
// (row stride cs) is formed again with the shifted pivot, the node's minor times it goes to
// topm[D + 1] and the child's own entry (with the true pivot) to topown.  Returns the code.
template <class F, int N, int D>
__device__ __noinline__ int nand_top_slow(const typename F::E* P, typename F::E* C, int p, int ps, int cs,
                                          XorLds<F, kNand>& sh, double tau2, int es)
{
    using E = typename F::E;
    constexpr int m = 2 * (N - D), mc = m - 2;
    constexpr int cw = top_cols(mc), H = (mc + cw - 1) / cw;
    constexpr bool kEven = mc % cw == 0;
    const int lane = threadIdx.x;
    const int i = lane % mc, h = lane / mc, h0 = h * cw;
    const bool act = h < H;
    const E pv = P[p * ps + p];
    E pc = F::zero(), pr = F::zero();
    if (act) pc = P[i * ps + p];
    if (lane < mc) pr = P[p * ps + lane];
    const double rmax = wave_max_nonneg(lane < mc ? F::mag(pr) : 0.0);
    const double cmax = wave_max_nonneg(act ? F::mag(pc) : 0.0);
    const double pm = F::mag(pv);
    if (!(pm == 0.0 || pm * pm < tau2 * rmax * cmax)) return kNoEv;
    const int code = shift_code(rmax, cmax, es, F::re(pv) < 0.0);
    const E ps2 = F::shift(pv, shift_value(es, code));
    const typename F::R r2 = F::recip(ps2);
    wave_sync();   // every lane has read wv
    if (lane < mc) sh.wv[lane] = F::rowscale(pr, r2);
    if (lane == 0) {
        sh.topown = F::bmul(sh.topm[D], pv, 0);
        sh.topm[D + 1] = F::bmul(sh.topm[D], ps2, 0);
    }
    wave_sync();
    if (act) {
#pragma unroll
        for (int j = 0; j < cw; ++j)
            if (kEven || h0 + j < mc) C[i * cs + h0 + j] = F::upd(P[i * ps + h0 + j], pc, sh.wv[h0 + j]);
    }
    return code;
}

// Top level D of matrix order 2N: the child of the depth-D node on path s (a group of
// columns of a row of the child per lane), from the workspace (or the input at D = 0) to
// the workspace.
template <class F, int N, int T, int D, int MODE>
__device__ __forceinline__ void xor_top(int d0, int s, const typename F::E* A0, typename F::E* st,
                                        typename F::E* ob, XorLds<F, MODE>& sh, double& chk, XPiv& xp)
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
                if constexpr (MODE == kNand) {
                    // pivot shift (Sec. II test on the kept row and column of the child's Schur
                    // complement), checked once the child is written (its inputs are at hand by
                    // then); a shifted child is formed again and corrected once its subtree is
                    // complete.  No lane holding an entry kFastExp binary orders above p:
                    // the test passes without the maxima.
                    const int ep = xexp(pv);
                    const int le = max(lane < mc ? xexp(pr) : 0, act ? xexp(pc) : 0);
                    int code = kNoEv;
                    if (ballot(ep == 0 || le >= ep + kFastExp)) {
                        code = nand_top_slow<F, N, D>(P, C, p, ps, cs, sh, xp.tau2, xp.es);
                        if (code != kNoEv) {
                            xp.nsh += 1;
                            xp.top_own = true;
                        }
                    }
                    xp.set_tcode(D, code);
                }
            } else if (a == 0) {
                // XNOR or NAND, the block left out: the leading part of the node, minor unchanged
                if (lane == 0) sh.topm[D + 1] = sh.topm[D];
                if constexpr (MODE == kNand) xp.set_tcode(D, kNoEv);
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
        xor_top<F, N, T, D + 1, MODE>(d0, s, A0, st, ob, sh, chk, xp);
    }
}

// Update pass of subtree level J: the children's matrices (orders 2(Q - J) - 2) from the
// nodes in buf[J & 1] and the scaled pivot rows in wk.  Lane (h, k, i) writes columns
// [h cw, (h + 1) cw) of row i of child k: where the rows do not fill the wavefront, each row
// is split over H lanes.
template <class F, int Q, int J, int MODE>
__device__ __forceinline__ void xor_sub_update(XorLds<F, MODE>& sh)
{
    using E = typename F::E;
    constexpr int cur = J & 1, nxt = cur ^ 1;
    constexpr int m = 2 * (Q - J), mc = m - 2;
    constexpr int kids = MODE == kNand ? (int)pow3(J + 1) : 2 << J;
    constexpr int rows = kids * mc, H = col_groups(rows, mc), cw = mc / H;
    const int lane = threadIdx.x;
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

// NAND subtree level J whose fast pivot test failed (rare, out of line): each kept row tested
// on its row and column maxima; if any is shifted, the level's kept children are formed again
// with the shifted pivots.  Returns the shifts made (codes and own entries in sh).
template <class F, int Q, int J>
__device__ __noinline__ int nand_sub_slow(XorLds<F, kNand>& sh, double tau2, int es)
{
    using E = typename F::E;
    constexpr int cur = J & 1, nxt = cur ^ 1;
    constexpr int m = 2 * (Q - J), mc = m - 2;
    constexpr int kids = (int)pow3(J + 1);
    const int lane = threadIdx.x;
    XPiv xp{tau2, es, 0, 0, false, 0, 0};
    bool shifted = false;
    if (lane < 2 * (kids / 3)) {
        const int v = lane >> 1, p = mc + (lane & 1);
        const E* P = &sh.buf[cur][v * m * xs(m)];
        int8_t code;
        const E pv = nand_sub_pivot<F, m>(P, p, xp, code);
        const int ci = xsub_code_base(J) + 3 * v + (lane & 1) + 1;
        if (code != kNoEv) {
            sh.sown[ci] = F::bmul(sh.mn[cur][v], P[p * xs(m) + p], 0);
            shifted = true;
        }
        sh.scode[ci] = code;
        sh.pvs[lane] = pv;
    }
    const int ns = __builtin_popcountll(ballot(shifted));
    if (ns) {
        wave_sync();
        if (lane < kids) {
            const int v = lane / 3, c = lane - 3 * v;
            if (c) sh.mn[nxt][lane] = F::bmul(sh.mn[cur][v], sh.pvs[2 * v + c - 1], 0);
        }
        if (lane < 2 * (kids / 3) * mc) {
            const int v = lane / (2 * mc), rr = lane - v * 2 * mc, r = rr / mc, j = rr - r * mc;
            const E* P = &sh.buf[cur][v * m * xs(m)];
            sh.wk[lane] = F::rowscale(P[(mc + r) * xs(m) + j], F::recip(sh.pvs[2 * v + r]));
        }
        wave_sync();
        xor_sub_update<F, Q, J, kNand>(sh);
    }
    return ns;
}

// Subtree level J of a Q-level subtree: the children of the 2^J nodes in buf[J & 1]
// (order 2(Q - J)) into buf[(J + 1) & 1], one row (or column group) of a child per lane.
// base is where the children's depth T+J+1 starts in the output (2^(T+J+1) - 2; XOR
// only: the XNOR minors are the 2^N leaves, written at the last level in block-mask order).
template <class F, int Q, int J, int MODE>
__device__ __forceinline__ void xor_sub(int64_t base, int s, typename F::E* ob, XorLds<F, MODE>& sh, double& chk,
                                        XPiv& xp)
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
        bool maybe = false;   // NAND: this lane's fast pivot-shift test failed
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
            // (formed with the true pivots; the shift test comes after the update pass)
            for (int t = lane; t < kids; t += 64) {
                const int v = t / 3, c = t - 3 * v;
                E mk = sh.mn[cur][v];
                if (c) {
                    const int p = mc + c - 1;
                    mk = F::bmul(mk, sh.buf[cur][v * m * xs(m) + p * xs(m) + p], 0);
                }
                sh.mn[nxt][t] = mk;
                if constexpr (J == Q - 1) {
                    // leaves: written here unless the subtree's corrections come first
                    if (!xp.sub_mask) {
                        ob[(int64_t)s * pow3(Q) + t] = mk;
                        chk += F::fincheck(mk);
                    }
                } else {
                    chk += F::fincheck(mk);
                }
            }
            if constexpr (mc > 0) {
                static_assert(2 * (kids / 3) <= xsub_pairs_max() && 2 * (kids / 3) * mc <= 64 && kids <= 64,
                              "one pass per level");
                if (lane < 2 * (kids / 3) * mc) {
                    const int v = lane / (2 * mc), rr = lane - v * 2 * mc, r = rr / mc, j = rr - r * mc;
                    const E* P = &sh.buf[cur][v * m * xs(m)];
                    const int p = mc + r;
                    const E pv = P[p * xs(m) + p], pj = P[p * xs(m) + j];
                    sh.wk[lane] = F::rowscale(pj, F::recip(pv));
                    const int ep = xexp(pv);
                    maybe = ep == 0 || max(xexp(pj), xexp(P[j * xs(m) + p])) >= ep + kFastExp;
                }
            }
        }
        wave_sync();
        if constexpr (mc > 0) xor_sub_update<F, Q, J, MODE>(sh);
        if constexpr (MODE == kNand && mc > 0) {
            // the NAND pivot shift test (Sec. II), consumed after the children are formed (its
            // inputs are long loaded by then).  Fast test: each lane of the pivot-row pass
            // compared the exponents of one row and one column entry of its kept row with
            // p's; if no lane found one kFastExp above, no pivot of this level is shifted.  Otherwise each kept row
            // is tested on its row and column maxima, and if any is shifted the level's kept
            // children are formed again with the shifted pivots (pvs).
            if (ballot(maybe)) {
                const int ns = nand_sub_slow<F, Q, J>(sh, xp.tau2, xp.es);
                if (ns) {
                    xp.nsh += ns;
                    xp.sub_mask |= 1 << J;
                }
            }
        }
        xor_sub<F, Q, J + 1, MODE>(2 * base + 2, s, ob, sh, chk, xp);   // XOR depth T+J+2 starts at 2^(T+J+2) - 2
    }
}

// NAND pivot corrections (Sec. II, pivot correction; Sec. III, NAND case: applied once the
// subtree below the shifted node is complete, deepest node first).  A kept row l whose pivot
// was shifted by C makes every minor of the child's subtree det A~[S]; the true minor is
// det A~[S] - C det A[S \ {l}], and S \ {l} is the entry with the same choices except block
// l left out: digit 0 instead of the child's digit c, i.e. c spans earlier in the ternary
// order.  The child's own entry (no deeper row kept) is not corrected: it is the parent's
// minor times the true pivot, kept aside when the shift is made (as the minors tree records
// a node's own minor with the true pivot).

// Subtree levels, on the 3^Q leaves in LDS: child x of level J + 1 (digits of the leaf
// index above the span 3^(Q - 1 - J)).
template <class F, int Q, int MODE>
__device__ __noinline__ void nand_sub_fix(XorLds<F, MODE>& sh, int es, int mask)
{
    using E = typename F::E;
    constexpr int nl = (int)pow3(Q);
    E* mn = sh.mn[Q & 1];
    const int lane = threadIdx.x;
    for (int J = Q - 2; J >= 0; --J) {
        if (!((mask >> J) & 1)) continue;
        int span = 1;
        for (int k = 0; k < Q - 1 - J; ++k) span *= 3;
        for (int t = lane; t < nl; t += 64) {
            const int x = t / span, c = x % 3;
            if (c) {
                const int code = sh.scode[xsub_code_base(J) + x];
                if (code != kNoEv) {
                    // the child's own entry (t = x span) takes its minor with the true pivot
                    mn[t] = t == x * span ? sh.sown[xsub_code_base(J) + x]
                                          : F::sub_scaled(mn[t], shift_value(es, code), mn[t - c * span]);
                }
            }
        }
        wave_sync();
    }
}

// Top levels: the children chosen by path sp at depths T-1 .. dlo, whose subtrees end with
// path sp, on the outputs in global memory (this wavefront's own stores).
template <class F, int N, int T, int Q>
__device__ __noinline__ double nand_top_fix(int dlo, int sp, typename F::E* ob, uint64_t tc0, uint64_t tc1, int es)
{
    const XPiv xp{0.0, es, 0, 0, false, tc0, tc1};
    double chk = 0.0;
    using E = typename F::E;
    const int lane = threadIdx.x;
    constexpr int64_t q3 = pow3(Q);
    int64_t w = 1;                                  // top paths below a depth-D child: 3^(T-1-D)
    for (int D = T - 1; D >= dlo; --D, w *= 3) {
        const int code = xp.tcode(D);
        if (code == kNoEv) continue;
        wave_mem_fence();                           // the subtree's stores, and deeper corrections
        const int a = (int)((sp / w) % 3);
        const int64_t span = w * q3, base = (int64_t)(sp - sp % w) * q3;
        const double C = shift_value(xp.es, code);
        constexpr int kU = 2;
        for (int64_t i0 = base; i0 < base + span; i0 += 64 * kU) {
            E va[kU], vb[kU];
#pragma unroll
            for (int u = 0; u < kU; ++u) {
                const int64_t i = i0 + lane + 64 * u;
                if (i < base + span && i != base) {
                    va[u] = ob[i];
                    vb[u] = ob[i - a * span];
                }
            }
#pragma unroll
            for (int u = 0; u < kU; ++u) {
                const int64_t i = i0 + lane + 64 * u;
                if (i < base + span && i != base) {
                    const E r = F::sub_scaled(va[u], C, vb[u]);
                    ob[i] = r;
                    chk += F::fincheck(r);
                }
            }
        }
    }
    return chk;
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
    double amax = 0.0;
    for (int e = lane; e < w * w; e += 64) {
        fin = fin && F::in_finite(A0[e]);
        amax = fmax(amax, F::mag(A0[e]));
    }
    if (!__all(fin ? 1 : 0)) {
        for (int64_t i = lane; i < nout; i += 64) F::store_nan(ob, nullptr, i, false);
        if (info && lane == 0) info[b] = -2;
        return;
    }
    E* st = ws + (int64_t)b * ws_stride;
    double chk = 0.0;
    XPiv xp{kDefaultPivTol * kDefaultPivTol, 0, 0, 0, false, 0, 0};
    if constexpr (MODE == kNand) (void)frexp(wave_max(amax), &xp.es);
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
        if constexpr (MODE == kNand && T > 0) {
            if (s && (xp.tc0 | xp.tc1)) chk += nand_top_fix<F, N, T, Q>(d0, s - 1, ob, xp.tc0, xp.tc1, xp.es);
        }
        xor_top<F, N, T, 0, MODE>(d0, s, A0, st, ob, sh, chk, xp);
        // the subtree of depth-T node s, breadth first in LDS
        if constexpr (T == 0) {
            for (int e = lane; e < w * w; e += 64) sh.buf[0][(e / w) * xs(w) + e % w] = A0[e];
        }
        if (lane == 0) sh.mn[0][0] = sh.topm[T];
        wave_sync();
        xp.sub_mask = 0;
        xor_sub<F, Q, 0, MODE>((int64_t(2) << T) - 2, s, ob, sh, chk, xp);
        if constexpr (MODE == kNand) {
            if (xp.sub_mask) {
                nand_sub_fix<F, Q, MODE>(sh, xp.es, xp.sub_mask);
                for (int t = lane; t < (int)pow3(Q); t += 64) {
                    const E v = sh.mn[Q & 1][t];
                    ob[(int64_t)s * pow3(Q) + t] = v;
                    chk += F::fincheck(v);
                }
            }
            // a top-level child shifted on this path: its own entry (leaf 0 of this subtree,
            // written by lane 0 above) with the true pivot
            if (xp.top_own && lane == 0) {
                ob[(int64_t)s * pow3(Q)] = sh.topown;
                chk += F::fincheck(sh.topown);
            }
            xp.top_own = false;
        }
    }
    if constexpr (MODE == kNand && T > 0) {
        if (xp.tc0 | xp.tc1) chk += nand_top_fix<F, N, T, Q>(0, ntop - 1, ob, xp.tc0, xp.tc1, xp.es);
    }
    const bool bad = __any(chk == 0.0 ? 0 : 1);
    if (info && lane == 0) info[b] = bad ? -3 : xp.nsh;
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
