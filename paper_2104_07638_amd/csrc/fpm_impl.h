// fpm_impl.h -- all principal minors of a batch of small matrices on gfx950 (kernels).
//
// Method: the Griffin-Tsatsomeros binary tree of Schur complements (Sec. II,
// Eqs. (dets_schur)-(eq:minor) and Algorithm 1), traversed depth-first so that
// only one matrix per level is kept (Sec. II, the paragraph after Algorithm 1),
// with the near-zero-pivot shift C and its post-order back-propagation
//     det A[S] = det A~[S] - C det A[S \ {l}]          (Sec. II, pivot correction).
//
// Mapping (one matrix per wavefront, 64 lanes):
//   * the pivot order is a fixed permutation pi of the rows: first the T highest
//     rows n-1, n-2, ..., n-T ("top" levels), then rows 0, 1, 2, ... .  Every
//     level pivots on the first row of its (permuted) matrix, exactly as in the
//     paper; the permutation only decides which mask bit each level owns.
//   * top levels (bits n-1..n-T): cooperative depth-first walk in LDS; every
//     leaf of this walk is a "chunk" node of order K = MID + K0 whose subtree
//     owns the contiguous mask range [c 2^K, (c+1) 2^K).
//   * mid levels (bits 0..MID-1, MID = 6): the chunk node is expanded
//     breadth-first (first BF levels in LDS, the last two per lane in registers)
//     into 64 nodes of order K0 -- one per lane, lane = the 6 low mask bits.
//   * lane levels (bits MID..K-1): each lane walks its own subtree fully
//     unrolled in registers.  Minor j of lane l is mask c 2^K + j 2^6 + l, so
//     each store instruction of the wave writes 512 contiguous bytes (fp64).
//   * every mask is written exactly once, by the lane whose subtree contains it;
//     the node's recorded minor uses the true pivot (Algorithm 1 records before
//     it shifts), its right subtree uses the shifted one.
//   * shifted pivots (see analyse() for the test and the shift) are recorded as one byte
//     holding the signed power-of-two shift (top: one byte per chunk transition; mid:
//     one byte per node; lane: one byte per node packed in a 64-bit register) and
//     corrected after the stores, deepest level first, by read-modify-write passes
//     over the already written minors (rare path).
#pragma once
#include <stdlib.h>

#include "apm_device.h"
#include "apm_kernels.h"

namespace apm {

#ifndef APM_FPM_OCC
#define APM_FPM_OCC
#endif

constexpr int kMid = 6;

template <int N, int K0MAX>
struct Plan {
    static_assert(K0MAX >= 1 && K0MAX <= 5, "lane subtrees hold at most 15 shifted pivots per lane");
    static constexpr int mid = N < kMid ? N : kMid;
    static constexpr int k0 = (N - mid) < K0MAX ? (N - mid) : K0MAX;
    static constexpr int K = mid + k0;
    static constexpr int T = N - K;
    static constexpr int inl = mid < 2 ? mid : 2;
    static constexpr int bf = mid - inl;
    static constexpr int active = 1 << mid;
};

constexpr int sq(int x) { return x * x; }
constexpr int nz(int x) { return x > 0 ? x : 1; }

// Per-wave LDS layout: matrices (units of E), then small typed arrays.
template <class F, int N, int K0MAX>
struct Lay {
    using P = Plan<N, K0MAX>;
    using E = typename F::E;
    using R = typename F::R;
    using Bs = typename F::Bs;
    static constexpr int top_off(int d)
    {
        int s = 0;
        for (int i = 0; i < d; ++i) s += sq(N - i);
        return s;
    }
    // Mid levels 0..bf-1 are expanded breadth-first into compact matrices: BF level j
    // (1..bf) holds all 2^j nodes of order K-j; odd and even levels alternate buffers.
    // Rows are padded to an odd number of elements, so that lanes reading the same column
    // of consecutive rows (of one node or of consecutive nodes) hit distinct LDS banks.
    static constexpr int rs(int sz) { return sz | 1; }
    static constexpr int ns(int sz) { return sz * rs(sz); }
    static constexpr int lvl(int j) { return (1 << j) * ns(P::K - j); }
    static constexpr int bufA()
    {
        int m = 0;
        for (int j = 1; j <= P::bf; j += 2) m = lvl(j) > m ? lvl(j) : m;
        return m;
    }
    static constexpr int bufB()
    {
        int m = 0;
        for (int j = 2; j <= P::bf; j += 2) m = lvl(j) > m ? lvl(j) : m;
        return m;
    }
    static constexpr int nE = top_off(P::T + 1) + bufA() + bufB();
    static constexpr int nPiv = nz((1 << P::bf) - 1);   // mid nodes expanded breadth-first
    static constexpr size_t al(size_t x) { return (x + 15) & ~size_t(15); }
    static constexpr size_t oE = 0;
    static constexpr size_t oPt = al(oE + sizeof(E) * nE);
    static constexpr size_t oPu = al(oPt + sizeof(E) * nPiv);
    static constexpr size_t oRi = al(oPu + sizeof(E) * nPiv);
    static constexpr size_t oOff = al(oRi + sizeof(R) * nPiv);
    static constexpr size_t oLd = al(oOff + sizeof(int) * (P::T + 1));
    static constexpr size_t oBu = al(oLd + sizeof(int) * (P::T + 1));
    static constexpr size_t oRec = al(oBu + sizeof(Bs) * (P::T + 1));
    static constexpr size_t oTev = al(oRec + sizeof(Bs) * (P::T + 1));     // int8 [2^T]
    static constexpr size_t oMid = al(oTev + (size_t(1) << P::T));        // int8 [2][64]: two chunks
    static constexpr size_t bytes = al(oMid + 128);
    // element offset of BF level j (j >= 1); node q of that level starts at q ns(K-j)
    static constexpr int lvl_base(int j) { return top_off(P::T + 1) + ((j & 1) ? 0 : bufA()); }
};

struct Opts {
    double tau;      // relative pivot threshold
    bool perturb;
    bool out_f64;
    int* topq;       // deferred top-level corrections (NULL: applied by the wavefront itself)
    int topq_cap;    // matrices the queue holds (slot index = matrix index)
    int split;       // work items per matrix (a power of two dividing the chunk count); > 1 needs topq
    int* part;       // split > 1: per-item info codes, combined by the last deferred-correction launch
};

// Most work items per matrix of a uniform launch with deferred top-level corrections: each
// of g items takes 2^T / g consecutive chunks, so that one matrix with many shifted pivots
// (whose corrections reread its minors) spreads over several wavefronts instead of holding
// one.
constexpr int kSplit = 4;

// Deferred top-level corrections.  A wavefront whose matrix has shifted pivots in the top
// levels records them in the matrix's slot of a queue instead of applying the corrections
// itself, and lists the matrix once; a follow-up launch applies every level's corrections of
// the listed matrices in one pass.  Queue layout (int32, cap matrices): [0] listed matrices,
// [1] workgroups done; from int kTopHead on, one slot of kTopEntryInts per matrix: out (2),
// ex (2), es_true (1), the shift code of each top node by chunk (8 ints = 32 bytes), the
// listed flag (1); then the list (cap ints); then, for split launches, the info code of each
// work item (cap * kSplit ints).  Ints 2 .. 2 + kTopCounts - 1 of the head are the completion
// counts of the correction launch.  Codes, flags and counts are zero between uses.
constexpr int kTopDeferMaxT = 5;
constexpr int kTopEntryInts = 14;
constexpr int kTopCodes = 5;     // first int of the shift codes in a slot
constexpr int kTopFlag = 13;     // the listed flag
constexpr int kTopHead = 64;
constexpr int kTopCounts = 8;    // partial completion counts of the correction launch (ints 2 ..)
static_assert(2 + kTopCounts == kTopCounterInts && kTopCounterInts <= kTopHead, "the counters fit the queue head");

// Matrix-wide parameters of the pivot shift.
struct PivCtl {
    double tau2;     // tau^2
    int es;          // binary exponent of s = max |A_ij| in stored units
    int es_true;     // the same in true units (stored = true * 2^-e0)
    bool perturb;
};

// Largest value of v[0..M) by a pairwise tree (depth log2 M instead of a chain of M).
template <int M>
__device__ __forceinline__ double tree_max(double (&v)[M])
{
#pragma unroll
    for (int w = 1; w < M; w *= 2)
#pragma unroll
        for (int i = 0; i + w < M; i += 2 * w) v[i] = fmax(v[i], v[i + w]);
    return M > 0 ? v[0] : 0.0;
}

template <class F>
struct PivInfo {
    typename F::E pt, pu;
    typename F::R ri;
    bool pert;
    int8_t code;     // shift code (see shift_value), kNoEv if not shifted
};

// Pivot analysis of a node (Sec. II, pivot correction).  A pivot p is shifted when
// |p|^2 < tau^2 * rmax * cmax, rmax / cmax being the largest magnitudes in the pivot's
// row / column of the node's matrix (a test invariant under diagonal similarity), or
// when p == 0.  The shift C takes the sign of Re p, so that it never cancels the pivot;
// its magnitude is given above (s / 16 when the row or column vanishes: the right child
// then equals the left one exactly, times C).
template <class F>
__device__ __forceinline__ PivInfo<F> analyse(typename F::E p, double rmax, double cmax, int size,
                                              const PivCtl& pc)
{
    PivInfo<F> v;
    v.pt = p;
    v.code = kNoEv;
    const double prod = rmax * cmax;
    const double pm = F::mag(p);
    v.pert = pc.perturb && size >= 2 && (pm == 0.0 || pm * pm < pc.tau2 * prod);
    v.pu = p;
    if (v.pert) {
        v.code = shift_code(rmax, cmax, pc.es, F::re(p) < 0.0);
        v.pu = F::shift(p, shift_value(pc.es, v.code));
    }
    v.ri = F::recip(v.pu);
    return v;
}

template <class F>
struct Ctx {
    void* op;       // this lane's first output of the chunk (mask c 2^K + lane)
    int16_t* ep;    // the same for the exponents (scaled variants)
    bool active;    // lane < 2^MID (always true for N >= 6)
    bool f64;
    uint32_t ev;    // lane-level shifted pivots: bit = heap index of the node
    uint64_t lc0;   // their shift exponents, one byte per heap index 0..7
    uint64_t lc1;   // ... and 8..14
    double chk;     // sum of v * 0 over stored minors: NaN iff one was not finite
};

// Store lane minor j (mask c 2^K + j 2^MID + lane): 64 lanes write 64 consecutive masks.
template <class F, bool AL>
__device__ __forceinline__ void put(Ctx<F>& cx, int j, typename F::Bs v)
{
    if (AL || cx.active) F::store_rel(cx.op, cx.ep, j << kMid, v, cx.f64);
    cx.chk += (double)F::fincheck(v);
}

// Lane subtree: node of order KP - S0 held as the trailing view (S0.., S0..) of the
// register matrix M (KP x KP); DEP = depth below the lane root, Q = bits decided so far.
// Records the node's minor with the true pivot, then the left child (a view), then the
// right child (Schur complement, possibly with a shifted pivot).
template <class F, bool AL, int KP, int S0, int DEP, int Q>
__device__ __forceinline__ void lane_node(const typename F::E (&M)[KP * KP], typename F::Bs bu, Ctx<F>& cx,
                                          const PivCtl& pc, int e0)
{
    using E = typename F::E;
    constexpr int SZ = KP - S0;
    const E p = M[S0 * KP + S0];
    put<F, AL>(cx, Q | (1 << DEP), F::bmul(bu, p, e0));
    if constexpr (SZ == 2) {
        // a 2 x 2 node is finished without division: the left child's minor is bu d and
        // the right child's is bu (p d - c r), exact whatever the pivot, so no shift
        const E r = M[S0 * KP + S0 + 1], c = M[(S0 + 1) * KP + S0], d = M[(S0 + 1) * KP + S0 + 1];
        put<F, AL>(cx, Q | (1 << (DEP + 1)), F::bmul(bu, d, e0));
        // (the scaled variants store values times 2^-e0, so the product of two carries 2^-2 e0)
        put<F, AL>(cx, Q | (1 << DEP) | (1 << (DEP + 1)), F::bmul(bu, F::det2(p, r, c, d), 2 * e0));
    } else if constexpr (SZ > 2) {
        lane_node<F, AL, KP, S0 + 1, DEP + 1, Q>(M, bu, cx, pc, e0);
        constexpr int m = SZ - 1;
        double rv[m], cv[m];
#pragma unroll
        for (int b = 0; b < m; ++b) {
            rv[b] = F::mag(M[S0 * KP + S0 + 1 + b]);
            cv[b] = F::mag(M[(S0 + 1 + b) * KP + S0]);
        }
        const PivInfo<F> pv = analyse<F>(p, tree_max<m>(rv), tree_max<m>(cv), SZ, pc);
        constexpr int id = (1 << DEP) - 1 + Q;
        if (pv.pert) {
            cx.ev |= 1u << id;
            constexpr int sh = 8 * (id & 7);
            const uint64_t byte = (uint64_t)(uint8_t)pv.code << sh;
            if constexpr (id < 8)
                cx.lc0 = (cx.lc0 & ~(0xFFull << sh)) | byte;
            else
                cx.lc1 = (cx.lc1 & ~(0xFFull << sh)) | byte;
        }
        E w[m];
#pragma unroll
        for (int b = 0; b < m; ++b) w[b] = F::rowscale(M[S0 * KP + S0 + 1 + b], pv.ri);
        E S[m * m];
#pragma unroll
        for (int a = 0; a < m; ++a)
#pragma unroll
            for (int b = 0; b < m; ++b)
                S[a * m + b] = F::upd(M[(S0 + 1 + a) * KP + S0 + 1 + b], M[(S0 + 1 + a) * KP + S0], w[b]);
        lane_node<F, AL, m, 0, DEP + 1, Q | (1 << DEP)>(S, F::bmul(bu, pv.pu, e0), cx, pc, e0);
    }
}

// Row / column magnitude maxima of the pivot of a register matrix of order SZ.
template <class F, int SZ>
__device__ __forceinline__ void rc_max(const typename F::E (&M)[SZ * SZ], double& rmax, double& cmax)
{
    double rv[SZ - 1 > 0 ? SZ - 1 : 1], cv[SZ - 1 > 0 ? SZ - 1 : 1];
#pragma unroll
    for (int b = 1; b < SZ; ++b) {
        rv[b - 1] = F::mag(M[b]);
        cv[b - 1] = F::mag(M[b * SZ]);
    }
    rmax = SZ > 1 ? tree_max(rv) : 0.0;
    cmax = SZ > 1 ? tree_max(cv) : 0.0;
}

// One in-lane mid level: node M (order SZ, registers) -> the lane's child (order SZ-1):
// the Schur complement if the lane's bit of this level is set, else the trailing view.
template <class F, int SZ>
__device__ __forceinline__ void inlane_step(const typename F::E (&M)[SZ * SZ], typename F::E (&Q)[nz(sq(SZ - 1))],
                                            bool right, typename F::R ri)
{
    using E = typename F::E;
    constexpr int m = SZ - 1;
    E w[nz(m)];
#pragma unroll
    for (int b = 0; b < m; ++b) w[b] = right ? F::rowscale(M[1 + b], ri) : F::zero();
#pragma unroll
    for (int a = 0; a < m; ++a)
#pragma unroll
        for (int b = 0; b < m; ++b) Q[a * m + b] = F::upd(M[(1 + a) * SZ + 1 + b], M[(1 + a) * SZ], w[b]);
}

// Columns per lane of a breadth-first level of `rows` rows of m entries: as few as the
// wavefront allows, the column groups as even as that count permits.
constexpr int bf_cols(int rows, int m)
{
    const int hmax = kWave / rows < m ? kWave / rows : m;
    return (m + hmax - 1) / hmax;
}

// Breadth-first mid level J (and, recursively, the following ones) of a chunk: lane
// (t, a) writes row a of both children of node (J, t) -- the left child (the trailing
// block) and the right child (the Schur complement), or a group of its columns.  Every
// lane of a node repeats the node's pivot analysis; one lane publishes it.
template <class F, int N, int K0MAX, int J>
__device__ __forceinline__ void bf_levels(typename F::E* lds, typename F::E* pt_a, typename F::E* pu_a,
                                          typename F::R* ri_a, int8_t* midc, int x0o, int x0l, int lane,
                                          const PivCtl& pc, bool& mid_any)
{
    using P = Plan<N, K0MAX>;
    using L = Lay<F, N, K0MAX>;
    using E = typename F::E;
    if constexpr (J < P::bf) {
        constexpr int nodes = 1 << J;
        constexpr int sz = P::K - J;
        constexpr int m = sz - 1;
        static_assert(nodes * m <= kWave, "one row per lane");
        // where the rows do not fill the wavefront, each is split over H lanes: lane
        // (h, t, a) writes columns [h cw, (h + 1) cw) of row a of node t's children
        constexpr int rows = nodes * m, cw = bf_cols(rows, m), H = (m + cw - 1) / cw;
        constexpr bool kEven = m % cw == 0;
        bool pert = false;
        if (lane < rows * H) {
            const int r = lane % rows, h = lane / rows;
            const int t = r / m, a = r - t * m, j0 = h * cw;
            const E* Pm = (J == 0) ? lds + x0o : lds + L::lvl_base(J) + t * L::ns(sz);
            const int pl = (J == 0) ? x0l : L::rs(sz);
            E row[cw], mine[cw];
            double rv[m], cv[m];
#pragma unroll
            for (int b = 0; b < m; ++b) {
                rv[b] = F::mag(Pm[b + 1]);
                cv[b] = F::mag(Pm[(b + 1) * pl]);
            }
#pragma unroll
            for (int b = 0; b < cw; ++b) {
                if (kEven || j0 + b < m) {
                    row[b] = Pm[j0 + b + 1];
                    mine[b] = Pm[(a + 1) * pl + j0 + b + 1];
                }
            }
            const E c = Pm[(a + 1) * pl];
            const PivInfo<F> pv = analyse<F>(Pm[0], tree_max(rv), tree_max(cv), sz, pc);
            E* Lr = lds + L::lvl_base(J + 1) + t * L::ns(m) + a * L::rs(m) + j0;
            E* Rr = Lr + nodes * L::ns(m);
#pragma unroll
            for (int b = 0; b < cw; ++b) {
                if (kEven || j0 + b < m) {
                    Lr[b] = mine[b];
                    Rr[b] = F::upd(mine[b], c, F::rowscale(row[b], pv.ri));
                }
            }
            if (a == 0 && h == 0) {
                pt_a[nodes - 1 + t] = pv.pt;
                pu_a[nodes - 1 + t] = pv.pu;
                ri_a[nodes - 1 + t] = pv.ri;
                midc[nodes - 1 + t] = pv.code;
                pert = pv.pert;
            }
        }
        mid_any |= ballot(pert) != 0;
        wave_sync();
        bf_levels<F, N, K0MAX, J + 1>(lds, pt_a, pu_a, ri_a, midc, x0o, x0l, lane, pc, mid_any);
    }
}

// Top level D: take the right branch of the depth-D node (Schur complement of order
// N-D-1 into top storage D+1), a column per lane over groups of rows.  Returns the pivot
// analysis.
template <class F, int N, int K0MAX, int D>
__device__ __forceinline__ PivInfo<F> top_right(typename F::E* lds, int xo, int xl, int lane, const PivCtl& pc)
{
    using L = Lay<F, N, K0MAX>;
    using E = typename F::E;
    constexpr int m = N - D - 1;
    const E* X = lds + xo;
    double rv[m], cv[m];
#pragma unroll
    for (int b = 0; b < m; ++b) {      // every lane reads the same entries (broadcast)
        rv[b] = F::mag(X[b + 1]);
        cv[b] = F::mag(X[(b + 1) * xl]);
    }
    const PivInfo<F> pv = analyse<F>(X[0], tree_max(rv), tree_max(cv), m + 1, pc);
    E* S = lds + L::top_off(D + 1);
    // lane (a0, b): column b of rows a0, a0 + g, ... (g = 64 / m row groups)
    constexpr int g = kWave / m;
    if (lane < g * m) {
        const int b = lane % m, a0 = lane / m;
        const E wb = F::rowscale(X[b + 1], pv.ri);
        for (int a = a0; a < m; a += g) {
            const E* xr = X + (a + 1) * xl;
            S[a * m + b] = F::upd(xr[b + 1], xr[0], wb);
        }
    }
    return pv;
}

template <class F, int N, int K0MAX, int D>
__device__ __forceinline__ PivInfo<F> top_right_at(int d, typename F::E* lds, int xo, int xl, int lane,
                                                   const PivCtl& pc)
{
    if constexpr (D + 1 < Plan<N, K0MAX>::T) {
        if (d != D) return top_right_at<F, N, K0MAX, D + 1>(d, lds, xo, xl, lane, pc);
    }
    return top_right<F, N, K0MAX, D>(lds, xo, xl, lane, pc);
}

// Cross-lane exchange of a correction value (fp64, or the two halves of a complex value).
__device__ __forceinline__ double shfl_xor_v(double v, int m) { return __shfl_xor(v, m); }
__device__ __forceinline__ cd shfl_xor_v(cd v, int m) { return {__shfl_xor(v.x, m), __shfl_xor(v.y, m)}; }

// Lane-level corrections of depth DEP and above (deepest first), on a lane's minors held in
// registers: lane node (DEP, q) with a shifted pivot corrects the minors of its strict right
// subtree, j = q | 2^DEP | u 2^(DEP+1) with u >= 1, as m[j] -= C m[j - 2^DEP] (Sec. II, pivot
// correction).
template <class F, int K0, int DEP>
__device__ __forceinline__ void lane_fix_reg(typename F::V (&v)[1 << K0], uint32_t& touched, uint32_t ev,
                                             uint64_t lc0, uint64_t lc1, int es_true)
{
    if constexpr (DEP >= 0) {
        constexpr int nq = 1 << DEP, nu = 1 << (K0 - 1 - DEP);
#pragma unroll
        for (int q = 0; q < nq; ++q) {
            const int id = nq - 1 + q;
            if ((ev >> id) & 1u) {
                const uint64_t lw = id < 8 ? lc0 : lc1;
                const double Ct = shift_value(es_true, (int)(uint8_t)(lw >> (8 * (id & 7))));
#pragma unroll
                for (int u = 1; u < nu; ++u) {
                    const int j = q | nq | (u << (DEP + 1));
                    v[j] = F::sub_scaled(v[j], Ct, v[j - nq]);
                    touched |= 1u << j;
                }
            }
        }
        lane_fix_reg<F, K0, DEP - 1>(v, touched, ev, lc0, lc1, es_true);
    }
}

// Correct the minors of one chunk for its lane- and mid-level shifted pivots, deepest level
// first: det A[S] = det A~[S] - C det A[S \ {l}] over each shifted node's strict right subtree
// (Sec. II, pivot correction).  One pass: every lane loads its own 2^k0 minors of the chunk
// (all loads in flight together; a lane rereads only what it stored itself, so program order
// suffices), applies the lane-level corrections in registers, then the mid-level ones with the
// partner lane's values taken by cross-lane exchange (mid node (b, q) corrects lane l with bit
// b set from lane l - 2^b), and stores what changed.
template <class F, int N, int K0MAX>
__device__ __noinline__ void chunk_fixup(void* out, int16_t* ex, int64_t base, int lane, bool f64, uint32_t ev,
                                         uint64_t lc0, uint64_t lc1, const int8_t* midc, int es_true)
{
    using P = Plan<N, K0MAX>;
    constexpr int k0 = P::k0, J = 1 << k0;
    using V = typename F::V;
    const bool active = lane < P::active;
    V v[J];
#pragma unroll
    for (int j = 0; j < J; ++j) {
        if (active) v[j] = F::load_v(out, ex, base + ((int64_t)j << kMid) + lane, f64);
        else v[j] = V{};
    }
    uint32_t touched = 0;
    // lane subtree nodes of order >= 3 (depth <= k0 - 3) can be shifted; 2 x 2 nodes are not
    if constexpr (k0 >= 3) {
        if (active) lane_fix_reg<F, k0, k0 - 3>(v, touched, ev, lc0, lc1, es_true);
    }
    for (int b = P::mid - 1; b >= 0; --b) {
        const int q = lane & ((1 << b) - 1);
        const int code = midc[(1 << b) - 1 + q];
        const bool mine = active && ((lane >> b) & 1) && code != kNoEv;
        if (ballot(mine) == 0) continue;
        const double Ct = mine ? shift_value(es_true, code) : 0.0;
        const bool skip0 = (lane >> (b + 1)) == 0;   // the node's own recorded minor (j = 0)
#pragma unroll
        for (int j = 0; j < J; ++j) {
            const V pv = shfl_xor_v(v[j], 1 << b);
            if (mine && !(j == 0 && skip0)) {
                v[j] = F::sub_scaled(v[j], Ct, pv);
                touched |= 1u << j;
            }
        }
    }
#pragma unroll
    for (int j = 0; j < J; ++j)
        if (active && ((touched >> j) & 1u)) F::store_v(out, ex, base + ((int64_t)j << kMid) + lane, v[j], f64);
}

// Count and correct the shifted mid- and lane-level pivots of chunk c (whose shift codes are
// in midc and in the lane registers ev / lc0 / lc1).
template <class F, int N, int K0MAX>
__device__ __forceinline__ void fix_chunk(void* out, int16_t* ex, int c, int lane, bool f64, uint32_t ev,
                                          uint64_t lc0, uint64_t lc1, const int8_t* midc, int es_true, int& nev)
{
    using P = Plan<N, K0MAX>;
    const bool active = lane < P::active;
    int nm = 0;
    for (int i = lane; i < (1 << P::mid) - 1; i += kWave) nm += midc[i] != kNoEv;
    nev += wave_sum(nm + (active ? __builtin_popcount(ev) : 0));
    chunk_fixup<F, N, K0MAX>(out, ex, (int64_t)c << P::K, lane, f64, ev, lc0, lc1, midc, es_true);
}

// All principal minors of one N x N matrix by one wavefront.  Returns the info code.
template <class F, int N, int K0MAX>
__device__ __forceinline__ int fpm_wave(const typename F::In* __restrict__ A, void* out, int16_t* ex,
                                        unsigned char* lds_raw, const Opts& o, int g = 0, int mat = 0)
{
    using P = Plan<N, K0MAX>;
    using L = Lay<F, N, K0MAX>;
    using E = typename F::E;
    using R = typename F::R;
    using Bs = typename F::Bs;
    constexpr int K = P::K, T = P::T, bf = P::bf, k0 = P::k0;
    const int lane = lane_id();

    E* lds = reinterpret_cast<E*>(lds_raw + L::oE);
    E* pt_a = reinterpret_cast<E*>(lds_raw + L::oPt);
    E* pu_a = reinterpret_cast<E*>(lds_raw + L::oPu);
    R* ri_a = reinterpret_cast<R*>(lds_raw + L::oRi);
    int* off_a = reinterpret_cast<int*>(lds_raw + L::oOff);
    int* ld_a = reinterpret_cast<int*>(lds_raw + L::oLd);
    Bs* bu_a = reinterpret_cast<Bs*>(lds_raw + L::oBu);
    Bs* rec_a = reinterpret_cast<Bs*>(lds_raw + L::oRec);
    int8_t* tevc = reinterpret_cast<int8_t*>(lds_raw + L::oTev);
    int8_t* const midc_base = reinterpret_cast<int8_t*>(lds_raw + L::oMid);

    // ---- load, scale, finiteness ------------------------------------------------------
    double smax = 0.0;
    bool bad = false;
    for (int i = lane; i < N * N; i += kWave) {
        const typename F::In v = A[i];
        bad |= !F::in_finite(v);
        smax = fmax(smax, F::in_mag(v));
    }
    // this item's chunks [c0, c1) (the whole matrix unless it is split)
    const int nsplit = (T > 0 && o.split > 1) ? o.split : 1;
    const int c0 = g * ((1 << T) / nsplit), c1 = c0 + (1 << T) / nsplit;
    if (ballot(bad)) {
        for (int64_t i = ((int64_t)c0 << K) + lane; i < ((int64_t)c1 << K); i += kWave) F::store_nan(out, ex, i, o.out_f64);
        return -2;
    }
    double s = wave_max(smax);
    if (s == 0.0) s = 1.0;
    int e0 = 0;
    if constexpr (F::kScaled) (void)frexp(s, &e0);
    const double sc = ldexp(1.0, -e0);
    PivCtl pc;
    pc.tau2 = o.tau * o.tau;
    pc.perturb = o.perturb;
    (void)frexp(s * sc, &pc.es);
    pc.es_true = pc.es + e0;
    for (int i = lane; i < N * N; i += kWave) {
        const int a = i / N, b = i - (i / N) * N;
        const int pa = a < T ? N - 1 - a : a - T;
        const int pb = b < T ? N - 1 - b : b - T;
        lds[i] = F::conv(A[pa * N + pb], sc);
    }
    for (int c = lane; c < (1 << T); c += kWave) tevc[c] = kNoEv;
    if (lane <= T) {
        off_a[lane] = lane * (N + 1);
        ld_a[lane] = N;
        bu_a[lane] = F::one();
        rec_a[lane] = F::one();
    }
    wave_sync();

    int nev = 0;
    bool any_top = false;
    double chkf = 0.0;
    // Corrections of a chunk's shifted mid- and lane-level pivots are applied one chunk late,
    // after the next chunk's top and breadth-first levels (LDS work): by then the chunk's
    // stores have drained, and reading them back does not stall the wavefront.
    bool pend = false;           // the previous chunk has shifted pivots (wavefront-uniform)
    uint32_t pev = 0;
    uint64_t plc0 = 0, plc1 = 0;

    // Top step: take the right branch at top level d (Schur complement into top storage d+1).
    // A shift is counted and recorded (for the chunk c at which that branch is first taken)
    // only by the item that owns chunk c.
    auto top_step = [&](int d, int c, bool own) {
      if constexpr (T > 0) {
        const int m = N - d - 1;
        const PivInfo<F> pv = top_right_at<F, N, K0MAX, 0>(d, lds, off_a[d], ld_a[d], lane, pc);
        const Bs bud = bu_a[d];
        if (pv.pert && own) {
            nev += 1;
            any_top = true;
            if (lane == 0) tevc[c] = pv.code;
        }
        const Bs bnew = F::bmul(bud, pv.pu, e0);
        const Bs rnew = F::bmul(bud, pv.pt, e0);
        for (int dd = d + 1 + lane; dd <= T; dd += kWave) {
            off_a[dd] = L::top_off(d + 1) + (dd - d - 1) * (m + 1);
            ld_a[dd] = m;
            bu_a[dd] = bnew;
            rec_a[dd] = rnew;
        }
        wave_sync();
      }
    };
    if constexpr (T > 0) {
        // the path to the item's first chunk: a right branch for every set bit of c0
        for (int d = 0; d < T; ++d)
            if ((c0 >> (T - 1 - d)) & 1) top_step(d, c0, d == T - 1 - __builtin_ctz((unsigned)c0));
    }

    for (int c = c0; c < c1; ++c) {
        int8_t* const midc = midc_base + 64 * (c & 1);
        // ---- top: take the right branch at the deepest level that changes -----------
        if constexpr (T > 0) if (c > c0) top_step(T - 1 - __builtin_ctz((unsigned)c), c, true);
        const int x0o = off_a[T], x0l = ld_a[T];
        const Bs bu0 = bu_a[T], rec0 = rec_a[T];

        // ---- mid levels 0..bf-1: breadth-first in LDS --------------------------------
        bool mid_any = false;
        bf_levels<F, N, K0MAX, 0>(lds, pt_a, pu_a, ri_a, midc, x0o, x0l, lane, pc, mid_any);

        // ---- the previous chunk's pivot corrections -----------------------------------
        if (pend) fix_chunk<F, N, K0MAX>(out, ex, c - 1, lane, o.out_f64, pev, plc0, plc1,
                                         midc_base + 64 * ((c - 1) & 1), pc.es_true, nev);
        pend = false;

        // ---- mid levels bf.., per lane, in registers ---------------------------------
        constexpr bool AL = (P::active == kWave);
        constexpr int szb = K - bf;               // order of the lane's level-bf node
        const int tb = lane & ((1 << bf) - 1);
        const E* Pb = (bf == 0) ? lds + x0o : lds + L::lvl_base(bf) + tb * L::ns(szb);
        const int pbl = (bf == 0) ? x0l : L::rs(szb);
        E r0[nz(szb - 1)], c0[nz(szb - 1)];
#pragma unroll
        for (int b = 0; b < szb - 1; ++b) {
            r0[b] = Pb[b + 1];
            c0[b] = Pb[(b + 1) * pbl];
        }
        double rvm[nz(szb - 1)], cvm[nz(szb - 1)];
#pragma unroll
        for (int b = 0; b < szb - 1; ++b) {
            rvm[b] = F::mag(r0[b]);
            cvm[b] = F::mag(c0[b]);
        }
        const double rm = szb > 1 ? tree_max(rvm) : 0.0, cm = szb > 1 ? tree_max(cvm) : 0.0;
        const PivInfo<F> v0 = analyse<F>(Pb[0], rm, cm, szb, pc);
        mid_any |= ballot(lane < (1 << bf) && v0.pert) != 0;
        if (lane < (1 << bf)) midc[(1 << bf) - 1 + lane] = v0.code;
        const bool rb0 = (lane >> bf) & 1;
        E M1[nz(sq(szb - 1))];
#pragma unroll
        for (int b = 0; b < szb - 1; ++b) r0[b] = rb0 ? F::rowscale(r0[b], v0.ri) : F::zero();
#pragma unroll
        for (int a = 0; a < szb - 1; ++a)
#pragma unroll
            for (int b = 0; b < szb - 1; ++b)
                M1[a * (szb - 1) + b] = F::upd(Pb[(a + 1) * pbl + b + 1], c0[a], r0[b]);
        // lane base: product of the used pivots on the lane's right branches; the recorded
        // value of the lane's own mask uses the true pivot at its highest bit.
        Bs acc = bu0, rec = rec0;
        const int h = lane ? 31 - __builtin_clz((unsigned)lane) : -1;
#pragma unroll
        for (int j = 0; j < bf; ++j) {
            if ((lane >> j) & 1) {
                const int id = (1 << j) - 1 + (lane & ((1 << j) - 1));
                if (j == h) rec = F::bmul(acc, pt_a[id], e0);
                acc = F::bmul(acc, pu_a[id], e0);
            }
        }
        if (rb0) {
            if (bf == h) rec = F::bmul(acc, v0.pt, e0);
            acc = F::bmul(acc, v0.pu, e0);
        }

        Ctx<F> cx;
        cx.op = F::optr(out, ((int64_t)c << K) + lane, o.out_f64);
        cx.ep = ex ? ex + ((int64_t)c << K) + lane : nullptr;
        cx.active = lane < P::active;
        cx.f64 = o.out_f64;
        cx.ev = 0;
        cx.lc0 = 0;
        cx.lc1 = 0;
        cx.chk = 0.0;

        if constexpr (P::inl == 2) {
            constexpr int sz1 = szb - 1;
            double rm1, cm1;
            rc_max<F, sz1>(M1, rm1, cm1);
            const PivInfo<F> v1 = analyse<F>(M1[0], rm1, cm1, sz1, pc);
            mid_any |= ballot(lane < (2 << bf) && v1.pert) != 0;
            if (lane < (2 << bf)) midc[(2 << bf) - 1 + lane] = v1.code;
            if ((lane >> (bf + 1)) & 1) {
                if (bf + 1 == h) rec = F::bmul(acc, v1.pt, e0);
                acc = F::bmul(acc, v1.pu, e0);
            }
            put<F, AL>(cx, 0, rec);
            if constexpr (k0 > 0) {
                E M2[k0 * k0];
                inlane_step<F, sz1>(M1, M2, (lane >> (bf + 1)) & 1, v1.ri);
                lane_node<F, AL, k0, 0, 0, 0>(M2, acc, cx, pc, e0);
            }
        } else {
            put<F, AL>(cx, 0, rec);
        }

        // ---- rare path: shifted pivots inside this chunk, corrected after the next one's
        //      breadth-first levels (or after the loop for the last chunk)
        const bool lane_ev = ballot(cx.active && cx.ev != 0) != 0;
        pend = lane_ev || mid_any;
        pev = cx.ev;
        plc0 = cx.lc0;
        plc1 = cx.lc1;
        chkf += cx.chk;
    }
    if (pend) {
        const int cl = c1 - 1;
        wave_sync();
        fix_chunk<F, N, K0MAX>(out, ex, cl, lane, o.out_f64, pev, plc0, plc1, midc_base + 64 * (cl & 1), pc.es_true,
                               nev);
    }

    // ---- top-level corrections, deepest first ---------------------------------------
    if constexpr (T > 0) {
        bool deferred = false;
        if constexpr (T <= kTopDeferMaxT) {
            if (any_top && o.topq && mat < o.topq_cap) {
                // the matrix's slot: every item of a split matrix writes the same header and
                // the codes of its own chunks; the first to set the flag lists the matrix
                deferred = true;
                int* ent = o.topq + kTopHead + (int64_t)mat * kTopEntryInts;
                if (lane == 0) {
                    const uint64_t po = reinterpret_cast<uint64_t>(out), pe = reinterpret_cast<uint64_t>(ex);
                    ent[0] = (int)(uint32_t)po;
                    ent[1] = (int)(uint32_t)(po >> 32);
                    ent[2] = (int)(uint32_t)pe;
                    ent[3] = (int)(uint32_t)(pe >> 32);
                    ent[4] = pc.es_true;
                }
                int8_t* tv = reinterpret_cast<int8_t*>(ent + kTopCodes);
                for (int c = c0 + lane; c < c1; c += kWave) tv[c] = tevc[c];
                if (lane == 0) {
                    const bool first = nsplit == 1 || atomicExch(ent + kTopFlag, 1) == 0;
                    if (first) {
                        int* list = o.topq + kTopHead + (int64_t)o.topq_cap * kTopEntryInts;
                        list[atomicAdd(o.topq, 1)] = mat;
                    }
                }
            }
        }
        if (any_top && !deferred && nsplit > 1) return -3;   // cannot happen: the queue holds every item
        if (any_top && !deferred) {
            wave_mem_fence();
            for (int d = T - 1; d >= 0; --d) {
                const int step = 1 << (T - 1 - d);
                const int64_t half = int64_t(1) << (N - 1 - d);
                bool did = false;
                for (int c = step; c < (1 << T); c += 2 * step) {
                    const int de = tevc[c];
                    if (de == kNoEv) continue;
                    did = true;
                    const double Ct = shift_value(pc.es_true, de);
                    const int64_t start = (int64_t)c << K, end = start + half;
                    constexpr int kU = 8;
                    for (int64_t i0 = start + 1; i0 < end; i0 += kWave * kU) {
                        typename F::V va[kU], vb[kU];
#pragma unroll
                        for (int u = 0; u < kU; ++u) {
                            const int64_t i = i0 + lane + kWave * u;
                            if (i < end) {
                                va[u] = F::load_v(out, ex, i, o.out_f64);
                                vb[u] = F::load_v(out, ex, i - half, o.out_f64);
                            }
                        }
#pragma unroll
                        for (int u = 0; u < kU; ++u) {
                            const int64_t i = i0 + lane + kWave * u;
                            if (i < end) F::store_v(out, ex, i, F::sub_scaled(va[u], Ct, vb[u]), o.out_f64);
                        }
                    }
                }
                if (did) wave_mem_fence();
            }
        }
    }
    const bool nonfinite = ballot(!(chkf == chkf)) != 0;
    return nonfinite ? -3 : nev;
}

// ------------------------------------------------------------------------------ kernels
template <class F, int N, int K0MAX>
__global__ __launch_bounds__(64) APM_FPM_OCC void fpm_uniform_kernel(const typename F::In* __restrict__ A, void* out,
                                                         int16_t* ex, int32_t* info, int32_t batch,
                                                         const int64_t* __restrict__ in_off,
                                                         const int64_t* __restrict__ out_off, Opts o)
{
    extern __shared__ __align__(16) unsigned char lds_dyn[];
    const int G = o.split > 1 ? o.split : 1;
    const int b = (int)(blockIdx.x / G), g = (int)(blockIdx.x % G);
    if (b >= batch) return;
    const int64_t io = in_off ? in_off[b] : (int64_t)b * N * N;
    const int64_t oo = out_off ? out_off[b] : ((int64_t)b << N);
    void* ob;
    if constexpr (F::kComplex) {
        ob = (o.out_f64 || !F::kScaled) ? (void*)(static_cast<cd*>(out) + oo) : (void*)(static_cast<cf*>(out) + oo);
    } else {
        ob = (o.out_f64 || !F::kScaled) ? (void*)(static_cast<double*>(out) + oo)
                                        : (void*)(static_cast<float*>(out) + oo);
    }
    int16_t* eb = ex ? ex + oo : nullptr;
    const int r = fpm_wave<F, N, K0MAX>(A + io, ob, eb, lds_dyn, o, g, b);
    if (lane_id() == 0) {
        if (G > 1) o.part[blockIdx.x] = r;
        else if (info) info[b] = r;
    }
}

// Deferred top-level corrections (see Opts), every level in one launch.  The correction of a
// shifted level-d node c (step s = 2^(T-1-d) chunks) subtracts C times the minor one subtree to
// the left from each minor of its strict right subtree: chunk c + u, offset j takes chunk
// c + u - s, offset j (all but the node's own minor, u = j = 0).  For a fixed in-chunk offset j
// the corrections of all levels act on the 2^T values at offsets j of the chunks only, so a
// thread holds those values in registers and applies the levels deepest first, with the same
// operations as the in-wavefront path.  Work items: (listed matrix, tile of 256 offsets).
// The workgroups also combine the info codes of split matrices; the last one to finish clears
// the slots that were used and resets the queue's counters.
constexpr int kTopFixThreads = 512;   // two work items in flight per workgroup (256 threads each)

template <class F, int N, int K0MAX>
__global__ __launch_bounds__(kTopFixThreads) void fpm_topfix_kernel(int* topq, int cap, int f64, const int* part,
                                                                    int split, int32_t* info, int batch)
{
    using P = Plan<N, K0MAX>;
    constexpr int T = P::T, K = P::K;
    constexpr int kSub = kTopFixThreads / 256;
    const int tid = threadIdx.x;
    __shared__ int last_s;
    int count = 0;
    if constexpr (T > 0 && T <= kTopDeferMaxT) {
        constexpr int NC = 1 << T;
        constexpr int kTiles = (1 << K) / 256;
        static_assert(kTiles >= 1 && (1 << K) % 256 == 0, "chunks hold whole tiles");
        using V = typename F::V;
        const int* list = topq + kTopHead + (int64_t)cap * kTopEntryInts;
        count = __hip_atomic_load(topq, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        if (count > cap) count = cap;
        for (int64_t w = (int64_t)blockIdx.x * kSub + (tid >> 8); w < (int64_t)count * kTiles; w += (int64_t)gridDim.x * kSub) {
            const int* ent = topq + kTopHead + (int64_t)list[w / kTiles] * kTopEntryInts;
            const int64_t j = (w % kTiles) * 256 + (tid & 255);
            void* out = reinterpret_cast<void*>((uint64_t)(uint32_t)ent[0] | ((uint64_t)(uint32_t)ent[1] << 32));
            int16_t* ex = reinterpret_cast<int16_t*>((uint64_t)(uint32_t)ent[2] | ((uint64_t)(uint32_t)ent[3] << 32));
            const int es = ent[4];
            int cw[(NC + 3) / 4];
#pragma unroll
            for (int k = 0; k < (NC + 3) / 4; ++k) cw[k] = ent[kTopCodes + k];
            auto code = [&](int c) { return (int)(int8_t)(cw[c >> 2] >> (8 * (c & 3))); };
            // chunks written (right subtrees) and read (left subtrees)
            uint32_t wm = 0, rm = 0;
#pragma unroll
            for (int c = 1; c < NC; ++c) {
                if (code(c) != kNoEv) {
                    const int st = c & -c;
                    wm |= ((1u << st) - 1) << c;
                    rm |= ((1u << st) - 1) << (c - st);
                }
            }
            V x[NC];
#pragma unroll
            for (int c = 0; c < NC; ++c) {
                x[c] = V{};
                if (((wm | rm) >> c) & 1u) x[c] = F::load_v(out, ex, ((int64_t)c << K) + j, f64 != 0);
            }
#pragma unroll
            for (int lv = 0; lv < T; ++lv) {            // deepest level first: step 1, 2, 4, ...
                const int st = 1 << lv;
#pragma unroll
                for (int c = st; c < NC; c += 2 * st) {
                    const int de = code(c);
                    if (de == kNoEv) continue;
                    const double Ct = shift_value(es, de);
#pragma unroll
                    for (int u = 0; u < st; ++u)
                        if (u != 0 || j != 0) x[c + u] = F::sub_scaled(x[c + u], Ct, x[c + u - st]);
                }
            }
#pragma unroll
            for (int c = 0; c < NC; ++c)
                if ((wm >> c) & 1u) F::store_v(out, ex, ((int64_t)c << K) + j, x[c], f64 != 0);
        }
    }
    if (split > 1 && info) {
        // info of a split matrix: the first error code of its items, else their shift counts summed
        for (int b = blockIdx.x * kTopFixThreads + tid; b < batch; b += gridDim.x * kTopFixThreads) {
            int sum = 0, err = 0;
            for (int k = 0; k < split; ++k) {
                const int r = part[(int64_t)b * split + k];
                if (r < 0 && err == 0) err = r;
                sum += r < 0 ? 0 : r;
            }
            info[b] = err ? err : sum;
        }
    }
    // The group's reads of the queue are complete here (each wave used their values before
    // the barrier), so relaxed counts suffice: the last group clears only what every other
    // group has finished reading, and no group reads another's corrections.  (A device-scope
    // fence in every group would write back each XCD's L2 once per group.)  Two levels of
    // counts, kTopCounts partial ones (by group index modulo kTopCounts) and one over those,
    // so that no single address takes one atomic per group.
    __syncthreads();
    if (tid == 0) {
        const int np = (int)gridDim.x < kTopCounts ? (int)gridDim.x : kTopCounts;
        const int r = (int)(blockIdx.x % kTopCounts);
        const int per = ((int)gridDim.x - r + kTopCounts - 1) / kTopCounts;   // groups with index r mod kTopCounts
        bool last = false;
        if (__hip_atomic_fetch_add(topq + 2 + r, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) == per - 1)
            last = __hip_atomic_fetch_add(topq + 1, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) == np - 1;
        last_s = last;
    }
    __syncthreads();
    if (last_s) {
        if constexpr (T > 0 && T <= kTopDeferMaxT) {
            // clear the codes and flags of the listed slots (the next launch fills them anew)
            const int* list = topq + kTopHead + (int64_t)cap * kTopEntryInts;
            constexpr int kClr = kTopEntryInts - kTopCodes;
            for (int64_t k = tid; k < (int64_t)count * kClr; k += kTopFixThreads)
                topq[kTopHead + (int64_t)list[k / kClr] * kTopEntryInts + kTopCodes + k % kClr] = 0;
        }
        if (tid < kTopCounterInts) atomicExch(topq + tid, 0);
    }
}

}  // namespace apm


// ------------------------------------------------------------------------- host side
namespace apm {

// Lane-subtree order K0 per field and matrix order: an explicit request (autotuning), then
// APM_K0=<k>, then the value the autotuner installed for this (dtype, order), then the
// default table measured on MI355X.  Values outside the instantiated set fall back.
template <class F>
struct K0Set;
template <> struct K0Set<FR64> { static constexpr int lo = 3, hi = 5; };
template <> struct K0Set<FR32S> { static constexpr int lo = 3, hi = 5; };
template <> struct K0Set<FC128> { static constexpr int lo = 2, hi = 3; };
template <> struct K0Set<FC64S> { static constexpr int lo = 3, hi = 4; };

template <class F>
int default_k0(int n);

inline int env_k0()
{
    const char* e = getenv("APM_K0");
    return e ? atoi(e) : 0;
}

template <class F> struct SplitOf;
template <> struct SplitOf<FR64> { static constexpr int v = 2; };
template <> struct SplitOf<FR32S> { static constexpr int v = 4; };
template <> struct SplitOf<FC128> { static constexpr int v = 2; };
template <> struct SplitOf<FC64S> { static constexpr int v = 1; };
static_assert(SplitOf<FR64>::v <= kSplit && SplitOf<FR32S>::v <= kSplit && SplitOf<FC128>::v <= kSplit &&
                  SplitOf<FC64S>::v <= kSplit, "the queue holds kSplit info codes per matrix");

// Workgroups of the deferred-correction launch.  Few matrices with top-level shifts (the usual
// case) make a launch of many workgroups cost more than their work (8192 x 16 stressed batch:
// 1024 groups of 256 threads 19 us, 256 groups 11 us); two items per group keep the loads of
// a batch that is shifted throughout in flight.
constexpr int kTopFixGroups = 256;

template <class F, int N, int K0>
hipError_t launch_uniform(const LaunchMinors& L, hipStream_t st)
{
    using Ly = Lay<F, N, K0>;
    auto kern = fpm_uniform_kernel<F, N, K0>;
    if (Ly::bytes > 65536) {
        hipError_t e = hipFuncSetAttribute((const void*)kern, hipFuncAttributeMaxDynamicSharedMemorySize,
                                           (int)Ly::bytes);
        if (e != hipSuccess) return e;
    }
    constexpr int T = Plan<N, K0>::T;
    constexpr bool kDefer = T > 0 && T <= kTopDeferMaxT;
    int* topq = kDefer ? L.topq : nullptr;
    // split matrices into work items (the queue holds a slot per matrix and an info code
    // per item of kSplit): with one wavefront per matrix, a few matrices with many shifted
    // pivots (whose corrections reread their minors) or a batch of few matrices set the end
    // of the launch.  Items per matrix by type, measured on MI355X: fp64 2 (stressed 8192 x
    // 16 batch 1.00 -> 0.97 ms; unstressed 0.92 -> 0.935), fp32-scaled 4 (stressed batch
    // 1.46 -> 1.10 ms), complex128 2 (4096 x 14 Keldysh 0.602 -> 0.582 ms), complex64-scaled
    // 1 (the same batch 0.304 ms; 2 items 0.309, 4 items 0.327).
    const int split = (topq && !L.no_split) ? (SplitOf<F>::v < (1 << T) ? SplitOf<F>::v : (1 << T)) : 1;
    int* part = topq ? topq + kTopHead + (int64_t)L.topq_cap * (kTopEntryInts + 1) : nullptr;
    Opts o{L.tau, L.perturb, L.out_f64, topq, topq ? L.topq_cap : 0, split, part};
    hipLaunchKernelGGL(kern, dim3((unsigned)((int64_t)L.batch * split)), dim3(64), Ly::bytes, st,
                       static_cast<const typename F::In*>(L.A), L.out, L.ex, L.info, L.batch, L.in_off, L.out_off, o);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess || !topq) return e;
    hipLaunchKernelGGL((fpm_topfix_kernel<F, N, K0>), dim3(kTopFixGroups), dim3(kTopFixThreads), 0, st, topq, o.topq_cap,
                       L.out_f64 ? 1 : 0, part, split, L.info, L.batch);
    return hipGetLastError();
}

template <class F, int N, int K0>
hipError_t dispatch_k0(int k0, const LaunchMinors& L, hipStream_t st)
{
    if constexpr (K0 > K0Set<F>::hi) {
        return launch_uniform<F, N, K0Set<F>::hi>(L, st);
    } else {
        if (k0 <= K0) return launch_uniform<F, N, K0>(L, st);
        return dispatch_k0<F, N, K0 + 1>(k0, L, st);
    }
}

template <class F, int N>
hipError_t dispatch_n(const LaunchMinors& L, hipStream_t st)
{
    if constexpr (N > 20) {
        return hipErrorInvalidValue;
    } else {
        if (L.n_uniform == N) {
            int k = L.force_k0;
            if (k <= 0) k = env_k0();
            if (k <= 0) k = tuned_k0(F::kId, N);
            if (k <= 0) k = default_k0<F>(N);
            return dispatch_k0<F, N, K0Set<F>::lo>(k, L, st);
        }
        return dispatch_n<F, N + 1>(L, st);
    }
}

// ----------------------------------------------------------------- ragged batches
// Lane-subtree order of the persistent mixed-order kernel by default: one below the largest,
// which keeps the merged kernel at two wavefronts per SIMD.  Instantiated range (the
// autotuner picks within it): that order and the one below.
template <class F>
constexpr int ragged_k0()
{
    return K0Set<F>::hi > K0Set<F>::lo ? K0Set<F>::hi - 1 : K0Set<F>::hi;
}
template <class F> struct RaggedK0 {
    static constexpr int hi = ragged_k0<F>();
    static constexpr int lo = hi - 1 >= K0Set<F>::lo ? hi - 1 : hi;
};

// Orders run by fpm_ragged_big_kernel (below) when a mixed batch contains them; its lane-
// subtree order is the largest by default, and the one below is instantiated too.
constexpr int kBigLo = 14, kBigHi = 16;
template <class F> struct BigK0 {
    static constexpr int hi = K0Set<F>::hi;
    static constexpr int lo = hi - 1 >= K0Set<F>::lo ? hi - 1 : hi;
};

// One order per (non-inlined) function, so that each keeps its own register allocation.
template <class F, int N, int K0R>
__device__ __noinline__ int fpm_wave_n(const typename F::In* A, void* ob, int16_t* eb, unsigned char* lds, Opts o)
{
    return fpm_wave<F, N, K0R>(A, ob, eb, lds, o);
}

template <class F, int N, int K0R>
__device__ __forceinline__ int fpm_dispatch(int n, const typename F::In* A, void* ob, int16_t* eb, unsigned char* lds,
                                            const Opts& o)
{
    if constexpr (N > 20) {
        return -1;
    } else if constexpr (N >= kBigLo && N <= kBigHi) {
        return fpm_dispatch<F, kBigHi + 1, K0R>(n, A, ob, eb, lds, o);   // fpm_ragged_big_kernel's orders
    } else {
        if (n == N) return fpm_wave_n<F, N, K0R>(A, ob, eb, lds, o);
        return fpm_dispatch<F, N + 1, K0R>(n, A, ob, eb, lds, o);
    }
}

// A persistent kernel's positions in the queue are split into kStreams interleaved streams
// (position p in stream p mod kStreams); workgroup g serves stream g mod kStreams, which takes
// consecutive workgroups to different XCDs.  Its first position is g itself; later ones come
// from the stream's own head (an atomic counter), so that the heads' atomics are spread over
// kStreams addresses instead of one.  Each stream keeps the queue order (largest first).
constexpr int kStreams = 8;
constexpr int kSmallHeads = 32, kBigHeads = 48;   // heads (every second int) in the counter block
// queue position of a workgroup's first item (its own index) and of the later ones (from the
// head of its stream)
__device__ __forceinline__ int stream_first() { return (int)blockIdx.x; }

__device__ __forceinline__ int stream_pop(int32_t* heads)
{
    const int x = (int)(blockIdx.x % kStreams);
    int j = 0;
    if (lane_id() == 0) j = atomicAdd(heads + 2 * x, 1);
    // the stream's first positions are the first items of the workgroups that serve it
    j = __builtin_amdgcn_readfirstlane(__shfl(j, 0)) + ((int)gridDim.x - x + kStreams - 1) / kStreams;
    return x + kStreams * j;
}

// Persistent waves over the prepared queue, skipping the matrices of orders kBigLo..kBigHi
// (a contiguous range of the queue order, left to fpm_ragged_big_kernel); each matrix is
// handled by the code for its order.
template <class F, int K0R>
__global__ __launch_bounds__(64) __attribute__((amdgpu_waves_per_eu(2))) void fpm_ragged_kernel(const typename F::In* __restrict__ A, void* out, int16_t* ex,
                                                        int32_t* info, int32_t batch, const int32_t* __restrict__ nv,
                                                        const int64_t* __restrict__ in_off,
                                                        const int64_t* __restrict__ out_off,
                                                        const int32_t* __restrict__ order, int32_t* counter, Opts o)
{
    extern __shared__ __align__(16) unsigned char lds_dyn[];
    const int lo = counter[kBucketBase + 20 - kBigHi];
    const int gap = counter[kBucketBase + 21 - kBigLo] - lo;
    for (int p = stream_first();; p = stream_pop(counter + kSmallHeads)) {
        const int i = p >= lo ? p + gap : p;
        if (i >= batch) break;
        const int b = order[i];
        const int n = nv[b];
        int r = -1;
        if (n >= 1 && n <= 20 && !(n >= kBigLo && n <= kBigHi)) {
            const int64_t io = in_off[b];
            const int64_t oo = out_off[b];
            void* ob;
            if constexpr (F::kComplex) {
                ob = (o.out_f64 || !F::kScaled) ? (void*)(static_cast<cd*>(out) + oo)
                                                : (void*)(static_cast<cf*>(out) + oo);
            } else {
                ob = (o.out_f64 || !F::kScaled) ? (void*)(static_cast<double*>(out) + oo)
                                                : (void*)(static_cast<float*>(out) + oo);
            }
            int16_t* eb = ex ? ex + oo : nullptr;
            r = fpm_dispatch<F, 1, K0R>(n, A + io, ob, eb, lds_dyn, o);
        }
        if (info && lane_id() == 0) info[b] = r;
        wave_sync();
    }
}

// The large orders of a mixed batch (kBigLo..kBigHi) run in a kernel of their own with the
// largest lane-subtree order: with only these orders inlined, the merged kernel keeps two
// wavefronts per SIMD.  The matrices of these orders are a contiguous range of the queue
// order (sorted by decreasing order), which this kernel walks with its own counter.

template <class F, int N, int K0B>
__device__ __forceinline__ int fpm_dispatch_big(int n, const typename F::In* A, void* ob, int16_t* eb,
                                                unsigned char* lds, const Opts& o)
{
    if constexpr (N > kBigHi) {
        return -1;
    } else {
        if (n == N) return fpm_wave<F, N, K0B>(A, ob, eb, lds, o);
        return fpm_dispatch_big<F, N + 1, K0B>(n, A, ob, eb, lds, o);
    }
}

template <class F, int K0B>
__global__ __launch_bounds__(64) __attribute__((amdgpu_waves_per_eu(2))) void fpm_ragged_big_kernel(
    const typename F::In* __restrict__ A, void* out, int16_t* ex, int32_t* info, const int32_t* __restrict__ nv,
    const int64_t* __restrict__ in_off, const int64_t* __restrict__ out_off, const int32_t* __restrict__ order,
    int32_t* counter, Opts o)
{
    extern __shared__ __align__(16) unsigned char lds_dyn[];
    const int lo = counter[kBucketBase + 20 - kBigHi], hi = counter[kBucketBase + 21 - kBigLo];
    for (int p = stream_first();; p = stream_pop(counter + kBigHeads)) {
        const int i = p + lo;
        if (i >= hi) break;
        const int b = order[i];
        const int n = nv[b];
        const int64_t oo = out_off[b];
        void* ob;
        if constexpr (F::kComplex) {
            ob = (o.out_f64 || !F::kScaled) ? (void*)(static_cast<cd*>(out) + oo) : (void*)(static_cast<cf*>(out) + oo);
        } else {
            ob = (o.out_f64 || !F::kScaled) ? (void*)(static_cast<double*>(out) + oo)
                                            : (void*)(static_cast<float*>(out) + oo);
        }
        const int r = fpm_dispatch_big<F, kBigLo, K0B>(n, A + in_off[b], ob, ex ? ex + oo : nullptr, lds_dyn, o);
        if (info && lane_id() == 0) info[b] = r;
        wave_sync();
    }
}

// LDS of the orders up to nmax that each kernel runs
template <class F, int N, int K0R>
size_t lay_bytes_upto(int nmax)
{
    if constexpr (N > 20) {
        return 0;
    } else {
        const size_t a = (N <= nmax && !(N >= kBigLo && N <= kBigHi)) ? Lay<F, N, K0R>::bytes : 0;
        const size_t b = lay_bytes_upto<F, N + 1, K0R>(nmax);
        return a > b ? a : b;
    }
}

template <class F, int N, int K0B>
size_t big_lay_bytes_upto(int nmax)
{
    if constexpr (N > kBigHi) {
        return 0;
    } else {
        const size_t a = N <= nmax ? Lay<F, N, K0B>::bytes : 0;
        const size_t b = big_lay_bytes_upto<F, N + 1, K0B>(nmax);
        return a > b ? a : b;
    }
}

// Persistent grid: as many workgroups as fit on the compute units at once.
template <class Kern>
hipError_t ragged_grid(Kern kern, size_t bytes, int cus, int64_t batch, int64_t* grid)
{
    if (bytes > 65536) {
        const hipError_t e = hipFuncSetAttribute((const void*)kern, hipFuncAttributeMaxDynamicSharedMemorySize,
                                                 (int)bytes);
        if (e != hipSuccess) return e;
    }
    int per_cu = 0;
    const hipError_t e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, (const void*)kern, 64, bytes);
    if (e != hipSuccess) return e;
    if (per_cu < 1) per_cu = 1;
    *grid = (int64_t)per_cu * cus;
    if (*grid > batch) *grid = batch;
    return hipSuccess;
}

template <class F, int K0R>
hipError_t launch_ragged_small(int k0, const LaunchMinors& L, const int64_t* ioff, const int64_t* ooff, const Opts& o,
                               int cus, hipStream_t st)
{
    if constexpr (K0R < RaggedK0<F>::hi) {
        if (k0 > K0R) return launch_ragged_small<F, K0R + 1>(k0, L, ioff, ooff, o, cus, st);
    }
    const size_t bytes = lay_bytes_upto<F, 1, K0R>(L.n_max);
    auto kern = fpm_ragged_kernel<F, K0R>;
    int64_t grid = 0;
    hipError_t e = ragged_grid(kern, bytes, cus, L.batch, &grid);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(kern, dim3((unsigned)grid), dim3(64), bytes, st, static_cast<const typename F::In*>(L.A), L.out,
                       L.ex, L.info, L.batch, L.n, ioff, ooff, L.order, L.counter, o);
    return hipGetLastError();
}

template <class F, int K0B>
hipError_t launch_ragged_big(int k0, const LaunchMinors& L, const int64_t* ioff, const int64_t* ooff, const Opts& o,
                             int cus, hipStream_t st)
{
    if constexpr (K0B < BigK0<F>::hi) {
        if (k0 > K0B) return launch_ragged_big<F, K0B + 1>(k0, L, ioff, ooff, o, cus, st);
    }
    const size_t bytes = big_lay_bytes_upto<F, kBigLo, K0B>(L.n_max);
    auto kern = fpm_ragged_big_kernel<F, K0B>;
    int64_t grid = 0;
    hipError_t e = ragged_grid(kern, bytes, cus, L.batch, &grid);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(kern, dim3((unsigned)grid), dim3(64), bytes, st, static_cast<const typename F::In*>(L.A), L.out,
                       L.ex, L.info, L.n, ioff, ooff, L.order, L.counter, o);
    return hipGetLastError();
}

// Mixed orders: the queue preparation, then the orders kBigLo..kBigHi (their own kernel)
// and the rest.  Lane-subtree orders: an explicit request (force_k0 / force_k0_big,
// autotuning and plans), else the autotuner's choice for the type, else the defaults.
template <class F>
hipError_t fpm_launch_ragged(const LaunchMinors& L, hipStream_t st)
{
    const int64_t* ioff = L.in_off ? L.in_off : L.ioff_ws;
    const int64_t* ooff = L.out_off ? L.out_off : L.ooff_ws;
    hipError_t e = fpm_prep_launch(L, st);
    if (e != hipSuccess) return e;
    const int cus = L.n_workers > 0 ? L.n_workers : 256;
    Opts o{L.tau, L.perturb, L.out_f64, nullptr, 0, 1, nullptr};   // mixed orders: corrections in the wavefront
    auto pick = [](int forced, int tuned, int def, int lo, int hi) {
        int k = forced > 0 ? forced : (tuned > 0 ? tuned : def);
        return k < lo ? lo : (k > hi ? hi : k);
    };
    if (L.n_max >= kBigLo) {
        const int kb = pick(L.force_k0_big, tuned_mixed_k0(F::kId, 1), BigK0<F>::hi, BigK0<F>::lo, BigK0<F>::hi);
        e = launch_ragged_big<F, BigK0<F>::lo>(kb, L, ioff, ooff, o, cus, st);
        if (e != hipSuccess) return e;
    }
    const int ks = pick(L.force_k0, tuned_mixed_k0(F::kId, 0), RaggedK0<F>::hi, RaggedK0<F>::lo, RaggedK0<F>::hi);
    return launch_ragged_small<F, RaggedK0<F>::lo>(ks, L, ioff, ooff, o, cus, st);
}

template <class F>
hipError_t fpm_launch_field(const LaunchMinors& L, hipStream_t st)
{
    if (L.n_uniform <= 0) return fpm_launch_ragged<F>(L, st);
    return dispatch_n<F, 1>(L, st);
}

}  // namespace apm
